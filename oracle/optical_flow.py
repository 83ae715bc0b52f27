"""FP64 optical-flow temporal regulariser of dynamic NL-RMM-GKS (test infrastructure only).

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may use this module; it imports nothing from the product package.

What it computes (Section 7, "Optical Flow Regularization (OF)", eqs. "of_forward" and
"Theta_OF", and the OF branch of Alg. "dyn_nl_rmmgks"):
  * velocity estimation (SOLVE-OF) for one frame pair (u0 = u(t), u1 = u(t+1)): the
    minimiser of || Y(u0) s + u_t ||^2 + gamma || L s ||^2 + ridge || s ||^2 over the velocity
    s = (s_x, s_y) (one pair of values per pixel), with Y(u0) = [diag(d_x u0), diag(d_y u0)]
    the spatial image gradients, u_t = u1 - u0 the temporal difference and L the forward
    differences of each velocity component;
  * the bilinear warp M(s): (M(s) v) at pixel (k, l) is v sampled at (k + s_x, l + s_y)
    (pixel units) by bilinear interpolation;
  * the motion rows of Theta: for t = 0 .. F-2, the forward consistency u(t) - M(s(t)) u(t+1)
    and the reverse consistency u(t+1) - M(s'(t)) u(t), with the reverse flow s' = -s.

Readings where the paper is silent or does not compose (listed in the design notes):
  * p = q = 2 in eq. "of_forward" (the Horn-Schunck form), with gamma fixed (default 0.05)
    instead of GCV and a ridge (default 1e-3) that makes the normal equations definite
    where the image is flat; solved exactly (sparse LU of the normal equations);
  * Y(u0) from central differences of frame t (one-sided at the borders), in pixel units;
  * L = unscaled forward differences along x and y, none across the border;
  * the warp's sample position is clamped to the grid [0, nx-1] x [0, ny-1];
  * the reverse flow is s' = -s (the first-order form of the OFC relation between the two
    flows);
  * M_hat stacks the forward rows M_bar(s) and the reverse rows M_bar'(s') with the same
    shape ((F-1) frame blocks acting on the F frames): the transposed reverse block as
    printed maps the other way and cannot be stacked with M_bar as an operator on u.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def spatial_gradients(U):
    """Central differences of a frame U [ny, nx] along x (fast index) and y, one-sided at
    the borders, in pixel units."""
    U = np.asarray(U, dtype=np.float64)
    gx = np.empty_like(U)
    gy = np.empty_like(U)
    gx[:, 1:-1] = 0.5 * (U[:, 2:] - U[:, :-2])
    gx[:, 0] = U[:, 1] - U[:, 0]
    gx[:, -1] = U[:, -1] - U[:, -2]
    gy[1:-1, :] = 0.5 * (U[2:, :] - U[:-2, :])
    gy[0, :] = U[1, :] - U[0, :]
    gy[-1, :] = U[-1, :] - U[-2, :]
    return gx, gy


def forward_differences(ny, nx):
    """Sparse [D_x; D_y]: forward differences along x ((nx-1) per row) then along y."""
    dx1 = sp.diags([-np.ones(nx - 1), np.ones(nx - 1)], [0, 1], shape=(nx - 1, nx))
    dy1 = sp.diags([-np.ones(ny - 1), np.ones(ny - 1)], [0, 1], shape=(ny - 1, ny))
    return sp.vstack([sp.kron(sp.identity(ny), dx1), sp.kron(dy1, sp.identity(nx))]).tocsr()


def flow_system(u0, u1, gamma, ridge):
    """Normal equations (Y^T Y + gamma L_hat^T L_hat + ridge I) s = -Y^T u_t of the velocity
    problem, with L_hat = blockdiag(L, L) acting on s = [s_x; s_y]."""
    u0 = np.asarray(u0, dtype=np.float64)
    ny, nx = u0.shape
    gx, gy = spatial_gradients(u0)
    ut = (np.asarray(u1, dtype=np.float64) - u0).ravel()
    Y = sp.hstack([sp.diags(gx.ravel()), sp.diags(gy.ravel())]).tocsr()
    L = forward_differences(ny, nx)
    Lh = sp.block_diag([L, L]).tocsr()
    A = (Y.T @ Y + gamma * (Lh.T @ Lh) + ridge * sp.identity(2 * nx * ny)).tocsc()
    return A, -(Y.T @ ut), Y, Lh, ut


def flow_objective(s, Y, Lh, ut, gamma, ridge):
    """|| Y s + u_t ||^2 + gamma || L_hat s ||^2 + ridge || s ||^2."""
    r = Y @ s + ut
    g = Lh @ s
    return float(r @ r + gamma * (g @ g) + ridge * (s @ s))


def solve_flow(u0, u1, gamma=0.05, ridge=1e-3):
    """SOLVE-OF for one frame pair: velocity (s_x, s_y), each [ny, nx], from u0 to u1."""
    ny, nx = np.asarray(u0).shape
    A, rhs, _, _, _ = flow_system(u0, u1, gamma, ridge)
    s = spla.spsolve(A, rhs)
    n = nx * ny
    return s[:n].reshape(ny, nx), s[n:].reshape(ny, nx)


def warp_matrix(sx, sy):
    """Sparse bilinear warp M(s): row (l, k) samples at (k + s_x, l + s_y), clamped to the
    grid; cell corner (k0, l0) = the floor, kept at most (nx-2, ny-2)."""
    sx = np.asarray(sx, dtype=np.float64)
    sy = np.asarray(sy, dtype=np.float64)
    ny, nx = sx.shape
    K, Lr = np.meshgrid(np.arange(nx), np.arange(ny))
    px = np.clip(K + sx, 0.0, nx - 1.0)
    py = np.clip(Lr + sy, 0.0, ny - 1.0)
    k0 = np.minimum(np.floor(px).astype(np.int64), nx - 2)
    l0 = np.minimum(np.floor(py).astype(np.int64), ny - 2)
    fx = px - k0
    fy = py - l0
    rows = np.repeat(np.arange(nx * ny), 4)
    cols = np.stack([l0 * nx + k0, l0 * nx + k0 + 1, (l0 + 1) * nx + k0,
                     (l0 + 1) * nx + k0 + 1], axis=-1).reshape(-1)
    vals = np.stack([(1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy],
                    axis=-1).reshape(-1)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nx * ny, nx * ny))


class Flow:
    """Velocities of every frame pair and their warps (forward s, reverse s' = -s)."""

    def __init__(self, sx, sy):
        self.sx = [np.asarray(a, dtype=np.float64) for a in sx]
        self.sy = [np.asarray(a, dtype=np.float64) for a in sy]
        self.M = [warp_matrix(a, b) for a, b in zip(self.sx, self.sy)]
        self.Mr = [warp_matrix(-a, -b) for a, b in zip(self.sx, self.sy)]


def estimate_flow(U, gamma=0.05, ridge=1e-3):
    """SOLVE-OF for every consecutive pair of the frames U [F, ny, nx]."""
    sx, sy = [], []
    for t in range(U.shape[0] - 1):
        a, b = solve_flow(U[t], U[t + 1], gamma, ridge)
        sx.append(a)
        sy.append(b)
    return Flow(sx, sy)


def motion_rows(U, flow: Flow):
    """[M_bar(s) u; M_bar'(s') u] of frames U [F, ny, nx]: (F-1) blocks of forward
    consistency u(t) - M(s(t)) u(t+1), then (F-1) blocks of reverse consistency
    u(t+1) - M(s'(t)) u(t)."""
    F = U.shape[0]
    fwd = [U[t].ravel() - flow.M[t] @ U[t + 1].ravel() for t in range(F - 1)]
    rev = [U[t + 1].ravel() - flow.Mr[t] @ U[t].ravel() for t in range(F - 1)]
    return np.concatenate(fwd + rev)


def motion_rows_t(z, F, ny, nx, flow: Flow):
    """Transpose of ``motion_rows``: frames [F, ny, nx] from the stacked rows z."""
    n = nx * ny
    U = np.zeros((F, n))
    for t in range(F - 1):
        zf = z[t * n:(t + 1) * n]
        U[t] += zf
        U[t + 1] -= flow.M[t].T @ zf
    off = (F - 1) * n
    for t in range(F - 1):
        zr = z[off + t * n:off + (t + 1) * n]
        U[t + 1] += zr
        U[t] -= flow.Mr[t].T @ zr
    return U.reshape(F, ny, nx)
