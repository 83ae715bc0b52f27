"""FP64 NumPy oracle of NL-RMM-GKS (AltMin and VarPro, streaming, dynamic ANISO-TV).

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use this module.  It imports nothing
from the product package; its operator is the C oracle in ``strip_oracle.c``.

Each function follows the paper's algorithm in the paper's order:
  * majorant weights ......... Section 3.1 (P_eps) and Alg. "mmgks" (w = ((Psi u)^2 + eps^2)^(-1/2))
  * projected solve .......... Section 3.2, eq. "reduced_problem" (QR of HV and of P Psi V)
  * discrepancy principle .... Section 3.2 (lambda by DP on the reduced problem)
  * Enlarge / Compress ....... supplementary Alg. "enlarge", Alg. "compress", Section 3.3
  * RMM-GKS append ........... Alg. "rmmgks" (weights, residual, projection, append)
  * UPDATE-PARAM ............. Alg. "update_param" (damped Gauss-Newton + Armijo)
  * VarPro ................... Section 4.2 eqs. "u_closed_form", "GN_system", supplementary
                               Alg. "update_varpro"
  * full-space sensitivity ... Section 4.2, eq. "sensitivity" for one global offset (dense,
                               and by a fixed number of CG steps as a parameter update with
                               Armijo on the reduced objective with u(p) to first order)
  * grid-search start ........ experiments section, "Parameter initialization" (one
                               global offset, reduced least squares on a GKB basis)
  * NL-RMM-GKS ............... Alg. "nl_rmmgks_two_solves", with the optional
                               high-regularisation solve of Section 4.3 (lam_hi)
  * s-NL-RMM-GKS ............. Alg. "s_nl_rmmgks_final"
  * dynamic ANISO-TV ......... Section 7 (operator D1, block-diagonal H)
  * dynamic optical flow ..... Section 7 (SOLVE-OF, eq. "of_forward"; Theta = [Psi; M_hat],
                               eq. "Theta_OF"; velocities from the current image at the start
                               of every outer iteration, Alg. "dyn_nl_rmmgks"), in
                               ``optical_flow.py``

Readings where the paper is silent (all listed in the design notes):
  eps = 1e-3; Psi = unscaled forward differences, (N-1) per line; DP target
  tau*delta with tau = 1.01 and delta the exact noise norm, log-bisection on
  [1e-10, 1e10] * tr(RA^T RA)/tr(RP^T RP); S = kmax - kmin solves per Enlarge
  and no append after the last solve; compression keeps the kmin-1 largest
  right singular vectors plus the normalised remainder of u; GN damping
  mu = 1e-6 * mean(diag), c1 = 1e-4, beta = 1/2, alpha0 = 1, 10 trials,
  one global alpha, maxiter_p = 1; VarPro weights B = diag(sqrt(w)) Psi V with w
  from the current image; GKB start basis of kmin+1 vectors from b, u0 = 0; the
  high-regularisation solve is one RMM-GKS cycle of S fixed-lambda solves from the
  compressed primary basis (kmin columns) and u_{k+1}.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np
from scipy.linalg import solve_triangular, cho_factor, cho_solve

from . import optical_flow as OF
from . import projector as P

# status bits (same meaning as the HIP library's device status word)
ST_BREAKDOWN = 1
ST_DP_LOW = 2
ST_DP_HIGH = 4
ST_ARMIJO = 8
ST_NONFINITE = 16
ST_COMPRESS_SKIP = 32


# ----------------------------------------------------------------------------
# operators
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Geometry:
    """Image grid, detector and frame structure (N x N per frame)."""
    N: int
    nb: int
    view_off: np.ndarray           # int64 [F + 1]
    temporal: bool = False         # dynamic: add the temporal difference L_t
    flow: Optional[OF.Flow] = None  # dynamic OF: motion rows in place of L_t

    @property
    def F(self) -> int:
        return int(self.view_off.shape[0] - 1)

    @property
    def V(self) -> int:
        return int(self.view_off[-1])

    @property
    def n(self) -> int:
        return self.F * self.N * self.N

    @property
    def m(self) -> int:
        return self.V * self.nb


def A(geo: Geometry, theta, x):
    """Forward projection of an image vector (length n) -> sinogram vector (length m)."""
    X = np.asarray(x).reshape(geo.F, geo.N, geo.N)
    return P.project(X, theta, geo.nb, geo.view_off).reshape(-1)


def AT(geo: Geometry, theta, y):
    """Backprojection (exact adjoint of ``A``)."""
    Y = np.asarray(y).reshape(geo.V, geo.nb)
    return np.asarray(P.backproject(Y, theta, geo.N, geo.view_off)).reshape(-1)


def dA(geo: Geometry, theta, x):
    """Angle derivative: row block v of the result is d(A(theta) x)_v / d theta_v."""
    X = np.asarray(x).reshape(geo.F, geo.N, geo.N)
    return P.dtheta(X, theta, geo.nb, geo.view_off).reshape(-1)


def dAT(geo: Geometry, theta, y):
    """Transpose of ``dA``: sum over views of the angle-derivative weights times y."""
    Y = np.asarray(y).reshape(geo.V, geo.nb)
    return np.asarray(P.dtheta_t(Y, theta, geo.N, geo.view_off)).reshape(-1)


def A_cols(geo: Geometry, theta, X):
    """A applied to every column of X (n x k) -> m x k."""
    k = X.shape[1]
    cols = np.ascontiguousarray(X.T).reshape(k, geo.F, geo.N, geo.N)
    return P.project(cols, theta, geo.nb, geo.view_off).reshape(k, -1).T


def psi(geo: Geometry, u):
    """Regulariser Psi u (Section 2.2): per frame [D_x u; D_y u] (forward differences,
    unscaled, N-1 per line), then for dynamic problems L_t u (frame differences, ANISO-TV
    operator D1 of Section 7) or, with a velocity field, the motion rows M_hat u of the
    optical-flow operator Theta (eq. "Theta_OF")."""
    U = np.asarray(u).reshape(geo.F, geo.N, geo.N)
    parts = []
    for f in range(geo.F):
        parts.append((U[f, :, 1:] - U[f, :, :-1]).ravel())
        parts.append((U[f, 1:, :] - U[f, :-1, :]).ravel())
    if geo.flow is not None and geo.F > 1:
        parts.append(OF.motion_rows(U, geo.flow))
    elif geo.temporal and geo.F > 1:
        parts.append((U[1:] - U[:-1]).ravel())
    return np.concatenate(parts)


def psiT(geo: Geometry, s):
    """Adjoint of ``psi``."""
    N, F = geo.N, geo.F
    U = np.zeros((F, N, N))
    pos = 0
    nx = N * (N - 1)
    for f in range(F):
        dx = s[pos:pos + nx].reshape(N, N - 1)
        pos += nx
        dy = s[pos:pos + nx].reshape(N - 1, N)
        pos += nx
        U[f, :, 1:] += dx
        U[f, :, :-1] -= dx
        U[f, 1:, :] += dy
        U[f, :-1, :] -= dy
    if geo.flow is not None and F > 1:
        U += OF.motion_rows_t(s[pos:], F, N, N, geo.flow)
    elif geo.temporal and F > 1:
        dt = s[pos:].reshape(F - 1, N, N)
        U[1:] += dt
        U[:-1] -= dt
    return U.ravel()


def psi_cols(geo: Geometry, X):
    return np.stack([psi(geo, X[:, i]) for i in range(X.shape[1])], axis=1)


def npsi(geo: Geometry) -> int:
    n = geo.F * 2 * geo.N * (geo.N - 1)
    if geo.flow is not None and geo.F > 1:
        n += 2 * (geo.F - 1) * geo.N * geo.N
    elif geo.temporal and geo.F > 1:
        n += (geo.F - 1) * geo.N * geo.N
    return n


def weights(geo: Geometry, u, eps):
    """MM weights w = ((Psi u)^2 + eps^2)^(-1/2), i.e. P_eps^2 (Section 3.1)."""
    s = psi(geo, u)
    return 1.0 / np.sqrt(s * s + eps * eps)


def objective(geo: Geometry, theta, u, b, lam, eps):
    """Smoothed joint objective 1/2||A(theta)u - b||^2 + lam * sum sqrt((Psi u)^2 + eps^2)."""
    r = A(geo, theta, u) - b
    s = psi(geo, u)
    return 0.5 * float(r @ r) + lam * float(np.sum(np.sqrt(s * s + eps * eps)))


# ----------------------------------------------------------------------------
# configuration and state
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Config:
    kmin: int = 5
    kmax: int = 30
    solves: Optional[int] = None      # solves per Enlarge (default kmax - kmin)
    eps: float = 1e-3
    tau: float = 1.01                 # DP safety factor
    dp_iters: int = 200
    lam_fix: Optional[float] = None   # fixed lambda instead of DP
    lam_hi: Optional[float] = None    # high-regularisation solve for the parameter update
    gn: str = "altmin"                # "altmin" | "varpro" | "sensitivity" | "none"
    sens_iters: int = 50              # CG steps of the sensitivity equation ("sensitivity")
    param_mode: str = "per_view"      # "per_view" | "scalar" (one global shift)
    maxiter_p: int = 1
    mu_rel: float = 1e-6
    c1: float = 1e-4
    beta: float = 0.5
    alpha0: float = 1.0
    armijo_trials: int = 10
    breakdown_tol: float = 1e-10
    # optical-flow temporal regulariser (dynamic problems): velocity estimated from the
    # current image every of_every outer iterations (tau of Alg. "dyn_nl_rmmgks")
    of: bool = False
    of_gamma: float = 0.05
    of_ridge: float = 1e-3
    of_every: int = 1

    @property
    def S(self) -> int:
        return self.solves if self.solves is not None else self.kmax - self.kmin


@dataclasses.dataclass
class State:
    V: np.ndarray        # n x l, orthonormal
    AV: np.ndarray       # m x l, A(theta_k) V
    PV: np.ndarray       # npsi x l, Psi V
    u: np.ndarray        # image
    theta: np.ndarray    # angles
    z: Optional[np.ndarray] = None
    lam: float = 0.0
    status: int = 0
    log: list = dataclasses.field(default_factory=list)


# ----------------------------------------------------------------------------
# Krylov building blocks
# ----------------------------------------------------------------------------
def cgs2(V, r):
    """Classical Gram-Schmidt, applied twice, against the columns of V."""
    if V.shape[1] == 0:
        return r.copy()
    r = r - V @ (V.T @ r)
    r = r - V @ (V.T @ r)
    return r


def gkb_basis(geo: Geometry, theta, b, k):
    """Golub-Kahan bidiagonalisation of A(theta) started from b; returns the first k
    right vectors (n x k), fully reorthogonalised (Section 3.2, initial basis)."""
    beta = np.linalg.norm(b)
    U = [b / beta]
    v = AT(geo, theta, U[0])
    alpha = np.linalg.norm(v)
    Vs = [v / alpha]
    for _ in range(1, k):
        p = A(geo, theta, Vs[-1]) - alpha * U[-1]
        p = cgs2(np.stack(U, 1), p)
        beta = np.linalg.norm(p)
        U.append(p / beta)
        v = AT(geo, theta, U[-1]) - beta * Vs[-1]
        v = cgs2(np.stack(Vs, 1), v)
        alpha = np.linalg.norm(v)
        Vs.append(v / alpha)
    return np.stack(Vs, axis=1)


def solve_stacked(RA, RP, cA, lam):
    """z = argmin || [RA; sqrt(lam) RP] z - [cA; 0] || (eq. reduced_problem)."""
    l = RA.shape[1]
    M = np.vstack([RA, math.sqrt(lam) * RP])
    rhs = np.concatenate([cA, np.zeros(RP.shape[0])])
    Q, R = np.linalg.qr(M)
    return solve_triangular(R, Q.T @ rhs)


def dp_lambda(RA, RP, cA, out2, target, iters=200):
    """Discrepancy principle on the reduced problem: lambda with
    ||A V z(lambda) - b|| = target, where ||AVz - b||^2 = ||RA z - cA||^2 + out2.
    Log-bisection on a bracket scaled by tr(RA^T RA)/tr(RP^T RP); clamps to the
    bracket ends (status bit) when the root is outside it."""
    trA = float(np.sum(RA * RA))
    trP = max(float(np.sum(RP * RP)), 1e-300)
    lo = math.log(1e-10 * trA / trP)
    hi = math.log(1e10 * trA / trP)
    t2 = target * target

    def res2(lam):
        z = solve_stacked(RA, RP, cA, lam)
        d = RA @ z - cA
        return float(d @ d) + out2

    if res2(math.exp(lo)) >= t2:
        return math.exp(lo), ST_DP_LOW
    if res2(math.exp(hi)) <= t2:
        return math.exp(hi), ST_DP_HIGH
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if res2(math.exp(mid)) < t2:
            lo = mid
        else:
            hi = mid
    return math.exp(0.5 * (lo + hi)), 0


def projected_solve(st: State, b, w, cfg: Config, target):
    """One MM-GKS solve on the current basis (Alg. "enlarge", body up to u = V z):
    QR(AV), QR(P Psi V), lambda by DP (or lam_fix), reduced LS, u = V z."""
    QA, RA = np.linalg.qr(st.AV)
    RP = np.linalg.qr(np.sqrt(w)[:, None] * st.PV, mode="r")
    cA = QA.T @ b
    rout = b - QA @ cA
    out2 = float(rout @ rout)
    flag = 0
    if cfg.lam_fix is not None:
        lam = cfg.lam_fix
    else:
        lam, flag = dp_lambda(RA, RP, cA, out2, target, cfg.dp_iters)
    z = solve_stacked(RA, RP, cA, lam)
    return z, lam, RA, RP, flag


def mm_residual(geo, theta, st: State, b, w, lam, z):
    """r = A^T (A V z - b) + lam Psi^T (w * Psi u) with u = V z (normal-equation residual)."""
    u = st.V @ z
    r = AT(geo, theta, st.AV @ z - b) + lam * psiT(geo, w * psi(geo, u))
    return r


def append_direction(geo, theta, st: State, r, cfg: Config, with_projection=True):
    """Project r out of V (CGS2), normalise, append to V, A V and Psi V."""
    nr = np.linalg.norm(r)
    rp = cgs2(st.V, r)
    nrp = np.linalg.norm(rp)
    if not np.isfinite(nrp) or nrp <= cfg.breakdown_tol * max(nr, 1e-300):
        st.status |= ST_BREAKDOWN
        return False
    v = rp / nrp
    st.V = np.column_stack([st.V, v])
    if with_projection:
        st.AV = np.column_stack([st.AV, A(geo, theta, v)])
    st.PV = np.column_stack([st.PV, psi(geo, v)])
    return True


def compress(st: State, RA, RP, lam, z, kmin):
    """Alg. "compress": W = right singular vectors of the kmin-1 largest singular values of
    [RA; sqrt(lam) RP]; new basis [V W, normalised (u - V W W^T V^T u)].
    Sign rule: largest-magnitude entry of each singular vector positive."""
    H = np.vstack([RA, math.sqrt(lam) * RP])
    _, _, Wt = np.linalg.svd(H)
    W = Wt[:kmin - 1].T.copy()
    for i in range(W.shape[1]):
        j = int(np.argmax(np.abs(W[:, i])))
        if W[j, i] < 0:
            W[:, i] = -W[:, i]
    c = z - W @ (W.T @ z)
    nc = np.linalg.norm(c)
    if nc <= 1e-12 * np.linalg.norm(z):
        st.status |= ST_COMPRESS_SKIP
        T = W
        znew = W.T @ z
    else:
        T = np.column_stack([W, c / nc])
        znew = np.concatenate([W.T @ z, [nc]])
    st.V = st.V @ T
    st.AV = st.AV @ T
    st.PV = st.PV @ T
    st.z = znew
    st.u = st.V @ znew
    return T


# ----------------------------------------------------------------------------
# parameter updates
# ----------------------------------------------------------------------------
def gn_altmin(geo: Geometry, theta, u, b, cfg: Config):
    """Alg. "update_param": damped Gauss-Newton on f(theta) = 1/2||A(theta)u - b||^2.
    J's column v lives on view v's rows, so J^T J is diagonal (per-view angles)."""
    status = 0
    info = {}
    for _ in range(cfg.maxiter_p):
        r = A(geo, theta, u) - b
        D = dA(geo, theta, u).reshape(geo.V, geo.nb)
        R = r.reshape(geo.V, geo.nb)
        g = np.sum(D * R, axis=1)
        h = np.sum(D * D, axis=1)
        if cfg.param_mode == "scalar":
            g_s, h_s = g.sum(), h.sum()
            mu = cfg.mu_rel * h_s
            d = np.full(geo.V, -g_s / (h_s + mu))
            gd = g_s * d[0]
        else:
            mu = cfg.mu_rel * float(np.mean(h))
            d = -g / (h + mu)
            gd = float(g @ d)
        f0 = 0.5 * float(r @ r)
        alpha = 0.0
        for q in range(cfg.armijo_trials):
            a = cfg.alpha0 * cfg.beta ** q
            rt = A(geo, theta + a * d, u) - b
            if 0.5 * float(rt @ rt) <= f0 + cfg.c1 * a * gd:
                alpha = a
                break
        if alpha == 0.0:
            status |= ST_ARMIJO
        info = dict(g=g, h=h, d=d, alpha=alpha, f0=f0)
        theta = theta + alpha * d
    return theta, status, info


def varpro_parts(geo: Geometry, theta, V, b, Bw, lam):
    """Reduced VarPro quantities at theta on the basis V (supplementary Alg. "update_varpro"):
    A_hat = A(theta) V, M = A_hat^T A_hat + lam B^T B, y = M^-1 A_hat^T b, r = A_hat y - b."""
    Ah = A_cols(geo, theta, V)
    M = Ah.T @ Ah + lam * (Bw.T @ Bw)
    y = np.linalg.solve(M, Ah.T @ b)
    r = Ah @ y - b
    f = 0.5 * float(r @ r) + 0.5 * lam * float(np.sum((Bw @ y) ** 2))
    return Ah, M, y, r, f


def gn_varpro(geo: Geometry, theta, V, b, w, PV, lam, cfg: Config):
    """VarPro parameter update (Section 4.2, eq. "GN_system"; supplementary Alg.
    "update_varpro") with the Jacobians in the subspace V:
      Y[:, v] = -M^-1 (E_v^T r_v + A_hat_v^T e_v),   e_v = sum_c y_c E_{c,v},
      g_v = <e_v, r_v>,
      J = diag(||e_v||^2) + C Y + (C Y)^T + Y^T M Y + mu I,  C[v, c] = <e_v, A_hat_{c,v}>."""
    Bw = np.sqrt(w)[:, None] * PV
    status = 0
    info = {}
    k = V.shape[1]
    for _ in range(cfg.maxiter_p):
        Ah, M, y, r, f0 = varpro_parts(geo, theta, V, b, Bw, lam)
        E = np.stack([dA(geo, theta, V[:, c]).reshape(geo.V, geo.nb) for c in range(k)])
        R = r.reshape(geo.V, geo.nb)
        Ahv = Ah.T.reshape(k, geo.V, geo.nb)
        e = np.einsum("c,cvj->vj", y, E)
        g = np.sum(e * R, axis=1)
        ETr = np.sum(E * R[None], axis=2)            # [c, v]
        Ate = np.sum(Ahv * e[None], axis=2)          # [c, v]
        Y = -np.linalg.solve(M, ETr + Ate)           # [c, v]
        C = Ate.T                                    # [v, c]
        J = np.diag(np.sum(e * e, axis=1)) + C @ Y + (C @ Y).T + Y.T @ M @ Y
        mu = cfg.mu_rel * float(np.mean(np.diag(J)))
        J = J + mu * np.eye(geo.V)
        d = -cho_solve(cho_factor(J), g)
        gd = float(g @ d)
        alpha = 0.0
        for q in range(cfg.armijo_trials):
            a = cfg.alpha0 * cfg.beta ** q
            ft = varpro_parts(geo, theta + a * d, V, b, Bw, lam)[4]
            if ft <= f0 + cfg.c1 * a * gd:
                alpha = a
                break
        if alpha == 0.0:
            status |= ST_ARMIJO
        info = dict(g=g, d=d, alpha=alpha, f0=f0, J=J)
        theta = theta + alpha * d
    return theta, status, info


# ----------------------------------------------------------------------------
# drivers
# ----------------------------------------------------------------------------
def grid_search_shift(geo: Geometry, theta_nom, b, shifts, ell0: int = 10, V=None):
    """Parameter initialisation of the experiments section ("Parameter initialization"): a
    GKB basis V of ell0 vectors at the nominal geometry (or the given V); for every candidate
    global offset s on a coarse grid, the reduced problem min_z ||H(theta_nom + s) V z - b||
    (least squares, unregularised: ell0 is small); the candidate with the smallest data
    residual (first on ties).  Returns (theta_nom + s_best, residuals^2, best index)."""
    if V is None:
        V = gkb_basis(geo, theta_nom, b, ell0)
    res2 = []
    for s in shifts:
        AV = A_cols(geo, theta_nom + s, V)
        z, *_ = np.linalg.lstsq(AV, b, rcond=None)
        r = AV @ z - b
        res2.append(float(r @ r))
    res2 = np.array(res2)
    best = int(np.argmin(res2))
    return np.asarray(theta_nom) + shifts[best], res2, best


def offset_sensitivity(geo: Geometry, theta, u, b, w, lam):
    """Full-space sensitivity of the VarPro reduced problem for one global angle offset p
    (Section 4.2, eqs. "u_closed_form", "sensitivity", "GN_system"), dense (tiny grids):
    M = A^T A + lam Psi^T diag(w) Psi;  M u_p = -(A_p^T r + A^T A_p u) with r = A u - b and
    A_p = dA/dp = sum over views of dA/dtheta_v (every view moves with p);
    J_r = A_p u + A u_p, J_s = sqrt(w) Psi u_p;  g = J_r^T r + lam J_s^T s (s = sqrt(w) Psi u),
    h = J_r^T J_r + lam J_s^T J_s, dp = -g / h.  Returns (u_p, g, h, dp)."""
    A, dA = P.dense(geo.N, geo.nb, theta)
    n = geo.n
    Psi = np.stack([psi(geo, np.eye(n)[:, i]) for i in range(n)], axis=1)
    M = A.T @ A + lam * Psi.T @ (w[:, None] * Psi)
    r = A @ u - b
    up = np.linalg.solve(M, -(dA.T @ r + A.T @ (dA @ u)))
    Jr = dA @ u + A @ up
    Pu, Pp = Psi @ u, Psi @ up
    g = float(Jr @ r + lam * Pp @ (w * Pu))
    h = float(Jr @ Jr + lam * Pp @ (w * Pp))
    return up, g, h, -g / h


def offset_sensitivity_cg(geo: Geometry, theta, u, b, w, lam, iters):
    """The full-space sensitivity of one global angle offset p (Section 4.2, eqs.
    "sensitivity" and "GN_system") with u_p from `iters` conjugate-gradient steps started at
    0 on M = A^T A + lam Psi^T diag(w) Psi, applied matrix-free:
      M u_p = -(A_p^T r + A^T A_p u),  r = A u - b,  A_p u = dA u (every view moves with p),
      J_r = A_p u + A u_p,  g = J_r^T r + lam (Psi u_p)^T diag(w) Psi u,
      h = J_r^T J_r + lam (Psi u_p)^T diag(w) Psi u_p.
    Returns (u_p, g, h)."""
    r = A(geo, theta, u) - b
    Du = dA(geo, theta, u)
    rhs = -(dAT(geo, theta, r) + AT(geo, theta, Du))

    def Mv(x):
        return AT(geo, theta, A(geo, theta, x)) + lam * psiT(geo, w * psi(geo, x))

    x = np.zeros(geo.n)
    res = rhs.copy()
    p = res.copy()
    rr = float(res @ res)
    for _ in range(iters):
        q = Mv(p)
        pq = float(p @ q)
        alpha = rr / pq if pq != 0.0 else 0.0
        x = x + alpha * p
        res = res - alpha * q
        rr_new = float(res @ res)
        beta = rr_new / rr if rr != 0.0 else 0.0
        rr = rr_new
        p = res + beta * p
    Jr = Du + A(geo, theta, x)
    Pu, Pp = psi(geo, u), psi(geo, x)
    g = float(Jr @ r + lam * Pp @ (w * Pu))
    h = float(Jr @ Jr + lam * Pp @ (w * Pp))
    return x, g, h


def gn_sensitivity(geo: Geometry, theta, u, b, w, lam, cfg: Config):
    """Parameter update of one global angle offset from the full-space sensitivity equation
    (Section 4.2): the Gauss-Newton step dp = -g / (h + mu), mu = mu_rel h, of eq. "GN_system"
    for one parameter, with u_p, g, h from ``offset_sensitivity_cg`` at the image u, and
    Armijo backtracking on the reduced objective f(p) = 1/2||r(p)||^2 + lam/2 ||s(p)||^2 with
    u(p) replaced by its first-order expansion u + (p - p_k) u_p from the sensitivity equation
    (u(p) itself would need a full inner solve per trial); its slope at p_k is g dp.  Every
    view moves by the same alpha dp."""
    status = 0
    info = {}
    sw = np.sqrt(w)

    def f_lin(t, ua):
        r = A(geo, t, ua) - b
        s = sw * psi(geo, ua)
        return 0.5 * float(r @ r) + 0.5 * lam * float(s @ s)

    for _ in range(cfg.maxiter_p):
        up, g, h = offset_sensitivity_cg(geo, theta, u, b, w, lam, cfg.sens_iters)
        mu = cfg.mu_rel * h
        dp = -g / (h + mu) if h + mu > 0.0 else 0.0
        f0 = f_lin(theta, u)
        gd = g * dp
        alpha = 0.0
        for q in range(cfg.armijo_trials):
            a = cfg.alpha0 * cfg.beta ** q
            ft = f_lin(theta + a * dp, u + (a * dp) * up)
            if ft <= f0 + cfg.c1 * a * gd:
                alpha = a
                break
        if alpha == 0.0:
            status |= ST_ARMIJO
        info = dict(g=g, h=h, dp=dp, up=up, alpha=alpha, f0=f0)
        theta = theta + alpha * dp
    return theta, status, info


def init_state(geo: Geometry, theta0, b, cfg: Config) -> State:
    """GKB basis of kmin+1 vectors at the starting angles, u0 = 0."""
    V = gkb_basis(geo, theta0, b, cfg.kmin + 1)
    return State(V=V, AV=np.zeros((geo.m, 0)), PV=psi_cols(geo, V), u=np.zeros(geo.n),
                 theta=np.array(theta0, dtype=np.float64))


def hi_solve(geo: Geometry, theta_k, st: State, b, cfg: Config) -> State:
    """The optional high-regularisation solve of Alg. "nl_rmmgks_two_solves" (Section 4.3):
    one RMM-GKS cycle (Alg. "rmmgks") with lambda fixed at lam_hi, started from the primary
    image u_{k+1} and its compressed basis V_kmin (copies; the primary state is untouched):
    S projected solves on kmin, kmin+1, ... columns with an expansion between consecutive
    solves (Alg. "enlarge"), then Compress when the VarPro update needs the compressed basis
    (Compress leaves u = V z unchanged, so AltMin takes u_hat from the last solve).  Returns
    the state holding u_hat, its basis and lam_hi, which only the parameter update uses."""
    hs = State(V=st.V.copy(), AV=st.AV.copy(), PV=st.PV.copy(), u=st.u.copy(),
               theta=st.theta.copy())
    hcfg = dataclasses.replace(cfg, lam_fix=cfg.lam_hi)
    S = cfg.S
    for t in range(S):
        w = weights(geo, hs.u, cfg.eps)
        z, lam, RA, RP, flag = projected_solve(hs, b, w, hcfg, None)
        hs.status |= flag
        hs.z, hs.lam = z, lam
        hs.u = hs.V @ z
        if t < S - 1:
            r = mm_residual(geo, theta_k, hs, b, w, lam, z)
            append_direction(geo, theta_k, hs, r, cfg)
    if cfg.gn == "varpro":
        compress(hs, RA, RP, hs.lam, hs.z, cfg.kmin)
    return hs


def outer_step(geo: Geometry, st: State, b, delta, cfg: Config):
    """One outer iteration of NL-RMM-GKS (Alg. "nl_rmmgks_two_solves"): rebase A V at
    theta_k, Enlarge (S solves, S-1 appends), Compress, the optional high-regularisation
    solve (cfg.lam_hi), UPDATE-PARAM on u_{k+1} (or on u_hat when lam_hi is set), weights
    from u_{k+1}, residual with the old operator H_k and lambda_k, append."""
    theta_k = st.theta.copy()
    if cfg.of and geo.F > 1 and len(st.log) % cfg.of_every == 0:
        # OF branch of Alg. "dyn_nl_rmmgks": velocities of every frame pair from u^(k)
        # (SOLVE-OF, eq. "of_forward"), reverse flow, Theta^(k) = [Psi; M_hat]
        geo.flow = OF.estimate_flow(st.u.reshape(geo.F, geo.N, geo.N), cfg.of_gamma,
                                    cfg.of_ridge)
        st.PV = psi_cols(geo, st.V)
    st.AV = A_cols(geo, theta_k, st.V)
    target = cfg.tau * delta
    S = cfg.S
    for t in range(S):
        w = weights(geo, st.u, cfg.eps)
        z, lam, RA, RP, flag = projected_solve(st, b, w, cfg, target)
        st.status |= flag
        st.z, st.lam = z, lam
        st.u = st.V @ z
        if t < S - 1:
            r = mm_residual(geo, theta_k, st, b, w, lam, z)
            append_direction(geo, theta_k, st, r, cfg)
    compress(st, RA, RP, st.lam, st.z, cfg.kmin)
    # the state the parameter update works on: the primary one, or the smoother estimate of
    # the high-regularisation solve (its basis is discarded afterwards)
    ps = st
    if cfg.lam_hi is not None:
        ps = hi_solve(geo, theta_k, st, b, cfg)
        st.status |= ps.status
    if cfg.gn == "altmin":
        theta_new, flag, info = gn_altmin(geo, theta_k, ps.u, b, cfg)
    elif cfg.gn == "varpro":
        w = weights(geo, ps.u, cfg.eps)
        theta_new, flag, info = gn_varpro(geo, theta_k, ps.V, b, w, ps.PV, ps.lam, cfg)
    elif cfg.gn == "sensitivity":
        w = weights(geo, ps.u, cfg.eps)
        theta_new, flag, info = gn_sensitivity(geo, theta_k, ps.u, b, w, ps.lam, cfg)
    else:
        theta_new, flag, info = theta_k, 0, {}
    st.status |= flag
    w = weights(geo, st.u, cfg.eps)
    r = mm_residual(geo, theta_k, st, b, w, st.lam, st.z)
    append_direction(geo, theta_k, st, r, cfg, with_projection=False)
    st.theta = theta_new
    st.log.append(dict(lam=st.lam, alpha=info.get("alpha"), status=st.status,
                       u_hat=None if ps is st else ps.u))
    return st


def run(geo: Geometry, b, delta, theta0, cfg: Config, outer: int, callback=None) -> State:
    """NL-RMM-GKS with a fixed number of outer iterations."""
    st = init_state(geo, theta0, b, cfg)
    for k in range(outer):
        outer_step(geo, st, b, delta, cfg)
        if callback is not None:
            callback(k, st)
    return st


def block_geometry(geo: Geometry, idx) -> Geometry:
    return Geometry(N=geo.N, nb=geo.nb, view_off=np.array([0, len(idx)], dtype=np.int64))


def block_rows(nb, idx):
    return (np.asarray(idx)[:, None] * nb + np.arange(nb)[None, :]).reshape(-1)


def run_streaming(geo: Geometry, b, noise, theta0, blocks: List[np.ndarray], cfg: Config,
                  passes: int, max_blocks: Optional[int] = None) -> State:
    """s-NL-RMM-GKS (Alg. "s_nl_rmmgks_final"): blocks of views processed in order, carrying
    (u, theta, V) from block to block; each block runs one NL-RMM-GKS outer iteration on its
    rows with delta = the norm of the block's noise."""
    theta = np.array(theta0, dtype=np.float64)
    first = blocks[0]
    g0 = block_geometry(geo, first)
    rows0 = block_rows(geo.nb, first)
    st = init_state(g0, theta[first], b[rows0], cfg)
    st.theta = theta
    done = 0
    for _ in range(passes):
        for idx in blocks:
            if max_blocks is not None and done >= max_blocks:
                return st
            gj = block_geometry(geo, idx)
            rows = block_rows(geo.nb, idx)
            sub = State(V=st.V, AV=st.AV, PV=st.PV, u=st.u, theta=theta[idx].copy(),
                        z=st.z, lam=st.lam, status=st.status, log=st.log)
            outer_step(gj, sub, b[rows], float(np.linalg.norm(noise[rows])), cfg)
            theta[idx] = sub.theta
            st = State(V=sub.V, AV=sub.AV, PV=sub.PV, u=sub.u, theta=theta, z=sub.z,
                       lam=sub.lam, status=sub.status, log=sub.log)
            done += 1
    return st


def make_data(geo: Geometry, x_true, theta_true, g, eta):
    """b = A(theta_true) x_true + e with e = eta ||A x_true|| g/||g|| (inverse crime)."""
    bex = A(geo, theta_true, np.asarray(x_true).reshape(-1))
    e = eta * np.linalg.norm(bex) * g / np.linalg.norm(g)
    return bex + e, e
