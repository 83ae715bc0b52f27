"""Pins of the optical-flow oracle (CPU only): the bilinear warp, the velocity estimation of
eq. "of_forward" and the motion rows of eq. "Theta_OF", each against what the mathematics
fixes independently of the oracle's code."""
import dataclasses
import math

import numpy as np

from oracle import method as M
from oracle import optical_flow as OF


def test_warp_zero_flow_is_the_identity_and_integer_flow_a_shift():
    rng = np.random.default_rng(0)
    ny, nx = 9, 11
    v = rng.standard_normal((ny, nx))
    z = np.zeros((ny, nx))
    assert np.array_equal((OF.warp_matrix(z, z) @ v.ravel()).reshape(ny, nx), v)
    # s = (+2, -1): pixel (k, l) reads v at (k + 2, l - 1) wherever that lies on the grid
    Mw = OF.warp_matrix(z + 2.0, z - 1.0)
    w = (Mw @ v.ravel()).reshape(ny, nx)
    assert np.allclose(w[1:, :nx - 2], v[:ny - 1, 2:], rtol=0, atol=1e-15)
    # outside, the clamped position: column nx-1 and row 0
    assert np.allclose(w[1:, nx - 1], v[:ny - 1, nx - 1], rtol=0, atol=1e-15)
    assert np.allclose(w[0, :nx - 2], v[0, 2:], rtol=0, atol=1e-15)


def test_warp_is_exact_on_bilinear_functions_and_a_partition_of_unity():
    rng = np.random.default_rng(1)
    ny, nx = 12, 10
    K, L = np.meshgrid(np.arange(nx), np.arange(ny))
    a, b, c, d = rng.standard_normal(4)
    v = a + b * K + c * L + d * K * L
    sx = rng.uniform(-0.9, 0.9, (ny, nx))
    sy = rng.uniform(-0.9, 0.9, (ny, nx))
    w = (OF.warp_matrix(sx, sy) @ v.ravel()).reshape(ny, nx)
    X, Y = K + sx, L + sy
    want = a + b * X + c * Y + d * X * Y
    inner = (X >= 0) & (X <= nx - 1) & (Y >= 0) & (Y <= ny - 1)
    assert np.max(np.abs(w - want)[inner]) < 1e-12
    Mw = OF.warp_matrix(5 * sx, 5 * sy)        # large flows: clamped positions
    assert Mw.data.min() >= -1e-15
    assert np.allclose(np.asarray(Mw.sum(axis=1)).ravel(), 1.0, rtol=0, atol=1e-14)


def smooth_texture(x, y):
    """A smooth, textured analytic image (no flat regions, gradients in both directions)."""
    return (np.sin(0.45 * x + 0.2 * y) + 0.8 * np.cos(0.3 * y - 0.15 * x)
            + 0.5 * np.sin(0.23 * x * 0.9 + 0.37 * y * 1.1))


def test_image_gradients_are_exact_on_linear_and_quadratic_images():
    """Central differences are exact for quadratics inside the frame, the one-sided
    differences at the borders for linear images."""
    ny, nx = 7, 9
    K, L = np.meshgrid(np.arange(nx, dtype=np.float64), np.arange(ny, dtype=np.float64))
    gx, gy = OF.spatial_gradients(0.5 + 0.3 * K - 0.7 * L)
    assert np.allclose(gx, 0.3, rtol=0, atol=1e-14) and np.allclose(gy, -0.7, rtol=0, atol=1e-14)
    gx, gy = OF.spatial_gradients(K * K - 2.0 * K * L + 0.5 * L * L)
    assert np.allclose(gx[:, 1:-1], (2 * K - 2 * L)[:, 1:-1], rtol=0, atol=1e-12)
    assert np.allclose(gy[1:-1, :], (L - 2 * K)[1:-1, :], rtol=0, atol=1e-12)


def test_zero_motion_gives_zero_flow():
    rng = np.random.default_rng(2)
    u = rng.uniform(0, 1, (10, 13))
    sx, sy = OF.solve_flow(u, u)
    assert np.array_equal(sx, np.zeros_like(u)) and np.array_equal(sy, np.zeros_like(u))


def test_constant_translation_is_recovered():
    """u1(x) = u0(x - s0) for a smooth texture: the flow from u0 to u1 is s0 everywhere (the
    OFC and the warp both describe u1(x + s) = u0(x)).  Small gamma and ridge, sub-pixel
    shifts: the mean over the interior is within a few per cent of s0 (linearisation and
    regularisation bias), for both components and signs."""
    n = 40
    K, L = np.meshgrid(np.arange(n, dtype=np.float64), np.arange(n, dtype=np.float64))
    for s0 in ((0.3, -0.2), (-0.25, 0.15)):
        u0 = smooth_texture(K, L)
        u1 = smooth_texture(K - s0[0], L - s0[1])
        sx, sy = OF.solve_flow(u0, u1, gamma=0.01, ridge=1e-6)
        core = (slice(6, n - 6), slice(6, n - 6))
        mx, my = float(sx[core].mean()), float(sy[core].mean())
        assert abs(mx - s0[0]) < 0.05 * abs(s0[0]) and abs(my - s0[1]) < 0.05 * abs(s0[1]), \
            (s0, mx, my)


def test_flow_solution_is_stationary_for_the_stated_objective():
    """The solved s has zero directional derivative of the objective written out term by
    term (the objective is quadratic: central differences are exact up to rounding)."""
    rng = np.random.default_rng(3)
    u0 = rng.uniform(0, 1, (8, 9))
    u1 = u0 + 0.1 * rng.standard_normal(u0.shape)
    gamma, ridge = 0.05, 1e-3
    sx, sy = OF.solve_flow(u0, u1, gamma, ridge)
    s = np.concatenate([sx.ravel(), sy.ravel()])
    # the objective from its definition: data term with central-difference gradients,
    # forward differences of each component, ridge
    gx, gy = OF.spatial_gradients(u0)
    ut = u1 - u0

    def obj(sv):
        ax, ay = sv[:72].reshape(8, 9), sv[72:].reshape(8, 9)
        r = gx * ax + gy * ay + ut
        reg = sum(float(np.sum(np.diff(c, axis=ax_) ** 2)) for c in (ax, ay) for ax_ in (0, 1))
        return float(np.sum(r * r)) + gamma * reg + ridge * float(sv @ sv)

    f0 = obj(s)
    for _ in range(5):
        d = rng.standard_normal(s.size)
        h = 1e-3
        dd = (obj(s + h * d) - obj(s - h * d)) / (2 * h)
        curv = (obj(s + h * d) - 2 * f0 + obj(s - h * d)) / (h * h)
        assert abs(dd) <= 1e-7 * max(curv, 1e-12) * np.linalg.norm(d) + 1e-10, (dd, curv)


def test_motion_rows_with_zero_flow_are_frame_differences():
    rng = np.random.default_rng(4)
    F, n = 4, 7
    U = rng.standard_normal((F, n, n))
    z = [np.zeros((n, n))] * (F - 1)
    rows = OF.motion_rows(U, OF.Flow(z, z))
    dt = (U[1:] - U[:-1]).ravel()
    assert np.array_equal(rows, np.concatenate([-dt, dt]))


def test_motion_rows_vanish_on_an_exact_translation():
    """Frames U[t](x) = v(x - t s0) of a bilinear v moving at s0 per frame: both the forward
    rows (s = s0) and the reverse rows (s' = -s0) vanish wherever the sample stays on the
    grid."""
    F, n = 3, 10
    K, L = np.meshgrid(np.arange(n, dtype=np.float64), np.arange(n, dtype=np.float64))
    s0 = (0.4, -0.7)

    def v(x, y):
        return 0.3 + 0.2 * x - 0.1 * y + 0.05 * x * y

    U = np.stack([v(K - t * s0[0], L - t * s0[1]) for t in range(F)])
    flow = OF.Flow([np.full((n, n), s0[0])] * (F - 1), [np.full((n, n), s0[1])] * (F - 1))
    rows = OF.motion_rows(U, flow).reshape(2, F - 1, n, n)
    ok_f = (K + s0[0] >= 0) & (K + s0[0] <= n - 1) & (L + s0[1] >= 0) & (L + s0[1] <= n - 1)
    ok_r = (K - s0[0] >= 0) & (K - s0[0] <= n - 1) & (L - s0[1] >= 0) & (L - s0[1] <= n - 1)
    assert np.max(np.abs(rows[0][:, ok_f])) < 1e-12
    assert np.max(np.abs(rows[1][:, ok_r])) < 1e-12
    assert np.max(np.abs(rows)) > 1e-3          # the clamped border rows do not vanish


def test_theta_with_flow_is_adjoint_to_its_transpose():
    rng = np.random.default_rng(5)
    F, N = 3, 9
    geo = M.Geometry(N=N, nb=13, view_off=np.array([0, 4, 9, 12], dtype=np.int64),
                     temporal=True)
    geo.flow = OF.Flow([rng.uniform(-2, 2, (N, N)) for _ in range(F - 1)],
                       [rng.uniform(-2, 2, (N, N)) for _ in range(F - 1)])
    u = rng.standard_normal(geo.n)
    z = rng.standard_normal(M.npsi(geo))
    assert M.psi(geo, u).size == M.npsi(geo)
    lhs = float(M.psi(geo, u) @ z)
    rhs = float(u @ M.psiT(geo, z))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0)


def test_of_loop_estimates_flow_each_outer_iteration():
    """The dynamic loop with the OF operator on a tiny moving phantom: velocities from the
    current image at every outer iteration, Psi V rebuilt for the new operator (PV equals
    psi of V), finite iterates."""
    rng = np.random.default_rng(6)
    N, F = 16, 3
    K, L = np.meshgrid(np.arange(N), np.arange(N))
    frames = np.stack([((K - 6 - t) ** 2 + (L - 7) ** 2 < 16).astype(float) for t in range(F)])
    counts = [9, 8, 10]
    vo = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    geo = M.Geometry(N=N, nb=23, view_off=vo, temporal=True)
    theta = rng.uniform(0, math.pi, vo[-1])
    b, e = M.make_data(geo, frames.ravel(), theta, rng.standard_normal(vo[-1] * 23), 0.01)
    cfg = dataclasses.replace(M.Config(kmin=4, kmax=9), of=True, gn="none")
    seen = []

    def cb(k, st):
        assert geo.flow is not None
        assert np.allclose(st.PV, M.psi_cols(geo, st.V), rtol=0, atol=1e-10)
        seen.append(k)

    st = M.run(geo, b, float(np.linalg.norm(e)), theta, cfg, 3, callback=cb)
    assert seen == [0, 1, 2] and np.all(np.isfinite(st.u))
    assert M.npsi(geo) == F * 2 * N * (N - 1) + 2 * (F - 1) * N * N
