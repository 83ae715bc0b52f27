"""Pins of the FP64 method oracle (regulariser, MM-GKS step, DP, compress, GN, VarPro).

Checks use dense linear algebra written independently of the oracle's QR/SVD
path, the majorant properties of Section 3.1, the descent property of the
image update with lambda fixed, quadratic convergence of Gauss-Newton on a
zero-residual problem, and finite differences of the VarPro reduced objective.
"""
import dataclasses
import math

import numpy as np
import pytest

from oracle import method as M
from oracle import projector as P
from paper_2605_06336_amd import synth


def small_problem(N=12, nb=19, V=10, seed=0, noise=0.01, F=1, temporal=False):
    rng = np.random.default_rng(seed)
    if F == 1:
        vo = np.array([0, V], dtype=np.int64)
    else:
        counts = rng.integers(3, 6, F)
        vo = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    geo = M.Geometry(N=N, nb=nb, view_off=vo, temporal=temporal)
    x = synth.ellipse_image(N, [0.1, -0.3], [0.0, 0.2], [0.5, 0.2], [0.3, 0.25], [0.3, 1.0],
                            [1.0, 0.5])
    x = np.stack([np.roll(x, f, axis=1) for f in range(geo.F)])
    th_nom = np.arange(geo.V) * math.pi / geo.V
    th_true = th_nom + rng.normal(0, math.radians(1.0), geo.V)
    g = rng.standard_normal(geo.m)
    b, e = M.make_data(geo, x.ravel(), th_true, g, noise)
    return geo, x.ravel(), th_nom, th_true, b, e


def dense_psi(geo):
    n = geo.n
    return np.stack([M.psi(geo, np.eye(n)[:, i]) for i in range(n)], axis=1)


@pytest.mark.parametrize("F,temporal", [(1, False), (3, True)])
def test_psi_adjoint_and_ramps(F, temporal):
    geo = M.Geometry(N=7, nb=11, view_off=np.arange(F + 1, dtype=np.int64), temporal=temporal)
    rng = np.random.default_rng(1)
    u = rng.standard_normal(geo.n)
    s = rng.standard_normal(M.npsi(geo))
    assert abs(M.psi(geo, u) @ s - u @ M.psiT(geo, s)) < 1e-12
    # linear ramp a*k + b*l + c*f has constant differences a, b, c
    f, l, k = np.meshgrid(np.arange(F), np.arange(7), np.arange(7), indexing="ij")
    ramp = (2.0 * k + 3.0 * l + 5.0 * f).ravel()
    d = M.psi(geo, ramp)
    nx = 7 * 6
    assert np.allclose(d[:nx], 2.0) and np.allclose(d[nx:2 * nx], 3.0)
    if temporal:
        assert np.allclose(d[F * 2 * nx:], 5.0)
        assert d.size == F * 2 * nx + (F - 1) * 49


def test_majorant_properties():
    """Q(u|uk) >= J(u), equality and equal gradients at uk (Section 3.1 (i)-(iii))."""
    geo, x, th, _, b, _ = small_problem()
    eps, lam = 1e-2, 0.3
    rng = np.random.default_rng(2)
    uk = x + 0.1 * rng.standard_normal(geo.n)
    w = M.weights(geo, uk, eps)
    sk = M.psi(geo, uk)
    phi_k = np.sqrt(sk ** 2 + eps ** 2)
    # constant c so that Q(uk|uk) = J(uk): c = lam * sum(phi_k - sk^2 w / 2)
    c = lam * np.sum(phi_k - 0.5 * sk ** 2 * w)

    def J(u):
        return M.objective(geo, th, u, b, lam, eps)

    def Q(u):
        r = M.A(geo, th, u) - b
        s = M.psi(geo, u)
        return 0.5 * r @ r + 0.5 * lam * np.sum(w * s * s) + c

    assert abs(Q(uk) - J(uk)) < 1e-12 * abs(J(uk))
    for _ in range(20):
        u = uk + rng.standard_normal(geo.n) * rng.uniform(0.01, 1.0)
        assert Q(u) >= J(u) - 1e-12 * abs(J(u))
    h = 1e-6
    for i in rng.choice(geo.n, 5, replace=False):
        e = np.zeros(geo.n)
        e[i] = h
        gq = (Q(uk + e) - Q(uk - e)) / (2 * h)
        gj = (J(uk + e) - J(uk - e)) / (2 * h)
        assert abs(gq - gj) < 1e-5 * max(1.0, abs(gj))


def test_projected_solve_matches_dense_normal_equations():
    geo, x, th, _, b, _ = small_problem()
    rng = np.random.default_rng(3)
    A, _ = P.dense(geo.N, geo.nb, th)
    Psi = dense_psi(geo)
    w = M.weights(geo, x + 0.05 * rng.standard_normal(geo.n), 1e-2)
    lam = 0.05
    cfg = M.Config(lam_fix=lam)
    Qm = A.T @ A + lam * Psi.T @ (w[:, None] * Psi)
    # a random 9-dimensional subspace
    V, _ = np.linalg.qr(rng.standard_normal((geo.n, 9)))
    st = M.State(V=V, AV=A @ V, PV=Psi @ V, u=np.zeros(geo.n), theta=th)
    z, *_ = M.projected_solve(st, b, w, cfg, 0.0)
    u_dense = V @ np.linalg.solve(V.T @ Qm @ V, V.T @ A.T @ b)
    assert np.linalg.norm(V @ z - u_dense) < 1e-12 * np.linalg.norm(u_dense)
    # V spanning R^n: the projected solve is the majorant minimiser (eq. normal_equations)
    Vf = np.eye(geo.n)
    st = M.State(V=Vf, AV=A, PV=Psi, u=np.zeros(geo.n), theta=th)
    z, *_ = M.projected_solve(st, b, w, cfg, 0.0)
    u_full = np.linalg.solve(Qm, A.T @ b)
    assert np.linalg.norm(z - u_full) < 1e-10 * np.linalg.norm(u_full)


def test_discrepancy_principle_hits_target():
    geo, x, th, _, b, e = small_problem(noise=0.05)
    rng = np.random.default_rng(4)
    A, _ = P.dense(geo.N, geo.nb, th)
    Psi = dense_psi(geo)
    V, _ = np.linalg.qr(rng.standard_normal((geo.n, 30)))
    V = np.column_stack([M.gkb_basis(geo, th, b, 12), V])
    V, _ = np.linalg.qr(V)
    st = M.State(V=V, AV=A @ V, PV=Psi @ V, u=np.zeros(geo.n), theta=th)
    w = M.weights(geo, x, 1e-2)
    delta = np.linalg.norm(e)
    cfg = M.Config()
    z, lam, _, _, flag = M.projected_solve(st, b, w, cfg, 1.01 * delta)
    assert flag == 0
    res = np.linalg.norm(A @ (V @ z) - b)
    assert abs(res - 1.01 * delta) < 1e-10 * delta
    # clamping: an unreachable target sets the low-end flag
    _, _, _, _, flag = M.projected_solve(st, b, w, cfg, 1e-9 * delta)
    assert flag == M.ST_DP_LOW


def test_gkb_basis_relations():
    geo, x, th, _, b, _ = small_problem()
    k = 6
    V = M.gkb_basis(geo, th, b, k)
    assert np.linalg.norm(V.T @ V - np.eye(k)) < 1e-13
    # span(V) = K_k(A^T A, A^T b)
    A, _ = P.dense(geo.N, geo.nb, th)
    K = [A.T @ b]
    for _ in range(k - 1):
        K.append(A.T @ (A @ K[-1]))
    Kq, _ = np.linalg.qr(np.stack(K, 1))
    s = np.linalg.svd(V.T @ Kq, compute_uv=False)
    assert np.min(s) > 1 - 1e-8


def test_compress_invariants_and_objective():
    geo, x, th, _, b, e = small_problem()
    cfg = M.Config(kmin=4, kmax=12, lam_fix=0.02, eps=1e-2)
    st = M.init_state(geo, th, b, cfg)
    st.AV = M.A_cols(geo, th, st.V)
    for t in range(cfg.S):
        w = M.weights(geo, st.u, cfg.eps)
        z, lam, RA, RP, _ = M.projected_solve(st, b, w, cfg, 0.0)
        st.z, st.lam, st.u = z, lam, st.V @ z
        if t < cfg.S - 1:
            M.append_direction(geo, th, st, M.mm_residual(geo, th, st, b, w, lam, z), cfg)
    u_before = st.u.copy()
    V_before = st.V.copy()
    J_before = M.objective(geo, th, u_before, b, cfg.lam_fix, cfg.eps)
    M.compress(st, RA, RP, st.lam, st.z, cfg.kmin)
    assert st.V.shape[1] == cfg.kmin
    assert np.linalg.norm(st.V.T @ st.V - np.eye(cfg.kmin)) < 1e-13
    assert np.linalg.norm(st.u - u_before) < 1e-13 * np.linalg.norm(u_before)
    assert np.linalg.norm(st.AV - M.A_cols(geo, th, st.V)) < 1e-12 * np.linalg.norm(st.AV)
    assert abs(M.objective(geo, th, st.u, b, cfg.lam_fix, cfg.eps) - J_before) < 1e-12 * J_before
    # the kept directions are V times the kmin-1 dominant eigenvectors of H^T H,
    # H = [RA; sqrt(lam) RP] (computed here by a symmetric eigensolver, not an SVD)
    H = np.vstack([RA, math.sqrt(st.lam) * RP])
    ev, U = np.linalg.eigh(H.T @ H)
    Wref = U[:, ::-1][:, :cfg.kmin - 1]
    kept = V_before.T @ st.V[:, :cfg.kmin - 1]
    s = np.linalg.svd(Wref.T @ kept, compute_uv=False)
    assert np.min(s) > 1 - 1e-9


def test_fixed_lambda_descent():
    """With lambda fixed each MM-GKS step does not increase J_eps (Section 3.1, MM property)."""
    geo, x, th, _, b, _ = small_problem(N=16, nb=23, V=14)
    cfg = M.Config(kmin=3, kmax=20, lam_fix=0.01, eps=1e-2)
    st = M.init_state(geo, th, b, cfg)
    st.AV = M.A_cols(geo, th, st.V)
    Js = []
    for t in range(cfg.S):
        w = M.weights(geo, st.u, cfg.eps)
        z, lam, RA, RP, _ = M.projected_solve(st, b, w, cfg, 0.0)
        st.z, st.u = z, st.V @ z
        Js.append(M.objective(geo, th, st.u, b, lam, cfg.eps))
        M.append_direction(geo, th, st, M.mm_residual(geo, th, st, b, w, lam, z), cfg)
    assert all(Js[i + 1] <= Js[i] * (1 + 1e-12) for i in range(len(Js) - 1))
    assert Js[-1] < 0.5 * Js[0]


def test_mm_residual_is_majorant_gradient():
    """r = A^T(Au - b) + lam Psi^T (w * Psi u) is the gradient of Q(.|uk) at u (eq. normal_equations)."""
    geo, x, th, _, b, _ = small_problem()
    A, _ = P.dense(geo.N, geo.nb, th)
    Psi = dense_psi(geo)
    rng = np.random.default_rng(5)
    V, _ = np.linalg.qr(rng.standard_normal((geo.n, 5)))
    z = rng.standard_normal(5)
    w = rng.uniform(0.5, 2.0, M.npsi(geo))
    st = M.State(V=V, AV=A @ V, PV=Psi @ V, u=V @ z, theta=th)
    r = M.mm_residual(geo, th, st, b, w, 0.7, z)
    u = V @ z
    ref = A.T @ (A @ u - b) + 0.7 * Psi.T @ (w * (Psi @ u))
    assert np.linalg.norm(r - ref) < 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("mode", ["per_view", "scalar"])
def test_gauss_newton_quadratic_convergence(mode):
    """Zero noise, u = x_true: theta -> theta_true quadratically from the nominal angles."""
    N, nb = 32, 47
    geo = M.Geometry(N=N, nb=nb, view_off=np.array([0, 16], dtype=np.int64))
    x = synth.ellipse_image(N, [0.1, -0.3], [0.0, 0.2], [0.5, 0.2], [0.3, 0.25], [0.3, 1.0],
                            [1.0, 0.5]).ravel()
    th_nom = np.arange(16) * math.pi / 16
    rng = np.random.default_rng(6)
    if mode == "scalar":
        th_true = th_nom + math.radians(0.7)
    else:
        th_true = th_nom + rng.normal(0, math.radians(1.0), 16)
    b = M.A(geo, th_true, x)
    cfg = M.Config(maxiter_p=1, param_mode=mode, mu_rel=1e-12)
    th = th_nom.copy()
    errs = [np.max(np.abs(th - th_true))]
    for _ in range(6):
        th, status, info = M.gn_altmin(geo, th, x, b, cfg)
        if info["f0"] > 0:
            assert info["g"] @ info["d"] < 0 or mode == "scalar"
        errs.append(np.max(np.abs(th - th_true)))
    assert errs[-1] < 1e-10
    assert errs[2] < errs[1] ** 1.5 * 10


def test_varpro_gradient_and_gn_matrix_by_finite_differences():
    geo, x, th, _, b, _ = small_problem(N=10, nb=15, V=6)
    rng = np.random.default_rng(7)
    V, _ = np.linalg.qr(np.column_stack([x, rng.standard_normal((geo.n, 3))]))
    PV = M.psi_cols(geo, V)
    w = M.weights(geo, x, 1e-2)
    lam = 0.03
    Bw = np.sqrt(w)[:, None] * PV
    cfg = M.Config(maxiter_p=1, armijo_trials=1, mu_rel=0.0)
    _, _, info = M.gn_varpro(geo, th, V, b, w, PV, lam, cfg)
    h = 1e-6
    gfd = np.zeros(geo.V)
    Jr = np.zeros((geo.m, geo.V))
    Js = np.zeros((Bw.shape[0], geo.V))
    for v in range(geo.V):
        e = np.zeros(geo.V)
        e[v] = h
        _, _, yp, rp, fp = M.varpro_parts(geo, th + e, V, b, Bw, lam)
        _, _, ym, rm, fm = M.varpro_parts(geo, th - e, V, b, Bw, lam)
        gfd[v] = (fp - fm) / (2 * h)
        Jr[:, v] = (rp - rm) / (2 * h)
        Js[:, v] = (Bw @ yp - Bw @ ym) / (2 * h)
    assert np.linalg.norm(info["g"] - gfd) < 1e-6 * np.linalg.norm(gfd)
    Jfd = Jr.T @ Jr + lam * Js.T @ Js
    assert np.linalg.norm(info["J"] - Jfd) < 1e-5 * np.linalg.norm(Jfd)


def test_reductions():
    """gn='none' keeps the angles (RMM-GKS); one streaming block equals the plain driver."""
    geo, x, th, _, b, e = small_problem(N=12, nb=19, V=8)
    delta = np.linalg.norm(e)
    cfg = M.Config(kmin=3, kmax=8, gn="none")
    st = M.run(geo, b, delta, th, cfg, 2)
    assert np.array_equal(st.theta, th)
    cfg = M.Config(kmin=3, kmax=8)
    st1 = M.run(geo, b, delta, th, cfg, 2)
    st2 = M.run_streaming(geo, b, e, th, [np.arange(geo.V)], cfg, passes=2)
    assert np.allclose(st1.u, st2.u, rtol=0, atol=1e-12 * np.abs(st1.u).max())
    assert np.allclose(st1.theta, st2.theta, rtol=0, atol=1e-14)


def test_altmin_reduces_angle_error_on_small_problem():
    geo, x, th_nom, th_true, b, e = small_problem(N=24, nb=35, V=30, noise=0.005)
    delta = np.linalg.norm(e)
    cfg = M.Config(kmin=4, kmax=14)
    st = M.run(geo, b, delta, th_nom, cfg, 6)
    e0 = np.linalg.norm(th_nom - th_true)
    assert np.linalg.norm(st.theta - th_true) < 0.6 * e0
    assert np.linalg.norm(st.V.T @ st.V - np.eye(st.V.shape[1])) < 1e-10


def test_hi_solve_matches_dense_fixed_lambda_steps():
    """High-regularisation solve (Section 4.3): from a compressed basis V and u in its span,
    two fixed-lambda MM-GKS steps written out with dense A and Psi (normal equations of the
    reduced problem, residual with the step's weights, two Gram-Schmidt passes); the primary
    state is left as it was."""
    geo, x, th, _, b, _ = small_problem(N=12, nb=19, V=10)
    A, _ = P.dense(geo.N, geo.nb, th)
    Psi = dense_psi(geo)
    lam, eps = 0.3, 1e-2
    cfg = M.Config(kmin=3, kmax=6, solves=2, eps=eps, lam_hi=lam, gn="altmin")
    rng = np.random.default_rng(8)
    V, _ = np.linalg.qr(rng.standard_normal((geo.n, cfg.kmin)))
    u0 = V @ rng.standard_normal(cfg.kmin)
    st = M.State(V=V.copy(), AV=A @ V, PV=Psi @ V, u=u0.copy(), theta=th.copy())
    hs = M.hi_solve(geo, th, st, b, cfg)

    def wts(u):
        return 1.0 / np.sqrt((Psi @ u) ** 2 + eps ** 2)

    def solve(B, w):
        AB, PB = A @ B, Psi @ B
        return np.linalg.solve(AB.T @ AB + lam * PB.T @ (w[:, None] * PB), AB.T @ b)

    w0 = wts(u0)
    u1 = V @ solve(V, w0)
    r = A.T @ (A @ u1 - b) + lam * Psi.T @ (w0 * (Psi @ u1))
    for _ in range(2):
        r = r - V @ (V.T @ r)
    V2 = np.column_stack([V, r / np.linalg.norm(r)])
    u2 = V2 @ solve(V2, wts(u1))
    assert np.linalg.norm(hs.u - u2) <= 1e-9 * np.linalg.norm(u2)
    assert hs.lam == lam and hs.V.shape[1] == cfg.kmin + 1
    assert np.array_equal(st.V, V) and np.array_equal(st.u, u0)


def test_hi_solve_leaves_primary_trajectory():
    """With the angles fixed, the high-regularisation solve changes nothing the outer iteration
    carries (its image only feeds the parameter update), and its image is smoother (smaller
    total variation) than the primary one for lam_hi well above the DP lambda."""
    geo, x, th_nom, _, b, e = small_problem(N=16, nb=23, V=14)
    delta = np.linalg.norm(e)
    base = M.Config(kmin=3, kmax=10, gn="none")
    st0 = M.run(geo, b, delta, th_nom, base, 3)
    hi = dataclasses.replace(base, lam_hi=100.0 * st0.lam)
    st1 = M.run(geo, b, delta, th_nom, hi, 3)
    assert np.array_equal(st0.u, st1.u) and np.array_equal(st0.V, st1.V)
    assert st0.lam == st1.lam
    uh = st1.log[-1]["u_hat"]
    assert uh is not None and st0.log[-1]["u_hat"] is None
    tv = lambda u: float(np.sum(np.abs(M.psi(geo, u))))   # noqa: E731
    assert tv(uh) < tv(st1.u)


def test_grid_search_offset_sign_and_residual():
    """Coarse grid search of the experiments section on a basis that contains the image:
    noise-free data from the angles offset by s*, so the reduced residual vanishes at s*
    (and only there on the grid), and the returned angles are the nominal ones plus s*.
    (With the GKB basis at the nominal angles a global offset of a parallel-beam operator is
    an image rotation that the basis absorbs; see the next test for that basis.)"""
    geo, x, th_nom, _, _, _ = small_problem(N=16, nb=23, V=20)
    s_true = math.radians(1.5)
    b = M.A(geo, th_nom + s_true, x)
    rng = np.random.default_rng(4)
    V, _ = np.linalg.qr(np.column_stack([x, rng.standard_normal((geo.n, 5))]))
    shifts = np.radians(np.arange(-3.0, 3.01, 0.5))
    th0, res2, best = M.grid_search_shift(geo, th_nom, b, shifts, V=V)
    assert shifts[best] == s_true
    assert np.array_equal(th0, th_nom + s_true)
    assert res2[best] <= 1e-20 * (b @ b)
    assert np.min(np.delete(res2, best)) > 1e-8 * (b @ b)


def test_grid_search_residual_bounds():
    """Each candidate's reduced residual lies between the full-space least-squares residual
    of the same operator (dense, tiny problem) and ||b||^2."""
    geo, x, th_nom, _, b, _ = small_problem(N=8, nb=13, V=12)
    shifts = np.radians(np.array([-2.0, 0.0, 2.0]))
    _, res2, _ = M.grid_search_shift(geo, th_nom, b, shifts, ell0=6)
    for s, r2 in zip(shifts, res2):
        A, _ = P.dense(geo.N, geo.nb, th_nom + s)
        xf, *_ = np.linalg.lstsq(A, b, rcond=None)
        full = float(np.sum((A @ xf - b) ** 2))
        assert full - 1e-9 * (b @ b) <= r2 <= b @ b


def test_offset_sensitivity_by_finite_differences():
    """Full-space sensitivity for a global offset (eq. "sensitivity"): at the closed-form
    u(p) = M(p)^-1 A(p)^T b of eq. "u_closed_form" (weights fixed), u_p equals the central
    difference of u(p), and g equals the derivative of the reduced objective
    f(p) = 1/2 ||A(p) u(p) - b||^2 + lam/2 ||sqrt(w) Psi u(p)||^2."""
    geo, x, th, _, b, _ = small_problem(N=8, nb=13, V=10)
    lam = 0.05
    w = M.weights(geo, x, 0.05)
    Psi = dense_psi(geo)

    def closed(p):
        A, _ = P.dense(geo.N, geo.nb, th + p)
        Mm = A.T @ A + lam * Psi.T @ (w[:, None] * Psi)
        u = np.linalg.solve(Mm, A.T @ b)
        f = 0.5 * np.sum((A @ u - b) ** 2) + 0.5 * lam * np.sum(w * (Psi @ u) ** 2)
        return u, f

    u0, _ = closed(0.0)
    up, g, hh, dp = M.offset_sensitivity(geo, th, u0, b, w, lam)
    e = 1e-6
    (u1, f1), (u2, f2) = closed(e), closed(-e)
    fd_u = (u1 - u2) / (2 * e)
    assert np.linalg.norm(up - fd_u) <= 1e-6 * np.linalg.norm(fd_u)
    assert abs(g - (f1 - f2) / (2 * e)) <= 1e-6 * abs(g)
    assert hh > 0 and dp == -g / hh
