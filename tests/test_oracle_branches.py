"""Pins of the oracle's decision branches (CPU only).

* Armijo backtracking of the parameter update (Alg. "update_param"; Section 4.2 for the
  variable-projection objective): when the first trial step is rejected, the accepted step
  is the first alpha0 * beta^q that satisfies f(theta + a d) <= f(theta) + c1 a g^T d, with
  the gradient g taken here by central differences of f (not from the oracle's angle
  derivative) and f evaluated with the dense operator; when every trial fails the angles
  are unchanged and the Armijo status bit is set.
* The discrepancy principle's high-end clamp (Section 3.2): a target above ||b|| cannot be
  met (the residual rises to ||b|| as lambda grows), so lambda is the bracket's top,
  1e10 * ||A V||_F^2 / ||sqrt(w) Psi V||_F^2, with the DP_HIGH bit.
* The streaming driver with several blocks (Alg. "s_nl_rmmgks_final"): its row, angle and
  noise mapping equals a loop written here with two-dimensional indexing of the sinogram,
  and its result does not depend on the order in which the views are stored.
* The full-space sensitivity step of one global offset (Section 4.2, eqs. "sensitivity",
  "GN_system"): u_p by conjugate gradients equals the dense solve; with the image at the
  minimiser of the majorised problem and a basis spanning the image space, g is the
  derivative of the reduced objective the line search uses; and that line search
  backtracks and rejects like the others.
"""
import dataclasses
import math

import numpy as np
import pytest

from oracle import method as M
from oracle import projector as P
from paper_2605_06336_amd import synth


def problem(N=12, nb=19, V=10, seed=0, noise=0.01, shift_deg=1.0):
    rng = np.random.default_rng(seed)
    geo = M.Geometry(N=N, nb=nb, view_off=np.array([0, V], dtype=np.int64))
    x = synth.ellipse_image(N, [0.1, -0.3], [0.0, 0.2], [0.5, 0.2], [0.3, 0.25], [0.3, 1.0],
                            [1.0, 0.5]).ravel()
    th_nom = np.arange(V) * math.pi / V
    th_true = th_nom + rng.normal(0, math.radians(shift_deg), V)
    g = rng.standard_normal(geo.m)
    b, e = M.make_data(geo, x, th_true, g, noise)
    return geo, x, th_nom, th_true, b, e


def first_accepted(f, f0, gd, alpha0, beta, c1, trials):
    """Index of the first trial step alpha0 beta^q meeting the sufficient-decrease test."""
    for q in range(trials):
        a = alpha0 * beta ** q
        if f(a) <= f0 + c1 * a * gd:
            return q
    return None


def fd_gradient(f, th, h=1e-6):
    g = np.zeros(th.size)
    for v in range(th.size):
        e = np.zeros(th.size)
        e[v] = h
        g[v] = (f(th + e) - f(th - e)) / (2 * h)
    return g


def check_backtracking(f, th, info, cfg, alpha):
    """alpha (the oracle's step) must be the first accepted trial of the Armijo sequence
    built from f and a finite-difference gradient; also checks that the sign of the
    sufficient-decrease term matters for this case (the pin would see it flipped)."""
    g = fd_gradient(f, th)
    d = info["d"]
    gd = float(g @ d)
    assert gd < 0, "not a descent direction"
    assert abs(gd - float(info["g"] @ d)) < 1e-5 * abs(gd)
    f0 = f(th)
    phi = lambda a: f(th + a * d)  # noqa: E731
    q = first_accepted(phi, f0, gd, cfg.alpha0, cfg.beta, cfg.c1, cfg.armijo_trials)
    assert q is not None and q >= 2, q        # the first steps were rejected
    assert alpha == cfg.alpha0 * cfg.beta ** q
    # the decisions at q-1 (rejected) and q (accepted) are not within finite-difference noise
    for qq in (q - 1, q):
        a = cfg.alpha0 * cfg.beta ** qq
        assert abs(phi(a) - (f0 + cfg.c1 * a * gd)) > 1e-6 * f0
    q_flip = first_accepted(phi, f0, -gd, cfg.alpha0, cfg.beta, cfg.c1, cfg.armijo_trials)
    q_beta = first_accepted(phi, f0, gd, cfg.alpha0, 0.6, cfg.c1, cfg.armijo_trials)
    assert q_flip != q and cfg.alpha0 * 0.6 ** q_beta != alpha
    return q


def test_armijo_backtracking_altmin():
    geo, x, th, th_true, b, _ = problem(V=10, shift_deg=2.0, noise=0.0)
    A = P.dense(geo.N, geo.nb, th)[0]   # only to size-check the dense evaluation below

    def f(t):
        At, _ = P.dense(geo.N, geo.nb, t)
        r = At @ x - b
        return 0.5 * float(r @ r)

    assert A.shape == (geo.m, geo.n)
    cfg = M.Config(maxiter_p=1, alpha0=16.0, beta=0.5, c1=0.3, armijo_trials=10, mu_rel=1e-6)
    th_new, status, info = M.gn_altmin(geo, th, x, b, cfg)
    assert not status & M.ST_ARMIJO
    q = check_backtracking(f, th, info, cfg, info["alpha"])
    assert np.array_equal(th_new, th + info["alpha"] * info["d"])
    assert f(th_new) < f(th)
    print(f"AltMin: accepted alpha = 16 * 0.5^{q}")


def test_armijo_rejection_altmin_keeps_angles():
    geo, x, th, _, b, _ = problem(V=10, shift_deg=2.0, noise=0.0)
    cfg = M.Config(maxiter_p=1, alpha0=1e4, beta=0.5, c1=1e-4, armijo_trials=3, mu_rel=1e-6)
    th_new, status, info = M.gn_altmin(geo, th, x, b, cfg)
    assert status & M.ST_ARMIJO
    assert info["alpha"] == 0.0
    assert np.array_equal(th_new, th)


def varpro_setup():
    geo, x, th, _, b, _ = problem(N=10, nb=15, V=6, shift_deg=2.0, noise=0.0)
    rng = np.random.default_rng(7)
    V, _ = np.linalg.qr(np.column_stack([x, rng.standard_normal((geo.n, 3))]))
    PV = M.psi_cols(geo, V)
    w = M.weights(geo, x, 1e-2)
    lam = 0.03
    Bw = np.sqrt(w)[:, None] * PV

    def f(t):
        """Reduced variable-projection objective with the dense operator: the image
        coefficients minimise 1/2||A(t) V y - b||^2 + lam/2 ||B y||^2."""
        At, _ = P.dense(geo.N, geo.nb, t)
        Ah = At @ V
        K = np.vstack([Ah, math.sqrt(lam) * Bw])
        rhs = np.concatenate([b, np.zeros(Bw.shape[0])])
        y = np.linalg.lstsq(K, rhs, rcond=None)[0]
        r = Ah @ y - b
        return 0.5 * float(r @ r) + 0.5 * lam * float(np.sum((Bw @ y) ** 2))

    return geo, th, V, b, w, PV, lam, f


def test_armijo_backtracking_varpro():
    geo, th, V, b, w, PV, lam, f = varpro_setup()
    cfg = M.Config(maxiter_p=1, alpha0=16.0, beta=0.5, c1=0.3, armijo_trials=10, mu_rel=1e-6)
    th_new, status, info = M.gn_varpro(geo, th, V, b, w, PV, lam, cfg)
    assert not status & M.ST_ARMIJO
    assert abs(info["f0"] - f(th)) < 1e-10 * f(th)
    q = check_backtracking(f, th, info, cfg, info["alpha"])
    assert np.array_equal(th_new, th + info["alpha"] * info["d"])
    print(f"VarPro: accepted alpha = 16 * 0.5^{q}")


def test_armijo_rejection_varpro_keeps_angles():
    geo, th, V, b, w, PV, lam, f = varpro_setup()
    cfg = M.Config(maxiter_p=1, alpha0=1e4, beta=0.5, c1=1e-4, armijo_trials=3, mu_rel=1e-6)
    th_new, status, info = M.gn_varpro(geo, th, V, b, w, PV, lam, cfg)
    assert status & M.ST_ARMIJO
    assert info["alpha"] == 0.0
    assert np.array_equal(th_new, th)


def test_discrepancy_principle_high_clamp():
    geo, x, th, _, b, e = problem(N=12, nb=19, V=10)
    cfg = M.Config(kmin=3, kmax=8)
    st = M.init_state(geo, th, b, cfg)
    st.AV = M.A_cols(geo, th, st.V)
    w = M.weights(geo, x, cfg.eps)
    target = 2.0 * np.linalg.norm(b)
    z, lam, RA, RP, flag = M.projected_solve(st, b, w, cfg, target)
    assert flag == M.ST_DP_HIGH
    # the bracket's top from the Frobenius norms of the two stacked blocks (no QR)
    top = 1e10 * np.sum(st.AV ** 2) / np.sum(w[:, None] * st.PV ** 2)
    assert abs(lam - top) <= 1e-12 * top
    # and the solve is the one of that lambda: the residual sits just below ||b||
    r = st.AV @ z - b
    assert np.linalg.norm(r) <= np.linalg.norm(b) and np.linalg.norm(r) < target
    # a whole outer iteration reports the clamp in its status word
    st = M.init_state(geo, th, b, cfg)
    M.outer_step(geo, st, b, 2.0 * np.linalg.norm(b) / cfg.tau, cfg)
    assert st.status & M.ST_DP_HIGH
    assert not st.status & M.ST_DP_LOW


def blocks_of(V, sizes, seed):
    perm = np.random.default_rng(seed).permutation(V)
    cuts = np.concatenate([[0], np.cumsum(sizes)])
    assert cuts[-1] == V
    return [np.sort(perm[cuts[i]:cuts[i + 1]]) for i in range(len(sizes))]


def streaming_by_hand(geo, b, e, th0, blocks, cfg, passes):
    """The streaming schedule written out with the sinogram as a [views, bins] array: per
    block, its rows B[idx], its angles and the norm of its noise rows; the angles written
    back view by view."""
    B = b.reshape(geo.V, geo.nb)
    E = e.reshape(geo.V, geo.nb)
    theta = np.array(th0, dtype=np.float64)
    g0 = M.Geometry(N=geo.N, nb=geo.nb, view_off=np.array([0, len(blocks[0])], dtype=np.int64))
    st = M.init_state(g0, theta[blocks[0]], B[blocks[0]].ravel(), cfg)
    for _ in range(passes):
        for idx in blocks:
            gj = M.Geometry(N=geo.N, nb=geo.nb, view_off=np.array([0, len(idx)], dtype=np.int64))
            st.theta = np.array([theta[v] for v in idx])
            M.outer_step(gj, st, B[idx].ravel(), float(np.sqrt(np.sum(E[idx] ** 2))), cfg)
            for k, v in enumerate(idx):
                theta[v] = st.theta[k]
    return st.u, theta


@pytest.mark.parametrize("lam_fix", [0.05, None])
def test_streaming_several_blocks_mapping(lam_fix):
    geo, x, th, _, b, e = problem(N=12, nb=19, V=14, noise=0.02)
    cfg = M.Config(kmin=3, kmax=7, lam_fix=lam_fix)
    blocks = blocks_of(geo.V, [4, 3, 5, 2], seed=3)
    st = M.run_streaming(geo, b, e, th, blocks, cfg, passes=2)
    u_ref, th_ref = streaming_by_hand(geo, b, e, th, blocks, cfg, passes=2)
    assert np.allclose(st.u, u_ref, rtol=0, atol=1e-12 * np.abs(u_ref).max())
    assert np.allclose(st.theta, th_ref, rtol=0, atol=1e-13)
    # views outside every block of a partial pass keep their angles
    st1 = M.run_streaming(geo, b, e, th, blocks, cfg, passes=1, max_blocks=2)
    untouched = np.setdiff1d(np.arange(geo.V), np.concatenate(blocks[:2]))
    assert np.array_equal(st1.theta[untouched], th[untouched])
    assert not np.array_equal(st1.theta[blocks[0]], th[blocks[0]])


def test_streaming_invariant_under_view_storage_order():
    """Storing the views in another order (angles, sinogram rows and noise rows permuted
    together, block lists renamed accordingly) gives the same image and the same angle per
    view: the driver addresses views only through their indices."""
    geo, x, th, _, b, e = problem(N=12, nb=19, V=14, noise=0.02)
    cfg = M.Config(kmin=3, kmax=7, lam_fix=0.05)
    blocks = blocks_of(geo.V, [5, 4, 5], seed=11)
    st = M.run_streaming(geo, b, e, th, blocks, cfg, passes=2)
    perm = np.random.default_rng(12).permutation(geo.V)   # new position i holds view perm[i]
    inv = np.argsort(perm)
    Bp = b.reshape(geo.V, geo.nb)[perm].ravel()
    Ep = e.reshape(geo.V, geo.nb)[perm].ravel()
    blocks_p = [inv[idx] for idx in blocks]   # same views, same order inside each block
    stp = M.run_streaming(geo, Bp, Ep, th[perm], blocks_p, cfg, passes=2)
    assert np.allclose(stp.u, st.u, rtol=0, atol=1e-10 * np.abs(st.u).max())
    assert np.allclose(stp.theta[inv], st.theta, rtol=0, atol=1e-12)


def sens_setup(N=6, nb=9, V=5, lam=0.05):
    geo, x, th, _, b, _ = problem(N=N, nb=nb, V=V, shift_deg=0.0, noise=0.0)
    b = M.A(geo, th + math.radians(1.5), x)          # data at a global offset of 1.5 degrees
    w = M.weights(geo, x + 0.1 * np.cos(np.arange(geo.n)), 1e-2)
    A, _ = P.dense(geo.N, geo.nb, th)
    n = geo.n
    Psi = np.stack([M.psi(geo, np.eye(n)[:, i]) for i in range(n)], axis=1)
    u_star = np.linalg.solve(A.T @ A + lam * Psi.T @ (w[:, None] * Psi), A.T @ b)
    return geo, th, b, w, lam, u_star


def test_sensitivity_cg_matches_dense_solve():
    """u_p by conjugate gradients (enough steps to converge on a tiny grid) equals the dense
    solve of the sensitivity equation, and so do g and h."""
    geo, th, b, w, lam, u = sens_setup()
    up_d, g_d, h_d, _ = M.offset_sensitivity(geo, th, u, b, w, lam)
    up, g, h = M.offset_sensitivity_cg(geo, th, u, b, w, lam, iters=400)
    assert np.linalg.norm(up - up_d) <= 1e-8 * np.linalg.norm(up_d)
    assert abs(g - g_d) <= 1e-8 * abs(g_d) and abs(h - h_d) <= 1e-8 * h_d


def test_sensitivity_gradient_is_derivative_of_reduced_objective():
    """With the image at the exact minimiser of the majorised problem and a basis spanning the
    whole image space, the reduced objective used by the line search is the paper's f(p)
    (Section 4.2), and the sensitivity gradient g is its derivative (central differences)."""
    geo, th, b, w, lam, u = sens_setup()
    V = np.eye(geo.n)
    PV = M.psi_cols(geo, V)
    Bw = np.sqrt(w)[:, None] * PV
    _, g, h = M.offset_sensitivity_cg(geo, th, u, b, w, lam, iters=400)
    f = lambda p: M.varpro_parts(geo, th + p, V, b, Bw, lam)[4]   # noqa: E731
    hstep = 1e-6
    gfd = (f(hstep) - f(-hstep)) / (2 * hstep)
    assert abs(g - gfd) <= 1e-5 * abs(gfd), (g, gfd)
    assert g != 0.0 and h > 0.0


def test_sensitivity_step_armijo_backtracking():
    """The sensitivity step's line search, written out with the dense operator and the dense
    solve of the sensitivity equation: the reduced objective with u(p) to first order,
    phi(a) = 1/2||A(theta + a dp)(u + a dp u_p) - b||^2 + lam/2 ||sqrt(w) Psi (u + a dp u_p)||^2;
    its slope at 0 (central differences) is g dp, and the accepted step is the first
    alpha0 beta^q meeting the sufficient-decrease test (a sign error in that test would
    change it here).  All trials rejected: the angles stay."""
    geo, th, b, w, lam, u = sens_setup()
    n = geo.n
    Psi = np.stack([M.psi(geo, np.eye(n)[:, i]) for i in range(n)], axis=1)
    up_d, g_d, h_d, _ = M.offset_sensitivity(geo, th, u, b, w, lam)
    cfg = M.Config(maxiter_p=1, alpha0=16.0, beta=0.5, c1=0.3, armijo_trials=10, mu_rel=1e-6,
                   sens_iters=400)
    th_new, status, info = M.gn_sensitivity(geo, th, u, b, w, lam, cfg)
    dp = info["dp"]
    assert abs(dp - (-g_d / (h_d * (1 + cfg.mu_rel)))) <= 1e-8 * abs(dp)

    def phi(a):
        A_a, _ = P.dense(geo.N, geo.nb, th + a * dp)
        ua = u + a * dp * up_d
        r = A_a @ ua - b
        sv = Psi @ ua
        return 0.5 * float(r @ r) + 0.5 * lam * float(np.sum(w * sv * sv))

    hstep = 1e-6
    gd = (phi(hstep) - phi(-hstep)) / (2 * hstep)
    assert gd < 0 and abs(gd - g_d * dp) <= 1e-5 * abs(gd)
    f0 = phi(0.0)
    q = first_accepted(phi, f0, gd, cfg.alpha0, cfg.beta, cfg.c1, cfg.armijo_trials)
    assert q is not None and q >= 1, q
    assert info["alpha"] == cfg.alpha0 * cfg.beta ** q
    assert first_accepted(phi, f0, -gd, cfg.alpha0, cfg.beta, cfg.c1, cfg.armijo_trials) != q
    assert np.array_equal(th_new, th + info["alpha"] * dp)
    assert phi(info["alpha"]) < f0
    cfg = dataclasses.replace(cfg, alpha0=1e4, armijo_trials=2)
    th_rej, status, info = M.gn_sensitivity(geo, th, u, b, w, lam, cfg)
    assert status & M.ST_ARMIJO and np.array_equal(th_rej, th)
