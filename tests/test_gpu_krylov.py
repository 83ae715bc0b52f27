"""GPU parity of the Krylov-side entry points and of the NL-RMM-GKS outer loop against the
FP64 oracle.  Bars: primitives on identical FP64 inputs to ~1e-9; the loop after a fixed
number of outer iterations: ||u_gpu - u_ora|| / ||u_ora|| <= 1e-3, max |theta diff| <= 1e-4 rad."""
import dataclasses
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import method as M  # noqa: E402
from oracle import projector as P  # noqa: E402
from paper_2605_06336_amd import ops, synth  # noqa: E402
from paper_2605_06336_amd.solver import Config, Solver  # noqa: E402


def dev(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt).cuda()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def small(N=48, nb=69, V=40, seed=0, F=1, temporal=False):
    rng = np.random.default_rng(seed)
    if F == 1:
        vo = np.array([0, V], dtype=np.int64)
    else:
        vo = np.concatenate([[0], np.cumsum(rng.integers(5, 12, F))]).astype(np.int64)
    geo = M.Geometry(N=N, nb=nb, view_off=vo, temporal=temporal)
    x = synth.ellipse_image(N, [0.1, -0.3], [0.0, 0.2], [0.5, 0.2], [0.3, 0.25], [0.3, 1.0],
                            [1.0, 0.5])
    x = np.stack([np.roll(x, 2 * f, axis=1) for f in range(geo.F)])
    th = rng.uniform(0, math.pi, geo.V)
    return geo, x.reshape(-1), th, rng


@pytest.mark.parametrize("F,temporal", [(1, 0), (3, 1)])
def test_tv_weights_and_gram(F, temporal):
    geo, x, th, rng = small(N=40, nb=59, F=F, temporal=bool(temporal))
    g = ops.geom(geo.N, geo.nb)
    u = (x + 0.05 * rng.standard_normal(x.size)).astype(np.float32)
    w = ops.tv_weights(dev(u, torch.float32), g, geo.F, bool(temporal), eps=1e-2).cpu().numpy()
    w_ref = M.weights(geo, u.astype(np.float64), 1e-2)
    assert w.shape == w_ref.shape
    assert rel(w, w_ref) <= 1e-6
    ell = 13
    V = rng.standard_normal((ell, geo.n)).astype(np.float32)
    G = ops.gram_psi(dev(V, torch.float32), dev(w, torch.float32), g, ell, geo.F,
                     bool(temporal)).cpu().numpy()
    PV = M.psi_cols(geo, V.T.astype(np.float64))
    G_ref = PV.T @ (w.astype(np.float64)[:, None] * PV)
    assert rel(G, G_ref) <= 1e-12


@pytest.mark.parametrize("ell,F,temporal", [(7, 1, 0), (40, 1, 0), (64, 1, 0), (33, 3, 1)])
def test_gram_mfma_precisions(ell, F, temporal):
    """FP32-MFMA and BF16-MFMA regulariser Grams against the FP64 definition."""
    geo, x, th, rng = small(N=72, nb=103, F=F, temporal=bool(temporal))
    g = ops.geom(geo.N, geo.nb)
    u = (x + 0.05 * rng.standard_normal(x.size)).astype(np.float32)
    w = ops.tv_weights(dev(u, torch.float32), g, geo.F, bool(temporal), eps=1e-3)
    V = np.linalg.qr(rng.standard_normal((geo.n, ell)))[0].T.astype(np.float32)
    Vd = dev(V, torch.float32)
    PV = M.psi_cols(geo, V.T.astype(np.float64))
    G_ref = PV.T @ (w.cpu().numpy().astype(np.float64)[:, None] * PV)
    for prec, tol in ((0, 1e-12), (1, 1e-6), (2, 3e-3)):
        G = ops.gram_psi(Vd, w, g, ell, geo.F, bool(temporal), precision=prec).cpu().numpy()
        assert rel(G, G_ref) <= tol, (prec, rel(G, G_ref))


@pytest.mark.parametrize("ell,noise,lam_fix", [(6, 0.01, -1.0), (20, 0.05, -1.0), (33, 0.01, -1.0),
                                               (12, 0.01, 0.37), (1, 0.01, -1.0), (2, 0.05, -1.0),
                                               (47, 0.01, -1.0), (55, 0.01, -1.0)])
def test_gks_solve_matches_oracle(ell, noise, lam_fix):
    geo, x, th, rng = small()
    b, e = M.make_data(geo, x, th, rng.standard_normal(geo.m), noise)
    V = M.gkb_basis(geo, th, b, min(ell, 8))
    if ell > V.shape[1]:
        V, _ = np.linalg.qr(np.column_stack([V, rng.standard_normal((geo.n, ell - V.shape[1]))]))
    AV = M.A_cols(geo, th, V)
    PV = M.psi_cols(geo, V)
    w = M.weights(geo, x + 0.02 * rng.standard_normal(geo.n), 1e-3)
    st = M.State(V=V, AV=AV, PV=PV, u=np.zeros(geo.n), theta=th)
    target = 1.01 * np.linalg.norm(e)
    cfg = M.Config(lam_fix=None if lam_fix < 0 else lam_fix)
    z_ref, lam_ref, _, _, flag_ref = M.projected_solve(st, b, w, cfg, target)
    GA = AV.T @ AV
    GP = PV.T @ (w[:, None] * PV)
    rb = AV.T @ b
    scal = np.array([b @ b, target])
    z, out, status = ops.gks_solve(dev(GA, torch.float64), dev(GP, torch.float64),
                                   dev(rb, torch.float64), dev(scal, torch.float64), ell, lam_fix)
    z = z.cpu().numpy()
    lam = out.cpu().numpy()[0]
    assert int(status.cpu()[0]) == flag_ref
    assert abs(lam - lam_ref) <= 1e-8 * lam_ref
    assert rel(V @ z, V @ z_ref) <= 1e-7
    if lam_fix < 0 and flag_ref == 0:
        res = np.linalg.norm(AV @ z - b)
        assert abs(res - target) <= 1e-8 * target


def test_gks_expand_and_compress_match_oracle():
    geo, x, th, rng = small(N=40, nb=59, V=30)
    g = ops.geom(geo.N, geo.nb)
    b, e = M.make_data(geo, x, th, rng.standard_normal(geo.m), 0.01)
    b32 = b.astype(np.float32)
    ell, kmax, kmin = 6, 12, 4
    V = M.gkb_basis(geo, th, b32.astype(np.float64), ell)
    V32 = V.astype(np.float32)
    Vd = torch.zeros((kmax, geo.n), dtype=torch.float32, device="cuda")
    Vd[:ell] = dev(V32.T, torch.float32)
    AVd = torch.zeros((kmax, geo.m), dtype=torch.float32, device="cuda")
    tht = dev(th, torch.float64)
    AVd[:ell] = ops.project(Vd[:ell].contiguous().view(ell, 1, geo.N, geo.N), tht, g).view(ell, -1)
    V64 = Vd[:ell].cpu().numpy().astype(np.float64).T
    AV64 = AVd[:ell].cpu().numpy().astype(np.float64).T
    GA = np.zeros((kmax, kmax))
    GA[:ell, :ell] = AV64.T @ AV64
    rb = np.zeros(kmax)
    rb[:ell] = AV64.T @ b32.astype(np.float64)
    z = rng.standard_normal(ell) * 0.1
    u = (V64 @ z).astype(np.float32)
    w = M.weights(geo, u.astype(np.float64), 1e-3).astype(np.float32)
    lam = 0.02
    GAd, rbd = dev(GA, torch.float64), dev(rb, torch.float64)
    lamd = dev(np.array([lam]), torch.float64)
    status = ops.gks_expand(Vd, AVd, dev(z, torch.float64), dev(b32, torch.float32),
                            dev(w, torch.float32), lamd, GAd, rbd, tht, g, ell)
    torch.cuda.synchronize()
    # oracle: residual from the same FP32 basis, CGS2, normalise
    st = M.State(V=V64, AV=AV64, PV=M.psi_cols(geo, V64), u=V64 @ z, theta=th)
    r = M.mm_residual(geo, th, st, b32.astype(np.float64), w.astype(np.float64), lam, z)
    v_ref = M.cgs2(V64, r)
    v_ref /= np.linalg.norm(v_ref)
    v = Vd[ell].cpu().numpy().astype(np.float64)
    assert int(status.cpu()[0]) == 0
    assert rel(v, v_ref) <= 2e-5
    Av = AVd[ell].cpu().numpy().astype(np.float64)
    assert rel(Av, M.A(geo, th, v)) <= 1e-5
    GAn = GAd.cpu().numpy()
    AVn = AVd[:ell + 1].cpu().numpy().astype(np.float64).T
    assert rel(GAn[:ell + 1, :ell + 1], AVn.T @ AVn) <= 1e-12
    assert abs(rbd.cpu().numpy()[ell] - AVn[:, ell] @ b32.astype(np.float64)) <= 1e-10 * np.abs(rb).max()
    # compress the (ell+1)-column basis to kmin with a DP-free lambda and a GP from weights
    ell1 = ell + 1
    PV = M.psi_cols(geo, Vd[:ell1].cpu().numpy().astype(np.float64).T)
    GP = PV.T @ (w.astype(np.float64)[:, None] * PV)
    GPf = np.zeros((kmax, kmax))
    GPf[:ell1, :ell1] = GP
    z1 = np.concatenate([z, [0.05]])
    V_before = Vd[:ell1].cpu().numpy().astype(np.float64).T
    u_before = V_before @ z1
    zd = torch.zeros(kmax, dtype=torch.float64, device="cuda")
    zd[:ell1] = dev(z1, torch.float64)
    st2 = ops.recycle_compress(Vd, AVd, GAd, dev(GPf, torch.float64), rbd, lamd, zd, ell1, kmin)
    torch.cuda.synchronize()
    Vn = Vd[:kmin].cpu().numpy().astype(np.float64).T
    zn = zd[:kmin].cpu().numpy()
    assert int(st2.cpu()[0]) == 0
    assert np.linalg.norm(Vn.T @ Vn - np.eye(kmin)) <= 1e-5
    assert rel(Vn @ zn, u_before) <= 1e-5
    # oracle compress on the same inputs (RA, RP from the Grams' Cholesky factors)
    RA = np.linalg.cholesky(AVn.T @ AVn).T
    RP = np.linalg.cholesky(GP).T
    ost = M.State(V=V_before, AV=AVn, PV=PV, u=u_before, theta=th)
    Vold = ost.V.copy()
    M.compress(ost, RA, RP, lam, z1, kmin)
    s = np.linalg.svd(ost.V.T @ Vn, compute_uv=False)
    assert np.min(s) > 1 - 1e-5
    assert rel(zn, ost.z) <= 1e-5
    assert rel(AVd[:kmin].cpu().numpy().astype(np.float64).T, AVn @ (Vold.T @ Vn)) <= 1e-5


def run_pair(key, N=None, outer=None, kmax=None, trace=False, gram_precision=0, lam_hi=None,
             gn="altmin", wl=None, sens_iters=50, ret_state=False):
    wl = wl or synth.WORKLOADS[key]
    inst = synth.draw(wl, N=N)
    N = inst.x_true.shape[-1]
    outer = outer or wl.outer
    kmax = kmax or wl.kmax
    geo = M.Geometry(N=N, nb=wl.nb, view_off=inst.view_off)
    x64 = inst.x_true.reshape(-1)
    b_ora, e_ora = M.make_data(geo, x64, inst.theta_true, inst.g, wl.noise)
    cfg = M.Config(kmin=wl.kmin, kmax=kmax, eps=wl.eps, lam_hi=lam_hi, gn=gn,
                   sens_iters=sens_iters)
    # GPU data: own projector, same noise direction
    g = ops.geom(N, wl.nb)
    x32 = inst.x_true.astype(np.float32)
    bex = ops.project(dev(x32, torch.float32), dev(inst.theta_true, torch.float64),
                      g).cpu().numpy().reshape(-1).astype(np.float64)
    e = wl.noise * np.linalg.norm(bex) * inst.g / np.linalg.norm(inst.g)
    b_gpu = dev((bex + e).astype(np.float32), torch.float32)
    th = dev(inst.theta_nom, torch.float64)
    sol = Solver(g, 1, geo.V, Config(kmin=wl.kmin, kmax=kmax, eps=wl.eps,
                                     gram_precision=gram_precision,
                                     lam_hi=lam_hi if lam_hi is not None else 0.0,
                                     param_update={"altmin": 1, "varpro": 2,
                                                   "sensitivity": 3}[gn],
                                     param_mode=1 if gn == "sensitivity" else 0,
                                     sens_iters=sens_iters))
    sol.init(th, b_gpu)
    ora_log = []
    st = M.init_state(geo, inst.theta_nom, b_ora, cfg)
    out = []
    for k in range(outer):
        M.outer_step(geo, st, b_ora, np.linalg.norm(e_ora), cfg)
        sol.outer(th, b_gpu, float(np.linalg.norm(e)))
        if trace or k == outer - 1:
            u, sc, status = sol.read()
            u = u.cpu().numpy().astype(np.float64)
            du = rel(u, st.u)
            dth = float(np.max(np.abs(th.cpu().numpy() - st.theta)))
            lam = float(sc.cpu().numpy()[2])
            out.append((k, du, dth, lam, st.lam, int(status.cpu()[0]), st.status))
            print(f"outer {k}: u rel diff {du:.3e}  theta max diff {dth:.3e}  lam gpu {lam:.6e} "
                  f"ora {st.lam:.6e} status {int(status.cpu()[0])}/{st.status}", flush=True)
    th_gpu = th.cpu().numpy()
    sol.close()
    rre_ora = np.linalg.norm(st.u - x64) / np.linalg.norm(x64)
    if ret_state:
        return out, rre_ora, st, th_gpu, inst
    return out, rre_ora


@pytest.mark.parametrize("gram_precision", [0, 1])
def test_loop_parity_c1(gram_precision):
    """64x64, 90 views, 91 bins, 20 outer iterations, basis cap 30 (the FP64 CPU workload);
    regulariser Gram in FP64 on the vector units, or on the FP32 matrix cores."""
    out, rre = run_pair("c1", trace=True, gram_precision=gram_precision)
    k, du, dth, *_ = out[-1]
    print(f"c1 final: u rel diff {du:.3e}, theta max diff {dth:.3e} rad, oracle RRE {rre:.4f}")
    assert du <= 1e-3
    assert dth <= 1e-4


@pytest.mark.parametrize("gn", ["altmin", "varpro"])
def test_loop_parity_c1_high_regularisation(gn):
    """The optional high-regularisation solve (Section 4.3, lam_hi = 3e-3, about twice the DP
    lambda of this workload): 8 outer iterations of the c1 workload, AltMin or VarPro angle
    update on u_hat, against the oracle."""
    out, rre = run_pair("c1", outer=8, trace=True, lam_hi=3e-3, gn=gn)
    k, du, dth, *_ = out[-1]
    print(f"c1 lam_hi {gn}: u rel diff {du:.3e}, theta max diff {dth:.3e} rad, "
          f"oracle RRE {rre:.4f}")
    assert du <= 1e-3
    assert dth <= 1e-4


@pytest.mark.parametrize("lam_hi", [None, 3e-3])
def test_loop_parity_c1_sensitivity_update(lam_hi):
    """Parameter update of one global offset by the full-space sensitivity equation (Section
    4.2, eqs. "sensitivity" and "GN_system"; 50 conjugate-gradient steps for u_p, Armijo on
    the compressed-basis reduced objective), alone and after the high-regularisation solve,
    on the c1 workload with every true angle shifted by 0.5 degrees and no per-view
    perturbation: 20 (8 with lam_hi) outer iterations against the oracle; the offset found
    moves most of the way to the true one."""
    wl = dataclasses.replace(synth.WORKLOADS["c1"], sigma_deg=0.0, offset_deg=0.5)
    outer = 20 if lam_hi is None else 8
    out, rre, st, th_gpu, inst = run_pair("c1", outer=outer, trace=True, gn="sensitivity",
                                          wl=wl, lam_hi=lam_hi, ret_state=True)
    k, du, dth, *_ = out[-1]
    off_g = float(np.mean(th_gpu - inst.theta_nom))
    off_o = float(np.mean(st.theta - inst.theta_nom))
    print(f"c1 sensitivity update (lam_hi {lam_hi}): u rel diff {du:.3e}, theta max diff "
          f"{dth:.3e} rad; offset gpu {math.degrees(off_g):.5f} oracle {math.degrees(off_o):.5f}"
          f" true 0.5 deg; oracle RRE {rre:.4f}")
    assert du <= 1e-3
    assert dth <= 1e-4
    # one offset for all views
    assert np.ptp(th_gpu - inst.theta_nom) <= 1e-12
    if lam_hi is None:
        assert abs(math.degrees(off_o) - 0.5) < 0.25


@pytest.mark.parametrize("ell,kmin", [(6, 2), (20, 5), (41, 5), (48, 16), (55, 16)])
def test_compress_sizes_match_oracle(ell, kmin):
    """Compression at every padded size of the one-wave kernel, kmin up to 16, against the
    oracle's SVD-based Alg. "compress" on the same FP64 Grams."""
    rng = np.random.default_rng(ell * 100 + kmin)
    n, m = 300, 400
    V = np.linalg.qr(rng.standard_normal((n, ell)))[0].astype(np.float32).astype(np.float64)
    AV = rng.standard_normal((m, ell)).astype(np.float32).astype(np.float64)
    Pm = rng.standard_normal((2 * n, ell)) * 0.3
    GA = AV.T @ AV
    GP = Pm.T @ Pm
    z = rng.standard_normal(ell)
    lam = 0.7
    kmax = 56
    Vd = torch.zeros((kmax, n), dtype=torch.float32, device="cuda")
    Vd[:ell] = dev(V.T, torch.float32)
    AVd = torch.zeros((kmax, m), dtype=torch.float32, device="cuda")
    AVd[:ell] = dev(AV.T, torch.float32)
    GAf = np.zeros((kmax, kmax))
    GAf[:ell, :ell] = GA
    GPf = np.zeros((kmax, kmax))
    GPf[:ell, :ell] = GP
    zd = torch.zeros(kmax, dtype=torch.float64, device="cuda")
    zd[:ell] = dev(z, torch.float64)
    rbd = torch.zeros(kmax, dtype=torch.float64, device="cuda")
    st = ops.recycle_compress(Vd, AVd, dev(GAf, torch.float64), dev(GPf, torch.float64), rbd,
                              dev(np.array([lam]), torch.float64), zd, ell, kmin)
    torch.cuda.synchronize()
    assert int(st.cpu()[0]) == 0
    Vn = Vd[:kmin].cpu().numpy().astype(np.float64).T
    zn = zd[:kmin].cpu().numpy()
    ost = M.State(V=V.copy(), AV=AV.copy(), PV=np.zeros((1, ell)), u=V @ z, theta=np.zeros(1))
    T_ref = M.compress(ost, np.linalg.cholesky(GA).T, np.linalg.cholesky(GP).T, lam, z, kmin)
    print(f"compress ell={ell} kmin={kmin}: V {rel(Vn, V @ T_ref):.2e} z {rel(zn, ost.z):.2e}")
    assert rel(Vn, V @ T_ref) <= 1e-5
    assert rel(zn, ost.z) <= 1e-5


@pytest.mark.parametrize("ell,kmin", [(20, 5), (55, 16)])
def test_compress_bf16_products(ell, kmin):
    """The mixed-precision compression (BF16 operands, FP32 accumulation on the matrix cores
    for V [W, c] and A V [W, c]) against the FP32/FP64 one on the same inputs: relL2 of the new
    bases and of u = V z within the BF16 basis-path bar 3e-3; z (FP64 eigen-problem) equal."""
    rng = np.random.default_rng(ell + 7 * kmin)
    n, m, kmax = 5000, 3000, 56
    V = np.linalg.qr(rng.standard_normal((n, ell)))[0].astype(np.float32)
    AV = rng.standard_normal((m, ell)).astype(np.float32)
    Pm = rng.standard_normal((2 * n, ell)) * 0.3
    GAf = np.zeros((kmax, kmax))
    GAf[:ell, :ell] = AV.T.astype(np.float64) @ AV.astype(np.float64)
    GPf = np.zeros((kmax, kmax))
    GPf[:ell, :ell] = Pm.T @ Pm
    z = rng.standard_normal(ell)
    outs = []
    for prec in (0, 2):
        Vd = torch.zeros((kmax, n), dtype=torch.float32, device="cuda")
        Vd[:ell] = dev(V.T, torch.float32)
        AVd = torch.zeros((kmax, m), dtype=torch.float32, device="cuda")
        AVd[:ell] = dev(AV.T, torch.float32)
        zd = torch.zeros(kmax, dtype=torch.float64, device="cuda")
        zd[:ell] = dev(z, torch.float64)
        st = ops.recycle_compress(Vd, AVd, dev(GAf, torch.float64), dev(GPf, torch.float64),
                                  torch.zeros(kmax, dtype=torch.float64, device="cuda"),
                                  dev(np.array([0.5]), torch.float64), zd, ell, kmin,
                                  precision=prec)
        torch.cuda.synchronize()
        assert int(st.cpu()[0]) == 0
        outs.append((Vd[:kmin].cpu().numpy().astype(np.float64),
                     AVd[:kmin].cpu().numpy().astype(np.float64), zd[:kmin].cpu().numpy()))
    (V0, A0, z0), (V2, A2, z2) = outs
    u0, u2 = V0.T @ z0, V2.T @ z2
    print(f"bf16 compress ell={ell} kmin={kmin}: V {rel(V2, V0):.2e} AV {rel(A2, A0):.2e} "
          f"u {rel(u2, u0):.2e}")
    assert rel(V2, V0) <= 3e-3 and rel(A2, A0) <= 3e-3 and rel(u2, u0) <= 3e-3
    assert rel(z2, z0) <= 1e-12
    assert rel(u0, V.astype(np.float64) @ z) <= 1e-5


def test_grid_search_matches_oracle():
    """Coarse grid search of one global offset (nlrmm_solver_grid_search) on the c1 workload
    with its per-view angle errors plus a 0.8 degree offset: the reduced residual of every
    candidate against the oracle (GKB basis of 10 vectors in both; the residual is ||b||^2
    minus a fit of nearly equal size, so the bar is absolute: 1e-6 ||b||^2, FP32 basis
    vectors), the same best candidate, and theta shifted by it."""
    wl = synth.WORKLOADS["c1"]
    inst = synth.draw(wl)
    N = wl.N
    geo = M.Geometry(N=N, nb=wl.nb, view_off=inst.view_off)
    s_true = math.radians(0.8)
    th_data = inst.theta_true + s_true
    g = ops.geom(N, wl.nb)
    x32 = inst.x_true.astype(np.float32)
    bex = ops.project(dev(x32, torch.float32), dev(th_data, torch.float64),
                      g).cpu().numpy().reshape(-1).astype(np.float64)
    e = wl.noise * np.linalg.norm(bex) * inst.g / np.linalg.norm(inst.g)
    b32 = (bex + e).astype(np.float32)
    shifts = np.radians(np.arange(-2.0, 2.01, 0.25))
    _, res_ora, best_ora = M.grid_search_shift(geo, inst.theta_nom, b32.astype(np.float64),
                                               shifts, ell0=10)
    sol = Solver(g, 1, geo.V, Config(kmin=wl.kmin, kmax=wl.kmax, eps=wl.eps))
    th = dev(inst.theta_nom, torch.float64)
    res2, best = sol.grid_search(th, dev(b32, torch.float32), dev(shifts, torch.float64), 10)
    torch.cuda.synchronize()
    sol.close()
    res2 = res2.cpu().numpy()
    bb = float(b32.astype(np.float64) @ b32.astype(np.float64))
    err = float(np.max(np.abs(res2 - res_ora))) / bb
    order = np.sort(res_ora)
    print(f"grid search: max |res2 diff| / ||b||^2 {err:.2e}, best gpu {int(best.cpu()[0])} "
          f"ora {best_ora} ({math.degrees(shifts[best_ora]):+.2f} deg), runner-up gap "
          f"{(order[1] - order[0]) / bb:.2e}", flush=True)
    assert err <= 1e-6
    if (order[1] - order[0]) / bb > 1e-5:
        assert int(best.cpu()[0]) == best_ora
    assert np.array_equal(th.cpu().numpy(), inst.theta_nom + shifts[int(best.cpu()[0])])


def test_offset_sensitivity_matches_oracle():
    """Full-space sensitivity for one global offset (nlrmm_solver_offset_sensitivity) at the
    image and lambda of one outer iteration, against the dense oracle of eq. "sensitivity" on
    the same u (FP32 values), weights of u and lambda: u_p, g, h and dp."""
    N, nb, V = 24, 35, 30
    rng = np.random.default_rng(31)
    geo = M.Geometry(N=N, nb=nb, view_off=np.array([0, V], dtype=np.int64))
    x = synth.ellipse_image(N, [0.1, -0.3], [0.0, 0.2], [0.5, 0.2], [0.3, 0.25], [0.3, 1.0],
                            [1.0, 0.5]).reshape(-1)
    th = np.arange(V) * math.pi / V + rng.normal(0, 0.01, V)
    g = ops.geom(N, nb)
    b64, e = M.make_data(geo, x, th, rng.standard_normal(geo.m), 0.01)
    b32 = b64.astype(np.float32)
    cfg = Config(kmin=3, kmax=12, eps=1e-2, param_update=0)
    sol = Solver(g, 1, V, cfg)
    tht, bt = dev(th, torch.float64), dev(b32, torch.float32)
    sol.init(tht, bt)
    sol.outer(tht, bt, float(np.linalg.norm(e)))
    u, sc, _ = sol.read()
    out, up = sol.offset_sensitivity(tht, bt, iters=400)
    torch.cuda.synchronize()
    sol.close()
    u64 = u.cpu().numpy().astype(np.float64)
    lam = float(sc.cpu().numpy()[2])
    w = M.weights(geo, u64, 1e-2)
    up_ref, g_ref, h_ref, dp_ref = M.offset_sensitivity(geo, th, u64, b32.astype(np.float64), w,
                                                         lam)
    o = out.cpu().numpy()
    up = up.cpu().numpy().astype(np.float64)
    print(f"offset sensitivity: u_p {rel(up, up_ref):.2e}  g {o[0]:.6e}/{g_ref:.6e}  "
          f"h {o[1]:.6e}/{h_ref:.6e}  dp {o[2]:.6e}/{dp_ref:.6e}  lam {lam:.3e}", flush=True)
    assert rel(up, up_ref) <= 1e-3
    assert abs(o[0] - g_ref) <= 1e-3 * abs(g_ref)
    assert abs(o[1] - h_ref) <= 1e-3 * abs(h_ref)
    assert abs(o[2] - dp_ref) <= 2e-3 * abs(dp_ref)
