"""GPU parity of the optical-flow temporal regulariser (nlrmm_of_estimate, nlrmm_theta_*,
nlrmm_gram_theta and the solver's temporal mode 2) against the FP64 oracle
(oracle/optical_flow.py) on the same seeded inputs.

Bars: the operators on the same velocities to 1e-5 (FP32 with FP32 bilinear weights against
FP64 weights); the velocity estimate (300 FP32 conjugate-gradient steps) against the exact
minimiser to 1e-4 per pair; the dynamic loop with the OF operator to the loop bars of the
static workloads (u 1e-3, theta 1e-4 rad)."""
import dataclasses
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import method as M  # noqa: E402
from oracle import optical_flow as OF  # noqa: E402
from paper_2605_06336_amd import _lib, ops, synth  # noqa: E402
from paper_2605_06336_amd.solver import Config, Solver  # noqa: E402


def dev(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt).cuda()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def moving_frames(N, F, seed=0):
    """Frames of the dynamic workload's moving-ellipse phantom at N x N."""
    wl = dataclasses.replace(synth.WORKLOADS["c4"], N=N, frames=F, seed=4001 + seed)
    return synth.draw(wl).x_true


def flow_of(frames):
    """Oracle velocities of every pair: [F-1, 2, N, N] float64 and the oracle Flow."""
    fl = OF.estimate_flow(frames)
    arr = np.stack([np.stack([a, b]) for a, b in zip(fl.sx, fl.sy)])
    return arr, fl


@pytest.mark.parametrize("N,F", [(24, 3), (48, 4), (37, 2)])
def test_velocity_estimate_matches_the_exact_minimiser(N, F):
    u32 = moving_frames(N, F).astype(np.float32)
    g = ops.geom(N, 2 * N + 1)
    print(f"case N={N} F={F}", flush=True)
    flow = ops.of_estimate(dev(u32, torch.float32), g, F, 0.05, 1e-3, 300).cpu().numpy()
    ref, _ = flow_of(u32.astype(np.float64))
    assert flow.shape == ref.shape
    errs = [rel(flow[t], ref[t]) for t in range(F - 1)]
    print(f"  per-pair relL2 {['%.2e' % e for e in errs]}", flush=True)
    assert max(errs) <= 1e-4


def test_velocity_estimate_recovers_a_translation():
    """A smooth texture shifted by a known sub-pixel displacement: the device's velocity
    averages to it within a few per cent inside the frame (the same check as the oracle's)."""
    n = 40
    K, L = np.meshgrid(np.arange(n, dtype=np.float64), np.arange(n, dtype=np.float64))

    def tex(x, y):
        return (np.sin(0.45 * x + 0.2 * y) + 0.8 * np.cos(0.3 * y - 0.15 * x)
                + 0.5 * np.sin(0.207 * x + 0.407 * y))

    s0 = (0.3, -0.2)
    u = np.stack([tex(K, L), tex(K - s0[0], L - s0[1])]).astype(np.float32)
    flow = ops.of_estimate(dev(u, torch.float32), ops.geom(n, 57), 2, 0.01, 1e-6,
                           1500).cpu().numpy()
    core = (slice(6, n - 6), slice(6, n - 6))
    mx, my = float(flow[0, 0][core].mean()), float(flow[0, 1][core].mean())
    assert abs(mx - s0[0]) < 0.05 * abs(s0[0]) and abs(my - s0[1]) < 0.05 * abs(s0[1]), (mx, my)


@pytest.mark.parametrize("N,F,kind", [(24, 3, "estimated"), (33, 4, "random"),
                                      (16, 2, "large")])
def test_theta_rows_weights_and_gradient(N, F, kind):
    """Theta u, its MM weights and r + lam Theta^T (w Theta u) (stored and formed weights) on
    the same velocities as the oracle: estimated ones, random ones, and large ones whose
    samples are clamped at the borders."""
    rng = np.random.default_rng(N)
    frames = moving_frames(N, F)
    u = (frames + 0.05 * rng.standard_normal(frames.shape)).astype(np.float32)
    if kind == "estimated":
        flow64, _ = flow_of(frames)
    else:
        amp = 1.5 if kind == "random" else 6.0
        flow64 = rng.uniform(-amp, amp, (F - 1, 2, N, N))
    flow32 = flow64.astype(np.float32)
    geo = M.Geometry(N=N, nb=13, view_off=np.arange(F + 1, dtype=np.int64), temporal=True)
    geo.flow = OF.Flow([f[0].astype(np.float64) for f in flow32],
                       [f[1].astype(np.float64) for f in flow32])
    g = ops.geom(N, 13)
    ud, fd = dev(u, torch.float32), dev(flow32, torch.float32)
    u64 = u.astype(np.float64).reshape(-1)
    print(f"case N={N} F={F} flow={kind}", flush=True)
    t = ops.theta_apply(ud, g, F, 2, fd).cpu().numpy()
    t_ref = M.psi(geo, u64)
    assert t.shape == t_ref.shape and rel(t, t_ref) <= 1e-5, rel(t, t_ref)
    w = ops.theta_weights(ud, g, F, 2, fd, eps=1e-2).cpu().numpy()
    w_ref = M.weights(geo, u64, 1e-2)
    assert rel(w, w_ref) <= 1e-5, rel(w, w_ref)
    r0 = rng.standard_normal(u.size).astype(np.float32)
    lam = 0.37
    lamd = torch.tensor([lam], dtype=torch.float64, device="cuda")
    for wd in (dev(w, torch.float32), None):
        r = ops.theta_grad_add(ud, dev(r0, torch.float32), lamd, g, F, 2, fd, w=wd,
                               eps=1e-2).cpu().numpy().reshape(-1)
        ww = w.astype(np.float64) if wd is not None else w_ref
        r_ref = r0.astype(np.float64) + lam * M.psiT(geo, ww * M.psi(geo, u64))
        d = rel(r - r0, r_ref - r0)
        print(f"  rows {rel(t, t_ref):.2e} weights {rel(w, w_ref):.2e} gradient {d:.2e}",
              flush=True)
        assert d <= 1e-5, d


@pytest.mark.parametrize("ell,N,F", [(9, 24, 3), (33, 40, 4)])
def test_gram_theta_precisions(ell, N, F):
    """(Theta V)^T diag(w) (Theta V) with the motion rows: FP64, FP32-MFMA and BF16-MFMA
    against the oracle's definition on the same velocities and weights."""
    rng = np.random.default_rng(ell)
    frames = moving_frames(N, F, seed=1)
    flow64, _ = flow_of(frames)
    flow32 = flow64.astype(np.float32)
    geo = M.Geometry(N=N, nb=13, view_off=np.arange(F + 1, dtype=np.int64), temporal=True)
    geo.flow = OF.Flow([f[0].astype(np.float64) for f in flow32],
                       [f[1].astype(np.float64) for f in flow32])
    g = ops.geom(N, 13)
    fd = dev(flow32, torch.float32)
    u = frames.astype(np.float32)
    w = ops.theta_weights(dev(u, torch.float32), g, F, 2, fd, eps=1e-3)
    V = np.linalg.qr(rng.standard_normal((geo.n, ell)))[0].T.astype(np.float32)
    Vd = dev(V, torch.float32)
    PV = M.psi_cols(geo, V.T.astype(np.float64))
    G_ref = PV.T @ (w.cpu().numpy().astype(np.float64)[:, None] * PV)
    for prec, tol in ((0, 1e-5), (1, 1e-5), (2, 3e-3)):
        G = ops.gram_theta(Vd, w, g, ell, F, 2, fd, precision=prec).cpu().numpy()
        print(f"  ell={ell} precision {prec}: relL2 {rel(G, G_ref):.2e}", flush=True)
        assert rel(G, G_ref) <= tol, (prec, rel(G, G_ref))


def test_theta_refusals_without_velocities():
    g = ops.geom(16, 23)
    u = torch.zeros((3, 16, 16), dtype=torch.float32, device="cuda")
    with pytest.raises(_lib.NlrmmError):
        ops.theta_apply(u, g, 3, 2, None)
    with pytest.raises(_lib.NlrmmError):
        ops.tv_weights(u, g, 3, 2)        # the velocity-free entry point refuses mode 2
    g1 = ops.geom(1, 23, ny=16)
    with pytest.raises(_lib.NlrmmError):
        ops.of_estimate(torch.zeros((3, 16, 1), dtype=torch.float32, device="cuda"), g1, 3)


def run_of_loop(N, F, outer, kmax, gn):
    c4 = synth.WORKLOADS["c4"]
    # bins scaled with the grid as in the workload (363 bins for 256 pixels)
    wl = dataclasses.replace(c4, N=N, frames=F, nb=int(round(c4.nb * N / c4.N)) | 1)
    inst = synth.draw(wl)
    geo = M.Geometry(N=N, nb=wl.nb, view_off=inst.view_off, temporal=True)
    x64 = inst.x_true.reshape(-1)
    b_ora, e_ora = M.make_data(geo, x64, inst.theta_true, inst.g, wl.noise)
    cfg = M.Config(kmin=wl.kmin, kmax=kmax, eps=wl.eps, gn=gn, of=True)
    g = ops.geom(N, wl.nb)
    fr = ops.Frames(inst.view_off)
    bex = ops.project(dev(inst.x_true.astype(np.float32), torch.float32),
                      dev(inst.theta_true, torch.float64), g, fr).cpu().numpy()
    bex = bex.reshape(-1).astype(np.float64)
    e = wl.noise * np.linalg.norm(bex) * inst.g / np.linalg.norm(inst.g)
    b_gpu = dev((bex + e).astype(np.float32), torch.float32)
    th = dev(inst.theta_nom, torch.float64)
    sol = Solver(g, F, geo.V, Config(kmin=wl.kmin, kmax=kmax, eps=wl.eps, temporal=2,
                                     param_update={"altmin": 1, "none": 0}[gn], of_iters=300))
    sol.init(th, b_gpu, fr)
    st = M.init_state(geo, inst.theta_nom, b_ora, cfg)
    res = []
    for k in range(outer):
        M.outer_step(geo, st, b_ora, np.linalg.norm(e_ora), cfg)
        sol.outer(th, b_gpu, float(np.linalg.norm(e)), fr)
        u, sc, status = sol.read()
        du = rel(u.cpu().numpy().astype(np.float64), st.u)
        dth = float(np.max(np.abs(th.cpu().numpy() - st.theta)))
        res.append((du, dth))
        print(f"outer {k}: u rel diff {du:.3e} theta max diff {dth:.3e} lam gpu "
              f"{float(sc.cpu().numpy()[2]):.5e} ora {st.lam:.5e} status "
              f"{int(status.cpu()[0])}/{st.status}", flush=True)
    sol.close()
    rre = float(np.linalg.norm(st.u - x64) / np.linalg.norm(x64))
    return res, rre


@pytest.mark.parametrize("gn", ["none", "altmin"])
def test_dynamic_loop_with_optical_flow_scaled_c4(gn):
    """The dynamic workload's phantom at 32x32 over 4 frames (30-120 views per frame, 45
    bins), kmax 12, 5 outer iterations of NL-RMM-GKS with Theta = [Psi; M_hat] re-estimated
    from the current image every outer iteration, angles fixed or by AltMin, against the
    oracle's loop."""
    res, rre = run_of_loop(32, 4, 5, 12, gn)
    du, dth = res[-1]
    print(f"OF loop ({gn}): u rel diff {du:.3e}, theta max diff {dth:.3e}, oracle RRE {rre:.4f}")
    assert du <= 1e-3
    assert dth <= 1e-4
