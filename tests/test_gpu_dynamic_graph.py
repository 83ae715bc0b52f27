"""GPU tests of the batched multi-frame path: the dynamic workload (block-diagonal operator
over frames with uneven view counts, ANISO-TV with frame differences) against the oracle,
batched single launches against plain per-frame launches, and HIP-graph replays of the outer
iteration against eager execution (bitwise)."""
import dataclasses

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import method as M  # noqa: E402
from paper_2605_06336_amd import ops, synth  # noqa: E402
from paper_2605_06336_amd.solver import Config, OuterGraph, Solver  # noqa: E402


def dev(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt).cuda()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def dyn_instance(N=64, frames=6):
    wl = dataclasses.replace(synth.WORKLOADS["c4"], N=N, frames=frames)
    inst = synth.draw(wl)
    geo = M.Geometry(N=N, nb=wl.nb if N == 256 else int(np.ceil(np.sqrt(2) * N)) + 1,
                     view_off=inst.view_off, temporal=True)
    return wl, inst, geo


def gpu_data(inst, geo, wl, fr):
    g = ops.geom(geo.N, geo.nb)
    x32 = inst.x_true.astype(np.float32)
    g_noise = np.random.default_rng(wl.seed).standard_normal(geo.m)
    bex = ops.project(dev(x32, torch.float32), dev(inst.theta_true, torch.float64), g,
                      fr).cpu().numpy().reshape(-1).astype(np.float64)
    e = wl.noise * np.linalg.norm(bex) * g_noise / np.linalg.norm(g_noise)
    return g, g_noise, dev((bex + e).astype(np.float32), torch.float32), float(np.linalg.norm(e))


def saturated_start(st, geo, seed=11, pert=1e-9):
    rng = np.random.default_rng(seed)
    st.V = np.linalg.qr(st.V + pert * rng.standard_normal(st.V.shape))[0]
    st.PV = M.psi_cols(geo, st.V)


def test_dynamic_batched_and_plain_match_oracle():
    wl, inst, geo = dyn_instance()
    fr = ops.Frames(inst.view_off)
    g, g_noise, b_gpu, delta = gpu_data(inst, geo, wl, fr)
    kmax, outer = 20, 3
    cfg = M.Config(kmin=5, kmax=kmax, eps=wl.eps)
    b_ora, e_ora = M.make_data(geo, inst.x_true.reshape(-1), inst.theta_true, g_noise, wl.noise)
    st = M.init_state(geo, inst.theta_nom, b_ora, cfg)
    saturated_start(st, geo)
    sols = {}
    for mode in ("batched", "plain"):
        sol = Solver(g, geo.F, geo.V, Config(kmin=5, kmax=kmax, eps=wl.eps, temporal=1))
        if mode == "plain":
            sol.set_per_frame(inst.view_off)
        th = dev(inst.theta_nom, torch.float64)
        sol.init(th, b_gpu, fr)
        sols[mode] = (sol, th)
    for k in range(outer):
        M.outer_step(geo, st, b_ora, np.linalg.norm(e_ora), cfg)
        for mode, (sol, th) in sols.items():
            sol.outer(th, b_gpu, delta, fr)
        res = {}
        for mode, (sol, th) in sols.items():
            u, sc, status = sol.read()
            res[mode] = (u.cpu().numpy(), th.cpu().numpy())
            print(f"dynamic outer {k} {mode}: u rel diff {rel(res[mode][0], st.u):.3e} "
                  f"theta max diff {np.max(np.abs(res[mode][1] - st.theta)):.3e}", flush=True)
    for mode in sols:
        assert rel(res[mode][0], st.u) <= 1e-3
        assert np.max(np.abs(res[mode][1] - st.theta)) <= 1e-4
    for sol, _ in sols.values():
        sol.close()


def test_graph_replay_equals_eager_bitwise():
    wl, inst, geo = dyn_instance(N=48, frames=4)
    fr = ops.Frames(inst.view_off)
    g, _, b_gpu, delta = gpu_data(inst, geo, wl, fr)
    cfg = Config(kmin=4, kmax=14, eps=wl.eps, temporal=1)
    runs = []
    for use_graph in (False, True):
        sol = Solver(g, geo.F, geo.V, cfg)
        th = dev(inst.theta_nom, torch.float64)
        sol.init(th, b_gpu, fr)
        sol.outer(th, b_gpu, delta, fr)            # eager warm-up iteration
        snaps = []
        if use_graph:
            gr = OuterGraph(sol, th, b_gpu, delta, fr)   # capture does not execute
            for _ in range(4):
                gr.replay()
                torch.cuda.synchronize()
                _ = torch.ones(1000, device="cuda").sum()   # unrelated eager work in between
                snaps.append((sol.read()[0].cpu().numpy(), th.cpu().numpy()))
        else:
            for _ in range(4):
                sol.outer(th, b_gpu, delta, fr)
                snaps.append((sol.read()[0].cpu().numpy(), th.cpu().numpy()))
        runs.append(snaps)
        sol.close()
    for (ue, te), (ug, tg) in zip(*runs):
        assert np.array_equal(ue, ug)
        assert np.array_equal(te, tg)
