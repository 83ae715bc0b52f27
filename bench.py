"""Benchmark of the NL-RMM-GKS hot path on one MI355X.

One step = one outer iteration of NL-RMM-GKS (AltMin, per-view angles) on the 256x256 /
360-view / 363-bin workload: rebase A V, Enlarge (35 projected solves, 34 Krylov
expansions, each with a projection and a backprojection), Compress, Gauss-Newton angle
update with Armijo trials, residual append.  Inputs are resident in HBM before timing.

Also reported: Gsamples/s of the projector family (one sample = one nonzero (ray, pixel)
weight applied) at the same workload, the roofline of the dominant kernel, and the FP64
oracle timed on a bounded sample on the host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_NONPACKED_PEAK_TFLOPS = 78.6   # 256 CU x 64 FP32 FMA lanes x 2 flop x 2.4 GHz
FLOP_PER_SAMPLE = 10.0              # algorithmic FP32 flops per applied strip-area weight
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--reps", type=int, default=20, help="repetitions per operator timing")
    ap.add_argument("--gram-precision", type=int, default=0, choices=(0, 1, 2),
                    help="regulariser Gram: 0 FP64 vector, 1 FP32 MFMA, 2 BF16 MFMA")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path has no "
              "multi-GPU mode in this build", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2605_06336_amd import metrics, ops, synth
    from paper_2605_06336_amd.solver import Config, Solver

    wl = synth.WORKLOADS["c2"]
    inst = synth.draw(wl)
    N, nb, V = wl.N, wl.nb, wl.n_views
    g = ops.geom(N, nb)
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    x32 = torch.as_tensor(inst.x_true.astype(np.float32), device=dev)
    th_true = torch.as_tensor(inst.theta_true, device=dev)
    bex = ops.project(x32, th_true, g).cpu().numpy().reshape(-1).astype(np.float64)
    e = wl.noise * np.linalg.norm(bex) * inst.g / np.linalg.norm(inst.g)
    delta = float(np.linalg.norm(e))
    b = torch.as_tensor((bex + e).astype(np.float32), device=dev)
    theta = torch.as_tensor(inst.theta_nom.copy(), device=dev)

    cfg = Config(kmin=wl.kmin, kmax=wl.kmax, eps=wl.eps, gram_precision=args.gram_precision)
    sol = Solver(g, 1, V, cfg)
    sol.init(theta, b)
    for _ in range(args.warmup):
        sol.outer(theta, b, delta)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for k in range(args.steps):
        sol.outer(theta, b, delta)
        print(f"# step {k + 1}/{args.steps} enqueued", file=sys.stderr, flush=True)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    ms_per_step = max(gpu_ms, wall * 1e3) / args.steps
    u, sc, status = sol.read()
    torch.cuda.synchronize()
    x_true = inst.x_true.reshape(-1)
    rre = float(np.linalg.norm(u.cpu().numpy() - x_true) / np.linalg.norm(x_true))
    dth0 = inst.theta_true - inst.theta_nom
    perr = float(np.linalg.norm(theta.cpu().numpy() - inst.theta_true) / np.linalg.norm(dth0))
    sol.close()

    # ---- projector family at the same workload -------------------------------------
    nnz = metrics.nnz(N, nb, inst.theta_true)
    y = torch.empty((1, V, nb), dtype=torch.float32, device=dev)
    xb = torch.empty((1, 1, N, N), dtype=torch.float32, device=dev)
    ysrc = b.view(1, V, nb)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a0 = torch.cuda.Event(enable_timing=True)
        a1 = torch.cuda.Event(enable_timing=True)
        a0.record(stream)
        for _ in range(args.reps):
            fn()
        a1.record(stream)
        torch.cuda.synchronize()
        return a0.elapsed_time(a1) / args.reps

    t_proj = timed(lambda: ops.project(x32, th_true, g, out=y))
    t_back = timed(lambda: ops.backproject(ysrc, th_true, g, out=xb))
    t_dth = timed(lambda: ops.project_dtheta(x32, th_true, g, want_dy=True))
    gs = {
        "project": nnz / (t_proj * 1e-3) / 1e9,
        "backproject": nnz / (t_back * 1e-3) / 1e9,
        "dtheta": nnz / (t_dth * 1e-3) / 1e9,
    }
    # dominant kernel: the backprojection (one kernel per call; launched as often as the
    # projection in every Krylov expansion and once more per outer iteration)
    dom_ms = t_back
    achieved = nnz * FLOP_PER_SAMPLE / (dom_ms * 1e-3) / 1e12
    roofline = {
        "bound": "alu",
        "kernel": "bwd_tiles_k (nlrmm_backproject)",
        "achieved": round(achieved, 3),
        "peak": FP32_NONPACKED_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(achieved / FP32_NONPACKED_PEAK_TFLOPS, 4),
        "traffic": None,
        "launch_ms": round(dom_ms, 5),
        "samples_per_launch": int(nnz),
    }

    # ---- FP64 oracle on a bounded sample ---------------------------------------------
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import method as OM
        from oracle import projector as OP
        geo = OM.Geometry(N=N, nb=nb, view_off=inst.view_off)
        b_ora, e_ora = OM.make_data(geo, x_true, inst.theta_true, inst.g, wl.noise)
        ocfg = OM.Config(kmin=wl.kmin, kmax=wl.kmax, eps=wl.eps)
        st = OM.init_state(geo, inst.theta_nom, b_ora, ocfg)
        c0 = time.perf_counter()
        OM.outer_step(geo, st, b_ora, float(np.linalg.norm(e_ora)), ocfg)
        csec = time.perf_counter() - c0
        cpu = {"value": round(1.0 / csec, 5), "unit": "outer it/s", "cores": OP.max_threads(),
               "kind": "oracle",
               "sample": f"one outer iteration (first after the GKB start basis) of the same "
                         f"workload, {csec:.1f} s"}

    out = {
        "metric": "proj+backproj+∂θ Gsamples/s & outer it/s, batched vs plain, relL2≤1e-5",
        "value": round(1000.0 / ms_per_step, 4),
        "unit": "outer it/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "c2-256px-360v: 256x256 image of 25 seeded ellipses, 360 views "
                               "(nominal + N(0,1 deg)), 363 bins, 1% noise, AltMin NL-RMM-GKS "
                               "kmin 5 kmax 40, TV, discrepancy principle",
                   "global_batch": 1, "parallelism": "none"},
        "gsamples_per_s": {k: round(v, 2) for k, v in gs.items()},
        "operator_ms": {"project": round(t_proj, 5), "backproject": round(t_back, 5),
                        "dtheta": round(t_dth, 5)},
        "nnz": int(nnz),
        "quality": {"rre": round(rre, 5), "angle_err_rel": round(perr, 5),
                    "outer_done": args.warmup + args.steps,
                    "lambda": float(sc.cpu().numpy()[2]), "status": int(status.cpu()[0])},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
