"""Benchmark of the NL-RMM-GKS hot path on one MI355X.

One step = one outer iteration of NL-RMM-GKS (AltMin, per-view angles) on the 256x256 /
360-view / 363-bin workload: rebase A V, Enlarge (35 projected solves, 34 Krylov
expansions, each with a projection and a backprojection), Compress, Gauss-Newton angle
update with Armijo trials, residual append.  Inputs are resident in HBM before timing.  The
rate of the same iteration captured once as a HIP graph and replayed is reported beside it.

Also reported:
  * the in-loop duration per launch of the two projector kernels (HIP events recorded by the
    library on the launch stream around every single one-column launch during the timed
    outer iterations), and the roofline of the one with the most time per outer iteration
    (algorithmic FP32 flops per launch over that duration, against the published FP32 vector
    peak, with the unpacked-FP32 rate beside it), with the HBM bytes and VALU instructions per
    launch of the same launch shape from the committed counter runs
    (profiles/projector_c2_counters.json): the traffic over the algorithmic bytes and the
    fraction of the chip's VALU issue rate the launch uses;
  * parity: the same iteration run for the workload's full outer count against the FP64
    oracle's run stored under tests/golden, and the four operators against the oracle on the
    same inputs (in the host-baseline leg);
  * Gsamples/s of the projector family (project, backproject, angle derivative and its
    transpose; one sample = one nonzero (ray, pixel) weight applied) at the same workload,
    per call and per kernel (single launches between HIP events);
  * outer it/s of the 32-frame dynamic workload, batched (one launch over all frames, the
    outer iteration replayed as a HIP graph) against plain (per-frame launches, eager), with
    the difference of the two reconstructions after the same iterations; the same workload
    with the optical-flow regulariser (velocities re-estimated every outer iteration) and the
    time of one velocity estimation;
  * ms of the full-space sensitivity solve of one global offset (50 CG steps) at the same
    workload;
  * Gsamples/s of the three operators at the shape of every workload (64x64 up to
    2048x2048 / 1440 views, and one 22-view block of the streaming workload);
  * outer it/s of VarPro NL-RMM-GKS on the 512x512 / 720-view workload;
  * ms per forward + backward of the autograd data loss at that workload;
  * outer it/s of the 256x256 iteration under each precision policy (FP64 Grams, FP32
    matrix-core Grams, BF16 matrix-core Grams and compression products);
  * ms per block of streaming NL-RMM-GKS at 2048x2048 / 1440 views in 64 blocks;
  * ms per call of the four fan-beam operators at the 256x256 / 360-view shape (source at
    four image half-widths);
  * the FP64 oracle timed on a bounded sample on the host: the median of three outer
    iterations and one application of each operator.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-dynamic]
                       [--no-workloads]
       python bench.py --ops-only     (operators and a copy calibration only, for counters)
       python bench.py --streaming-only --steps K   (K blocks of the streaming workload only)
       python bench.py --dynamic-only --steps K --warmup W   (the 32-frame dynamic leg only)
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK_TFLOPS = 157.3     # published MI355X FP32 vector peak (packed FMA)
FP32_NONPACKED_PEAK_TFLOPS = 78.6   # 256 CU x 64 FP32 FMA lanes x 2 flop x 2.4 GHz (unpacked)
FLOP_PER_SAMPLE = 10.0              # algorithmic FP32 flops per applied strip-area weight
LOOP_FIXTURE = os.path.join(ROOT, "tests", "golden", "loop_c2_oracle.npz")
TIMING_PERIOD = 4                   # in-loop kernel timing samples every 4th launch
COUNTER_FILE = os.path.join(ROOT, "profiles", "projector_c2_counters.json")
VALU_ISSUE_PER_US = 1024 * 2400 / 4.0   # wave64 VALU instructions the chip issues per us
COPY_BYTES = 256 << 20              # calibration copy for the HBM byte counters
HBM_PEAK_GBS = 8000.0               # MI355X HBM3E
MFMA_PEAK_TFLOPS = {1: 157.3, 2: 2500.0}   # dense matrix-core peaks: FP32, BF16


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dynamic", action="store_true", help="skip the batched-vs-plain leg")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the extra legs: operator rates at every workload shape, VarPro, "
                         "autograd, precision policy, streaming and the sensitivity solve")
    ap.add_argument("--ops-only", action="store_true",
                    help="only the operator timings and the copy calibration")
    ap.add_argument("--dynamic-only", action="store_true",
                    help="only the 32-frame dynamic leg (plain, batched, optical flow)")
    ap.add_argument("--streaming-only", action="store_true",
                    help="only the streaming block timing (for a kernel trace of one block)")
    ap.add_argument("--gram-only", action="store_true",
                    help="only the regulariser-Gram timings on the matrix cores")
    ap.add_argument("--reps", type=int, default=20, help="repetitions per operator timing")
    ap.add_argument("--gram-precision", type=int, default=1, choices=(0, 1, 2),
                    help="regulariser Gram: 0 FP64 vector, 1 FP32 MFMA, 2 BF16 MFMA")
    return ap.parse_args()


def source_digest():
    """Digest of the projector source and the headers it includes: counters recorded for
    another version are void."""
    h = hashlib.sha256()
    for name in ("proj.hip", "internal.h", "multidot.h", "tv.h", "wave.h"):
        with open(os.path.join(ROOT, "paper_2605_06336_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def make_data(torch, ops, inst, wl, g, fr=None):
    dev = torch.device("cuda", 0)
    x32 = torch.as_tensor(inst.x_true.astype(np.float32), device=dev)
    th_true = torch.as_tensor(inst.theta_true, device=dev)
    bex = ops.project(x32, th_true, g, fr).cpu().numpy().reshape(-1).astype(np.float64)
    e = wl.noise * np.linalg.norm(bex) * inst.g / np.linalg.norm(inst.g)
    b = torch.as_tensor((bex + e).astype(np.float32), device=dev)
    return x32, th_true, b, float(np.linalg.norm(e))


def timed_steps(torch, step, steps, stream, label):
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for k in range(steps):
        step()
        print(f"# {label} step {k + 1}/{steps} enqueued", file=sys.stderr, flush=True)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return max(e0.elapsed_time(e1), wall * 1e3) / steps


def operators(torch, ops, metrics, inst, wl, g, x32, th_true, b, reps, stream):
    """Per-call and per-kernel times of project / backproject / dtheta at one workload."""
    dev = x32.device
    N, nb, V = wl.N, wl.nb, wl.n_views
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
        for _ in range(reps):
            fn()
        a1.record(stream)
        torch.cuda.synchronize()
        return a0.elapsed_time(a1) / reps

    proj = lambda: ops.project(x32, th_true, g, out=y)              # noqa: E731
    back = lambda: ops.backproject(ysrc, th_true, g, out=xb)        # noqa: E731
    dth = lambda: ops.project_dtheta(x32, th_true, g, want_dy=True)  # noqa: E731
    dtt = lambda: ops.backproject_dtheta(ysrc, th_true, g, out=xb)   # noqa: E731
    call_ms = {"project": timed(proj), "backproject": timed(back), "dtheta": timed(dth),
               "dtheta_transpose": timed(dtt)}
    # the two projector kernels alone: HIP events around every single launch
    ops.set_kernel_timing(-1)
    for _ in range(reps):
        proj()
    fwd_ms, _ = ops.kernel_avg("project")
    for _ in range(reps):
        back()
    bwd_ms, _ = ops.kernel_avg("backproject")
    ops.set_kernel_timing(False)
    kern_ms = {"fwd_edges_k": fwd_ms, "bwd_tiles_k": bwd_ms}
    return nnz, call_ms, kern_ms


def copy_calibration(torch):
    """A plain device copy of known size: the scale of the HBM byte counters."""
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def counters_for(kernel, tuned):
    """HBM bytes and VALU instructions per launch of `kernel` at the c2 shape, in the launch
    shape the autotuner chose, from the committed counter runs; None when absent or recorded
    for another version of the projector source."""
    try:
        with open(COUNTER_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha") != source_digest():
        return None
    k = rec.get("kernels", {}).get(kernel, {})
    if kernel == "fwd_edges_k":
        return k.get("by_waves_per_block", {}).get(str(tuned.get("fwd_waves_per_block_1col")))
    return k.get("by_view_split", {}).get(str(tuned.get("bwd_view_split")))


def loop_parity(torch, ops, inst, wl, g, b, delta, Config, Solver, gram_precision):
    """The benchmark's iteration run from the GKB start for the workload's full outer count
    against the FP64 oracle's run stored by tests/golden/make_loops.py: relative L2 of the
    image and the largest angle difference."""
    try:
        fx = np.load(LOOP_FIXTURE)
    except OSError:
        return None
    theta = torch.as_tensor(inst.theta_nom.copy(), device="cuda")
    sol = Solver(g, 1, wl.n_views, Config(kmin=wl.kmin, kmax=wl.kmax, eps=wl.eps,
                                          gram_precision=gram_precision))
    sol.init(theta, b)
    for _ in range(int(fx["outer"])):
        sol.outer(theta, b, delta)
    u, sc, status = sol.read()
    torch.cuda.synchronize()
    u = u.cpu().numpy()[::int(fx["stride"])].astype(np.float64)
    uo = fx["u_sample"].astype(np.float64)
    out = {"outer_iterations": int(fx["outer"]),
           "u_rel_l2": float(np.linalg.norm(u - uo) / np.linalg.norm(uo)),
           "theta_max_abs_rad": float(np.max(np.abs(theta.cpu().numpy() - fx["theta"][-1]))),
           "lambda_rel": float(abs(float(sc.cpu()[2]) - fx["lam"][-1]) / fx["lam"][-1]),
           "reference": "FP64 oracle from the exact GKB start (tests/golden/loop_c2_oracle.npz)",
           "bars": {"u_rel_l2": 1e-3, "theta_max_abs_rad": 1e-4}}
    sol.close()
    return out


def autotune(torch, ops, g, x, theta, b, kmin, fr=None):
    """Tune the projector launch shapes for the column counts the solver uses (one column for
    the Krylov expansions, kmin + 1 for the rebase) and for the backprojection."""
    npix = g.nx * g.ny * (fr.nframes if fr is not None else 1)
    xs = x.reshape(-1)[:npix]
    ops.autotune_project(xs, theta, g, fr)
    ops.autotune_project(xs.repeat(kmin + 1), theta, g, fr)
    ops.autotune_backproject(b, theta, g, fr)
    V = theta.numel()
    return {"fwd_waves_per_block_1col": ops.tune_query("project", g, V, 1, fr),
            f"fwd_waves_per_block_{kmin + 1}col": ops.tune_query("project", g, V, kmin + 1, fr),
            "bwd_view_split": ops.tune_query("backproject", g, V, 1, fr)}


def workload_operators(torch, ops, metrics, synth, reps):
    """Gsamples/s of the three operators (one column) at the shape of every workload: its
    grid, bins, views and frames, with the workload's true angles and a random image and
    sinogram; for the streaming workload also one block of its views.  The launch shapes are
    tuned for each shape first; nnz is counted exactly."""
    dev = torch.device("cuda", 0)
    gen = torch.Generator(device=dev)
    gen.manual_seed(12345)
    stream = torch.cuda.current_stream()
    out = {}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a0 = torch.cuda.Event(enable_timing=True)
        a1 = torch.cuda.Event(enable_timing=True)
        a0.record(stream)
        for _ in range(reps):
            fn()
        a1.record(stream)
        torch.cuda.synchronize()
        return a0.elapsed_time(a1) / reps

    cases = [("c1", None), ("c2", None), ("c3", None), ("c4", None), ("c5", None),
             ("c5", 0)]
    for key, block in cases:
        wl = synth.WORKLOADS[key]
        inst = synth.draw(wl, with_image=False)
        th_host = inst.theta_true if block is None else inst.theta_true[inst.blocks[block]]
        V = th_host.size
        F = wl.frames
        fr = ops.Frames(inst.view_off) if F > 1 else None
        g = ops.geom(wl.N, wl.nb)
        th = torch.as_tensor(th_host, device=dev)
        x = torch.rand((1, F, wl.N, wl.N), generator=gen, device=dev, dtype=torch.float32)
        y = torch.randn((1, V, wl.nb), generator=gen, device=dev, dtype=torch.float32)
        nnz = metrics.nnz_torch(torch, wl.N, wl.nb, th_host, device=dev)
        ops.autotune_project(x, th, g, fr)
        ops.autotune_backproject(y, th, g, fr)
        yo = torch.empty_like(y)
        xo = torch.empty_like(x)
        ms = {"project": timed(lambda: ops.project(x, th, g, fr, out=yo)),
              "backproject": timed(lambda: ops.backproject(y, th, g, fr, out=xo)),
              "dtheta": timed(lambda: ops.project_dtheta(x, th, g, fr, want_dy=True)),
              "dtheta_transpose": timed(lambda: ops.backproject_dtheta(y, th, g, fr, out=xo))}
        name = key if block is None else f"{key}_block{block}"
        out[name] = {"grid": f"{F}x{wl.N}x{wl.N}" if F > 1 else f"{wl.N}x{wl.N}",
                     "views": int(V), "bins": wl.nb, "nnz": int(nnz),
                     "gsamples_per_s": {k: round(nnz / (v * 1e-3) / 1e9, 1)
                                        for k, v in ms.items()},
                     "ms": {k: round(v, 4) for k, v in ms.items()}}
        print(f"# operators at {name}: {out[name]['gsamples_per_s']}", file=sys.stderr,
              flush=True)
        del x, y, xo, yo
    torch.cuda.synchronize()
    return out


def fan_leg(torch, ops, synth, reps):
    """ms per call of the four fan-beam operators at the 256x256 / 360-view / 363-bin shape
    with the source at R = 4 (one kernel per call), pixel-views per second, and the parallel
    projector's calls at the same shape beside them."""
    wl = synth.WORKLOADS["c2"]
    inst = synth.draw(wl)
    g = ops.geom(wl.N, wl.nb)
    dev = torch.device("cuda", 0)
    x = torch.as_tensor(inst.x_true[0].astype(np.float32), device=dev).contiguous()
    th = torch.as_tensor(inst.theta_true, device=dev)
    R = 4.0
    y = ops.fan_project(x, th, g, R)
    xb = torch.empty((1, 1, wl.N, wl.N), dtype=torch.float32, device=dev)
    yb = torch.empty_like(y)
    stream = torch.cuda.current_stream()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a0 = torch.cuda.Event(enable_timing=True)
        a1 = torch.cuda.Event(enable_timing=True)
        a0.record(stream)
        for _ in range(reps):
            fn()
        a1.record(stream)
        torch.cuda.synchronize()
        return a0.elapsed_time(a1) / reps

    ms = {"project": timed(lambda: ops.fan_project(x, th, g, R, out=yb)),
          "backproject": timed(lambda: ops.fan_backproject(y, th, g, R, out=xb)),
          "dtheta": timed(lambda: ops.fan_project_dtheta(x, th, g, R, out=yb)),
          "dtheta_transpose": timed(lambda: ops.fan_backproject_dtheta(y, th, g, R, out=xb))}
    pv = wl.N * wl.N * wl.n_views
    return {"workload": "256x256 image, 360 views, 363 bins, source at R = 4 image half-widths",
            "ms_per_call": {k: round(v, 4) for k, v in ms.items()},
            "gpixelviews_per_s": {k: round(pv / (v * 1e-3) / 1e9, 2) for k, v in ms.items()}}


def pat_leg(torch, ops, synth, reps):
    """ms per call of the photoacoustic circular-means operators (projection, its derivative in
    the radial shift, transpose) at the 64x64 shape (64 sensors, 64 radii, 512 samples per
    circle, p = 0.432) and the 50x50 frames (32 sensors, 50 radii, 256 samples, p = 0.1924,
    20 frames in one call), with circle samples per second."""
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a0 = torch.cuda.Event(enable_timing=True)
        a1 = torch.cuda.Event(enable_timing=True)
        a0.record(stream)
        for _ in range(reps):
            fn()
        a1.record(stream)
        torch.cuda.synchronize()
        return a0.elapsed_time(a1) / reps

    res = {}
    for name, (N, na, nc, K, p, cols) in {"64x64": (64, 64, 64, 512, 0.432, 1),
                                          "50x50_frames": (50, 32, 50, 256, 0.1924, 20)}.items():
        x = torch.as_tensor(synth.random_image(N, seed=N, frames=cols).astype(np.float32),
                            device=dev).contiguous()
        g = ops.geom(N, 3)
        pg = ops.pat_geom(na, nc, K)
        y = ops.pat_project(x, g, pg, p)
        yb = torch.empty_like(y)
        xb = torch.empty((cols, N, N), dtype=torch.float32, device=dev)
        ms = {"project": timed(lambda: ops.pat_project(x, g, pg, p, out=yb)),
              "project_dp": timed(lambda: ops.pat_project_dp(x, g, pg, p, out=yb)),
              "backproject": timed(lambda: ops.pat_backproject(y, g, pg, p, out=xb))}
        samples = cols * na * nc * K
        res[name] = {"image": N, "sensors": na, "radii": nc, "samples_per_circle": K,
                     "columns": cols, "ms_per_call": {k: round(v, 4) for k, v in ms.items()},
                     "gsamples_per_s": {k: round(samples / (v * 1e-3) / 1e9, 2)
                                        for k, v in ms.items()}}
    return res


def varpro_leg(torch, ops, synth, Config, Solver, steps, warmup, gram_precision):
    """Outer it/s of VarPro NL-RMM-GKS on the 512x512 / 720-view / 725-bin workload (S = 15
    projected solves per outer iteration, kmax 25)."""
    wl = synth.WORKLOADS["c3"]
    inst = synth.draw(wl)
    g = ops.geom(wl.N, wl.nb)
    x32, th_true, b, delta = make_data(torch, ops, inst, wl, g)
    autotune(torch, ops, g, x32, th_true, b, wl.kmin)
    stream = torch.cuda.current_stream()
    theta = torch.as_tensor(inst.theta_nom.copy(), device="cuda")
    cfg = Config(kmin=wl.kmin, kmax=wl.kmax, solves=wl.solves, eps=wl.eps, param_update=2,
                 gram_precision=gram_precision)
    sol = Solver(g, 1, wl.n_views, cfg)
    sol.init(theta, b)
    for _ in range(warmup):
        sol.outer(theta, b, delta)
    ms = timed_steps(torch, lambda: sol.outer(theta, b, delta), steps, stream, "c3 varpro")
    u, _, status = sol.read()
    torch.cuda.synchronize()
    x_true = inst.x_true.reshape(-1)
    rre = float(np.linalg.norm(u.cpu().numpy() - x_true) / np.linalg.norm(x_true))
    dth0 = inst.theta_true - inst.theta_nom
    perr = float(np.linalg.norm(theta.cpu().numpy() - inst.theta_true) / np.linalg.norm(dth0))
    sol.close()
    return {"outer_it_s": round(1000.0 / ms, 4), "ms_per_step": round(ms, 3),
            "rre": round(rre, 5), "angle_err_rel": round(perr, 5), "status": int(status.cpu()[0]),
            "workload": f"c3: 512x512, 720 views, 725 bins, VarPro, S = {wl.solves}, kmax "
                        f"{wl.kmax}, regulariser Gram precision {gram_precision}; {warmup} "
                        f"warm-up + {steps} timed outer iterations"}


def autograd_leg(torch, ops, synth, reps):
    """ms per forward + backward of the data loss 1/2 ||A(theta) x - b||^2 through the
    autograd Function (gradients for x and theta) at the 512x512 / 720-view workload."""
    from paper_2605_06336_amd import autograd as AG
    wl = synth.WORKLOADS["c3"]
    inst = synth.draw(wl, with_image=False)
    g = ops.geom(wl.N, wl.nb)
    dev = torch.device("cuda", 0)
    gen = torch.Generator(device=dev)
    gen.manual_seed(7)
    x = torch.rand((1, wl.N, wl.N), generator=gen, device=dev, dtype=torch.float32)
    b = torch.randn((wl.n_views, wl.nb), generator=gen, device=dev, dtype=torch.float32)
    th0 = torch.as_tensor(inst.theta_true, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        xr = x.clone().requires_grad_(True)
        th = th0.clone().requires_grad_(True)
        y = AG.project(xr, th, g)
        loss = 0.5 * ((y.view(wl.n_views, wl.nb) - b) ** 2).sum()
        loss.backward()
        return xr.grad, th.grad

    step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"ms_forward_backward": round(ms, 4),
            "workload": "c3 shape: 512x512, 720 views, 725 bins; loss 1/2||A(theta)x - b||^2, "
                        "gradients for x (backprojection) and theta (fused per-view <D, g>)"}


def precision_leg(torch, ops, synth, Config, Solver, steps, warmup):
    """Outer it/s of the c2 iteration under each precision policy of the Krylov side."""
    wl = synth.WORKLOADS["c2"]
    inst = synth.draw(wl)
    g = ops.geom(wl.N, wl.nb)
    x32, th_true, b, delta = make_data(torch, ops, inst, wl, g)
    stream = torch.cuda.current_stream()
    x_true = inst.x_true.reshape(-1)
    out = {}
    for name, gp, cp in (("fp64_grams", 0, 0), ("fp32_mfma_grams", 1, 0),
                         ("bf16_mfma_grams_and_compression", 2, 2)):
        theta = torch.as_tensor(inst.theta_nom.copy(), device="cuda")
        sol = Solver(g, 1, wl.n_views, Config(kmin=wl.kmin, kmax=wl.kmax, eps=wl.eps,
                                              gram_precision=gp, compress_precision=cp))
        sol.init(theta, b)
        for _ in range(warmup):
            sol.outer(theta, b, delta)
        ms = timed_steps(torch, lambda: sol.outer(theta, b, delta), steps, stream,
                         f"c2 {name}")
        u, _, _ = sol.read()
        torch.cuda.synchronize()
        rre = float(np.linalg.norm(u.cpu().numpy() - x_true) / np.linalg.norm(x_true))
        sol.close()
        out[name] = {"outer_it_s": round(1000.0 / ms, 4), "rre": round(rre, 5)}
    return out


def gram_leg(torch, ops, synth, reps):
    """The weighted regulariser Gram (Psi V)^T diag(w) (Psi V) on the matrix cores at the c2
    and c5 image sizes with the basis widths their solvers reach (kmax), FP32 and BF16
    operands.  Algorithmic work: the symmetric half, npsi * ell * (ell + 1) flop; algorithmic
    bytes: V (4 n ell) and w (4 npsi) read once."""
    res = {}
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    for name in ("c2", "c5"):
        wl = synth.WORKLOADS[name]
        g = ops.geom(wl.N, wl.nb)
        n = wl.N * wl.N
        ell = wl.kmax
        V = torch.randn((ell, n), generator=gen, device="cuda", dtype=torch.float32)
        u = torch.rand(n, generator=gen, device="cuda", dtype=torch.float32)
        w = ops.tv_weights(u, g, eps=wl.eps)
        npsi = w.numel()
        flop = float(npsi) * ell * (ell + 1)
        nbytes = 4.0 * n * ell + 4.0 * npsi
        entry = {"n": n, "ell": ell, "npsi": npsi}
        for label, prec in (("fp32_mfma", 1), ("bf16_mfma", 2)):
            for _ in range(2):
                ops.gram_psi(V, w, g, ell, precision=prec)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                ops.gram_psi(V, w, g, ell, precision=prec)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            tf = flop / (ms * 1e-3) / 1e12
            gbs = nbytes / (ms * 1e-3) / 1e9
            entry[label] = {"ms": round(ms, 4), "tflops": round(tf, 2),
                            "mfma_peak_tflops": MFMA_PEAK_TFLOPS[prec],
                            "mfma_frac": round(tf / MFMA_PEAK_TFLOPS[prec], 4),
                            "gb_s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
        res[name] = entry
        del V, u, w
    return res


def streaming_leg(torch, ops, synth, Config, steps):
    """ms per block of s-NL-RMM-GKS at the full streaming shape (2048x2048, 1440 views in 64
    blocks of 22-23, 2897 bins, kmax 50, BF16 Grams and compression products).  The image is
    random (timing at fixed iteration counts does not depend on it)."""
    from paper_2605_06336_amd.streaming import Streaming
    wl = synth.WORKLOADS["c5"]
    inst = synth.draw(wl, with_image=False)
    g = ops.geom(wl.N, wl.nb)
    dev = torch.device("cuda", 0)
    gen = torch.Generator(device=dev)
    gen.manual_seed(11)
    x = torch.rand((1, 1, wl.N, wl.N), generator=gen, device=dev, dtype=torch.float32)
    bex = ops.project(x, torch.as_tensor(inst.theta_true, device=dev), g).cpu().numpy()
    bex = bex.reshape(-1).astype(np.float64)
    e = wl.noise * np.linalg.norm(bex) * inst.g / np.linalg.norm(inst.g)
    cfg = Config(kmin=wl.kmin, kmax=wl.kmax, eps=wl.eps, gram_precision=2, compress_precision=2)
    st = Streaming(g, inst.blocks, cfg)
    st.load(inst.theta_nom, bex + e, e)
    st.init()
    st.run(1, max_blocks=1)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ms = timed_steps(torch, lambda: st.solver.outer(*st._block(1), st.deltas[1]), steps, stream,
                     "c5 block")
    st.solver.close()
    return {"ms_per_block": round(ms, 3), "blocks_per_pass": len(inst.blocks),
            "pass_s_estimate": round(ms * len(inst.blocks) / 1000.0, 3),
            "workload": "c5 shape: 2048x2048, 1440 views in 64 blocks, 2897 bins, kmax 50, "
                        "BF16 Grams and compression products; random image"}


def dynamic_leg(torch, ops, synth, Config, OuterGraph, Solver, steps, warmup, gram_precision):
    """Outer it/s of the 32-frame dynamic workload: batched + graph replay vs plain."""
    wl = synth.WORKLOADS["c4"]
    inst = synth.draw(wl)
    fr = ops.Frames(inst.view_off)
    g = ops.geom(wl.N, wl.nb)
    x32, th_true, b, delta = make_data(torch, ops, inst, wl, g, fr)
    stream = torch.cuda.current_stream()
    V = int(inst.view_off[-1])
    tuned = autotune(torch, ops, g, x32, th_true, b, wl.kmin, fr)
    out = {}
    us = {}
    for mode in ("plain", "batched"):
        cfg = Config(kmin=wl.kmin, kmax=wl.kmax, eps=wl.eps, temporal=1,
                     gram_precision=gram_precision)
        sol = Solver(g, wl.frames, V, cfg)
        if mode == "plain":
            sol.set_per_frame(inst.view_off)
        th = torch.as_tensor(inst.theta_nom.copy(), device="cuda")
        sol.init(th, b, fr)
        for _ in range(warmup):
            sol.outer(th, b, delta, fr)
        if mode == "batched":
            gr = OuterGraph(sol, th, b, delta, fr)
            step = gr.replay
        else:
            step = lambda: sol.outer(th, b, delta, fr)   # noqa: E731
        ms = timed_steps(torch, step, steps, stream, f"dynamic {mode}")
        u, _, status = sol.read()
        torch.cuda.synchronize()
        us[mode] = u.cpu().numpy().astype(np.float64)
        x_true = inst.x_true.reshape(-1)
        out[mode] = {"outer_it_s": round(1000.0 / ms, 4), "ms_per_step": round(ms, 3),
                     "rre": round(float(np.linalg.norm(us[mode] - x_true) /
                                        np.linalg.norm(x_true)), 5),
                     "status": int(status.cpu()[0])}
        sol.close()
    # the optical-flow temporal regulariser at the same shape (batched, graph replay): the
    # velocities of all 31 frame pairs re-estimated (200 CG steps) at every outer iteration
    cfg = Config(kmin=wl.kmin, kmax=wl.kmax, eps=wl.eps, temporal=2,
                 gram_precision=gram_precision)
    sol = Solver(g, wl.frames, V, cfg)
    th = torch.as_tensor(inst.theta_nom.copy(), device="cuda")
    sol.init(th, b, fr)
    for _ in range(warmup):
        sol.outer(th, b, delta, fr)
    gr = OuterGraph(sol, th, b, delta, fr)
    ms = timed_steps(torch, gr.replay, steps, stream, "dynamic optical flow")
    u, _, status = sol.read()
    torch.cuda.synchronize()
    u_of = u.cpu().numpy().astype(np.float64)
    uu = u.view(wl.frames, wl.N, wl.N)
    flow = ops.of_estimate(uu, g, wl.frames, 0.05, 1e-3, 200)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ops.of_estimate(uu, g, wl.frames, 0.05, 1e-3, 200, out=flow)
    e1.record(stream)
    torch.cuda.synchronize()
    sol.close()
    x_true = inst.x_true.reshape(-1)
    out["optical_flow"] = {"outer_it_s": round(1000.0 / ms, 4), "ms_per_step": round(ms, 3),
                           "velocity_estimate_ms": round(e0.elapsed_time(e1), 3),
                           "rre": round(float(np.linalg.norm(u_of - x_true) /
                                              np.linalg.norm(x_true)), 5),
                           "status": int(status.cpu()[0])}
    out["speedup"] = round(out["batched"]["outer_it_s"] / out["plain"]["outer_it_s"], 3)
    out["u_rel_diff_batched_vs_plain"] = float(
        np.linalg.norm(us["batched"] - us["plain"]) / np.linalg.norm(us["plain"]))
    out["autotune_batched"] = tuned
    out["workload"] = (f"c4: 32 frames of 256x256 (moving ellipses), {V} views in total "
                       f"(30..120 per frame, golden-angle), 363 bins, 2% noise, ANISO-TV with "
                       f"frame differences, kmin {wl.kmin} kmax {wl.kmax}; "
                       f"{warmup} warm-up + {steps} timed outer iterations per mode")
    return out


def cpu_baseline_leg(torch, ops, inst, wl, g, x32, th_true, b, x_true):
    """The FP64 oracle on the host's cores: the median of three outer iterations of the same
    workload (after the GKB start) and one application of each operator at its shape; the
    operators' outputs also give the library's error against FP64 on the same inputs."""
    from oracle import method as OM
    from oracle import projector as OP
    from paper_2605_06336_amd import metrics
    geo = OM.Geometry(N=wl.N, nb=wl.nb, view_off=inst.view_off)
    b_ora, e_ora = OM.make_data(geo, x_true, inst.theta_true, inst.g, wl.noise)
    ocfg = OM.Config(kmin=wl.kmin, kmax=wl.kmax, eps=wl.eps)
    st = OM.init_state(geo, inst.theta_nom, b_ora, ocfg)
    secs = []
    for k in range(3):
        c0 = time.perf_counter()
        OM.outer_step(geo, st, b_ora, float(np.linalg.norm(e_ora)), ocfg)
        secs.append(time.perf_counter() - c0)
        print(f"# oracle outer iteration {k + 1}/3: {secs[-1]:.1f} s", file=sys.stderr, flush=True)
    med = float(np.median(secs))
    # operators at the same shape: the image and angles the library projected, a sinogram
    x64 = x32.cpu().numpy().astype(np.float64).reshape(wl.N, wl.N)
    th = th_true.cpu().numpy()
    ys32 = b.cpu().numpy().reshape(wl.n_views, wl.nb)
    ys = ys32.astype(np.float64)
    nnz = metrics.nnz(wl.N, wl.nb, inst.theta_true)
    ora = {}
    t = {}
    for name, fn in (("project", lambda: OP.project(x64, th, wl.nb)),
                     ("backproject", lambda: OP.backproject(ys, th, wl.N)),
                     ("dtheta", lambda: OP.dtheta(x64, th, wl.nb)),
                     ("dtheta_transpose", lambda: OP.dtheta_t(ys, th, wl.N))):
        c0 = time.perf_counter()
        ora[name] = fn()
        t[name] = time.perf_counter() - c0
    cpu = {"value": round(1.0 / med, 5), "unit": "outer it/s", "cores": OP.max_threads(),
           "kind": "oracle",
           "sample": f"median of 3 outer iterations (the first three after the GKB start basis) "
                     f"of the same 256x256 / 360-view workload in FP64 on the host: "
                     + ", ".join(f"{v:.1f}" for v in secs) + " s",
           "operators_gsamples_per_s": {k: round(nnz / v / 1e9, 4) for k, v in t.items()}}
    dev = torch.device("cuda", 0)
    bt = torch.as_tensor(ys32, device=dev).view(1, wl.n_views, wl.nb)
    lib = {"project": ops.project(x32, th_true, g).cpu().numpy(),
           "backproject": ops.backproject(bt, th_true, g).cpu().numpy(),
           "dtheta": ops.project_dtheta(x32, th_true, g, want_dy=True)["dy"].cpu().numpy(),
           "dtheta_transpose": ops.backproject_dtheta(bt, th_true, g).cpu().numpy()}

    def rel(a, ref):
        a = np.asarray(a, np.float64).reshape(ref.shape)
        return float(np.linalg.norm(a - ref) / np.linalg.norm(ref))

    op_parity = {k: rel(lib[k], ora[k]) for k in ora}
    op_parity["bar"] = 1e-5
    return cpu, op_parity


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): this build "
              "measures the path on a single device and has no multi-GPU mode", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2605_06336_amd import metrics, ops, synth
    from paper_2605_06336_amd.solver import Config, OuterGraph, Solver

    if args.dynamic_only:
        print(json.dumps({"dynamic_only": True,
                          "batched_vs_plain": dynamic_leg(torch, ops, synth, Config, OuterGraph,
                                                          Solver, args.steps, args.warmup,
                                                          args.gram_precision)}), flush=True)
        return

    if args.streaming_only:
        print(json.dumps({"streaming_only": True,
                          "streaming": streaming_leg(torch, ops, synth, Config, args.steps)}),
              flush=True)
        return

    if args.gram_only:
        print(json.dumps({"gram_only": True, "gram_mfma": gram_leg(torch, ops, synth, args.reps)}),
              flush=True)
        return

    wl = synth.WORKLOADS["c2"]
    inst = synth.draw(wl)
    V = wl.n_views
    g = ops.geom(wl.N, wl.nb)
    stream = torch.cuda.current_stream()
    x32, th_true, b, delta = make_data(torch, ops, inst, wl, g)
    tuned = autotune(torch, ops, g, x32, th_true, b, wl.kmin)

    if args.ops_only:
        nnz, call_ms, kern_ms = operators(torch, ops, metrics, inst, wl, g, x32, th_true, b,
                                          args.reps, stream)
        copy_calibration(torch)
        print(json.dumps({"ops_only": True, "autotune": tuned, "nnz": int(nnz), "call_ms": call_ms,
                          "kernel_ms": kern_ms, "copy_bytes": COPY_BYTES,
                          "source_sha": source_digest()}), flush=True)
        return

    theta = torch.as_tensor(inst.theta_nom.copy(), device="cuda")
    cfg = Config(kmin=wl.kmin, kmax=wl.kmax, eps=wl.eps, gram_precision=args.gram_precision)
    sol = Solver(g, 1, V, cfg)
    sol.init(theta, b)
    for _ in range(args.warmup):
        sol.outer(theta, b, delta)
    # over the timed steps, every 4th one-column projection and backprojection records a HIP
    # event pair around its single kernel launch on the launch stream: the in-loop duration
    # per launch of the two projector kernels (sampled, so that the events cost little)
    ops.set_kernel_timing(-TIMING_PERIOD)
    ms_per_step = timed_steps(torch, lambda: sol.outer(theta, b, delta), args.steps, stream,
                              "c2")
    loop_kernels = {}
    for which, kname in (("project", "fwd_edges_k"), ("backproject", "bwd_tiles_k")):
        avg, n = ops.kernel_avg(which)
        loop_kernels[kname] = {"avg_launch_ms": round(avg, 5), "launches_timed": n,
                               "ms_per_outer_iteration":
                                   round(avg * n * TIMING_PERIOD / args.steps, 4)}
    ops.set_kernel_timing(False)
    # the same iteration captured once as a HIP graph and replayed (bitwise equal to eager
    # execution, no timing events), reported beside the eager rate
    graph_steps = max(2, args.steps // 2)
    graph = OuterGraph(sol, theta, b, delta)
    ms_graph = timed_steps(torch, graph.replay, graph_steps, stream, "c2 graph")
    u, sc, status = sol.read()
    torch.cuda.synchronize()
    x_true = inst.x_true.reshape(-1)
    rre = float(np.linalg.norm(u.cpu().numpy() - x_true) / np.linalg.norm(x_true))
    dth0 = inst.theta_true - inst.theta_nom
    perr = float(np.linalg.norm(theta.cpu().numpy() - inst.theta_true) / np.linalg.norm(dth0))
    # full-space sensitivity of one global offset at the current image (CG on A^T A + lam R)
    sensitivity = None
    if not args.no_workloads:
        sens_iters = 50
        sol.offset_sensitivity(theta, b, iters=sens_iters)
        sens_ms = timed_steps(torch, lambda: sol.offset_sensitivity(theta, b, iters=sens_iters),
                              3, stream, "c2 offset sensitivity")
        sens_out, _ = sol.offset_sensitivity(theta, b, iters=sens_iters)
        sensitivity = {"ms_per_solve": round(sens_ms, 3), "cg_iterations": sens_iters,
                       "ms_per_cg_iteration": round(sens_ms / sens_iters, 4),
                       "g_h_dp": [float(v) for v in sens_out.cpu().numpy()]}
    sol.close()
    parity = loop_parity(torch, ops, inst, wl, g, b, delta, Config, Solver, args.gram_precision)

    nnz, call_ms, kern_ms = operators(torch, ops, metrics, inst, wl, g, x32, th_true, b,
                                      args.reps, stream)
    gs = {k: round(nnz / (v * 1e-3) / 1e9, 2) for k, v in call_ms.items()}
    gs_kernel = {k: round(nnz / (v * 1e-3) / 1e9, 2) for k, v in kern_ms.items()}

    def roof(kernel):
        ms = loop_kernels[kernel]["avg_launch_ms"]
        achieved = nnz * FLOP_PER_SAMPLE / (ms * 1e-3) / 1e12
        ctr = counters_for(kernel, tuned) or {}
        traffic = ctr.get("bytes_per_launch")
        valu = ctr.get("valu_wave_insts")
        alg_bytes = 4 * (wl.N * wl.N + V * wl.nb)
        return {"bound": "alu", "kernel": kernel, "achieved": round(achieved, 3),
                "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                "frac_of_unpacked_fp32": round(achieved / FP32_NONPACKED_PEAK_TFLOPS, 4),
                "traffic": traffic,
                "hbm_gb_s": round(traffic / (ms * 1e-3) / 1e9, 1) if traffic else None,
                "traffic_x_algorithmic": round(traffic / alg_bytes, 2) if traffic else None,
                "valu_wave_insts": valu,
                "valu_issue_frac": round(valu / (ms * 1e3 * VALU_ISSUE_PER_US), 3) if valu
                else None,
                "launch_ms": round(ms, 5), "launches_timed": loop_kernels[kernel]["launches_timed"],
                "timing": f"HIP events around every {TIMING_PERIOD}th single launch in the timed "
                          "outer iterations",
                "samples_per_launch": int(nnz), "flop_per_sample": FLOP_PER_SAMPLE}

    # dominant kernel: the projector kernel with the most time per outer iteration
    dominant = max(loop_kernels, key=lambda k: loop_kernels[k]["ms_per_outer_iteration"])
    other = [k for k in loop_kernels if k != dominant][0]
    roofline = roof(dominant)
    roofline_other = roof(other)

    dyn = None
    if not args.no_dynamic:
        dyn = dynamic_leg(torch, ops, synth, Config, OuterGraph, Solver, max(3, args.steps // 2),
                          2, args.gram_precision)

    per_workload = varpro = autograd_r = precision = streaming = gram = fan = pat = None
    if not args.no_workloads:
        gram = gram_leg(torch, ops, synth, max(3, args.reps // 2))
        fan = fan_leg(torch, ops, synth, max(3, args.reps // 2))
        pat = pat_leg(torch, ops, synth, max(3, args.reps // 2))
        per_workload = workload_operators(torch, ops, metrics, synth, max(3, args.reps // 4))
        varpro = varpro_leg(torch, ops, synth, Config, Solver, max(3, args.steps // 2), 2,
                            args.gram_precision)
        autograd_r = autograd_leg(torch, ops, synth, max(3, args.reps // 2))
        precision = precision_leg(torch, ops, synth, Config, Solver, max(3, args.steps // 2), 2)
        streaming = streaming_leg(torch, ops, synth, Config, 3)

    cpu = None
    op_parity = None
    if not args.no_cpu_baseline:
        cpu, op_parity = cpu_baseline_leg(torch, ops, inst, wl, g, x32, th_true, b, x_true)

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
                               "kmin 5 kmax 40, TV, discrepancy principle, FP32 projector, "
                               f"regulariser Gram precision {args.gram_precision}, FP64 "
                               "projected solves",
                   "global_batch": 1, "parallelism": "none"},
        "graph_replay_outer_it_s": round(1000.0 / ms_graph, 4),
        "gsamples_per_s": gs,
        "gsamples_per_s_kernel": gs_kernel,
        "operator_ms": {k: round(v, 5) for k, v in call_ms.items()},
        "kernel_ms": {k: round(v, 5) for k, v in kern_ms.items()},
        "nnz": int(nnz),
        "quality": {"rre": round(rre, 5), "angle_err_rel": round(perr, 5),
                    "outer_done": args.warmup + args.steps + graph_steps,
                    "lambda": float(sc.cpu().numpy()[2]), "status": int(status.cpu()[0])},
        "autotune": tuned,
        "batched_vs_plain": dyn,
        "offset_sensitivity_c2": sensitivity,
        "operators_by_workload": per_workload,
        "varpro_c3": varpro,
        "autograd_c3": autograd_r,
        "precision_policy_c2": precision,
        "streaming_c5": streaming,
        "gram_mfma": gram,
        "fan_beam_c2": fan,
        "photoacoustic": pat,
        "roofline": roofline,
        "roofline_" + other: roofline_other,
        "loop_kernels": loop_kernels,
        "parity": {"loop_c2": parity, "operators_c2": op_parity},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
