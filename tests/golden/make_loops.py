"""Write loop_<workload>_oracle.npz: the FP64 oracle's NL-RMM-GKS run at a workload's full
size and full outer-iteration count, from the exact GKB start basis.

Inputs come from the seeded generators (paper_2605_06336_amd.synth: phantom, angles, noise
direction); every step of the method is the oracle's (oracle.method, the C strip-area
projector).  Stored: the angles after every outer iteration (or after the last one for the
dynamic workload), lambda and the status word after every outer iteration, and the final
image at every `stride`-th pixel (float32; the full image when it has at most 65536
pixels).  The GPU loop-parity tests compare against these values; nothing here touches the
HIP library.

Usage: python tests/golden/make_loops.py c2 [c3 c4 ...]   (c2 takes ~10 min on 8 cores)
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import method as M  # noqa: E402
from paper_2605_06336_amd import synth  # noqa: E402

MAX_SAMPLES = 65536


def image_stride(n: int) -> int:
    return max(1, n // MAX_SAMPLES)


def run(name: str) -> str:
    wl = synth.WORKLOADS[name]
    inst = synth.draw(wl)
    geo = M.Geometry(N=wl.N, nb=wl.nb, view_off=inst.view_off, temporal=wl.frames > 1)
    b, e = M.make_data(geo, inst.x_true.reshape(-1), inst.theta_true, inst.g, wl.noise)
    gn = {"altmin": "altmin", "varpro": "varpro", "dynamic": "altmin"}[wl.method]
    cfg = M.Config(kmin=wl.kmin, kmax=wl.kmax, solves=wl.solves, eps=wl.eps, gn=gn)
    st = M.init_state(geo, inst.theta_nom, b, cfg)
    delta = float(np.linalg.norm(e))
    thetas, lams, status = [], [], []
    t0 = time.time()
    for k in range(wl.outer):
        M.outer_step(geo, st, b, delta, cfg)
        thetas.append(st.theta.copy())
        lams.append(st.lam)
        status.append(st.status)
        print(f"{name} outer {k + 1}/{wl.outer}: lambda {st.lam:.4e} status {st.status} "
              f"({time.time() - t0:.0f} s)", flush=True)
    stride = image_stride(geo.n)
    if wl.frames > 1:
        thetas = thetas[-1:]
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"loop_{name}_oracle.npz")
    np.savez_compressed(path, u_sample=st.u[::stride].astype(np.float32), stride=stride,
                        u_norm=float(np.linalg.norm(st.u)), theta=np.array(thetas),
                        lam=np.array(lams), status=np.array(status, dtype=np.int32),
                        outer=wl.outer, seed=wl.seed)
    return path


if __name__ == "__main__":
    for w in sys.argv[1:] or ["c2"]:
        print("wrote", run(w), flush=True)
