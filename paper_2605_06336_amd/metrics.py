"""Host-side workload metrics: exact number of nonzero weights of A(theta).

One "sample" is one nonzero (ray, pixel) weight applied; Gsamples/s of the projector
family = nnz(A(theta)) * columns / kernel time.
"""
from __future__ import annotations

import numpy as np


def nnz(N: int, nb: int, theta, ny: int = None, s_half: float = 1.42) -> int:
    """Count pairs (bin, pixel) whose strip and pixel square overlap with positive area."""
    ny = N if ny is None else ny
    d = 2.0 / N
    ds = 2.0 * s_half / nb
    xs = -1.0 + (np.arange(N) + 0.5) * d
    ys = -1.0 * ny / N + (np.arange(ny) + 0.5) * d
    total = 0
    for th in np.asarray(theta, dtype=np.float64):
        c, s = np.cos(th), np.sin(th)
        wo = 0.5 * d * (abs(c) + abs(s))
        cc = xs[None, :] * c + ys[:, None] * s
        lo = np.floor((cc - wo + s_half) / ds)
        hi = np.ceil((cc + wo + s_half) / ds) - 1
        lo = np.clip(lo, 0, nb - 1)
        hi = np.clip(hi, 0, nb - 1)
        total += int(np.sum(hi - lo + 1))
    return total
