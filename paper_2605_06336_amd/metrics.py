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


def nnz_torch(torch, N: int, nb: int, theta, device="cpu", ny: int = None,
              s_half: float = 1.42, chunk: int = 16) -> int:
    """nnz() with the same FP64 operations on torch tensors (a device makes the count of
    large grids fast); the result is identical to nnz()."""
    ny = N if ny is None else ny
    d = 2.0 / N
    ds = 2.0 * s_half / nb
    xs = -1.0 + (torch.arange(N, dtype=torch.float64, device=device) + 0.5) * d
    ys = -1.0 * ny / N + (torch.arange(ny, dtype=torch.float64, device=device) + 0.5) * d
    th = np.asarray(theta, dtype=np.float64)
    total = 0
    for v0 in range(0, th.size, chunk):
        t = th[v0:v0 + chunk]
        c = torch.as_tensor(np.cos(t), device=device)[:, None, None]
        s = torch.as_tensor(np.sin(t), device=device)[:, None, None]
        wo = torch.as_tensor(0.5 * d * (np.abs(np.cos(t)) + np.abs(np.sin(t))),
                             device=device)[:, None, None]
        cc = xs[None, None, :] * c + ys[None, :, None] * s
        lo = torch.clamp(torch.floor((cc - wo + s_half) / ds), 0, nb - 1)
        hi = torch.clamp(torch.ceil((cc + wo + s_half) / ds) - 1, 0, nb - 1)
        total += int(torch.sum(hi - lo + 1).item())
    return total
