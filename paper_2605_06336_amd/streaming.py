"""Streaming NL-RMM-GKS (Alg. "s_nl_rmmgks_final"): measurement blocks of views processed
in sequence, each with one outer iteration on its own rows, carrying (u, theta, V) from
block to block in the native solver.

The views are permuted once at setup so that every block is a contiguous range: a block's
angles and data are then plain sub-ranges of device arrays, and no gather happens inside
the passes.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np
import torch

from . import ops
from .solver import Config, Solver


class Streaming:
    def __init__(self, g: ops.Geom, blocks: Sequence[np.ndarray], cfg: Config, device: int = 0):
        self.g = g
        self.blocks = [np.asarray(b, dtype=np.int64) for b in blocks]
        self.perm = np.concatenate(self.blocks)
        self.off = np.concatenate([[0], np.cumsum([len(b) for b in self.blocks])]).astype(np.int64)
        self.V = int(self.off[-1])
        self.dev = torch.device("cuda", device)
        maxv = int(max(len(b) for b in self.blocks))
        self.solver = Solver(g, 1, maxv, cfg, device)
        self.theta = None
        self.b = None
        self.deltas = None

    def load(self, theta0: np.ndarray, b: np.ndarray, noise: np.ndarray) -> None:
        """Angles (view order), data [V, nb] and the noise realisation (for per-block DP
        targets) in the original view order; stored permuted on the device."""
        nb = self.g.nbins
        self.theta = torch.as_tensor(np.asarray(theta0, np.float64)[self.perm], device=self.dev)
        bp = np.asarray(b, np.float32).reshape(-1, nb)[self.perm]
        self.b = torch.as_tensor(np.ascontiguousarray(bp), device=self.dev)
        ep = np.asarray(noise, np.float64).reshape(-1, nb)[self.perm]
        self.deltas = [float(np.linalg.norm(ep[self.off[j]:self.off[j + 1]]))
                       for j in range(len(self.blocks))]

    def _block(self, j):
        v0, v1 = int(self.off[j]), int(self.off[j + 1])
        return self.theta[v0:v1], self.b[v0:v1]

    def init(self) -> None:
        th, bb = self._block(0)
        self.solver.init(th, bb)

    def run(self, passes: int, max_blocks: int = None) -> int:
        done = 0
        for _ in range(passes):
            for j in range(len(self.blocks)):
                if max_blocks is not None and done >= max_blocks:
                    return done
                th, bb = self._block(j)
                self.solver.outer(th, bb, self.deltas[j])
                done += 1
        return done

    def angles(self) -> np.ndarray:
        """Current angles in the original view order (host)."""
        out = np.empty(self.V)
        out[self.perm] = self.theta.cpu().numpy()
        return out

    def image(self) -> torch.Tensor:
        return self.solver.read()[0]
