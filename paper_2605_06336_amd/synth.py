"""Seeded synthetic inputs for the angle-uncertain parallel-beam CT problem.

This module draws random numbers and rasterises phantoms; it holds none of the
method's arithmetic (no projector, no regulariser, no solver).  Both the HIP
path and the FP64 oracle receive its arrays as inputs, so a mismatch between
the two can never come from the random number generator.

Workloads stand in for the paper's CT experiments (Section 6.2: Shepp-Logan
256x256 with 180 views, Section 7 dynamic Moving-MNIST frames): seeded random
ellipse phantoms with the same grid sizes, view counts and noise levels.

Geometry shared by every workload (the paper delegates the discretisation to a
toolbox; this is the parallel-beam reading used throughout the package):
  * image domain [-1, 1]^2, N x N pixels, pixel width D = 2/N, stored row-major
    with x fastest: pixel (k, l) covers [-1 + kD, -1 + (k+1)D] x [-1 + lD, ...]
    and lives at x[l * N + k];
  * detector coordinate s in [-1.42, 1.42], nb bins of width ds = 2.84 / nb;
  * view angle theta (radians), ray normal n = (cos theta, sin theta).

Random draw order (PCG64, seed fixed per workload): ellipses (cx, cy, a, b,
phi, rho[, vx, vy]) -> per-frame view counts -> golden-angle start offset ->
angle perturbations -> streaming block permutation -> noise direction g.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

S_HALF = 1.42          # detector half-width
DOMAIN_HALF = 1.0      # image half-width


@dataclasses.dataclass(frozen=True)
class Workload:
    """Sizes and iteration counts of one synthetic CT workload."""
    name: str
    N: int                      # image is N x N per frame
    n_ellipses: int
    n_views: int                # total views (all frames)
    nb: int                     # detector bins
    sigma_deg: float            # std of the true-angle perturbation
    noise: float                # relative noise level eta
    seed: int
    method: str                 # "altmin" | "varpro" | "dynamic" | "streaming"
    outer: int                  # outer iterations (fixed count, stopping off)
    kmax: int
    kmin: int = 5
    inner_solves: Optional[int] = None   # S per Enlarge; default kmax - kmin
    frames: int = 1
    views_per_frame: Optional[tuple] = None   # (lo, hi) inclusive, dynamic only
    blocks: int = 1             # streaming blocks
    passes: int = 1             # streaming passes
    eps: float = 1e-3           # smoothing of the l1 penalty
    velocity: float = 0.0       # dynamic: centre velocity bound per frame
    offset_deg: float = 0.0     # global shift of every true angle (the experiments' parameter)

    @property
    def D(self) -> float:
        return 2.0 * DOMAIN_HALF / self.N

    @property
    def ds(self) -> float:
        return 2.0 * S_HALF / self.nb

    @property
    def s0(self) -> float:
        return -S_HALF

    @property
    def n_pix(self) -> int:
        return self.N * self.N

    @property
    def solves(self) -> int:
        return self.inner_solves if self.inner_solves is not None else self.kmax - self.kmin


# The five workloads: sizes as in the project's target configurations.
WORKLOADS = {
    "c1": Workload("c1-64px-90v", N=64, n_ellipses=10, n_views=90, nb=91, sigma_deg=0.5,
                   noise=0.01, seed=1001, method="altmin", outer=20, kmax=30),
    "c2": Workload("c2-256px-360v", N=256, n_ellipses=25, n_views=360, nb=363, sigma_deg=1.0,
                   noise=0.01, seed=2001, method="altmin", outer=30, kmax=40),
    "c3": Workload("c3-512px-720v", N=512, n_ellipses=40, n_views=720, nb=725, sigma_deg=1.0,
                   noise=0.01, seed=3001, method="varpro", outer=10, kmax=25, inner_solves=15),
    "c4": Workload("c4-32x256px-dyn", N=256, n_ellipses=25, n_views=0, nb=363, sigma_deg=0.5,
                   noise=0.02, seed=4001, method="dynamic", outer=20, kmax=25, frames=32,
                   views_per_frame=(30, 120), velocity=0.01),
    "c5": Workload("c5-2048px-1440v", N=2048, n_ellipses=80, n_views=1440, nb=2897, sigma_deg=0.5,
                   noise=0.01, seed=5001, method="streaming", outer=1, kmax=50, blocks=64,
                   passes=2),
}


@dataclasses.dataclass
class Instance:
    """One drawn problem instance (all arrays host numpy)."""
    wl: Workload
    x_true: Optional[np.ndarray]   # float64 [frames, N, N] (None: drawn without the image)
    theta_nom: np.ndarray       # float64 [V]
    theta_true: np.ndarray      # float64 [V]
    view_off: np.ndarray        # int64 [frames + 1]
    g: np.ndarray               # float64 [V * nb], standard normal noise direction
    blocks: Optional[List[np.ndarray]] = None   # streaming: view indices per block


def ellipse_image(N: int, cx, cy, a, b, phi, rho, sub: int = 4) -> np.ndarray:
    """Additive ellipse phantom on [-1,1]^2, each pixel the mean over a sub x sub grid."""
    D = 2.0 / N
    off = (np.arange(sub) + 0.5) / sub
    coords = -1.0 + (np.arange(N)[:, None] + off[None, :]).reshape(-1) * D   # N*sub points
    X = coords[None, :]
    Y = coords[:, None]
    img = np.zeros((N * sub, N * sub))
    for e in range(len(cx)):
        c, s = math.cos(phi[e]), math.sin(phi[e])
        xr = (X - cx[e]) * c + (Y - cy[e]) * s
        yr = -(X - cx[e]) * s + (Y - cy[e]) * c
        img += rho[e] * ((xr / a[e]) ** 2 + (yr / b[e]) ** 2 <= 1.0)
    return img.reshape(N, sub, N, sub).mean(axis=(1, 3))


def draw(wl: Workload, N: Optional[int] = None, with_image: bool = True) -> Instance:
    """Draw the instance of a workload.  ``N`` overrides the grid (for scaled tests);
    ``with_image=False`` skips building the phantom (x_true is None) and draws everything
    else identically (the random stream does not depend on the image)."""
    rng = np.random.Generator(np.random.PCG64(wl.seed))
    N = wl.N if N is None else N
    ne = wl.n_ellipses
    cx = rng.uniform(-0.6, 0.6, ne)
    cy = rng.uniform(-0.6, 0.6, ne)
    a = rng.uniform(0.05, 0.4, ne)
    b = rng.uniform(0.05, 0.4, ne)
    phi = rng.uniform(0.0, math.pi, ne)
    rho = rng.uniform(0.1, 1.0, ne)
    if wl.frames > 1:
        vx = rng.uniform(-wl.velocity, wl.velocity, ne)
        vy = rng.uniform(-wl.velocity, wl.velocity, ne)
        lo, hi = wl.views_per_frame
        counts = rng.integers(lo, hi + 1, wl.frames)
        start = rng.uniform(0.0, math.pi)
        golden = math.pi * (math.sqrt(5.0) - 1.0) / 2.0
        V = int(counts.sum())
        theta_nom = np.mod(start + golden * np.arange(V), math.pi)
        x_true = None
        if with_image:
            x_true = np.stack([ellipse_image(N, cx + t * vx, cy + t * vy, a, b, phi, rho)
                               for t in range(wl.frames)])
        view_off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    else:
        V = wl.n_views
        theta_nom = np.arange(V) * (math.pi / V)
        x_true = ellipse_image(N, cx, cy, a, b, phi, rho)[None] if with_image else None
        view_off = np.array([0, V], dtype=np.int64)
    theta_true = theta_nom + rng.normal(0.0, math.radians(wl.sigma_deg), V)
    theta_true = theta_true + math.radians(wl.offset_deg)
    blocks = None
    if wl.blocks > 1:
        perm = rng.permutation(V)
        nbig = V - (V // wl.blocks) * wl.blocks
        sizes = [V // wl.blocks + 1] * nbig + [V // wl.blocks] * (wl.blocks - nbig)
        blocks, pos = [], 0
        for sz in sizes:
            blocks.append(np.sort(perm[pos:pos + sz]).astype(np.int64))
            pos += sz
    g = rng.standard_normal(V * wl.nb)
    return Instance(wl=wl, x_true=x_true, theta_nom=theta_nom, theta_true=theta_true,
                    view_off=view_off, g=g, blocks=blocks)


def random_image(N: int, seed: int, frames: int = 1) -> np.ndarray:
    """Uniform random image(s) in [0, 1) for operator tests (float64 [frames, N, N])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(0.0, 1.0, (frames, N, N))


def random_sinogram(V: int, nb: int, seed: int) -> np.ndarray:
    """Standard-normal sinogram for adjoint tests (float64 [V, nb])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((V, nb))


def random_angles(V: int, seed: int, lo: float = 0.0, hi: float = math.pi) -> np.ndarray:
    """Uniform random view angles (float64 [V])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, V)
