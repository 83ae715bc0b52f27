"""FP64 photoacoustic (circular-means) operator with a global radial shift (test
infrastructure only).

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may use this module; it imports nothing from the product package.

What it computes (Section 6.3, "Photoacoustic Tomography with Sensor Radius Uncertainty"):
the image is integrated along circles centred at the sensors, with the nominal radii
r_j = 2 j / n_c (j = 1 .. n_c) all shifted by one global p, r_j(p) = r_j + p.

Readings where the paper leaves the operator to its toolbox (listed in the design notes):
  * the image lives on [-1, 1]^2 with N x N pixels (width d = 2 / N); between pixel centres
    it is the bilinear interpolant of the pixel values, with value 0 for indices outside the
    grid (the interpolant falls to zero over the half pixel beyond the outer centres);
  * n_a sensors at angles 2 pi a / n_a on the circle of radius 1.5 around the centre (outside
    the image);
  * a circle integral is the K-point trapezoid rule, K the same for every circle:
    y[a][j] = (2 pi r / K) sum_k I(x_a + r (cos psi_k, sin psi_k)), psi_k = 2 pi k / K,
    r = r_j(p); a shift that takes r below zero is used as it stands (the circle of radius
    |r| traced from the opposite side, with the negative factor r), which keeps the operator
    smooth in p through r = 0;
  * its derivative in p is the derivative of that sum, (2 pi / K) sum_k [I + r grad I . e_k]
    with e_k = (cos psi_k, sin psi_k) and grad I the gradient of the bilinear interpolant of
    the sample's cell.
"""
from __future__ import annotations

import math

import numpy as np

SENSOR_RADIUS = 1.5


def sensors(n_a):
    ang = 2.0 * math.pi * np.arange(n_a) / n_a
    return SENSOR_RADIUS * np.cos(ang), SENSOR_RADIUS * np.sin(ang)


def radii(n_c, p):
    return 2.0 * np.arange(1, n_c + 1) / n_c + p


def _samples(N, n_a, n_c, K, p):
    """Sample points [n_a, n_c, K] (x, y), the radii [n_c] and the unit directions [K]."""
    sx, sy = sensors(n_a)
    r = radii(n_c, p)
    psi = 2.0 * math.pi * np.arange(K) / K
    ex, ey = np.cos(psi), np.sin(psi)
    X = sx[:, None, None] + r[None, :, None] * ex[None, None, :]
    Y = sy[:, None, None] + r[None, :, None] * ey[None, None, :]
    return X, Y, r, ex, ey


def _cells(N, X, Y):
    """Cell corner indices and fractions of points (fractional pixel indices)."""
    d = 2.0 / N
    fx = (X + 1.0) / d - 0.5
    fy = (Y + 1.0) / d - 0.5
    k0 = np.floor(fx).astype(np.int64)
    l0 = np.floor(fy).astype(np.int64)
    return k0, l0, fx - k0, fy - l0


def _val(img, k, l):
    N = img.shape[0]
    ok = (k >= 0) & (k < N) & (l >= 0) & (l < N)
    return np.where(ok, img[np.clip(l, 0, N - 1), np.clip(k, 0, N - 1)], 0.0)


def interp(img, X, Y):
    """The bilinear interpolant I (and its gradient) of img [N, N] (row l along y, column k
    along x) at points X, Y."""
    N = img.shape[0]
    d = 2.0 / N
    k0, l0, tx, ty = _cells(N, X, Y)
    v00, v10 = _val(img, k0, l0), _val(img, k0 + 1, l0)
    v01, v11 = _val(img, k0, l0 + 1), _val(img, k0 + 1, l0 + 1)
    I = (1 - tx) * (1 - ty) * v00 + tx * (1 - ty) * v10 + (1 - tx) * ty * v01 + tx * ty * v11
    gx = ((1 - ty) * (v10 - v00) + ty * (v11 - v01)) / d
    gy = ((1 - tx) * (v01 - v00) + tx * (v11 - v10)) / d
    return I, gx, gy


def project(img, n_a, n_c, K, p):
    """y [n_a, n_c]: the circle integrals of the image."""
    X, Y, r, ex, ey = _samples(img.shape[0], n_a, n_c, K, p)
    I, _, _ = interp(np.asarray(img, dtype=np.float64), X, Y)
    return (2.0 * math.pi * r / K)[None, :] * I.sum(axis=2)


def project_dp(img, n_a, n_c, K, p):
    """dy/dp [n_a, n_c]: the derivative of ``project`` in the global radial shift."""
    X, Y, r, ex, ey = _samples(img.shape[0], n_a, n_c, K, p)
    I, gx, gy = interp(np.asarray(img, dtype=np.float64), X, Y)
    radial = gx * ex[None, None, :] + gy * ey[None, None, :]
    return (2.0 * math.pi / K) * (I + r[None, :, None] * radial).sum(axis=2)


def matrix(N, n_a, n_c, K, p):
    """Dense A [n_a * n_c, N * N] (tiny sizes): the transpose of ``project`` is A^T."""
    X, Y, r, ex, ey = _samples(N, n_a, n_c, K, p)
    k0, l0, tx, ty = _cells(N, X, Y)
    A = np.zeros((n_a * n_c, N * N))
    scale = (2.0 * math.pi * r / K)
    for a in range(n_a):
        for j in range(n_c):
            row = a * n_c + j
            for q in range(K):
                for dk, dl, w in ((0, 0, (1 - tx) * (1 - ty)), (1, 0, tx * (1 - ty)),
                                  (0, 1, (1 - tx) * ty), (1, 1, tx * ty)):
                    k, l = k0[a, j, q] + dk, l0[a, j, q] + dl
                    if 0 <= k < N and 0 <= l < N:
                        A[row, l * N + k] += scale[j] * w[a, j, q]
    return A


def backproject(y, N, n_a, n_c, K, p):
    """x = A^T y [N, N]: every sample's value y[a][j] 2 pi r / K spread on the four corners
    of its cell with the bilinear weights (the transpose of the interpolation)."""
    X, Y, r, ex, ey = _samples(N, n_a, n_c, K, p)
    k0, l0, tx, ty = _cells(N, X, Y)
    val = (np.asarray(y, dtype=np.float64).reshape(n_a, n_c) * (2.0 * math.pi * r / K)[None, :])
    val = np.broadcast_to(val[:, :, None], X.shape)
    out = np.zeros(N * N)
    for dk, dl, w in ((0, 0, (1 - tx) * (1 - ty)), (1, 0, tx * (1 - ty)),
                      (0, 1, (1 - tx) * ty), (1, 1, tx * ty)):
        k, l = k0 + dk, l0 + dl
        ok = (k >= 0) & (k < N) & (l >= 0) & (l < N)
        np.add.at(out, (l * N + k)[ok], (val * w)[ok])
    return out.reshape(N, N)
