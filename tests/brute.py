"""Brute-force references used to pin the oracle (tests only).

Polygon clipping (Sutherland-Hodgman) of a pixel square against the two
half-planes of a detector strip, with the shoelace area; this computes the
strip-area weight from its geometric definition without the closed-form
trapezoid profile the oracle uses.
"""
import math

import numpy as np


def clip(poly, n, e, keep_ge):
    """Clip polygon (list of (x, y)) to {p : p.n >= e} (keep_ge) or {p : p.n <= e}."""
    out = []
    m = len(poly)
    for i in range(m):
        p, q = poly[i], poly[(i + 1) % m]
        fp = (p[0] * n[0] + p[1] * n[1]) - e
        fq = (q[0] * n[0] + q[1] * n[1]) - e
        if not keep_ge:
            fp, fq = -fp, -fq
        if fp >= 0:
            out.append(p)
        if (fp >= 0) != (fq >= 0):
            t = fp / (fp - fq)
            out.append((p[0] + t * (q[0] - p[0]), p[1] + t * (q[1] - p[1])))
    return out


def area(poly):
    if len(poly) < 3:
        return 0.0
    s = 0.0
    for i in range(len(poly)):
        x0, y0 = poly[i]
        x1, y1 = poly[(i + 1) % len(poly)]
        s += x0 * y1 - x1 * y0
    return 0.5 * abs(s)


def strip_area(x0, y0, x1, y1, theta, e0, e1):
    n = (math.cos(theta), math.sin(theta))
    poly = [(x0, y0), (x1, y0), (x1, y1), (x0, y1)]
    poly = clip(poly, n, e0, True)
    if poly:
        poly = clip(poly, n, e1, False)
    return area(poly)


def dense_matrix(N, nb, thetas):
    """A[v*nb + j, l*N + k] = |pixel ∩ strip_j| / ds, by polygon clipping."""
    D = 2.0 / N
    ds = 2.84 / nb
    A = np.zeros((len(thetas) * nb, N * N))
    for v, th in enumerate(thetas):
        for l in range(N):
            for k in range(N):
                x0, y0 = -1 + k * D, -1 + l * D
                for j in range(nb):
                    e0 = -1.42 + j * ds
                    a = strip_area(x0, y0, x0 + D, y0 + D, th, e0, e0 + ds)
                    if a:
                        A[v * nb + j, l * N + k] = a / ds
    return A


def big_square_projection(nb, theta):
    """Projection of the all-ones image = |[-1,1]^2 ∩ strip_j| / ds (one clip per bin)."""
    ds = 2.84 / nb
    return np.array([strip_area(-1, -1, 1, 1, theta, -1.42 + j * ds, -1.42 + (j + 1) * ds) / ds
                     for j in range(nb)])


def disk_bin_average(nb, r):
    """(1/ds) * integral over each bin of the disk chord 2 sqrt(r^2 - s^2)."""
    ds = 2.84 / nb
    e = -1.42 + np.arange(nb + 1) * ds
    s = np.clip(e, -r, r)
    F = s * np.sqrt(np.maximum(r * r - s * s, 0)) + r * r * np.arcsin(s / r)
    return np.diff(F) / ds


def disk_area_image(N, r):
    """Exact area fraction of the centred disk of radius r in each pixel (adaptive quadrature
    of the clipped chord height over the pixel's x-range)."""
    from scipy.integrate import quad
    D = 2.0 / N
    img = np.zeros((N, N))
    for l in range(N):
        y0, y1 = -1 + l * D, -1 + (l + 1) * D
        for k in range(N):
            x0, x1 = -1 + k * D, -1 + (k + 1) * D
            # corners fully inside / outside
            dmin = math.hypot(max(x0, 0, -x1), max(y0, 0, -y1))
            dmax = math.hypot(max(abs(x0), abs(x1)), max(abs(y0), abs(y1)))
            if dmin >= r:
                continue
            if dmax <= r:
                img[l, k] = 1.0
                continue
            a, b = max(x0, -r), min(x1, r)
            if b <= a:
                continue

            def h(t):
                s = math.sqrt(max(r * r - t * t, 0.0))
                return max(0.0, min(y1, s) - max(y0, -s))

            pts = [p for yy in (y0, y1) if abs(yy) < r
                   for p in (math.sqrt(r * r - yy * yy), -math.sqrt(r * r - yy * yy)) if a < p < b]
            val, _ = quad(h, a, b, points=pts or None, epsabs=1e-15, epsrel=1e-13, limit=200)
            img[l, k] = val / (D * D)
    return img
