"""Pins of the fan-beam oracle (CPU only).

The fan-beam operator of the C oracle (Section 6.2's CT geometry; source at distance R from
the rotation centre; near each pixel the rays are taken as parallel along the ray through its
centre, so the weight is the strip-area weight for that ray's direction, centred at the
pixel's perspective projection and scaled by its magnification) is checked against:
  * the parallel-beam strip model, which it must become as R grows (projection, backprojection
    and angle derivative; the gap is first order in 1/R);
  * mass: every pixel whose footprint lies on the detector puts m x (pixel area) into each
    view, m = R l / (R + c.t)^2 (l the source-to-pixel distance) the detector length per unit
    length across the rays at the pixel, computed here from the geometry;
  * the analytic fan-beam projection of a disk, the bin average of its chord lengths
    2 sqrt(r^2 - d(s)^2) along the rays through the source (d the distance from the disk's
    centre to the ray), which the pixelised disk approaches at second order in the pixel size
    (a model off at first order, e.g. with the wrong magnification or footprint direction,
    stalls at a fixed gap instead);
  * one off-axis pixel on a fine detector against the exact chord lengths of the square along
    the diverging rays: the local-parallel model is off by a shape error of the order of the
    ray spread across the pixel (pixel size over source distance), so the gap halves with the
    pixel, where a footprint taken along the wrong direction (the central ray's, or the tilt
    with the wrong sign) stays off by the tilt itself;
  * central differences in the angle for the derivative, and the adjoint identity for both
    transposes.
"""
import math

import numpy as np

from oracle import projector as P


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - b) / np.linalg.norm(b))


def test_large_source_distance_is_the_parallel_beam():
    rng = np.random.default_rng(0)
    N, nb = 24, 35
    x = rng.uniform(0, 1, (N, N))
    th = np.concatenate([[0.0, math.pi / 4, math.pi / 2, 1e-7], rng.uniform(0, math.pi, 6)])
    y = rng.standard_normal((th.size, nb))
    gaps = []
    for R in (1e8, 1e10):
        gp = rel(P.fan_project(x, th, nb, R), P.project(x, th, nb))
        gd = rel(P.fan_dtheta(x, th, nb, R), P.dtheta(x, th, nb))
        gb = rel(P.fan_backproject(y, th, N, R), P.backproject(y, th, N))
        gaps.append((gp, gd, gb))
    # first order in 1/R: a hundredfold distance leaves a hundredth of every gap
    for g8, g10 in zip(*gaps):
        assert g10 < 1e-8 and 80.0 < g8 / g10 < 120.0, (g8, g10)


def test_mass_is_magnified_pixel_area():
    rng = np.random.default_rng(1)
    N, nb, R = 20, 41, 3.0
    d = 2.0 / N
    ds = 2.84 / nb
    c = -1.0 + (np.arange(N) + 0.5) * d
    X, Y = np.meshgrid(c, c)   # X along k (fast), Y along l
    # an image inside the disk of radius 0.7, whose magnified footprints stay on the detector
    x = rng.uniform(0, 1, (N, N)) * (X * X + Y * Y < 0.49)
    th = rng.uniform(0, 2 * math.pi, 7)
    y = P.fan_project(x, th, nb, R)
    for v, t in enumerate(th):
        ct = -X * math.sin(t) + Y * math.cos(t)
        cn = X * math.cos(t) + Y * math.sin(t)
        b = R + ct
        m = R * np.sqrt(cn * cn + b * b) / (b * b)
        half = m * d / math.sqrt(2.0)   # bounds the footprint's half-width in any direction
        assert np.all((np.abs(R * cn / b) + half < 1.42)[x > 0])
        want = np.sum(x * m) * d * d
        assert abs(y[v].sum() * ds - want) <= 1e-12 * want


def disk_fan_bins(cx, cy, r, th, nb, R, n_quad=64):
    """Bin averages over s of the disk's chord length along the fan rays of view th."""
    ds = 2.84 / nb
    n = np.array([math.cos(th), math.sin(th)])
    t = np.array([-math.sin(th), math.cos(th)])
    S = -R * t
    C = np.array([cx, cy])
    g, w = np.polynomial.legendre.leggauss(n_quad)
    out = np.zeros(nb)
    for j in range(nb):
        e0 = -1.42 + j * ds
        s = e0 + 0.5 * ds * (g + 1.0)
        acc = 0.0
        for si, wi in zip(s, w):
            u = si * n - S
            u /= np.linalg.norm(u)
            dvec = C - S
            dist = abs(dvec[0] * u[1] - dvec[1] * u[0])
            acc += wi * 2.0 * math.sqrt(max(r * r - dist * dist, 0.0))
        out[j] = 0.5 * acc
    return out


def disk_image(N, cx, cy, r, sub=8):
    """Area fraction of the disk in every pixel (sub x sub sampling)."""
    d = 2.0 / N
    o = (np.arange(sub) + 0.5) / sub
    c = -1.0 + d * (np.arange(N)[:, None] + o[None, :])
    X = c.reshape(-1)
    inside = ((X[None, :] - cx) ** 2 + (X[:, None] - cy) ** 2) <= r * r
    return inside.reshape(N, sub, N, sub).mean(axis=(1, 3))


def test_disk_projection_converges_to_the_fan_chords():
    cx, cy, r, R, nb = 0.15, -0.2, 0.45, 2.5, 57
    th = np.array([0.3, 1.2, 2.0])
    ref = np.stack([disk_fan_bins(cx, cy, r, t, nb, R) for t in th])
    errs = []
    for N in (32, 64, 128):
        y = P.fan_project(disk_image(N, cx, cy, r), th, nb, R)
        errs.append(rel(y, ref))
    # second order: each halving of the pixel cuts the gap by about four (3.1 and 3.5 seen)
    assert errs[0] > 2.5 * errs[1] and errs[1] > 2.5 * errs[2], errs
    assert errs[2] < 3e-3, errs


def square_fan_bins(cx, cy, hw, th, nb, R, n_quad=24):
    """Bin averages of the chord lengths of the square [cx +- hw] x [cy +- hw] along the rays
    from the source S = -R t(th) to the detector points s n(th)."""
    ds = 2.84 / nb
    n = np.array([math.cos(th), math.sin(th)])
    S = R * np.array([math.sin(th), -math.cos(th)])
    g, w = np.polynomial.legendre.leggauss(n_quad)
    s = (-1.42 + np.arange(nb) * ds)[:, None] + 0.5 * ds * (g[None, :] + 1.0)
    px, py = s * n[0] - S[0], s * n[1] - S[1]
    norm = np.hypot(px, py)
    lo = np.full(s.shape, -np.inf)
    hi = np.full(s.shape, np.inf)
    for o, u in ((S[0] - cx, px / norm), (S[1] - cy, py / norm)):
        with np.errstate(divide="ignore", invalid="ignore"):
            a, b = (-hw - o) / u, (hw - o) / u
        lo = np.maximum(lo, np.minimum(a, b))
        hi = np.minimum(hi, np.maximum(a, b))
    return 0.5 * (np.clip(hi - lo, 0.0, None) * w[None, :]).sum(axis=1)


def test_off_axis_pixel_follows_its_own_ray():
    R, nb = 2.5, 4000
    errs = []
    for N in (8, 16, 32):
        d = 2.0 / N
        k = int(1.6 / d)                 # the pixel nearest (0.6, 0.6): far off the axis
        c = -1.0 + (k + 0.5) * d
        x = np.zeros((N, N))
        x[k, k] = 1.0
        th = np.array([0.3, 2.0])        # tilts of about 0.26 and 0.2 rad
        y = P.fan_project(x, th, nb, R)
        errs.append([rel(y[v], square_fan_bins(c, c, d / 2, t, nb, R)) for v, t in enumerate(th)])
    errs = np.array(errs)
    # seen: 0.075/0.057, 0.036/0.025, 0.019/0.013; the wrong tilt sign stays near 0.2-0.28
    assert np.all(errs[:-1] > 1.7 * errs[1:]), errs
    assert np.all(errs[-1] < 0.03), errs


def test_angle_derivative_by_central_differences():
    rng = np.random.default_rng(2)
    N, nb, R = 24, 35, 3.0
    x = rng.uniform(0, 1, (N, N))
    th = np.concatenate([[0.0, math.pi / 2, 0.7], rng.uniform(0, 2 * math.pi, 4)])
    D = P.fan_dtheta(x, th, nb, R)
    errs = []
    for h in (1e-5, 1e-6):
        fd = (P.fan_project(x, th + h, nb, R) - P.fan_project(x, th - h, nb, R)) / (2 * h)
        errs.append(rel(D, fd))
    # the discrepancy is the differences' own error (5.6e-6, then 2.6e-8): it falls faster
    # than the step, where a missing or wrong term would leave a fixed gap
    assert errs[0] > 20.0 * errs[1] and errs[1] < 1e-6, errs


def test_adjoint_identities():
    rng = np.random.default_rng(3)
    N, nb, R = 18, 27, 2.2
    x = rng.uniform(0, 1, (N, N))
    th = rng.uniform(0, 2 * math.pi, 9)
    y = rng.standard_normal((th.size, nb))
    for fwd, bwd in ((P.fan_project, P.fan_backproject), (P.fan_dtheta, P.fan_dtheta_t)):
        lhs = float(np.sum(fwd(x, th, nb, R) * y))
        rhs = float(np.sum(x * bwd(y, th, N, R)))
        assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
