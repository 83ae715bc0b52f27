"""Pins of the FP64 projector oracle against geometry, closed forms and calculus.

Each check is independent of the oracle's own formulas: polygon clipping for the
strip-area weights, the projection of the whole square and of a disk in closed
form, mass conservation, the adjoint identity, rotation/reflection symmetries,
central finite differences of clipped areas for the angle derivative, and the stored
hand-derived weights of a 2x2 image (tests/golden/).
"""
import math
import os

import numpy as np
import pytest

from oracle import projector as P
from paper_2605_06336_amd import synth
from tests import brute

SPECIAL = [0.0, math.pi / 4, math.pi / 2, 3 * math.pi / 4, 1e-7, math.pi / 2 - 1e-9,
           0.3, 1.1, 2.0, 2.9, math.pi - 1e-3]


def test_golden_strip_weights_2x2():
    """The stored strip-area weights of a 2x2 image at 0, pi/4 and pi/2 (written out from
    interval overlaps and corner-triangle areas by tests/golden/make_strip_weights.py) equal
    the oracle's weights, read as its projection of each unit pixel."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "strip_weights_2x2.txt")
    names = {"0": 0.0, "pi/4": math.pi / 4, "pi/2": math.pi / 2}
    want = {}
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, j, l, k, w = line.split()
            want[(name, int(j), int(l), int(k))] = float(w)
    assert len(want) == 3 * 5 * 4
    th = np.array(list(names.values()))
    for l in range(2):
        for k in range(2):
            img = np.zeros((2, 2))
            img[l, k] = 1.0
            y = P.project(img, th, 5)
            for v, name in enumerate(names):
                for j in range(5):
                    assert abs(y[v, j] - want[(name, j, l, k)]) < 1e-13, (name, j, l, k)
    # each pixel's weights integrate to its area in every view
    for name in names:
        for l in range(2):
            for k in range(2):
                tot = sum(want[(name, j, l, k)] for j in range(5)) * (2.84 / 5)
                assert abs(tot - 1.0) < 1e-13


def test_golden_dtheta_2x2():
    """The stored angle derivatives of the 2x2 weights at 0 and pi/2 (chord moments of the
    strip boundaries written out by tests/golden/make_strip_weights.py) equal the oracle's
    derivative of the projection of each unit pixel; this fixes the sign convention."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "dtheta_2x2.txt")
    want = {}
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, j, l, k, w = line.split()
            want[(name, int(j), int(l), int(k))] = float(w)
    assert len(want) == 2 * 5 * 4
    names = ["0", "pi/2"]
    th = np.array([0.0, math.pi / 2])
    for l in range(2):
        for k in range(2):
            img = np.zeros((2, 2))
            img[l, k] = 1.0
            dy = P.dtheta(img, th, 5)
            for v, name in enumerate(names):
                for j in range(5):
                    assert abs(dy[v, j] - want[(name, j, l, k)]) < 1e-13, (name, j, l, k)


@pytest.mark.parametrize("N,nb", [(8, 13), (6, 11), (10, 9)])
def test_weights_match_polygon_clipping(N, nb):
    th = np.array(SPECIAL + list(synth.random_angles(6, seed=N)))
    A, _ = P.dense(N, nb, th)
    B = brute.dense_matrix(N, nb, th)
    assert np.max(np.abs(A - B)) < 1e-13


def test_all_ones_image_closed_form():
    N, nb = 32, 47
    th = np.array(SPECIAL)
    y = P.project(np.ones((N, N)), th, nb)
    for v, t in enumerate(th):
        ref = brute.big_square_projection(nb, t)
        assert np.max(np.abs(y[v] - ref)) < 1e-12


def test_disk_converges_to_chord_integral():
    """Projection of the exactly pixelised disk vs the bin-averaged chord 2 sqrt(r^2 - s^2).
    The discretisation error is O(D) for bins crossing the circle transversally; the
    bins tangent to it carry a phase-dependent O(sqrt(D)) error and are excluded."""
    r = 0.6
    errs = []
    for N, nb in [(64, 91), (128, 181), (256, 363)]:
        img = brute.disk_area_image(N, r)
        th = np.array([0.0, 0.4, math.pi / 4, 1.9])
        y = P.project(img, th, nb)
        ref = brute.disk_bin_average(nb, r)
        s = -1.42 + (np.arange(nb) + 0.5) * 2.84 / nb
        m = np.abs(s) < r - 0.05
        errs.append(np.mean([np.linalg.norm((y[v] - ref)[m]) / np.linalg.norm(ref[m])
                             for v in range(4)]))
    assert errs[0] < 3e-3
    assert errs[2] < errs[1] < errs[0]
    assert errs[2] < 0.4 * errs[0]


@pytest.mark.parametrize("N,nb", [(16, 23), (31, 45), (64, 91)])
def test_mass_conservation(N, nb):
    x = synth.random_image(N, seed=N)[0]
    th = synth.random_angles(17, seed=3)
    y = P.project(x, th, nb)
    ds, D = 2.84 / nb, 2.0 / N
    mass = y.sum(axis=1) * ds
    assert np.max(np.abs(mass - D * D * x.sum())) <= 1e-13 * D * D * x.sum()


@pytest.mark.parametrize("N,nb,F", [(16, 23, 1), (24, 35, 3)])
def test_adjoint_identity(N, nb, F):
    rng = np.random.default_rng(0)
    counts = rng.integers(3, 9, F)
    vo = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    V = int(vo[-1])
    th = synth.random_angles(V, seed=1)
    x = synth.random_image(N, seed=2, frames=F)
    y = synth.random_sinogram(V, nb, seed=3)
    Ax = P.project(x, th, nb, vo)
    ATy = P.backproject(y, th, N, vo)
    lhs, rhs = float((Ax * y).sum()), float((x.reshape(ATy.shape) * ATy).sum())
    assert abs(lhs - rhs) <= 1e-14 * np.linalg.norm(Ax) * np.linalg.norm(y)


def test_symmetries():
    N, nb = 32, 47
    x = synth.random_image(N, seed=5)[0]
    th = synth.random_angles(9, seed=6, hi=math.pi / 2)
    y = P.project(x, th, nb)
    y_pi = P.project(x, th + math.pi, nb)
    assert np.max(np.abs(y_pi - y[:, ::-1])) < 1e-12
    # xr[l, k] = x[k, N-1-l], i.e. xr(p) = x(R p) with R the +90 degree rotation, so
    # the projection of xr at theta - pi/2 is the projection of x at theta
    xr = np.rot90(x)
    y_rot = P.project(xr, th - math.pi / 2, nb)
    assert np.max(np.abs(y_rot - y)) < 1e-12


def test_dtheta_matches_clipped_area_differences():
    N, nb = 6, 11
    th = np.array([0.2, 0.9, 1.7, 2.6, math.pi / 4 + 0.01])
    _, dA = P.dense(N, nb, th)
    h = 1e-6
    Ap = brute.dense_matrix(N, nb, th + h)
    Am = brute.dense_matrix(N, nb, th - h)
    fd = (Ap - Am) / (2 * h)
    assert np.max(np.abs(dA - fd)) < 1e-7 * max(1.0, np.max(np.abs(dA)))


@pytest.mark.parametrize("N,nb", [(32, 47), (128, 181)])
def test_dtheta_finite_differences_and_zero_sum(N, nb):
    inst = synth.draw(synth.WORKLOADS["c1"], N=N)
    x = inst.x_true[0]
    th = synth.random_angles(12, seed=7)
    D = P.dtheta(x, th, nb)
    errs = []
    for h in (1e-5, 1e-6):
        fd = (P.project(x, th + h, nb) - P.project(x, th - h, nb)) / (2 * h)
        errs.append(np.linalg.norm(D - fd) / np.linalg.norm(D))
    assert errs[1] < 1e-4
    assert np.max(np.abs(D.sum(axis=1))) < 1e-12 * np.abs(D).max() * nb


def test_dtheta_transpose_by_finite_differences_and_adjoint():
    """D^T r (the adjoint-derivative operator of the full-space sensitivity equation): for
    random x, r, <x, D^T r> = d/de <A(theta + e) x, r> at e = 0 (central differences of the
    area projector, which does not use the chord moments), and <D x, r> = <x, D^T r> against
    the forward derivative's loop."""
    rng = np.random.default_rng(12)
    N, nb, V = 12, 19, 9
    th = np.concatenate([rng.uniform(0, np.pi, V - 3), [0.0, np.pi / 4, np.pi / 2 + 1e-3]])
    x = rng.standard_normal((N, N))
    r = rng.standard_normal((V, nb))
    xt = P.dtheta_t(r, th, N)
    lhs = float(np.sum(x * xt))
    h = 1e-6
    fd = (np.sum(P.project(x, th + h, nb) * r) - np.sum(P.project(x, th - h, nb) * r)) / (2 * h)
    assert abs(lhs - fd) <= 1e-6 * (abs(fd) + np.linalg.norm(x) * np.linalg.norm(r) * 1e-3)
    assert abs(float(np.sum(P.dtheta(x, th, nb) * r)) - lhs) <= 1e-12 * np.abs(xt).sum() * np.abs(x).max()
