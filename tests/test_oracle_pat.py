"""Pins of the photoacoustic (circular-means) oracle, CPU only: closed forms on images whose
bilinear interpolant is exact, the dense matrix against the vectorised transpose, central
differences in the radial shift and the adjoint identity."""
import math

import numpy as np

from oracle import pat as PA


def grid(N):
    d = 2.0 / N
    c = -1.0 + (np.arange(N) + 0.5) * d
    return np.meshgrid(c, c)   # X along k (columns), Y along l (rows)


def inside(N, n_a, n_c, K, p):
    """Circles whose samples all lie inside the hull of the pixel centres."""
    X, Y, r, _, _ = PA._samples(N, n_a, n_c, K, p)
    h = 1.0 - 1.0 / N
    return np.all((np.abs(X) <= h) & (np.abs(Y) <= h), axis=2)


def test_interpolant_is_exact_on_linear_images():
    rng = np.random.default_rng(2)
    N = 24
    X, Y = grid(N)
    a, b, c = 0.7, -0.3, 0.45
    img = a + b * X + c * Y
    h = 1.0 - 1.0 / N
    px, py = rng.uniform(-h, h, 200), rng.uniform(-h, h, 200)
    I, gx, gy = PA.interp(img, px, py)
    assert np.max(np.abs(I - (a + b * px + c * py))) < 1e-13
    assert np.max(np.abs(gx - b)) < 1e-12 and np.max(np.abs(gy - c)) < 1e-12


def bump(N):
    X, Y = grid(N)
    return np.exp(-12 * ((X - 0.1) ** 2 + (Y + 0.15) ** 2)) * ((X - 0.1) ** 2 + (Y + 0.15) ** 2 < 0.36)


def test_circle_integrals_over_all_radii_give_the_image_mass():
    """Polar coordinates around a sensor: integrating the circle integrals over the radius
    gives the area integral of the interpolant, d^2 times the sum of the pixel values (each
    bilinear hat integrates to d^2).  The bump's support (within 0.6 of (0.1, -0.15)) lies
    between 0.7 and 2.4 from every sensor, inside the radii [0.7 + 2/n_c, 2.7] at p = 0.7; the
    radius sum converges to the mass as the radii get denser, for every sensor."""
    N, n_a, p = 48, 8, 0.7
    img = bump(N)
    mass = (2.0 / N) ** 2 * img.sum()
    errs = []
    for n_c in (40, 80, 160):
        y = PA.project(img, n_a, n_c, 4 * n_c, p)
        errs.append(float(np.max(np.abs(y.sum(axis=1) * (2.0 / n_c) - mass)) / mass))
    assert errs[2] < 1e-3 and errs[2] < errs[1] < errs[0], errs
    # that sum does not depend on p: its derivative vanishes in the limit
    n_c = 160
    D = PA.project_dp(img, n_a, n_c, 4 * n_c, p)
    y = PA.project(img, n_a, n_c, 4 * n_c, p)
    assert np.max(np.abs(D.sum(axis=1))) < 1e-2 * np.max(np.abs(y.sum(axis=1)))


def test_sensor_geometry_and_shift():
    sx, sy = PA.sensors(8)
    assert np.allclose(np.hypot(sx, sy), 1.5) and np.isclose(sx[0], 1.5) and np.isclose(sy[2], 1.5)
    assert np.allclose(PA.radii(4, 0.1), [0.6, 1.1, 1.6, 2.1])
    # a circle that misses the image entirely sees nothing
    img = np.ones((16, 16))
    y = PA.project(img, 4, 8, 32, -0.2)   # the first radii stay outside [-1, 1]^2
    assert y[0, 0] == 0.0


def test_dense_matrix_equals_projection_and_transpose():
    rng = np.random.default_rng(0)
    N, n_a, n_c, K, p = 10, 6, 7, 24, 0.13
    A = PA.matrix(N, n_a, n_c, K, p)
    img = rng.uniform(0, 1, (N, N))
    yv = rng.standard_normal((n_a, n_c))
    assert np.allclose(A @ img.ravel(), PA.project(img, n_a, n_c, K, p).ravel(), rtol=0,
                       atol=1e-12)
    assert np.allclose(A.T @ yv.ravel(), PA.backproject(yv, N, n_a, n_c, K, p).ravel(), rtol=0,
                       atol=1e-12)


def test_radial_derivative_by_central_differences():
    """A smooth image (no cell-boundary kinks matter at this step): the derivative in p matches
    central differences, and the gap falls with the step."""
    N, n_a, n_c, K, p = 48, 12, 16, 96, 0.07
    X, Y = grid(N)
    img = np.exp(-3 * ((X - 0.2) ** 2 + (Y + 0.1) ** 2)) + 0.3 * np.sin(2 * X) * np.cos(3 * Y)
    D = PA.project_dp(img, n_a, n_c, K, p)
    errs = []
    for h in (1e-4, 1e-5):
        fd = (PA.project(img, n_a, n_c, K, p + h) - PA.project(img, n_a, n_c, K, p - h)) / (2 * h)
        errs.append(float(np.linalg.norm(D - fd) / np.linalg.norm(fd)))
    # the sampled interpolant is piecewise smooth in p: the differences converge to it
    assert errs[1] < 1e-3 and errs[1] < errs[0], errs


def test_adjoint_identity():
    rng = np.random.default_rng(1)
    N, n_a, n_c, K, p = 20, 10, 12, 48, -0.04
    img = rng.uniform(0, 1, (N, N))
    yv = rng.standard_normal((n_a, n_c))
    lhs = float(np.sum(PA.project(img, n_a, n_c, K, p) * yv))
    rhs = float(np.sum(img * PA.backproject(yv, N, n_a, n_c, K, p)))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
