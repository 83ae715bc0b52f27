"""Write strip_weights_2x2.txt: the strip-area weights of a 2x2 image written out from
elementary geometry (no projector code, neither the oracle's nor the library's).

Operator (Section 1, eq. "nonlinear_forward", parallel beam with the strip-area reading of
the toolbox discretisation): a[v][j][l][k] = |Q_lk  ∩  {e_j <= x cos(theta_v) + y sin(theta_v)
< e_{j+1}}| / ds, image on [-1, 1]^2 with pixel (l, k) = [-1 + k D, -1 + (k+1) D] x
[-1 + l D, -1 + (l+1) D], D = 2 / N, bin edges e_j = -1.42 + j ds, ds = 2.84 / nb.

theta = 0 and pi/2: the strip meets the pixel in a rectangle, D times the overlap of the
pixel's x (y) interval with the bin.  theta = pi/4: s = (x + y) / sqrt 2, and the part of the
pixel with x + y <= t has area u^2 / 2 (0 <= u <= D), D^2 - (2D - u)^2 / 2 (D <= u <= 2D),
with u = t - x0 - y0 and (x0, y0) the pixel's lower-left corner.

Also writes dtheta_2x2.txt: d a[v][j][l][k] / d theta_v = (M(e_j) - M(e_{j+1})) / ds, with
M(e) the integral of p . t (t = (-sin, cos)) along the chord {p in Q : p . n = e} (the
boundaries of the strip turn with theta, and a point p of a boundary line moves across it at
rate p . t).  At theta = 0 the chord is the vertical segment x = e across the pixel and
M(e) = D * (y centre); at theta = pi/2 it is the horizontal segment y = e and
M(e) = -D * (x centre); M(e) = 0 when the line misses the pixel.

Run from the repository root: python tests/golden/make_strip_weights.py
"""
import math
import os

N, NB = 2, 5
D = 2.0 / N
DS = 2.84 / NB
THETAS = [("0", 0.0), ("pi/4", math.pi / 4), ("pi/2", math.pi / 2)]


def overlap(a0, a1, b0, b1):
    return max(0.0, min(a1, b1) - max(a0, b0))


def below(u):
    """Area of {x + y <= x0 + y0 + u} inside a D x D square."""
    if u <= 0.0:
        return 0.0
    if u <= D:
        return 0.5 * u * u
    if u <= 2.0 * D:
        return D * D - 0.5 * (2.0 * D - u) ** 2
    return D * D


def weight(name, j, l, k):
    x0, y0 = -1.0 + k * D, -1.0 + l * D
    e0, e1 = -1.42 + j * DS, -1.42 + (j + 1) * DS
    if name == "0":
        area = D * overlap(x0, x0 + D, e0, e1)
    elif name == "pi/2":
        area = D * overlap(y0, y0 + D, e0, e1)
    else:
        r2 = math.sqrt(2.0)
        area = below(r2 * e1 - x0 - y0) - below(r2 * e0 - x0 - y0)
    return area / DS


def moment(name, e, l, k):
    x0, y0 = -1.0 + k * D, -1.0 + l * D
    if name == "0":
        return D * (y0 + 0.5 * D) if x0 < e < x0 + D else 0.0
    return -D * (x0 + 0.5 * D) if y0 < e < y0 + D else 0.0


def main():
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "strip_weights_2x2.txt")
    with open(out, "w") as f:
        f.write("# strip-area weights a[v][j][l][k] of a 2x2 image, 5 bins on [-1.42, 1.42]\n")
        f.write("# (Section 1, eq. nonlinear_forward; elementary geometry, see make_strip_weights.py)\n")
        f.write("# theta j l k weight\n")
        for name, _ in THETAS:
            for j in range(NB):
                for l in range(N):
                    for k in range(N):
                        f.write(f"{name} {j} {l} {k} {weight(name, j, l, k):.17g}\n")
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "dtheta_2x2.txt")
    with open(out, "w") as f:
        f.write("# d a[v][j][l][k] / d theta_v of a 2x2 image, 5 bins on [-1.42, 1.42]\n")
        f.write("# (Section 1, eq. nonlinear_forward; chord moments, see make_strip_weights.py)\n")
        f.write("# theta j l k derivative\n")
        for name in ("0", "pi/2"):
            for j in range(NB):
                e0, e1 = -1.42 + j * DS, -1.42 + (j + 1) * DS
                for l in range(N):
                    for k in range(N):
                        dv = (moment(name, e0, l, k) - moment(name, e1, l, k)) / DS
                        f.write(f"{name} {j} {l} {k} {dv:.17g}\n")


if __name__ == "__main__":
    main()
