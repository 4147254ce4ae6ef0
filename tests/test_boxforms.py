"""Pins of the closed-form static box integrals in ``boxforms`` (the checker
behind the small-box and lag-moment pins of the oracle's Green dyad), and a
brute-force pin of individual G_k(d) on boxes that cross the knot spheres.

The antiderivatives are checked against adaptive cubature (scipy.integrate)
of their defining integrands on boxes away from the observation point,
against finite differences of ``inv_r`` (for both Hessians, through the
shift of the box), and against exact values for the box around the point.
"""

import math

import numpy as np
import pytest
from scipy import integrate

import boxforms as bf
from oracle import basis, green

BOXES = [((0.5, 1.5), (-0.5, 0.5), (-0.5, 0.5)),
         ((1.5, 2.5), (0.5, 1.5), (-0.5, 0.5)),
         ((-3.5, -2.5), (1.5, 2.5), (0.5, 1.5)),
         ((0.3, 1.1), (-0.7, 0.4), (0.2, 0.9))]


def _cub(f, box, eps=1e-11):
    (x1, x2), (y1, y2), (z1, z2) = box
    val, _ = integrate.nquad(lambda x, y, z: f(x, y, z), [[x1, x2], [y1, y2], [z1, z2]],
                             opts={"epsabs": 0.0, "epsrel": eps, "limit": 200})
    return val


@pytest.mark.parametrize("box", BOXES)
def test_inv_r_against_cubature(box):
    ref = _cub(lambda x, y, z: 1.0 / math.sqrt(x * x + y * y + z * z), box)
    assert bf.inv_r(box) == pytest.approx(ref, rel=1e-10)


@pytest.mark.parametrize("box", BOXES)
def test_hessians_against_cubature(box):
    # d_p d_q of int 1/|r - x'| at r = 0 is int (3 x_p x_q - delta R^2)/R^5;
    # d_p d_q of int |r - x'| at r = 0 is int (delta R^2 - x_p x_q)/R^3
    H1, H2 = bf.hess_inv_r(box), bf.hess_r(box)
    for p in range(3):
        for q in range(p, 3):
            def k1(x, y, z, p=p, q=q):
                v = (x, y, z)
                r2 = x * x + y * y + z * z
                return (3 * v[p] * v[q] - (r2 if p == q else 0.0)) / r2 ** 2.5

            def k2(x, y, z, p=p, q=q):
                v = (x, y, z)
                r2 = x * x + y * y + z * z
                return ((r2 if p == q else 0.0) - v[p] * v[q]) / r2 ** 1.5
            assert H1[p, q] == pytest.approx(_cub(k1, box), rel=1e-8, abs=1e-12)
            assert H2[p, q] == pytest.approx(_cub(k2, box), rel=1e-8, abs=1e-12)
            assert H1[p, q] == H1[q, p] and H2[p, q] == H2[q, p]


def _shift(box, v):
    return tuple((a - s, b - s) for (a, b), s in zip(box, v))


@pytest.mark.parametrize("box", BOXES + [((-0.5, 0.5),) * 3])
def test_hess_inv_r_is_second_difference_of_inv_r(box):
    # moving the observation point by r is moving the box by -r; central
    # second differences at steps h and h/2, Richardson-extrapolated
    H = bf.hess_inv_r(box)

    def fd(p, q, h):
        ep, eq = np.eye(3)[p] * h, np.eye(3)[q] * h
        return (bf.inv_r(_shift(box, ep + eq)) - bf.inv_r(_shift(box, ep - eq))
                - bf.inv_r(_shift(box, -ep + eq)) + bf.inv_r(_shift(box, -ep - eq))) / (4 * h * h)
    for p in range(3):
        for q in range(3):
            h = 8e-3
            est = (4 * fd(p, q, h / 2) - fd(p, q, h)) / 3
            assert H[p, q] == pytest.approx(est, rel=2e-6, abs=1e-7)


def test_self_box_values():
    # the unit box around the point: grad grad int 1/(4 pi R) = -I/3 (Laplacian
    # -1 shared by symmetry), int 1/R = 3 ln(2 + sqrt 3) - pi/2, and by
    # symmetry d_p d_q int R is 2/3 int 1/R on the diagonal, 0 off it
    b = ((-0.5, 0.5),) * 3
    c = 3 * math.log(2 + math.sqrt(3)) - math.pi / 2
    assert bf.inv_r(b) == pytest.approx(c, rel=1e-14)
    assert np.abs(bf.hess_inv_r(b) / (4 * math.pi) + np.eye(3) / 3).max() < 1e-14
    assert np.abs(bf.hess_r(b) - 2.0 / 3.0 * c * np.eye(3)).max() < 1e-13


# ---- P5: brute-force face sums of individual G_k(d)
def _f_prime(R, k, L):
    """f'(R) for f(R) = T(k - R/L)/(4 pi R), from the spline of ``basis``."""
    s = k - R / L
    T = basis.spline(s)
    # dT/ds on the three pieces: s+1, 1-2s, s-2
    dT = np.where((s >= -1) & (s < 0), s + 1, np.where((s >= 0) & (s < 1), 1 - 2 * s,
                  np.where((s >= 1) & (s < 2), s - 2, 0.0)))
    return (-dT / L / R - T / (R * R)) / (4 * math.pi)


def _hess_pi_faces(d, k, L, n):
    """d_p d_q Pi_k(0) = sum_s s int_{F_q^s} f'(R) x_p / R dS by n x n midpoint sums."""
    u = (np.arange(n) + 0.5) / n - 0.5
    A = np.zeros((3, 3))
    for q in range(3):
        a, b = [i for i in range(3) if i != q]
        U, V = np.meshgrid(d[a] + u, d[b] + u, indexing="ij")
        for s in (1.0, -1.0):
            X = [None] * 3
            X[q] = np.full_like(U, d[q] + 0.5 * s)
            X[a], X[b] = U, V
            R = np.sqrt(X[0] ** 2 + X[1] ** 2 + X[2] ** 2)
            w = _f_prime(R, k, L) / R / (n * n)
            for p in range(3):
                A[p, q] += s * np.sum(w * X[p])
    return 0.5 * (A + A.T)


@pytest.mark.parametrize("alpha,d,k", [(1, (1, 0, 0), 2), (1, (2, 1, 0), 4), (2, (1, 1, 0), 1),
                                       (2, (2, 1, 1), 2), (2, (3, 0, 2), 3), (5, (2, 2, 1), 1)])
def test_green_dyad_brute_force_faces(alpha, d, k):
    # For d != 0 the observation point lies outside the source box, where the
    # retarded potential solves the wave equation: d_t^2 Pi_k = trace of its
    # Hessian.  So G_k(d) = H - trace(H) I with H the Hessian, which is a
    # face integral of f' (continuous for the C^1 spline); plain midpoint sums,
    # Richardson-extrapolated in the face resolution, give G_k(d) with none of
    # the oracle's closed-form pieces.
    L = basis.cdt_from_alpha(alpha)
    R = [(_hess_pi_faces(d, k, L, n)) for n in (200, 400)]
    H = (4 * R[1] - R[0]) / 3
    ref = H - np.trace(H) * np.eye(3)
    got = green.dyad_at([d[0]], [d[1]], [d[2]], k, L)[:, 0]
    G = np.zeros((3, 3))
    for c, (p, q) in enumerate(green.PAIR):
        G[p, q] = G[q, p] = got[c]
    # the box must actually meet a knot sphere R = (k - j) L for this to test the splitting
    dmin = math.sqrt(sum(max(abs(x) - 0.5, 0) ** 2 for x in d))
    dmax = math.sqrt(sum((abs(x) + 0.5) ** 2 for x in d))
    assert any(dmin < (k - j) * L < dmax for j in (-1, 0, 1, 2))
    assert np.abs(G - ref).max() <= 2e-6 * np.abs(ref).max()
