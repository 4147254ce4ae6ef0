"""Closed-form static integrals over a box, used as pins for the oracle.

Observation point at the origin, box B = [x1,x2] x [y1,y2] x [z1,z2] (no
coordinate of a corner may be zero).  Each quantity is a signed sum over the
eight corners, S[F] = sum s_x s_y s_z F(x, y, z) with s = +1 at the upper
and -1 at the lower bound, of an antiderivative F written out below.  They are
independent of the oracle's quadrature and are themselves checked against
brute-force numerical integration in ``test_boxforms.py``.
"""

import math

import numpy as np


def _corner_sum(box, F):
    (x1, x2), (y1, y2), (z1, z2) = box
    tot = 0.0
    for sx, x in ((-1, x1), (1, x2)):
        for sy, y in ((-1, y1), (1, y2)):
            for sz, z in ((-1, z1), (1, z2)):
                tot += sx * sy * sz * F(x, y, z)
    return tot


def _r(x, y, z):
    return math.sqrt(x * x + y * y + z * z)


def inv_r(box):
    """int_B 1/R dV (gravitational potential of a rectangular prism)."""
    def F(x, y, z):
        R = _r(x, y, z)
        return (y * z * math.log(x + R) + x * z * math.log(y + R) + x * y * math.log(z + R)
                - 0.5 * x * x * math.atan(y * z / (x * R))
                - 0.5 * y * y * math.atan(x * z / (y * R))
                - 0.5 * z * z * math.atan(x * y / (z * R)))
    return _corner_sum(box, F)


def _perm(box, p, q):
    """Reorder box axes so that (p, q, r) become (x, y, z)."""
    r = 3 - p - q
    return (box[p], box[q], box[r])


def hess_inv_r(box):
    """3x3 matrix d_p d_q int_B 1/R dV' (derivatives in the observation point)."""
    H = np.zeros((3, 3))
    for p in range(3):
        q = (p + 1) % 3
        bp = _perm(box, p, q)
        H[p, p] = -_corner_sum(bp, lambda x, y, z: math.atan(y * z / (x * _r(x, y, z))))
    for p, q in ((0, 1), (0, 2), (1, 2)):
        bp = _perm(box, p, q)
        H[p, q] = H[q, p] = _corner_sum(bp, lambda x, y, z: math.log(z + _r(x, y, z)))
    return H


def hess_r(box):
    """3x3 matrix d_p d_q int_B R dV'."""
    H = np.zeros((3, 3))
    for p in range(3):
        q = (p + 1) % 3
        bp = _perm(box, p, q)

        def F(x, y, z):
            R = _r(x, y, z)
            return x * (y * math.log(z + R) + z * math.log(y + R)) - x * x * math.atan(y * z / (x * R))
        H[p, p] = _corner_sum(bp, F)
    for p, q in ((0, 1), (0, 2), (1, 2)):
        bp = _perm(box, p, q)

        def F(x, y, z):
            R = _r(x, y, z)
            return 0.5 * (z * R + (x * x + y * y) * math.log(z + R))
        H[p, q] = H[q, p] = _corner_sum(bp, F)
    return H


def box_of(d):
    return tuple((di - 0.5, di + 0.5) for di in d)


def static_dyad(d):
    """N(d) = d_p d_q int_B 1/(4 pi R) + delta_pq [d = 0]: the alpha-independent
    sum over lags of the retarded dyad (partition of unity of the spline)."""
    N = hess_inv_r(box_of(d)) / (4 * math.pi)
    if tuple(d) == (0, 0, 0):
        N = N + np.eye(3)
    return N


def small_box_dyads(d, L):
    """G_0, G_1, G_2 in closed form when the whole box lies inside R < L."""
    b = box_of(d)
    NA = hess_inv_r(b) / (4 * math.pi)
    M = hess_r(b)
    P = inv_r(b) / (4 * math.pi)
    I = np.eye(3)
    selfb = 1.0 if tuple(d) == (0, 0, 0) else 0.0
    g0 = 0.5 * NA + M / (8 * math.pi * L * L) + I * (-P / (L * L) + 0.5 * selfb)
    g1 = 0.5 * NA - M / (4 * math.pi * L * L) + I * (2 * P / (L * L) + 0.5 * selfb)
    g2 = M / (8 * math.pi * L * L) - I * P / (L * L)
    return g0, g1, g2
