"""Time step, lag count and temporal basis (oracle; test infrastructure only).

Units: c0 = eps0 = h = 1 (h the voxel edge), time in h/c0.  A time step is
given by L = c0*dt/h.  With dt = alpha*dt_CFL and dt_CFL = h/(c0*sqrt(3)) --
the convention that reproduces the paper's 0.0193 fs at 10 nm (Sec. V-B) --
L = alpha/sqrt(3).

Temporal basis (Sec. II, discretization paragraph: causal quadratic spline,
p = 2).  Reading: the uniform quadratic B-spline on integer knots, shifted so
that its support is [-dt, 2dt); in step units s = t/dt

    T(s) = (s+1)^2/2        -1 <= s < 0
           3/4 - (s-1/2)^2   0 <= s < 1
           (2-s)^2/2         1 <= s < 2
           0                 otherwise,

so T(0) = T(1) = 1/2 and T(k) = 0 for every other integer k.  The current is
J(r, t) = sum_n J_n(r) T(t/dt - n).
"""

import math

import numpy as np

SQRT3 = math.sqrt(3.0)

# Polynomial coefficients (a0, a1, a2) of T on its three pieces, in s:
#   T(s) = a0 + a1*s + a2*s^2 for piece j covering s in [j-1, j).
SPLINE_PIECES = (
    (0.5, 1.0, 0.5),    # (s+1)^2/2
    (0.5, 1.0, -1.0),   # 3/4 - (s-1/2)^2
    (2.0, -2.0, 0.5),   # (2-s)^2/2
)


def cdt_from_alpha(alpha):
    """L = c0*dt/h for dt = alpha*dt_CFL, dt_CFL = h/(c0*sqrt(3)) (Eq. 9 scale)."""
    return float(alpha) / SQRT3


def spline(s):
    """T(s) of the module docstring, elementwise, FP64."""
    s = np.asarray(s, dtype=np.float64)
    out = np.zeros_like(s)
    for j, (a0, a1, a2) in enumerate(SPLINE_PIECES):
        m = (s >= j - 1) & (s < j)
        sj = s[m]
        out[m] = a0 + a1 * sj + a2 * sj * sj
    return out


def spline_d2(s):
    """Second derivative of T in s: 1, -2, 1 on the three pieces, else 0."""
    s = np.asarray(s, dtype=np.float64)
    out = np.zeros_like(s)
    for j, (_, _, a2) in enumerate(SPLINE_PIECES):
        out[(s >= j - 1) & (s < j)] = 2.0 * a2
    return out


def nlags(nx, ny, nz, alpha=None, cdt=None, p=2):
    """Maximum lag ell of Eq. 4: ceil(R_max / (c0 dt)) + p.

    Reading: R_max is the largest distance from an observation point (a voxel
    centre) to a source point of the domain (anywhere in a voxel),
    sqrt(sum_i (N_i - 1/2)^2) in units of h.  With the spline support
    [-dt, 2dt) every lag k with a nonzero Z_k then satisfies k <= ell.  For an
    integer alpha the ceiling is exact in integers:
    ceil(R_max/L) = least c with (2 c alpha)^2 >= 3 sum_i (2 N_i - 1)^2.
    """
    if alpha is not None and float(alpha) == int(alpha):
        a = int(alpha)
        m = 3 * ((2 * nx - 1) ** 2 + (2 * ny - 1) ** 2 + (2 * nz - 1) ** 2)
        c = math.isqrt(m) // (2 * a)
        while (2 * c * a) ** 2 < m:
            c += 1
        while c > 0 and (2 * (c - 1) * a) ** 2 >= m:
            c -= 1
        return c + p
    if cdt is None:
        cdt = cdt_from_alpha(alpha)
    rmax = math.sqrt((nx - 0.5) ** 2 + (ny - 0.5) ** 2 + (nz - 0.5) ** 2)
    return int(math.ceil(rmax / cdt)) + p
