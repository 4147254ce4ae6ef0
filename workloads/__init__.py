"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds input recipes only -- grid shapes, permittivity maps,
random currents and plane-wave parameters -- and none of the method's
arithmetic.  Every array is drawn from NumPy's PCG64 with a fixed seed on the
host and handed to either implementation unchanged.

Pulse recipe (stand-in for the paper's modulated Gaussian of Eq. 7 / Table II,
peak-normalized): the -20 dB full width of the amplitude spectrum is 0.8 f0,
so sigma_f = 0.4 f0 / sqrt(2 ln 10), sigma = 1/(2 pi sigma_f), t0 = 6 sigma
(the ratio t0/sigma = 6 of Table II), f_max = 1.4 f0 and the voxel edge is
h = lambda_min / ppw with lambda_min = c0 / f_max.  Units c0 = h = 1.
"""

import math
from dataclasses import dataclass, field

import numpy as np


def pulse(ppw, k_hat=(0.0, 0.0, 1.0), e_hat=(1.0, 0.0, 0.0), amp=1.0):
    """Plane-wave parameters for h = lambda_min / ppw."""
    f0 = 1.0 / (1.4 * ppw)
    sigma_f = 0.4 * f0 / math.sqrt(2.0 * math.log(10.0))
    sigma = 1.0 / (2.0 * math.pi * sigma_f)
    return {"e": np.array(e_hat, dtype=np.float64), "k": np.array(k_hat, dtype=np.float64),
            "f0": f0, "sigma": sigma, "t0": 6.0 * sigma, "amp": float(amp)}


def eps_uniform(n, value):
    nx, ny, nz = n
    return np.full((nz, ny, nx), float(value))


def eps_iid(n, lo, hi, seed):
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(nz, ny, nx))


def eps_nested(n, seed, layers=((16, 6.0), (32, 4.0), (48, 2.5)), noise=0.05):
    """Concentric cubes by Chebyshev distance from the centre, +-noise jitter."""
    nx, ny, nz = n
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cheb = np.maximum(np.maximum(np.abs(2 * x + 1 - nx), np.abs(2 * y + 1 - ny)),
                      np.abs(2 * z + 1 - nz)) / 2.0
    eps = np.ones((nz, ny, nx))
    for r, v in sorted(layers, reverse=True):
        eps[cheb < r] = v
    rng = np.random.default_rng(seed)
    return eps * (1.0 + noise * rng.uniform(-1.0, 1.0, size=eps.shape))


def eps_pillars(n=(320, 320, 48), seed=4, pitch=40, radius=12, z_range=(4, 44),
                core=6.0, shell=3.5, core_r=(6, 9)):
    """8x8 z-axis cylinders: core eps for rho < r_c (r_c seeded per pillar), shell to radius."""
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    ax, ay = nx // pitch, ny // pitch
    rc = rng.integers(core_r[0], core_r[1] + 1, size=(ay, ax))
    eps = np.ones((nz, ny, nx))
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    plane = np.ones((ny, nx))
    for b in range(ay):
        for a in range(ax):
            cx, cy = pitch // 2 + pitch * a, pitch // 2 + pitch * b
            r2x4 = (2 * x + 1 - 2 * cx) ** 2 + (2 * y + 1 - 2 * cy) ** 2  # (2 rho)^2
            plane[r2x4 < 4 * radius * radius] = shell
            plane[r2x4 < 4 * rc[b, a] * rc[b, a]] = core
    eps[z_range[0]:z_range[1]] = plane[None]
    return eps


def random_current(n, seed, dtype=np.float64):
    """i.i.d. standard-normal current [3][nz][ny][nx]."""
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    return rng.standard_normal((3, nz, ny, nx)).astype(dtype)


def sparse_current(n, seed, count):
    """Current that is nonzero on ``count`` random voxels only (all 3 components)."""
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    J = np.zeros((3, nz, ny, nx))
    idx = rng.choice(nx * ny * nz, size=count, replace=False)
    J.reshape(3, -1)[:, idx] = rng.standard_normal((3, count))
    return J, idx


# Regularization of the marches of these workloads: the second difference
# (d/2, -d, d/2) of the regularized interaction matrices (delta_n = d_n
# diag(eps_r) for n = 0, 1, 2), with d per time step dt = alpha dt_CFL.
# Values: about twice the smallest d that kept the 300-step 64^3 i.i.d. cube
# and the 96^3 nested cube of the time-step sweep (over two windows of
# 1600 dt_CFL) bounded.
DELTA_TABLE = {1: 1.5, 2: 0.4, 4: 0.1, 8: 0.01, 16: 0.002}


def delta_for(alpha):
    """d for dt = alpha dt_CFL: DELTA_TABLE, log-linear in alpha between entries."""
    a = float(alpha)
    keys = sorted(DELTA_TABLE)
    if a <= keys[0]:
        return DELTA_TABLE[keys[0]]
    if a >= keys[-1]:
        return DELTA_TABLE[keys[-1]]
    for lo, hi in zip(keys, keys[1:]):
        if lo <= a <= hi:
            t = math.log(a / lo) / math.log(hi / lo)
            return math.exp((1 - t) * math.log(DELTA_TABLE[lo]) + t * math.log(DELTA_TABLE[hi]))


def regularization_for(alpha):
    """(d_0, d_1, d_2) = (d/2, -d, d/2) with d = delta_for(alpha)."""
    d = delta_for(alpha)
    return (0.5 * d, -d, 0.5 * d)


@dataclass
class Workload:
    name: str
    n: tuple            # (nx, ny, nz)
    alpha: int          # dt = alpha * dt_CFL
    steps: int
    ppw: int            # voxels per minimum wavelength
    eps_fn: object = field(repr=False)

    def eps(self):
        return self.eps_fn(self.n)

    def unknowns(self):
        return 3 * self.n[0] * self.n[1] * self.n[2]


CUBE16 = Workload("cube16_eps4_a1", (16, 16, 16), 1, 200, 20, lambda n: eps_uniform(n, 4.0))
CUBE64 = Workload("cube64_iid2to6_a8", (64, 64, 64), 8, 300, 20, lambda n: eps_iid(n, 2.0, 6.0, 2))
CUBE96 = Workload("cube96_nested_sweep", (96, 96, 96), 16, 100, 40, lambda n: eps_nested(n, 3))
PILLARS = Workload("pillars8x8_320x320x48_a16", (320, 320, 48), 16, 120, 40,
                   lambda n: eps_pillars(n, 4))
WORKLOADS = {w.name: w for w in (CUBE16, CUBE64, CUBE96, PILLARS)}


@dataclass
class Scatterer:
    """One member of a batch: a cube with its own permittivity map and incidence."""
    n: tuple
    eps: np.ndarray = field(repr=False)
    k_hat: tuple
    e_hat: tuple


def cube_batch(count=32, sides=(24, 32, 40, 48, 64, 80), lo=1.5, hi=6.0, seed=5):
    """Batch of independent cubes: side drawn from ``sides``, eps_r i.i.d. U[lo, hi],
    incidence direction uniform on the sphere, polarization uniform on the
    circle orthogonal to it (all from one PCG64 stream)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        s = int(rng.choice(sides))
        eps = rng.uniform(lo, hi, size=(s, s, s))
        k = rng.standard_normal(3)
        k /= np.linalg.norm(k)
        a = rng.standard_normal(3)
        e = a - np.dot(a, k) * k
        e /= np.linalg.norm(e)
        out.append(Scatterer((s, s, s), eps, tuple(float(v) for v in k), tuple(float(v) for v in e)))
    return out


# batch of 32 cubes (sides 24..80), alpha = 4, 150 steps, h = lambda_min / 40
BATCH_ALPHA, BATCH_STEPS, BATCH_PPW = 4, 150, 40
