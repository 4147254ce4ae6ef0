"""Pins of the oracle's time step, lag count, temporal basis and causal masks."""

import math
import os

import numpy as np
import pytest

from oracle import basis, masks

C0_NM_PER_FS = 299.792458
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _table3():
    rows = []
    with open(os.path.join(GOLDEN, "table3_z0_nnz.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            g, a, v, st = line.split()
            rows.append((int(g), int(a), float(v), st))
    return rows


@pytest.mark.parametrize("grid,alpha,printed,status", [r for r in _table3() if r[3] == "pinned"])
def test_table3_z0_nnz(grid, alpha, printed, status):
    # Table III: 200 nm cube, dt = alpha * 0.005 fs on both meshes.
    h = 200.0 / grid
    cdt = alpha * 0.005 * C0_NM_PER_FS / h
    nnz = masks.zk_nnz(grid, grid, grid, k=0, cdt=cdt)
    assert round(nnz / 1e6, 2) == printed


def test_table3_exact_counts():
    # the exact integers behind the four reproduced rows
    exact = {(40, 4): 9236568, (40, 8): 45558792, (80, 2): 76092408, (80, 4): 382402152}
    for (grid, alpha), val in exact.items():
        cdt = alpha * 0.005 * C0_NM_PER_FS / (200.0 / grid)
        assert masks.zk_nnz(grid, grid, grid, k=0, cdt=cdt) == val


def test_printed_time_steps():
    # Sec. V-B: 10 nm voxels give dt_CFL = 0.0193 fs; dt = 16 dt_CFL = 0.308 fs;
    # f_max = 375 THz with kappa = 2 gives dt_Nyq = 0.67 fs ~ 34 dt_CFL (Eq. 5).
    dt_cfl = 10.0 / (C0_NM_PER_FS * math.sqrt(3.0))
    assert round(dt_cfl, 4) == 0.0193
    assert round(16 * dt_cfl, 3) == 0.308
    dt_nyq = 1.0 / (2 * 2 * 375e-3)  # fs, f in PHz
    assert round(dt_nyq, 2) == 0.67
    assert int(dt_nyq / dt_cfl) == 34
    # Sec. III-B: 2.5 nm voxels give ~0.005 fs
    assert round(2.5 / (C0_NM_PER_FS * math.sqrt(3.0)), 3) == 0.005
    # cdt of the oracle is alpha/sqrt(3) in units of h
    assert basis.cdt_from_alpha(16) == pytest.approx(16 * dt_cfl * C0_NM_PER_FS / 10.0, rel=1e-15)
    # Sec. V-B grid: 240 x 240 x 90 voxels = 5.184e6 cells, 1.56e7 unknowns
    assert 240 * 240 * 90 == 5_184_000
    assert round(3 * 240 * 240 * 90 / 1e7, 2) == 1.56


def test_spline_basis():
    s = np.linspace(-1.5, 2.5, 4001)
    T = basis.spline(s)
    # partition of unity and linear reproduction of the integer shifts
    tot = sum(basis.spline(s - n) for n in range(-4, 6))
    lin = sum(n * basis.spline(s - n) for n in range(-4, 6))
    inner = (s > 0.5) & (s < 1.0)
    assert np.allclose(tot[inner], 1.0, atol=1e-15)
    x = np.linspace(0.0, 1.0, 101)
    assert np.allclose(sum(basis.spline(k - x) for k in range(-3, 6)), 1.0, atol=1e-15)
    assert np.allclose(sum(k * basis.spline(k - x) for k in range(-3, 6)), x + 0.5, atol=1e-14)
    assert basis.spline(np.array([0.0]))[0] == 0.5 and basis.spline(np.array([1.0]))[0] == 0.5
    assert basis.spline(np.array([-1.0, 2.0, 3.0, -2.0])).tolist() == [0.0, 0.0, 0.0, 0.0]
    # causal support [-1, 2) and C1 continuity at the knots
    assert np.all(T[s < -1] == 0) and np.all(T[s >= 2] == 0)
    for knot in (-1.0, 0.0, 1.0, 2.0):
        e = 1e-7
        l, m, r = basis.spline(np.array([knot - e, knot, knot + e]))
        assert abs(l - r) < 1e-6
        assert abs((m - l) / e - (r - m) / e) < 1e-5
    d2 = basis.spline_d2(np.array([-0.5, 0.5, 1.5, 2.5]))
    assert d2.tolist() == [1.0, -2.0, 1.0, 0.0]


@pytest.mark.parametrize("alpha", [1, 2, 3, 8, 16])
def test_integer_mask_matches_fp64_rule(alpha):
    rng = np.random.default_rng(alpha)
    d = rng.integers(-60, 61, size=(3, 20000))
    L = basis.cdt_from_alpha(alpha)
    for k in (0, 1, 2, 3, 7, 20):
        mi = masks.mask(d[0], d[1], d[2], k, alpha=alpha)
        mf = masks.mask(d[0], d[1], d[2], k, cdt=L)
        assert np.array_equal(mi, mf)


def test_z0_self_and_stencil():
    # alpha = 1 (L = 0.577): the Z0 region holds the self voxel and its 6 face neighbours
    d = np.array([[0, 1, 0, 0, 1, 1], [0, 0, 1, 0, 1, 0], [0, 0, 0, 1, 0, 1]])
    m = masks.mask(d[0], d[1], d[2], 0, alpha=1)
    assert m.tolist() == [True, True, True, True, False, False]


@pytest.mark.parametrize("n,alpha", [((16, 16, 16), 1), ((9, 7, 5), 3), ((20, 6, 11), 8)])
def test_nlags_covers_last_nonzero_lag(n, alpha):
    nl = basis.nlags(*n, alpha=alpha)
    last = max(k for k, m in masks.lag_support(*n, nl + 6, alpha=alpha) if m.any())
    assert last <= nl <= last + 1


def test_nlags_integer_ceiling():
    # 16^3 at alpha = 1: R_max / L = 15.5 sqrt(3) * sqrt(3) = 46.5 -> 47 + 2
    assert basis.nlags(16, 16, 16, alpha=1) == 49
    assert basis.nlags(320, 320, 48, alpha=16) == 52
    assert basis.nlags(1, 1, 1, alpha=4) == 3
    # 8^3 at alpha = 3: R_max/L = 7.5*3/3 = 7.5 -> 8 + 2; the FP64 path agrees here
    assert basis.nlags(8, 8, 8, alpha=3) == 10 == basis.nlags(8, 8, 8, cdt=basis.cdt_from_alpha(3))


def test_sparse_z0_exceeds_two_terabytes():
    # Sec. V-B: explicit sparse Z0 for 240x240x90 at dt = 16 dt_CFL exceeds 2 TB.
    nnz = masks.zk_nnz(240, 240, 90, k=0, alpha=16)
    assert nnz > 1.5e11
    # MATLAB sparse (Sec. III-B) stores an FP64 value and a 64-bit row index per nonzero
    assert nnz == 163979728440
    assert nnz * 16 > 2e12
