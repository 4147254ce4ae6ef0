"""Pins of the oracle's Green dyad G_k(d) against closed forms and invariants."""

import math

import numpy as np
import pytest

import boxforms as bf
from oracle import basis, green, masks

C1 = (3.0 * math.log(2.0 + math.sqrt(3.0)) - math.pi / 2.0) / (2.0 * math.pi)


def _mat(v):
    M = np.zeros((3, 3))
    for c, (p, q) in enumerate(green.PAIR):
        M[p, q] = M[q, p] = v[c]
    return M


def _dyads(d, L, K):
    return [_mat(green.dyad_at([d[0]], [d[1]], [d[2]], k, L)[:, 0]) for k in range(K)]


@pytest.mark.parametrize("alpha", [2, 4, 16])
def test_self_term_closed_form(alpha):
    # For alpha >= 3/2 the self box lies inside R < c0 dt, one spline piece per lag:
    # G0(0) = (1/3 - c1/a^2) I, G1(0) = (1/3 + 2 c1/a^2) I, G2(0) = -(c1/a^2) I, G3(0) = 0,
    # with c1 = (3 ln(2+sqrt3) - pi/2)/(2 pi) from int_cube dV/|x| = 3 ln(2+sqrt3) - pi/2.
    L = basis.cdt_from_alpha(alpha)
    ref = [1 / 3 - C1 / alpha ** 2, 1 / 3 + 2 * C1 / alpha ** 2, -C1 / alpha ** 2, 0.0]
    for k in range(4):
        g = green.dyad_at([0], [0], [0], k, L)[:, 0]
        assert np.allclose(g[:3], ref[k], rtol=0, atol=2e-15)
        assert np.all(g[3:] == 0.0)
    assert green.dyad_at([0], [0], [0], 0, basis.cdt_from_alpha(16))[0, 0] == pytest.approx(
        0.3318536416246674, abs=1e-15)


@pytest.mark.parametrize("alpha", [5, 8, 16])
def test_small_box_closed_forms(alpha):
    # every box with dmax < L sits in one spline piece per lag: G0, G1, G2 in closed form
    L = basis.cdt_from_alpha(alpha)
    n = int(L) + 1
    checked = 0
    for dx in range(n):
        for dy in range(dx + 1):
            for dz in range(dy + 1):
                d = (dx, dy, dz)
                if math.sqrt(sum((x + 0.5) ** 2 for x in d)) >= L:
                    continue
                refs = bf.small_box_dyads(d, L)
                got = _dyads(d, L, 4)
                for k in range(3):
                    assert np.abs(got[k] - refs[k]).max() <= 1e-14 * max(1.0, np.abs(refs[k]).max())
                assert np.abs(got[3]).max() == 0.0
                checked += 1
    assert checked >= 3


@pytest.mark.parametrize("alpha", [1, 2, 3, 5, 8])
@pytest.mark.parametrize("d", [(0, 0, 0), (1, 0, 0), (1, 2, 0), (2, 1, 3), (0, 3, 4), (4, 5, 6)])
def test_lag_moment_sum_rules(alpha, d):
    # Quadratic B-splines reproduce 1, n and n^2 (sum_k k^j T(k - x) = 1, x + 1/2,
    # (x + 1/2)^2 + 1/4); hence for every offset and every dt:
    #   sum_k G_k = N,  sum_k k G_k = N/2,
    #   sum_k k^2 G_k = d d int_B R/(4 pi L^2) + N_A/2 + I (-2 P/L^2 + [d=0]/2),
    # with N_A = d d int_B 1/(4 pi R), N = N_A + I [d=0], P = int_B 1/(4 pi R).
    L = basis.cdt_from_alpha(alpha)
    dmax = math.sqrt(sum((x + 0.5) ** 2 for x in d))
    G = _dyads(d, L, int(dmax / L) + 4)
    b = bf.box_of(d)
    N = bf.static_dyad(d)
    NA = bf.hess_inv_r(b) / (4 * math.pi)
    M = bf.hess_r(b)
    P = bf.inv_r(b) / (4 * math.pi)
    sb = 1.0 if d == (0, 0, 0) else 0.0
    m2 = M / (4 * math.pi * L * L) + 0.5 * NA + np.eye(3) * (-2 * P / L ** 2 + 0.5 * sb)
    # the corner-sum closed forms cancel terms of size |d|^3 ln|d| down to |d|^-3
    tol = 1e-15 * max(1.0, float(sum(x * x for x in d))) ** 3
    s0 = sum(G)
    s1 = sum(k * g for k, g in enumerate(G))
    s2 = sum(k * k * g for k, g in enumerate(G))
    assert np.abs(s0 - N).max() <= tol * np.abs(N).max() + 1e-16
    assert np.abs(s1 - 0.5 * N).max() <= 10 * tol * np.abs(N).max() + 1e-16
    assert np.abs(s2 - m2).max() <= 10 * tol * np.abs(m2).max() + 1e-16


def test_static_dyad_limits():
    # N(0) = 2/3 I exactly; far field -> (3 dd - I)/(4 pi |d|^3)
    assert np.allclose(bf.static_dyad((0, 0, 0)), 2.0 / 3.0 * np.eye(3), atol=1e-15)
    d = np.array([9.0, 14.0, 20.0])
    r = np.linalg.norm(d)
    far = (3 * np.outer(d, d) / r ** 2 - np.eye(3)) / (4 * math.pi * r ** 3)
    assert np.abs(bf.static_dyad(tuple(int(x) for x in d)) - far).max() < 2e-3 * np.abs(far).max()


@pytest.mark.parametrize("alpha", [1, 4])
def test_symmetry_zeros_and_support(alpha):
    L = basis.cdt_from_alpha(alpha)
    rng = np.random.default_rng(7)
    d = rng.integers(0, 9, size=(3, 400))
    d[:, :40] = 0
    d[0, 40:80] = 0
    for k in range(0, int(15 * math.sqrt(3) / L) + 3, 2):
        G = green.dyad_at(d[0], d[1], d[2], k, L)
        m = masks.mask(d[0], d[1], d[2], k, alpha=alpha)
        # outside the causal shell the exact formulas vanish (rounding level)
        assert np.abs(G[:, ~m]).max(initial=0.0) < 1e-15
        # inside, the diagonal is generically nonzero
        if m.any():
            assert np.all(np.abs(G[:3, m]).max(axis=0) > 0)
        for c, (p, q) in enumerate(green.PAIR):
            if p != q:
                z = (d[p] == 0) | (d[q] == 0)
                assert np.all(G[c, z] == 0.0)


def test_quadrature_converged():
    rng = np.random.default_rng(3)
    d = rng.integers(0, 7, size=(3, 150))
    for alpha in (1, 2, 7):
        L = basis.cdt_from_alpha(alpha)
        for k in range(0, 10):
            a = green.dyad_at(d[0], d[1], d[2], k, L, nq=16)
            b = green.dyad_at(d[0], d[1], d[2], k, L, nq=40)
            assert np.abs(a - b).max() <= 1e-12 * max(np.abs(b).max(), 1e-300)


def test_octant_table_and_reflection():
    g = green.green_octant(5, 4, 3, 0, alpha=4)
    full = green.green_full(g)
    # G(-d) = G(d), G = G^T, and reflection of one axis flips the odd components
    assert np.allclose(full, full[:, :, ::-1, ::-1, ::-1], atol=0)
    assert np.allclose(full, np.transpose(full, (1, 0, 2, 3, 4)), atol=0)
    assert np.array_equal(full[0, 1, :, :, ::-1], -full[0, 1])
    assert np.array_equal(full[0, 0, :, :, ::-1], full[0, 0])
