"""Pins of the oracle's MOT march (Eq. 3) and excitation (Eq. 7, Eq. 8)."""

import math

import numpy as np
import pytest

import workloads as W
from oracle import basis, green, march

C1 = (3.0 * math.log(2.0 + math.sqrt(3.0)) - math.pi / 2.0) / (2.0 * math.pi)


def _greens(n, alpha):
    nl = basis.nlags(*n, alpha=alpha)
    return green.green_all(*n, nl, alpha=alpha)


def test_unit_contrast_gives_zero_current():
    # eps_r = 1: the right-hand side vanishes and every J_n is exactly zero
    n, alpha = (4, 3, 5), 4
    eps = W.eps_uniform(n, 1.0)
    J, iters = march.run(eps, _greens(n, alpha), basis.cdt_from_alpha(alpha), W.pulse(20), 12)
    assert np.all(J == 0.0) and iters == [0] * 12


@pytest.mark.parametrize("alpha,eps_r", [(2, 4.0), (16, 4.0), (8, 12.0)])
def test_single_voxel_recurrence(alpha, eps_r):
    # 1 voxel, alpha >= 3/2: z0 J_n = E_n - z1 J_{n-1} - z2 J_{n-2} with
    # z0 = e/2 - (e-1)(1/3 - c1/a^2), z1 = e/2 - (e-1)(1/3 + 2 c1/a^2), z2 = (e-1) c1/a^2
    n = (1, 1, 1)
    L = basis.cdt_from_alpha(alpha)
    eps = W.eps_uniform(n, eps_r)
    p = W.pulse(40)
    steps = 80
    J, _ = march.run(eps, _greens(n, alpha), L, p, steps, tol=1e-14)
    e = eps_r
    z0 = e / 2 - (e - 1) * (1 / 3 - C1 / alpha ** 2)
    z1 = e / 2 - (e - 1) * (1 / 3 + 2 * C1 / alpha ** 2)
    z2 = (e - 1) * C1 / alpha ** 2
    ref = np.zeros((steps, 3))
    for s in range(steps):
        E = march.dt_einc(p, eps, s * L)[:, 0, 0, 0]
        prev1 = ref[s - 1] if s >= 1 else 0.0
        prev2 = ref[s - 2] if s >= 2 else 0.0
        ref[s] = (E - z1 * prev1 - z2 * prev2) / z0
    got = J[:, :, 0, 0, 0]
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    # the recurrence is damped: both roots inside the unit circle
    roots = np.roots([z0, z1, z2])
    assert np.all(np.abs(roots) < 1.0)
    # DC gain 1/(z0+z1+z2) = 3/(e+2): the Clausius-Mossotti factor
    assert 1.0 / (z0 + z1 + z2) == pytest.approx(3.0 / (e + 2.0), rel=1e-14)


def test_excitation_plane_wave():
    # Eq. 7/8: tau = t - t0 - k.(r - r_c); x-polarized along +z, peak-normalized
    n = (4, 5, 6)
    p = W.pulse(20)
    eps = W.eps_iid(n, 2.0, 5.0, seed=1)
    t = 130.0
    E = march.dt_einc(p, eps, t)
    assert np.all(E[1] == 0.0) and np.all(E[2] == 0.0)
    # finite-difference check of the time derivative at one voxel
    z, y, x = 3, 1, 2
    zc = z + 0.5 - n[2] / 2.0

    def g(tt):
        tau = tt - p["t0"] - zc
        return math.exp(-tau * tau / (2 * p["sigma"] ** 2)) * math.cos(2 * math.pi * p["f0"] * tau)
    h = 1e-4
    fd = (g(t + h) - g(t - h)) / (2 * h)
    assert E[0, z, y, x] == pytest.approx((eps[z, y, x] - 1.0) * fd, rel=1e-7)
    # pulse recipe: -20 dB full width of 0.8 f0, t0 = 6 sigma
    sf = 1.0 / (2 * math.pi * p["sigma"])
    assert math.exp(-(0.4 * p["f0"]) ** 2 / (2 * sf * sf)) == pytest.approx(0.1, rel=1e-12)
    assert p["t0"] == pytest.approx(6 * p["sigma"])


def test_shift_invariance_bitwise():
    # delaying the excitation by m steps delays the whole response by m steps, bitwise
    n, alpha, m = (3, 4, 2), 4, 3
    L = basis.cdt_from_alpha(alpha)
    G = _greens(n, alpha)
    eps = W.eps_iid(n, 2.0, 6.0, seed=3)
    p = W.pulse(20)
    Es = [march.dt_einc(p, eps, 100.0 + s * L) for s in range(15)]
    a = march.Mot(eps, G, L)
    b = march.Mot(eps, G, L)
    Ja = [a.step(E)[0] for E in Es]
    Jb = [b.step(np.zeros_like(Es[0]))[0] for _ in range(m)] + [b.step(E)[0] for E in Es[:-m]]
    assert all(np.all(j == 0) for j in Jb[:m])
    for s in range(len(Es) - m):
        assert np.array_equal(Ja[s], Jb[s + m])


def test_linearity():
    n, alpha = (4, 3, 3), 8
    L = basis.cdt_from_alpha(alpha)
    G = _greens(n, alpha)
    eps = W.eps_iid(n, 2.0, 6.0, seed=4)
    p1 = W.pulse(20)
    p2 = W.pulse(30, k_hat=(1.0, 0.0, 0.0), e_hat=(0.0, 0.6, 0.8))
    runs = []
    for fn in (lambda t: march.dt_einc(p1, eps, t), lambda t: march.dt_einc(p2, eps, t),
               lambda t: 2.0 * march.dt_einc(p1, eps, t) - 3.0 * march.dt_einc(p2, eps, t)):
        mot = march.Mot(eps, G, L)
        runs.append(np.array([mot.step(fn(s * L), tol=1e-12)[0] for s in range(40)]))
    comb = 2.0 * runs[0] - 3.0 * runs[1]
    assert np.abs(runs[2] - comb).max() <= 1e-9 * np.abs(comb).max()


@pytest.mark.slow
def test_time_step_convergence():
    # Sec. III-B: responses at dt = 8 and 16 dt_CFL follow the finer-step reference.
    # Compare J(t) = (J_n + J_{n-1})/2 (the spline value at t_n) on a common time grid.
    n = (6, 6, 6)
    eps = W.eps_uniform(n, 4.0)
    p = W.pulse(40)
    T = 16 * 24
    traces = {}
    for alpha in (2, 4, 8, 16):
        L = basis.cdt_from_alpha(alpha)
        J, _ = march.run(eps, _greens(n, alpha), L, p, T // alpha + 1, tol=1e-10,
                         probe=(0, 3, 3, 3))
        Jt = 0.5 * (J + np.concatenate([[0.0], J[:-1]]))
        traces[alpha] = Jt[::16 // alpha][: T // 16 + 1]
    ref = traces[2]
    err = {a: np.abs(traces[a] - ref).max() / np.abs(ref).max() for a in (4, 8, 16)}
    assert err[4] < err[8] < err[16]
    assert err[8] < 0.01 and err[16] < 0.05
