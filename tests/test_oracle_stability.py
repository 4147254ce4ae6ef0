"""Stability of the MOT march (Eq. 3) under the spline reading of the temporal
basis, and of its regularized form (Sec. II, delta-notation).

The spline weights the constitutive term eps_r J at t_n by (1/2, 1/2) on
(J_n, J_{n-1}), so a current that alternates in sign from step to step is
invisible to that term (its symbol vanishes at z = -1).  The spatial coupling
then decides the sign of the remaining root: on grids of a few voxels the
unregularized march has roots outside the unit circle at dt = 1..4 dt_CFL.
The regularization delta_0 = +delta eps_r, delta_1 = -delta eps_r damps that
pattern.  These tests pin (i) the march against the companion matrix of the
dense Z_k (the same recurrence, assembled from ``operators.z0_dense``), (ii)
the single-voxel recurrence in closed form with delta, and (iii) boundedness
of long regularized marches with the per-alpha delta of the workloads.
"""

import math

import numpy as np
import pytest

import workloads as W
from oracle import basis, green, march, operators

C1 = (3.0 * math.log(2.0 + math.sqrt(3.0)) - math.pi / 2.0) / (2.0 * math.pi)


def _companion(n, alpha, eps_r, delta):
    """Companion matrix of sum_k Z_k J_{n-k} = 0 from the dense Z_k."""
    nl = basis.nlags(*n, alpha=alpha)
    eps = W.eps_uniform(n, eps_r)
    m = 3 * eps.size
    d = np.tile(eps.ravel(), 3)
    Z = []
    for k in range(nl + 1):
        g = green.green_octant(*n, k, alpha=alpha)
        # z0_dense(G, eps) = (1/2 + delta) diag(eps) - diag(eps - 1) G: strip the
        # diagonal and put the weight T(k) + delta_k of lag k back
        Zk = operators.z0_dense(g, eps) - np.diag(0.5 * d)
        Zk += np.diag(d * ({0: 0.5 + delta, 1: 0.5 - delta}.get(k, 0.0)))
        Z.append(Zk)
    Z0i = np.linalg.inv(Z[0])
    C = np.zeros((nl * m, nl * m))
    for k in range(1, nl + 1):
        C[:m, (k - 1) * m:k * m] = -Z0i @ Z[k]
    C[m:, :-m] = np.eye((nl - 1) * m)
    return C, eps, nl


@pytest.mark.slow
@pytest.mark.parametrize("alpha", [1, 2])
def test_companion_roots_and_march_growth(alpha):
    n, eps_r = (4, 4, 4), 12.0
    C, eps, nl = _companion(n, alpha, eps_r, 0.0)
    w = np.linalg.eigvals(C)
    r0 = np.abs(w).max()
    # the unregularized reading has a growing mode on this grid
    assert r0 > 1.02
    if alpha == 2:
        # ... at z = -1: the step-alternating pattern
        assert abs(np.angle(w[np.argmax(np.abs(w))])) == pytest.approx(math.pi, abs=1e-6)
    # the march grows at the rate of the dominant root (power iteration on
    # the homogeneous recurrence, zero excitation after a random start)
    L = basis.cdt_from_alpha(alpha)
    mot = march.Mot(eps, green.green_all(*n, nl, alpha=alpha), L)
    rng = np.random.default_rng(5)
    norms = []
    for s in range(420):
        e = rng.standard_normal((3,) + eps.shape) if s < 2 else np.zeros((3,) + eps.shape)
        J, _ = mot.step(e, tol=1e-13)
        norms.append(np.linalg.norm(J))
    # ratio over many periods of the dominant (possibly complex) pair
    rate = (np.mean(norms[-14:]) / np.mean(norms[-154:-140])) ** (1 / 140)
    assert rate == pytest.approx(r0, rel=2e-3)
    # regularized with delta = 0.1 dt_CFL / dt: every root inside the unit circle
    Cd, _, _ = _companion(n, alpha, eps_r, 0.1 / alpha)
    assert np.abs(np.linalg.eigvals(Cd)).max() < 0.999


@pytest.mark.parametrize("alpha,eps_r,delta", [(2, 4.0, (0.05, -0.05, 0.0)), (16, 4.0, (0.2, -0.2, 0.0)),
                                               (8, 12.0, (0.0125, -0.0125, 0.0)), (2, 12.0, (0.2, -0.4, 0.2))])
def test_single_voxel_recurrence_with_delta(alpha, eps_r, delta):
    # 1 voxel, alpha >= 3/2: z0 J_n = E_n - z1 J_{n-1} - z2 J_{n-2},
    # z0 = e (1/2 + d0) - (e-1)(1/3 - c1/a^2), z1 = e (1/2 + d1) - (e-1)(1/3 + 2 c1/a^2),
    # z2 = e d2 + (e-1) c1/a^2; the DC gain 1/(z0+z1+z2) = 3/(e+2) does not depend on
    # a regularization whose weights sum to zero
    n = (1, 1, 1)
    L = basis.cdt_from_alpha(alpha)
    eps = W.eps_uniform(n, eps_r)
    p = W.pulse(40)
    steps = 60
    nl = basis.nlags(*n, alpha=alpha)
    J, _ = march.run(eps, green.green_all(*n, nl, alpha=alpha), L, p, steps, tol=1e-14, delta=delta)
    e = eps_r
    d0, d1, d2 = delta
    z0 = e * (0.5 + d0) - (e - 1) * (1 / 3 - C1 / alpha ** 2)
    z1 = e * (0.5 + d1) - (e - 1) * (1 / 3 + 2 * C1 / alpha ** 2)
    z2 = e * d2 + (e - 1) * C1 / alpha ** 2
    ref = np.zeros((steps, 3))
    for s in range(steps):
        E = march.dt_einc(p, eps, s * L)[:, 0, 0, 0]
        ref[s] = (E - z1 * (ref[s - 1] if s else 0.0) - z2 * (ref[s - 2] if s > 1 else 0.0)) / z0
    assert np.abs(J[:, :, 0, 0, 0] - ref).max() <= 1e-12 * np.abs(ref).max()
    assert 1.0 / (z0 + z1 + z2) == pytest.approx(3.0 / (e + 2.0), rel=1e-14)
    assert np.all(np.abs(np.roots([z0, z1, z2])) < 1.0)


@pytest.mark.slow
@pytest.mark.parametrize("eps_r", [4.0, 12.0])
@pytest.mark.parametrize("alpha", [1, 2, 4, 8, 16])
def test_regularized_march_bounded_1500_steps(alpha, eps_r):
    # the cube of the time-step study at 8^3, x-polarized pulse along +z,
    # tol 1e-6 (Sec. V-A); delta from the workloads' table
    n = (8, 8, 8)
    L = basis.cdt_from_alpha(alpha)
    nl = basis.nlags(*n, alpha=alpha)
    eps = W.eps_uniform(n, eps_r)
    p = W.pulse(20)
    mot = march.Mot(eps, green.green_all(*n, nl, alpha=alpha), L, delta=W.regularization_for(alpha))
    norms = np.array([np.linalg.norm(mot.step(march.dt_einc(p, eps, s * L), tol=1e-6)[0])
                      for s in range(1500)])
    assert np.all(np.isfinite(norms))
    peak = norms.max()
    # the pulse has passed long before step 1000; what is left is the cube's
    # own ringing, which decays (slowly for eps_r = 12: the second difference
    # adds no damping in the physical band) and never grows back
    assert norms[1000:].max() <= 0.1 * peak
    assert norms[1300:].max() <= norms[1000:1300].max()
