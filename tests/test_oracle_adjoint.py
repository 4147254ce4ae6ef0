"""Pins of the oracle's adjoint march and far-field gradient (oracle/adjoint.py).

Each part is checked against something other than itself: the transposed Z0
against the dense matrix, the far field of one voxel in closed form, the
transposed far field and the adjoint march against dense linear algebra, and
the gradient against central finite differences of the forward march.
"""

import math

import numpy as np
import pytest

import workloads as W
from oracle import adjoint, basis, green, operators

PULSE = {"e": [0.6, 0.8, 0.0], "k": [0.0, 0.0, 1.0], "f0": 0.09, "sigma": 2.5, "t0": 5.0, "amp": 1.0}


def _dense_g(g_oct, shape):
    # z0_dense with eps = 2 is I - G exactly (D = I, X = 1)
    return np.eye(3 * int(np.prod(shape))) - operators.z0_dense(g_oct, W.eps_uniform(shape, 2.0))


@pytest.mark.parametrize("delta", [0.0, 0.07])
@pytest.mark.parametrize("n,alpha", [((3, 2, 2), 1), ((4, 3, 2), 4)])
def test_z0t_is_dense_transpose(n, alpha, delta):
    g0 = green.green_octant(*n, 0, alpha=alpha)
    eps = W.eps_iid(n, 1.5, 6.0, seed=21)
    v = W.random_current(n, seed=22)
    u = W.random_current(n, seed=23)
    Z = operators.z0_dense(g0, eps, delta=delta)
    yt = adjoint.z0t_apply(g0, eps, v, delta=delta)
    assert np.linalg.norm(yt.ravel() - Z.T @ v.ravel()) <= 1e-13 * np.linalg.norm(yt)
    # <Z0^T v, u> = <v, Z0 u>
    lhs = np.sum(yt * u)
    rhs = np.sum(v * operators.z0_apply(g0, eps, u, delta=delta))
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)


def test_dspline_is_derivative_of_spline():
    s = np.linspace(-1.5, 2.5, 4001)
    h = 1e-6
    fd = (basis.spline(s + h) - basis.spline(s - h)) / (2 * h)
    inner = np.all(np.abs(s[:, None] - np.array([-1.0, 0.0, 1.0, 2.0])[None]) > 2 * h, axis=1)
    assert np.abs(fd[inner] - adjoint.dspline(s[inner])).max() < 1e-8
    assert adjoint.dspline(np.array([0.0, 1.0, -1.0, 2.0])).tolist() == [1.0, -1.0, 0.0, 0.0]


def test_farfield_single_voxel_closed_form():
    # centre voxel of a 3x3x3 grid sits at r = 0: e_j = -(P J)/(4 pi dt) T'(j - n0)
    dt, n0 = 0.75, 2
    J = np.zeros((5, 3, 3, 3, 3))
    J[n0, :, 1, 1, 1] = [1.0, 0.0, 0.0]
    rhat = np.array([0.0, 0.6, 0.8])
    e = adjoint.farfield(J, rhat, dt, 0, 6)
    P = np.eye(3) - np.outer(rhat, rhat)
    want = np.zeros((6, 3))
    want[n0] = -(P @ [1.0, 0.0, 0.0]) / (4 * math.pi * dt)        # T'(0) = 1
    want[n0 + 1] = +(P @ [1.0, 0.0, 0.0]) / (4 * math.pi * dt)    # T'(1) = -1
    assert np.abs(e - want).max() <= 1e-15
    # half a step of retardation: voxel at z = +1/2 seen along z with dt = 1
    J2 = np.zeros((4, 3, 2, 1, 1))
    J2[1, 0, 1, 0, 0] = 1.0
    e2 = adjoint.farfield(J2, [0.0, 0.0, 1.0], 1.0, -1, 6)
    want2 = np.zeros((6, 3))
    want2[0 + 1, 0] = -0.5 / (4 * math.pi)    # j = 0: T'(-1/2) = 1/2
    want2[2 + 1, 0] = +0.5 / (4 * math.pi)    # j = 2: T'(3/2) = -1/2
    assert np.abs(e2 - want2).max() <= 1e-15
    # a current along the direction of observation does not radiate there
    J3 = np.zeros((3, 3, 2, 2, 2))
    J3[1, 2] = 1.0
    assert np.abs(adjoint.farfield(J3, [0.0, 0.0, 1.0], 0.5, -3, 9)).max() == 0.0


def test_farfield_adjoint_dot_product():
    rng = np.random.default_rng(31)
    shape, nt, dt = (2, 3, 4), 6, 0.8
    rhat = np.array([1.0, 2.0, 2.0]) / 3.0
    J = rng.standard_normal((nt, 3) + shape)
    j0, nj = -6, nt + 12
    w = rng.standard_normal((nj, 3))
    lhs = np.sum(adjoint.farfield(J, rhat, dt, j0, nj) * w)
    rhs = np.sum(J * adjoint.farfield_adjoint(w, rhat, dt, j0, nt, shape))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


@pytest.mark.parametrize("delta", [0.0, 0.07, (0.1, -0.2, 0.1)])
def test_adjoint_march_solves_transposed_spacetime_system(delta):
    n, alpha, nt = (2, 2, 2), 1, 7
    nl = basis.nlags(*n, alpha=alpha)
    greens = green.green_all(*n, nl, alpha=alpha)
    eps = W.eps_iid(n, 2.0, 5.0, seed=41)
    shape = eps.shape
    m3 = 3 * eps.size
    # local weights of Z_0, Z_1, Z_2: the spline's T(0) = T(1) = 1/2, T(2) = 0,
    # plus the regularization's (d, -d, 0) or (d_0, d_1, d_2)
    d = (delta, -delta, 0.0) if np.ndim(delta) == 0 else delta
    Tk = [0.5 + d[0], 0.5 + d[1], d[2]] + [0.0] * (nl - 2)
    d = np.tile(eps.ravel(), 3)
    x = d - 1.0
    Zk = [Tk[k] * np.diag(d) - x[:, None] * _dense_g(greens[k], n) for k in range(nl + 1)]
    A = np.zeros((nt * m3, nt * m3))
    for r in range(nt):
        for k in range(min(r, nl) + 1):
            A[r * m3:(r + 1) * m3, (r - k) * m3:(r - k + 1) * m3] = Zk[k]
    g = np.random.default_rng(42).standard_normal((nt, 3) + shape)
    lam_dense = np.linalg.solve(A.T, g.ravel()).reshape(g.shape)
    lam = adjoint.adjoint_march(eps, greens, g, tol=1e-14, delta=delta)
    assert np.linalg.norm(lam - lam_dense) <= 1e-10 * np.linalg.norm(lam_dense)
    # the forward march solves the same (untransposed) block-Toeplitz system
    from oracle import march
    J_dense = np.linalg.solve(A, g.ravel()).reshape(g.shape)
    mot = march.Mot(eps, greens, basis.cdt_from_alpha(alpha), delta=delta)
    J = np.array([mot.step(g[r], tol=1e-14)[0] for r in range(nt)])
    assert np.linalg.norm(J - J_dense) <= 1e-10 * np.linalg.norm(J_dense)


@pytest.mark.parametrize("delta", [0.0, 0.05, (0.1, -0.2, 0.1)])
def test_gradient_matches_central_differences(delta):
    n, alpha, nt = (3, 2, 2), 2, 12
    dt = basis.cdt_from_alpha(alpha)
    nl = basis.nlags(*n, alpha=alpha)
    greens = green.green_all(*n, nl, alpha=alpha)
    eps = W.eps_iid(n, 2.0, 5.0, seed=51)
    eps[0, 1, 2] = 1.0   # one air voxel: the gradient there is that of adding material
    rhat = np.array([0.48, -0.6, 0.64])
    j0, nj = -8, nt + 16
    W0, grad = adjoint.gradient(eps, greens, dt, PULSE, nt, rhat, j0, nj, delta=delta)
    assert W0 > 0.0
    assert abs(W0 - adjoint.energy_of(eps, greens, dt, PULSE, nt, rhat, j0, nj, delta=delta)) <= 1e-12 * W0
    h = 1e-4
    fd = np.zeros_like(eps)
    for idx in np.ndindex(eps.shape):
        ep, em = eps.copy(), eps.copy()
        ep[idx] += h
        em[idx] -= h
        fd[idx] = (adjoint.energy_of(ep, greens, dt, PULSE, nt, rhat, j0, nj, delta=delta)
                   - adjoint.energy_of(em, greens, dt, PULSE, nt, rhat, j0, nj, delta=delta)) / (2 * h)
    assert np.abs(fd - grad).max() <= 1e-6 * np.abs(grad).max()
    assert np.abs(grad).max() > 0.0
