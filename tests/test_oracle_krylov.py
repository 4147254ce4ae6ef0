"""Pins of the oracle's TFQMR: exact solves and agreement with SciPy's routine."""

import numpy as np
import pytest
from scipy.sparse.linalg import tfqmr as scipy_tfqmr

from oracle import krylov


def _system(n, seed, shift=3.0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) / np.sqrt(n) + shift * np.eye(n)
    b = rng.standard_normal(n)
    return A, b


@pytest.mark.parametrize("n,seed", [(10, 0), (60, 1), (200, 2)])
def test_matches_dense_solve(n, seed):
    A, b = _system(n, seed)
    r = krylov.tfqmr(lambda v: A @ v, b, tol=1e-12, max_iter=500)
    x = np.linalg.solve(A, b)
    assert r.converged
    assert np.linalg.norm(r.x - x) <= 1e-10 * np.linalg.cond(A) * np.linalg.norm(x)
    assert np.linalg.norm(b - A @ r.x) <= 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("seed", range(5))
def test_iteration_count_vs_scipy(seed):
    A, b = _system(150, seed, shift=1.5)
    r = krylov.tfqmr(lambda v: A @ v, b, tol=1e-6)
    counted = []
    x, info = scipy_tfqmr(A, b, rtol=1e-6, atol=0.0, callback=lambda xk: counted.append(1))
    assert info == 0 and r.converged
    # SciPy's callback fires once per half step
    assert abs(2 * r.iterations - len(counted)) <= 4
    assert np.linalg.norm(r.x - x) <= 5e-6 * np.linalg.norm(x)


def test_zero_rhs_and_exact_start():
    A, _ = _system(20, 3)
    r = krylov.tfqmr(lambda v: A @ v, np.zeros(20))
    assert r.iterations == 0 and r.matvecs == 0 and np.all(r.x == 0)


def test_identity_one_iteration():
    b = np.arange(1.0, 9.0)
    r = krylov.tfqmr(lambda v: 2.0 * v, b, tol=1e-14)
    assert r.iterations == 1 and np.allclose(r.x, b / 2, rtol=1e-15)


def test_breakdown_reported():
    # a skew-symmetric system: sigma = v . r~ = b^T A b = 0 at the first
    # iteration, which TFQMR cannot pass (the solver's breakdown exit)
    A = np.array([[0.0, 1.0], [-1.0, 0.0]])
    res = krylov.tfqmr(lambda v: A @ v, np.array([1.0, 0.0]), tol=1e-12)
    assert res.breakdown and not res.converged
