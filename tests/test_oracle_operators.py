"""Pins of the oracle's Z0 forms: dense matrix = direct Toeplitz sum = FFT (Eq. 11/12)."""

import numpy as np
import pytest

import workloads as W
from oracle import basis, green, operators


@pytest.mark.parametrize("n,alpha", [((2, 2, 2), 1), ((3, 2, 4), 4), ((5, 4, 3), 16), ((4, 4, 4), 2)])
def test_dense_direct_fft_agree(n, alpha):
    nx, ny, nz = n
    g0 = green.green_octant(nx, ny, nz, 0, alpha=alpha)
    eps = W.eps_iid(n, 1.5, 6.0, seed=11)
    J = W.random_current(n, seed=12)
    Z = operators.z0_dense(g0, eps)
    y_dense = (Z @ J.ravel()).reshape(J.shape)
    y_dir = operators.z0_apply(g0, eps, J, method="direct")
    y_fft = operators.z0_apply(g0, eps, J, method="fft")
    sc = np.linalg.norm(y_dense)
    assert np.linalg.norm(y_dir - y_dense) <= 1e-13 * sc
    assert np.linalg.norm(y_fft - y_dense) <= 1e-13 * sc


def test_reciprocity_and_real_spectra():
    # with eps = 2 (X = 1, D = I) Z0 = I - G is symmetric: G(m-m')[p,q] = G(m'-m)[q,p]
    n = (4, 3, 5)
    g0 = green.green_octant(*n, 0, alpha=8)
    Z = operators.z0_dense(g0, W.eps_uniform(n, 2.0))
    assert np.abs(Z - Z.T).max() == 0.0
    lam, imag = operators.embed_spectra(g0)
    assert imag <= 1e-12 * np.abs(lam).max()


def test_unit_contrast_gives_half_identity():
    # eps = 1: Z0 = D = I/2 exactly, for any current
    n = (6, 5, 4)
    g0 = green.green_octant(*n, 0, alpha=4)
    J = W.random_current(n, seed=5)
    y = operators.z0_apply(g0, W.eps_uniform(n, 1.0), J)
    assert np.array_equal(y, 0.5 * J)


def test_history_lag_convolution_forms_agree():
    n = (5, 4, 6)
    for k in (1, 2, 5):
        gk = green.green_octant(*n, k, alpha=2)
        J = W.random_current(n, seed=k)
        a = operators.gconv_direct(gk, J)
        b = operators.gconv_fft(gk, J)
        assert np.linalg.norm(a - b) <= 1e-13 * max(np.linalg.norm(a), 1e-300)
