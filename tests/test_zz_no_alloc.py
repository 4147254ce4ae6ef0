"""The allocation-free far field (mot_farfield_static) against mot_farfield:
the same samples and energy, bit for bit (the same kernels and partial
layout), over two calls in a row, the second with fewer samples and steps;
and its limit on the sample count."""

import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def test_farfield_static_matches_farfield(gpu_lib):
    import torch
    n, alpha = (16, 12, 8), 4
    eps = W.eps_iid(n, 1.5, 6.0, seed=71)
    c = gpu_lib.Context(*n, alpha=alpha, precision="f64")
    c.set_material(torch.from_numpy(eps.ravel()).cuda())
    c.build_green_spectra()
    N3 = 3 * int(np.prod(n))
    rng = np.random.default_rng(72)
    for nsteps, j0, nj, rhat in ((40, -20, 700, (0.3, -0.5, 0.81)), (9, 3, 17, (0.0, 0.0, 1.0))):
        J = torch.from_numpy(rng.standard_normal(nsteps * N3)).cuda()
        e_ref = torch.empty(3 * nj, dtype=torch.float64, device="cuda")
        e_st = torch.full((3 * nj,), float("nan"), dtype=torch.float64, device="cuda")
        w_ref = torch.empty(1, dtype=torch.float64, device="cuda")
        w_st = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        c.farfield(J, rhat, j0, nj, e_ref, w_ref)
        c.farfield_static(J, rhat, j0, nj, e_st, w_st)
        torch.cuda.synchronize()
        assert float(torch.abs(e_ref).max()) > 0.0
        assert torch.equal(e_st, e_ref) and torch.equal(w_st, w_ref)
    # at most 1024 samples
    e = torch.empty(3 * 1025, dtype=torch.float64, device="cuda")
    with pytest.raises(gpu_lib.MotError) as ei:
        c.farfield_static(J, (1.0, 0.0, 0.0), 0, 1025, e)
    assert ei.value.status == gpu_lib.MOT_EINVAL
    c.close()
