"""Tile-shape variants of the FFT passes and the autotuner (HIP library
through its C ABI).

Every variant computes the same pencil transforms, the same spectral multiply
and the same epilogue in the same order, so products and history updates
must agree bit for bit across variants; the FP64 products are also held to
the oracle (relative L2 <= 1e-10, as in the other parity tests).
"""

import math

import numpy as np
import pytest

import workloads as W
from oracle import green, operators

pytestmark = pytest.mark.gpu

KNOBS = ("x", "y", "z_history", "z_fused")
# grids whose tiles end in ragged tails, with tile widths that differ between variants
# (96, 48, 4): the 96-point plan (radices 8 and 12) in the x and y passes
GRIDS = [((40, 12, 6), 2), ((80, 24, 10), 4), ((48, 40, 24), 2), ((16, 16, 48), 4), ((96, 48, 4), 2)]


def _t(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return (t.to(dtype) if dtype is not None else t).cuda()


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def _eps(n, seed=31):
    e = W.eps_iid(n, 1.5, 6.0, seed)
    e.ravel()[::7] = 1.0
    return e


def _ctx(native, n, alpha, prec, eps):
    c = native.Context(*n, alpha=alpha, precision=prec)
    c.set_material(_t(eps.ravel()))
    c.build_green_spectra()
    return c


def _setting(on):
    """8 variants with the knobs named in `on` set to 1, in both precisions."""
    return [1 if k in on else 0 for _ in range(2) for k in KNOBS]


def _products(c, J):
    import torch
    y64 = torch.empty(J.size, dtype=torch.float64, device="cuda")
    y32 = torch.empty(J.size, dtype=torch.float32, device="cuda")
    yr = torch.empty(J.size, dtype=torch.float64, device="cuda")
    c.z0_matvec(_t(J.ravel()), y64, "f64")
    c.z0_matvec(_t(J.ravel(), torch.float32), y32, "f32")
    c.z0_matvec(_t(J.ravel()), yr, "f32_refined")
    torch.cuda.synchronize()
    return y64, y32, yr


@pytest.mark.parametrize("n,alpha", GRIDS)
def test_variants_give_identical_products(gpu_lib, n, alpha):
    import torch
    eps = _eps(n)
    c = _ctx(gpu_lib, n, alpha, "f32_refined", eps)
    assert c.variants() == {p: {k: 0 for k in KNOBS} for p in ("f32", "f64")}
    J = W.random_current(n, seed=32)
    base = _products(c, J)
    ref = operators.z0_apply(green.green_octant(*n, 0, alpha=alpha), eps, J)
    assert np.linalg.norm(_np(base[0]).reshape(J.shape) - ref) <= 1e-10 * np.linalg.norm(ref)
    for on in (("x",), ("y",), ("z_fused",), KNOBS, ()):
        c.set_variants(_setting(on))
        got = _products(c, J)
        for a, b in zip(got, base):
            assert torch.equal(a, b), on
    # a dict round trip
    v = c.variants()
    c.set_variants(v)
    assert c.variants() == v


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_variants_give_identical_history(gpu_lib, prec):
    import torch
    n, alpha = (40, 12, 6), 2
    eps = _eps(n, 33)
    cs = [_ctx(gpu_lib, n, alpha, prec, eps) for _ in range(2)]
    cs[1].set_variants(_setting(KNOBS))
    nl = cs[0].info()["nlags"]
    out = [torch.empty(3 * math.prod(n), dtype=torch.float64, device="cuda") for _ in range(2)]
    for c in cs:
        c.reset()
    for s in range(nl + 3):
        J = _t(W.random_current(n, seed=200 + s).ravel())
        for c, o in zip(cs, out):
            c.history_update(J)
            c.history_rhs(o)
        torch.cuda.synchronize()
        assert torch.equal(out[0], out[1]), s


def test_autotune(gpu_lib):
    import torch
    n, alpha = (48, 40, 24), 2
    eps = _eps(n, 34)
    c = _ctx(gpu_lib, n, alpha, "f32_refined", eps)
    J = W.random_current(n, seed=35)
    base = _products(c, J)
    ms = c.autotune(reps=5)
    for p in ("f32", "f64"):
        for k in KNOBS:
            if p == "f64" and k == "z_history":
                assert ms[p][k] is None    # the history of an FP32-refined context runs in FP32
            else:
                assert ms[p][k] is not None and all(t > 0.0 for t in ms[p][k]), (p, k)
    chosen = c.variants()
    assert all(v in (0, 1) for p in chosen.values() for v in p.values())
    got = _products(c, J)
    for a, b in zip(got, base):
        assert torch.equal(a, b)
    # the march starts from a clean history after tuning
    out = torch.empty(3 * math.prod(n), dtype=torch.float64, device="cuda")
    c.history_gfield(out)
    assert float(torch.abs(out).max()) == 0.0
    # tuning needs step 0
    c.history_update(_t(J.ravel()))
    with pytest.raises(gpu_lib.MotError):
        c.autotune(reps=1)
    c.reset()
    c.autotune(reps=1)


def test_variant_change_drops_graphs(gpu_lib):
    # a graph-replaying context whose variants change mid-march steps like a
    # context that launches stream by stream with the same changes
    import torch
    n, alpha = (16, 6, 4), 4
    eps = _eps(n, 36)
    cs = [_ctx(gpu_lib, n, alpha, "f32_refined", eps) for _ in range(2)]
    for c in cs:
        c.reset()
    cs[1].set_graphs(True)
    p = W.pulse(20)
    N = int(np.prod(n))
    e = torch.empty(3 * N, dtype=torch.float64, device="cuda")
    J = [torch.empty(3 * N, dtype=torch.float64, device="cuda") for _ in range(2)]
    for k in range(16):
        if k == 8:
            for c in cs:
                c.set_variants(_setting(KNOBS))
        cs[0].excitation(p, (60 + k) * alpha / math.sqrt(3.0), e)
        st = [c.step(e, Jc, tol=1e-6)[1] for c, Jc in zip(cs, J)]
        assert st[0]["iters"] == st[1]["iters"]
        assert torch.equal(J[0], J[1])


def test_invalid_variants(gpu_lib):
    c = gpu_lib.Context(8, 4, 4, alpha=2, precision="f64")
    with pytest.raises(gpu_lib.MotError):
        c.set_variants([0, 0, 0, 2, 0, 0, 0, 0])
    with pytest.raises(ValueError):
        c.set_variants([0, 0, 0])
    with pytest.raises(gpu_lib.MotError):
        c.autotune()                 # no material and spectra yet
