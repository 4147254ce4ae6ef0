"""Parity of the HIP library (through its C ABI) with the FP64 CPU oracle.

Tolerances (from the arithmetic of each comparison):
  * integer work (masks, lag counts, support of G_k): bit-exact;
  * G_k tables: |lib - oracle| <= 1e-11 max|G_k| (two independent FP64
    quadratures of the same integrals, each accurate to ~1e-13), widened by
    (|extent|/20)^2 on grids wider than 20 voxels (cancellation at far offsets);
  * FP64 products: relative L2 <= 1e-10;
  * FP32 products: relative L2 <= 1e-5 (FP32 FFT rounding over ~25 stages, with margin);
  * marched fields: max_n ||J_n - J_n^ref|| / max_n ||J_n^ref|| <= 1e-4.
"""

import functools
import math

import numpy as np
import pytest

import workloads as W
from oracle import basis, green, march, masks, operators

pytestmark = pytest.mark.gpu

GRIDS = [((8, 8, 8), 4), ((16, 16, 16), 1), ((24, 20, 12), 8), ((16, 6, 4), 16), ((40, 12, 6), 2),
         ((48, 40, 24), 2), ((80, 24, 10), 4)]


@functools.lru_cache(maxsize=None)
def og(n, k, alpha):
    return green.green_octant(*n, k, alpha=alpha)


def _t(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def _eps(n, seed=21):
    e = W.eps_iid(n, 1.5, 6.0, seed)
    e.ravel()[::7] = 1.0        # some background voxels
    return e


def _ctx(native, n, alpha, prec="f64", eps=None, **kw):
    c = native.Context(*n, alpha=alpha, precision=prec, **kw)
    c.set_material(_t((_eps(n) if eps is None else eps).ravel()))
    c.build_green_spectra()
    return c


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


@pytest.mark.parametrize("n,alpha", GRIDS)
def test_green_tables(gpu_lib, n, alpha):
    import torch
    c = _ctx(gpu_lib, n, alpha)
    nl = c.info()["nlags"]
    assert nl == basis.nlags(*n, alpha=alpha)
    out = torch.empty(6 * math.prod(n), dtype=torch.float64, device="cuda")
    for k in sorted({0, 1, 2, 3, nl // 2, nl}):
        c.green_table(k, out)
        lib = _np(out).reshape(6, n[2], n[1], n[0])
        ref = og(n, k, alpha)
        # support (causal mask and symmetry zeros) is bit-exact
        assert np.array_equal(lib != 0.0, ref != 0.0), k
        sc = max(np.abs(ref).max(), 1e-300)
        # far offsets cancel face contributions of size ~|d| times the entry
        # in both quadratures; allow for it beyond 20 voxels
        far = max(1.0, (math.sqrt(sum(x * x for x in n)) / 20.0) ** 2)
        assert np.abs(lib - ref).max() <= 1e-11 * far * sc, (k, np.abs(lib - ref).max() / sc)


@pytest.mark.parametrize("n,alpha", GRIDS)
def test_z0_matvec(gpu_lib, n, alpha):
    import torch
    eps = _eps(n)
    c = _ctx(gpu_lib, n, alpha, "f32_refined", eps)
    assert c.build_green_spectra() <= 1e-12
    J = W.random_current(n, seed=5)
    ref = operators.z0_apply(og(n, 0, alpha), eps, J)
    y = torch.empty(J.size, dtype=torch.float64, device="cuda")
    c.z0_matvec(_t(J.ravel()), y, "f64")
    assert _rel(_np(y).reshape(J.shape), ref) <= 1e-10
    c.z0_matvec(_t(J.ravel()), y, "f32_refined")
    assert _rel(_np(y).reshape(J.shape), ref) <= 1e-5
    y32 = torch.empty(J.size, dtype=torch.float32, device="cuda")
    c.z0_matvec(_t(J.ravel(), torch.float32), y32, "f32")
    assert _rel(_np(y32).reshape(J.shape), ref) <= 1e-5


def test_z0_matvec_direct_sum_and_dense(gpu_lib):
    # tiny grid: library vs the dense matrix and the direct Toeplitz sum
    import torch
    n, alpha = (8, 4, 4), 8
    eps = _eps(n, 3)
    c = _ctx(gpu_lib, n, alpha, "f64", eps)
    J = W.random_current(n, seed=9)
    Z = operators.z0_dense(og(n, 0, alpha), eps)
    ref = (Z @ J.ravel()).reshape(J.shape)
    y = torch.empty(J.size, dtype=torch.float64, device="cuda")
    c.z0_matvec(_t(J.ravel()), y, "f64")
    assert _rel(_np(y).reshape(J.shape), ref) <= 1e-10
    assert _rel(operators.z0_apply(og(n, 0, alpha), eps, J, method="direct"), ref) <= 1e-13


@pytest.mark.parametrize("prec", ["f64", "f32_refined"])
def test_history_lag_products(gpu_lib, prec):
    import torch
    n, alpha = (16, 6, 4), 2
    eps = _eps(n)
    c = _ctx(gpu_lib, n, alpha, prec, eps)
    nl = c.info()["nlags"]
    J = W.random_current(n, seed=2)
    y = torch.empty(J.size, dtype=torch.float64, device="cuda")
    tol = 1e-10 if prec == "f64" else 1e-5
    for k in (1, 2, 3, nl // 2, nl):
        ref = operators.gconv_fft(og(n, k, alpha), J)
        if not np.abs(ref).max() > 0:
            continue
        c.gk_matvec(k, _t(J.ravel()), y, "f64" if prec == "f64" else "f32_refined")
        assert _rel(_np(y).reshape(J.shape), ref) <= tol, k


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_history_update(gpu_lib, prec):
    # h_{n+1} = -(eps/2) J_n + (eps-1) sum_{k>=1} G_k * J_{n+1-k} after each push
    import torch
    n, alpha = (8, 6, 4), 2
    eps = _eps(n, 4)
    c = _ctx(gpu_lib, n, alpha, prec, eps)
    nl = c.info()["nlags"]
    Gs = [og(n, k, alpha) for k in range(nl + 1)]
    hist = []
    out = torch.empty(3 * math.prod(n), dtype=torch.float64, device="cuda")
    tol = 1e-10 if prec == "f64" else 1e-5
    for s in range(nl + 3):  # wraps the ring
        J = W.random_current(n, seed=100 + s)
        hist.insert(0, J)
        c.history_update(_t(J.ravel()))
        c.history_rhs(out)
        acc = np.zeros_like(J)
        for k in range(1, nl + 1):
            if k - 1 < len(hist):
                acc += operators.gconv_fft(Gs[k], hist[k - 1])
        ref = -0.5 * eps[None] * J + (eps[None] - 1.0) * acc
        assert _rel(_np(out).reshape(J.shape), ref) <= tol, s
    assert c.info()["steps"] == nl + 3
    # nl + 3 = 14 pushes span two history blocks of B = 8 (and the second level
    # of each, at its fifth step)
    assert c.info()["history_block"] == 8
    c.reset()
    c.history_rhs(out)
    assert not _np(out).any()


def test_excitation(gpu_lib):
    import torch
    n = (12, 10, 6)
    eps = _eps(n)
    c = _ctx(gpu_lib, n, 4, "f64", eps)
    out = torch.empty(3 * math.prod(n), dtype=torch.float64, device="cuda")
    for p in (W.pulse(20), W.pulse(40, k_hat=(0.6, 0.0, 0.8), e_hat=(0.0, 1.0, 0.0), amp=0.3)):
        for t in (0.0, 100.0, 143.5, 400.0):
            c.excitation(p, t, out)
            ref = march.dt_einc(p, eps, t)
            got = _np(out).reshape(ref.shape)
            assert np.abs(got - ref).max() <= 1e-13 * max(np.abs(ref).max(), 1e-300)


def _march_gpu(native, n, alpha, prec, eps, p, steps, tol=1e-6):
    import torch
    c = _ctx(native, n, alpha, prec, eps)
    L = basis.cdt_from_alpha(alpha)
    N3 = 3 * math.prod(n)
    einc = torch.empty(N3, dtype=torch.float64, device="cuda")
    J = torch.empty(N3, dtype=torch.float64, device="cuda")
    out, iters = [], []
    for s in range(steps):
        c.excitation(p, s * L, einc)
        _, st = c.step(einc, J, tol=tol)
        out.append(_np(J).reshape(3, n[2], n[1], n[0]))
        iters.append(st["iters"])
    return np.array(out), iters


def _field_err(a, b):
    num = max(np.linalg.norm(a[s] - b[s]) for s in range(len(b)))
    return num / max(np.linalg.norm(b[s]) for s in range(len(b)))


@pytest.mark.parametrize("prec", ["f64", "f32_refined"])
def test_march_cube16_alpha1(gpu_lib, prec):
    # 16^3 homogeneous cube, eps_r = 4, dt = dt_CFL, 200 steps, h = lambda_min/20
    w = W.CUBE16
    eps = w.eps()
    p = W.pulse(w.ppw)
    L = basis.cdt_from_alpha(w.alpha)
    Gs = [og(w.n, k, w.alpha) for k in range(basis.nlags(*w.n, alpha=w.alpha) + 1)]
    ref, ref_it = march.run(eps, Gs, L, p, w.steps, tol=1e-6)
    got, it = _march_gpu(gpu_lib, w.n, w.alpha, prec, eps, p, w.steps)
    assert _field_err(got, ref) <= 1e-4
    assert max(abs(a - b) for a, b in zip(it, ref_it)) <= 2 or prec != "f64"


@pytest.mark.parametrize("prec", ["f64", "f32_refined"])
def test_march_alpha8_inhomogeneous(gpu_lib, prec):
    n, alpha = (24, 20, 12), 8
    eps = W.eps_iid(n, 2.0, 6.0, 2)
    p = W.pulse(20)
    L = basis.cdt_from_alpha(alpha)
    Gs = [og(n, k, alpha) for k in range(basis.nlags(*n, alpha=alpha) + 1)]
    steps = 45
    ref, _ = march.run(eps, Gs, L, p, steps, tol=1e-6)
    got, it = _march_gpu(gpu_lib, n, alpha, prec, eps, p, steps)
    assert _field_err(got, ref) <= 1e-4
    assert max(it) >= 3


def test_edge_cases(gpu_lib):
    import torch
    native = gpu_lib
    n, alpha = (8, 6, 4), 4
    N3 = 3 * math.prod(n)
    # eps = 1 everywhere: no current, bitwise, and zero iterations
    c = _ctx(native, n, alpha, "f64", W.eps_uniform(n, 1.0))
    einc = torch.empty(N3, dtype=torch.float64, device="cuda")
    J = torch.full((N3,), 7.0, dtype=torch.float64, device="cuda")
    c.excitation(W.pulse(20), 140.0, einc)
    _, st = c.step(einc, J)
    assert st["iters"] == 0 and not _np(J).any()
    # zero right-hand side at the first step
    c2 = _ctx(native, n, alpha, "f32_refined")
    einc.zero_()
    _, st = c2.step(einc, J)
    assert st["iters"] == 0 and not _np(J).any()
    # max_iter = 1 with an unreachable tolerance: MOT_ENOCONV, history still advances
    c.set_material(_t(_eps(n).ravel()))
    c.excitation(W.pulse(20), 140.0, einc)
    rc, st = c.step(einc, J, tol=1e-14, max_iter=1, allow=(native.MOT_ENOCONV,))
    assert rc == native.MOT_ENOCONV and st["iters"] == 1
    assert c.info()["steps"] == 2
    # NaN in the excitation: MOT_ENONFINITE
    einc[5] = float("nan")
    rc, _ = c.step(einc, J, allow=(native.MOT_ENONFINITE,))
    assert rc == native.MOT_ENONFINITE
    # misuse is rejected before any work
    with pytest.raises(native.MotError):
        c.z0_matvec(J, J)
    c3 = native.Context(*n, alpha=alpha)
    with pytest.raises(native.MotError) as e:
        c3.step(einc, J)
    assert e.value.status == native.MOT_ESTATE


def test_determinism(gpu_lib):
    import torch
    n, alpha = (24, 20, 12), 8
    eps = _eps(n)
    outs = []
    for _ in range(2):
        c = _ctx(gpu_lib, n, alpha, "f32_refined", eps)
        N3 = 3 * math.prod(n)
        einc = torch.empty(N3, dtype=torch.float64, device="cuda")
        J = torch.empty(N3, dtype=torch.float64, device="cuda")
        L = basis.cdt_from_alpha(alpha)
        seq = []
        for s in range(12, 16):
            c.excitation(W.pulse(20), s * L, einc)
            c.step(einc, J)
            seq.append(_np(J))
        y = torch.empty(N3, dtype=torch.float64, device="cuda")
        c.z0_matvec(J, y, "f64")
        seq.append(_np(y))
        outs.append(seq)
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def _octant_blocks(goct):
    """Signed offsets (dz, dy, dx) of the nonzero entries of an octant table and
    their 3x3 blocks (reflection signs s_p s_q on the off-diagonal entries)."""
    offs, blks = [], []
    for dz, dy, dx in np.argwhere(np.abs(goct).sum(axis=0) > 0):
        v = goct[:, dz, dy, dx]
        for sz in ((1, -1) if dz else (1,)):
            for sy in ((1, -1) if dy else (1,)):
                for sx in ((1, -1) if dx else (1,)):
                    sg = (sx, sy, sz)
                    B = np.zeros((3, 3))
                    for cc, (pp, qq) in enumerate(green.PAIR):
                        B[pp, qq] = B[qq, pp] = v[cc] * (sg[pp] * sg[qq] if pp != qq else 1.0)
                    offs.append((sz * dz, sy * dy, sx * dx))
                    blks.append(B)
    return np.array(offs), np.array(blks)


def _direct_at(goct, J, samples):
    """(G J) at the sampled voxels (z, y, x) by the direct Toeplitz sum; (len, 3)."""
    offs, blks = _octant_blocks(goct)
    _, nz, ny, nx = J.shape
    out = []
    for (z, yy, x) in samples:
        src = np.array([z, yy, x]) - offs
        ok = np.all((src >= 0) & (src < np.array([nz, ny, nx])), axis=1)
        s_ = src[ok]
        out.append(np.einsum("mpq,qm->p", blks[ok], J[:, s_[:, 0], s_[:, 1], s_[:, 2]]))
    return np.array(out)


def _samples(n, seed, count=60):
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    out = [(0, 0, 0), (nz - 1, ny - 1, nx - 1), (nz // 2, ny // 8, nx // 8), (nz // 2, ny // 2, nx // 2 + 1)]
    return out + [tuple(int(rng.integers(0, s_)) for s_ in (nz, ny, nx)) for _ in range(count)]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_z0_matvec_pillars_full_size(gpu_lib, dtype):
    # 8x8 pillar array, 320x320x48 voxels (14.7M unknowns), dt = 16 dt_CFL: the
    # benchmarked size; checked on sampled voxels against the oracle's direct sum.
    import torch
    w = W.PILLARS
    n, alpha = w.n, w.alpha
    eps = w.eps()
    c = _ctx(gpu_lib, n, alpha, "f32_refined", eps, nlags=1)
    J = W.random_current(n, seed=44)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    y = torch.empty(J.size, dtype=tdt, device="cuda")
    c.z0_matvec(_t(J.ravel(), tdt), y, dtype)
    got = _np(y).reshape(J.shape)
    Jin = J.astype(np.float32).astype(np.float64) if dtype == "f32" else J
    samples = [(0, 0, 0), (n[2] - 1, n[1] - 1, n[0] - 1), (24, 20, 20), (24, 160, 161)] + _samples(n, 7)[4:]
    gj = _direct_at(og(n, 0, alpha), Jin, samples)
    err, scale = 0.0, 0.0
    for (z, yy, x), g in zip(samples, gj):
        e = eps[z, yy, x]
        ref = 0.5 * e * Jin[:, z, yy, x] - (e - 1.0) * g
        err = max(err, np.abs(got[:, z, yy, x] - ref).max())
        scale = max(scale, np.abs(ref).max())
    assert err <= (1e-10 if dtype == "f64" else 1e-5) * scale


@pytest.mark.parametrize("prec", ["f64", "f32_refined"])
def test_history_lags_pillars_full_size(gpu_lib, prec):
    # The history operators at the benchmarked size: G_k J for lags k = 1, 2, 3
    # through the octant-compressed history spectra (640 x 640 x 96 embedding,
    # the ring precision of the context), on sampled voxels against the
    # oracle's direct sum of G_k.
    import torch
    w = W.PILLARS
    n, alpha = w.n, w.alpha
    c = _ctx(gpu_lib, n, alpha, prec, w.eps())
    J = W.random_current(n, seed=45)
    y = torch.empty(J.size, dtype=torch.float64, device="cuda")
    samples = _samples(n, 8)
    tol = 1e-10 if prec == "f64" else 1e-5
    for k in (1, 2, 3):
        c.gk_matvec(k, _t(J.ravel()), y, "f64" if prec == "f64" else "f32_refined")
        got = _np(y).reshape(J.shape)
        ref = _direct_at(og(n, k, alpha), J, samples)
        sub = np.array([got[:, z, yy, x] for (z, yy, x) in samples])
        assert np.abs(sub - ref).max() <= tol * np.abs(ref).max(), (k, np.abs(sub - ref).max() / np.abs(ref).max())
    c.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_history_rhs_pillars_full_size(gpu_lib, prec):
    # The history right-hand side at the benchmarked size after four pushes,
    # started at step 40 so that the ring slots written (40..43 of ell = 52)
    # lie past 2^31 complex elements of the ring: h = -(1/2 + d1) eps_r J_new
    # - d2 eps_r J_before + (eps_r - 1) sum_k G_k J_{n+1-k}, on sampled voxels
    # against the oracle's direct sums, with the regularization of the workloads.
    import torch
    w = W.PILLARS
    n, alpha = w.n, w.alpha
    eps = w.eps()
    c = _ctx(gpu_lib, n, alpha, prec, eps)
    d0, d1, d2 = W.regularization_for(alpha)
    c.set_regularization((d0, d1, d2))
    c.reset()
    c.set_step(40)
    Js = [W.random_current(n, seed=60 + i) for i in range(4)]
    for J in Js:
        c.history_update(_t(J.ravel()))
    h = torch.empty(Js[0].size, dtype=torch.float64, device="cuda")
    c.history_rhs(h)
    got = _np(h).reshape(Js[0].shape)
    # half of the samples inside the pillars, where the contrast term is nonzero
    mat = np.argwhere(eps != 1.0)
    pick = np.random.default_rng(10).choice(len(mat), size=40, replace=False)
    samples = _samples(n, 9, count=24) + [tuple(int(v) for v in mat[i]) for i in pick]
    acc = np.zeros((len(samples), 3))
    for k in range(1, 5):
        acc += _direct_at(og(n, k, alpha), Js[-k], samples)
    err, scale = 0.0, 0.0
    for i, (z, yy, x) in enumerate(samples):
        e = eps[z, yy, x]
        ref = -(0.5 + d1) * e * Js[-1][:, z, yy, x] - d2 * e * Js[-2][:, z, yy, x] + (e - 1.0) * acc[i]
        err = max(err, np.abs(got[:, z, yy, x] - ref).max())
        scale = max(scale, np.abs(ref).max())
    assert err <= (1e-10 if prec == "f64" else 1e-5) * scale, err / scale
    c.close()


def test_march_pillars_full_size(gpu_lib):
    # The benchmarked march: 8x8 pillars, 320x320x48 voxels, dt = 16 dt_CFL,
    # autotuned tile shapes, started at step ell with zero past currents,
    # tol 1e-6, over 10 steps (one history block of 8 with its second-level
    # block, and the next block start); its vectors are large enough for the
    # streaming accesses.  At this size it is held to properties: every
    # current meets the residual bound under a separate FP64 product; the
    # history right-hand side from the blocked multiply-accumulate equals the
    # sum of the lag products (one FFT product per lag); the FP32-refined and
    # FP64 marches agree.
    import torch
    w = W.PILLARS
    n, alpha = w.n, w.alpha
    eps = w.eps()
    N3 = 3 * math.prod(n)
    p = W.pulse(w.ppw)
    L = basis.cdt_from_alpha(alpha)
    eps3 = _t(np.tile(eps.ravel(), 3))
    steps, tol = 10, 1e-6
    marches = {}
    for prec in ("f64", "f32_refined"):
        c = _ctx(gpu_lib, n, alpha, prec, eps)
        c.autotune()
        nl = c.info()["nlags"]
        c.reset()
        c.set_step(nl)
        einc, h, y, g = (torch.empty(N3, dtype=torch.float64, device="cuda") for _ in range(4))
        htol = 1e-10 if prec == "f64" else 1e-5
        gdt = "f64" if prec == "f64" else "f32_refined"
        Js = []                          # newest first
        for s in range(steps):
            c.history_rhs(h)
            if not Js:
                assert float(torch.abs(h).max()) == 0.0
            else:
                acc = torch.zeros_like(h)
                for k in range(1, min(len(Js), nl) + 1):
                    c.gk_matvec(k, Js[k - 1], g, gdt)
                    acc += g
                ref = -0.5 * eps3 * Js[0] + (eps3 - 1.0) * acc
                rel = float(torch.linalg.vector_norm(h - ref) / torch.linalg.vector_norm(ref))
                assert rel <= htol, (prec, s, rel)
            c.excitation(p, (22 + s) * L, einc)
            J = torch.empty_like(einc)
            status, st = c.step(einc, J, tol=tol)
            assert status == 0 and st["iters"] > 0, (prec, s, st)
            b = einc + h
            c.z0_matvec(J, y, "f64")
            rr = float(torch.linalg.vector_norm(y - b) / torch.linalg.vector_norm(b))
            assert rr <= 1.01 * tol, (prec, s, rr)
            Js.insert(0, J)
        marches[prec] = Js
        c.close()
    a, b = marches["f32_refined"], marches["f64"]
    num = max(float(torch.linalg.vector_norm(x - z)) for x, z in zip(a, b))
    den = max(float(torch.linalg.vector_norm(z)) for z in b)
    assert num <= 2e-5 * den, num / den


def test_march_cube64_refined_vs_f64_full_length(gpu_lib):
    # The 64^3 inhomogeneous cube (eps_r i.i.d. U[2, 6], seed 2), dt = 8 dt_CFL,
    # h = lambda_min/20, all 300 steps from t = 0, in FP64 and in FP32 with FP64
    # refinement side by side, with the regularized operator of the workloads
    # (delta = 0.1 dt_CFL/dt).  Every step of both marches meets the FP64
    # residual bound, the field-error bar (1e-4 of the largest current) holds
    # over all 300 steps, and after the pulse the medium's ringing stays well
    # below the peak (unregularized, a growing mode passes the peak by the
    # last steps).
    import torch
    w = W.CUBE64
    n, alpha = w.n, w.alpha
    eps = w.eps()
    N3 = 3 * math.prod(n)
    p = W.pulse(w.ppw)
    L = basis.cdt_from_alpha(alpha)
    tol = 1e-6
    ctx = {prec: _ctx(gpu_lib, n, alpha, prec, eps) for prec in ("f64", "f32_refined")}
    for c in ctx.values():
        c.set_regularization(W.regularization_for(alpha))
    einc = torch.empty(N3, dtype=torch.float64, device="cuda")
    J = {prec: torch.empty(N3, dtype=torch.float64, device="cuda") for prec in ctx}
    diff, norm = [], []
    for s in range(w.steps):
        ctx["f64"].excitation(p, s * L, einc)
        for prec, c in ctx.items():
            status, st = c.step(einc, J[prec], tol=tol)
            assert status == 0 and st["relres"] <= 1.01 * tol, (prec, s, st)
        diff.append(float(torch.linalg.vector_norm(J["f32_refined"] - J["f64"])))
        norm.append(float(torch.linalg.vector_norm(J["f64"])))
    for c in ctx.values():
        c.close()
    assert max(diff) <= 1e-4 * max(norm), max(diff) / max(norm)
    assert max(norm[-50:]) < 0.2 * max(norm), (max(norm[-50:]), max(norm))


def _trace(name):
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"oracle_trace_{name}.npz")
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def _march_vs_trace(gpu_lib, name, eps, prec, history="auto"):
    """March the workload of an oracle trace on the GPU (tol 1e-6) and return the
    field error max_n ||J_n - J_n^ref|| / max_n ||J_n^ref|| on the sampled voxels,
    and the largest relative difference of the full norms."""
    import torch
    tr = _trace(name)
    nx, ny, nz = (int(v) for v in tr["shape"])
    alpha, steps = int(tr["alpha"]), int(tr["steps"])
    n = (nx, ny, nz)
    ppw = {"cube32": W.CUBE64.ppw, "pillars80": W.PILLARS.ppw}.get(name, W.CUBE96.ppw)
    p = W.pulse(ppw)
    L = basis.cdt_from_alpha(alpha)
    c = _ctx(gpu_lib, n, alpha, prec, eps)
    c.set_regularization(tuple(float(v) for v in np.atleast_1d(tr["delta"])) if np.size(tr["delta"]) == 3
                         else float(tr["delta"]))
    c.set_history_scheme(history)
    c.reset()
    N3 = 3 * math.prod(n)
    einc = torch.empty(N3, dtype=torch.float64, device="cuda")
    J = torch.empty(N3, dtype=torch.float64, device="cuda")
    idx = _t(tr["idx"].astype(np.int64))
    num = den = nerr = 0.0
    for s in range(steps):
        c.excitation(p, s * L, einc)
        status, st = c.step(einc, J, tol=1e-6)
        assert status == 0, (s, st)
        sub = J.view(3, -1)[:, idx]
        ref = _t(tr["samples"][s])
        num = max(num, float(torch.linalg.vector_norm(sub - ref)))
        den = max(den, float(torch.linalg.vector_norm(ref)))
        nerr = max(nerr, abs(float(torch.linalg.vector_norm(J)) - float(tr["norms"][s])))
    c.close()
    err, nerr = num / den, nerr / float(tr["norms"].max())
    print(f"[trace] {name} {prec} history {history}: field error {err:.2e}, norm error {nerr:.2e}")
    return err, nerr


@pytest.mark.parametrize("prec", ["f64", "f32_refined"])
def test_march_cube32_config2_medium_vs_oracle(gpu_lib, prec):
    # a 32^3 cut of the 64^3 i.i.d. eps_r ~ U[2, 6] medium, dt = 8 dt_CFL, all
    # 300 steps from t = 0, against the oracle's FP64 march (stored trace, TFQMR
    # to 1e-10): field error <= 1e-4 on 192 sampled voxels and on the norms
    eps = np.ascontiguousarray(W.CUBE64.eps()[:32, :32, :32])
    err, nerr = _march_vs_trace(gpu_lib, "cube32", eps, prec)
    assert err <= 1e-4 and nerr <= 1e-4, (err, nerr)


@pytest.mark.parametrize("prec", ["f64", "f32_refined"])
def test_march_pillars80_vs_oracle(gpu_lib, prec):
    # a 2x2-pillar cut (80 x 80 x 48) of the benchmarked array, dt = 16 dt_CFL,
    # 120 steps from t = 0, against the oracle's FP64 march (stored trace)
    eps = np.ascontiguousarray(W.PILLARS.eps()[:, :80, :80])
    err, nerr = _march_vs_trace(gpu_lib, "pillars80", eps, prec)
    assert err <= 1e-4 and nerr <= 1e-4, (err, nerr)


@pytest.mark.parametrize("alpha,history", [(1, "auto"), (1, "fft_time"), (2, "auto"), (2, "fft_time"), (4, "auto"),
                                           (8, "auto"), (16, "auto")])
def test_march_nested24_time_step_sweep_vs_oracle(gpu_lib, alpha, history):
    # the time-step sweep on a 24^3 cut of the 96^3 nested cube (eps_r 6 core
    # and 4 layer, +-5 % noise), dt = alpha dt_CFL over the window of 1600
    # dt_CFL from t = 0 with the regularization of the workloads, FP32 refined,
    # against the oracle's FP64 march of each alpha (stored traces); at
    # alpha = 1 and 2 (ell = 73 and 37) also with the far lags by FFTs in time
    eps = np.ascontiguousarray(W.CUBE96.eps()[24:48, 24:48, 24:48])
    err, nerr = _march_vs_trace(gpu_lib, f"nested24_a{alpha}", eps, "f32_refined", history)
    assert err <= 1e-4 and nerr <= 1e-4, (err, nerr)


@pytest.mark.parametrize("prec,expect", [("f64", "MOT_EBREAKDOWN"), ("f32", "MOT_EBREAKDOWN"),
                                         ("f32_refined", "MOT_ENOCONV")])
def test_forced_breakdown_is_reported_and_recoverable(gpu_lib, prec, expect):
    # failure injection from the host: a near-breakdown tolerance that no
    # reduction passes ends every TFQMR solve at its first reduction.  The
    # FP64 and FP32 solves report MOT_EBREAKDOWN; the refined solve, whose
    # inner solves all break down, gives up after its refinement sweeps with
    # MOT_ENOCONV.  The history still advances, and with the tolerance back at
    # 0 the march is bit-identical to that of a context that never broke down.
    import torch
    n, alpha = (16, 6, 4), 4
    eps = _eps(n)
    p = W.pulse(20)
    L = basis.cdt_from_alpha(alpha)
    c = _ctx(gpu_lib, n, alpha, prec, eps)
    ref = _ctx(gpu_lib, n, alpha, prec, eps)
    N3 = 3 * math.prod(n)
    E = torch.empty(N3, dtype=torch.float64, device="cuda")
    J = torch.empty_like(E)
    Jr = torch.empty_like(E)
    code = getattr(gpu_lib, expect)
    c.set_breakdown_tolerance(1e300)
    c.reset()
    for s in range(3):
        c.excitation(p, (30 + s) * L, E)
        rc, _ = c.step(E, J, tol=1e-8, max_iter=60, allow=(code,))
        assert rc == code, (s, rc)
    assert c.info()["steps"] == 3
    with pytest.raises(gpu_lib.MotError) as ei:
        c.set_breakdown_tolerance(-1.0)
    assert ei.value.status == gpu_lib.MOT_EINVAL
    c.set_breakdown_tolerance(0.0)
    c.reset()
    ref.reset()
    tol = 1e-5 if prec == "f32" else 1e-8  # what a plain FP32 solve reaches
    for s in range(4):
        c.excitation(p, (30 + s) * L, E)
        assert c.step(E, J, tol=tol)[0] == 0
        assert ref.step(E, Jr, tol=tol)[0] == 0
        assert torch.equal(J, Jr), s
    c.close()
    ref.close()


def test_out_of_memory_is_reported(gpu_lib):
    # the largest grid the transforms support at dt = dt_CFL needs ell = 1359
    # history spectra (terabytes): creation fails with MOT_ENOMEM, frees what
    # it took, and a normal context still works afterwards
    with pytest.raises(gpu_lib.MotError) as ei:
        gpu_lib.Context(640, 320, 320, alpha=1, precision="f32")
    assert ei.value.status == gpu_lib.MOT_ENOMEM
    c = _ctx(gpu_lib, (8, 8, 8), 4)
    c.close()


@pytest.mark.parametrize("prec", ["f64", "f32_refined"])
def test_graph_replay_matches_stream_launches(gpu_lib, prec):
    # TFQMR iterations replayed from HIP graphs give the same currents, bit for bit
    import torch
    n, alpha = (16, 6, 4), 4
    eps = _eps(n)
    cs = [_ctx(gpu_lib, n, alpha, prec, eps=eps) for _ in range(2)]
    for c in cs:
        c.reset()
    cs[1].set_graphs(True)
    p = W.pulse(20)
    N = int(np.prod(n))
    e = torch.empty(3 * N, dtype=torch.float64, device="cuda")
    J = [torch.empty(3 * N, dtype=torch.float64, device="cuda") for _ in range(2)]
    for k in range(30):
        cs[0].excitation(p, (60 + k) * alpha / math.sqrt(3.0), e)
        st = [c.step(e, Jc, tol=1e-6)[1] for c, Jc in zip(cs, J)]
        assert st[0]["iters"] == st[1]["iters"]
        assert torch.equal(J[0], J[1])


def test_sweep_graph_matches_stream_launches(gpu_lib):
    # graph mode 2 (the refined first sweep as one graph with a fixed number of
    # gated iterations) gives the currents and counts of stream launches, bit
    # for bit, also in steps whose tighter tolerance needs a second sweep
    import torch
    n, alpha = (24, 20, 12), 8
    eps = _eps(n)
    cs = [_ctx(gpu_lib, n, alpha, "f32_refined", eps=eps) for _ in range(2)]
    for c in cs:
        c.reset()
    cs[1].set_graphs(2)
    p = W.pulse(20)
    N = int(np.prod(n))
    e = torch.empty(3 * N, dtype=torch.float64, device="cuda")
    J = [torch.empty(3 * N, dtype=torch.float64, device="cuda") for _ in range(2)]
    for k in range(40):
        tol = 1e-6 if k < 25 else 3e-7
        cs[0].excitation(p, (40 + k) * alpha / math.sqrt(3.0), e)
        st = [c.step(e, Jc, tol=tol)[1] for c, Jc in zip(cs, J)]
        for key in ("iters", "matvecs", "matvecs_f64", "refinements"):
            assert st[0][key] == st[1][key], (k, key)
        assert st[1]["relres"] <= tol
        assert torch.equal(J[0], J[1]), k
    for c in cs:
        c.close()


def test_last_stats_without_device_wait(gpu_lib):
    # a step without stats returns with its history update in flight; its
    # counts and residual are those a step with stats reports, bit for bit,
    # and its LHS/RHS times are -1
    import torch
    n, alpha = (16, 6, 4), 4
    eps = _eps(n)
    cs = [_ctx(gpu_lib, n, alpha, "f32_refined", eps=eps) for _ in range(2)]
    p = W.pulse(20)
    N = int(np.prod(n))
    e = torch.empty(3 * N, dtype=torch.float64, device="cuda")
    J = [torch.empty(3 * N, dtype=torch.float64, device="cuda") for _ in range(2)]
    for k in range(12):
        cs[0].excitation(p, (60 + k) * alpha / math.sqrt(3.0), e)
        st0 = cs[0].step(e, J[0], tol=1e-6)[1]
        assert cs[1].step(e, J[1], tol=1e-6, stats=False)[1] is None
        st1 = cs[1].last_stats()
        for key in ("iters", "matvecs", "matvecs_f64", "refinements", "relres"):
            assert st0[key] == st1[key], (k, key)
        assert st1["ms_lhs"] == -1.0 and st1["ms_rhs"] == -1.0
        assert cs[0].last_stats() == st0
    torch.cuda.synchronize()
    assert torch.equal(J[0], J[1])
    for c in cs:
        c.close()


def test_step_batch_matches_single_steps(gpu_lib):
    # contexts of uneven grids on their own streams, stepped together by the
    # library's thread pool, give the currents of one-by-one steps, bit for bit
    import torch
    shapes = [(8, 8, 8), (12, 12, 12), (16, 16, 16), (8, 12, 16)]
    rng = np.random.default_rng(7)
    eps = [rng.uniform(1.5, 6.0, size=n[::-1]) for n in shapes]
    pulses = [W.pulse(20, k_hat=(0.0, 0.0, 1.0), e_hat=(1.0, 0.0, 0.0)),
              W.pulse(20, k_hat=(1.0, 0.0, 0.0), e_hat=(0.0, 1.0, 0.0)),
              W.pulse(20, k_hat=(0.0, 1.0, 0.0), e_hat=(0.0, 0.0, 1.0)),
              W.pulse(20, k_hat=(0.6, 0.0, 0.8), e_hat=(0.0, 1.0, 0.0))]
    alpha = 4
    batch = [_ctx(gpu_lib, n, alpha, "f32_refined", eps=e, stream=torch.cuda.Stream()) for n, e in zip(shapes, eps)]
    single = [_ctx(gpu_lib, n, alpha, "f32_refined", eps=e) for n, e in zip(shapes, eps)]
    for c in batch + single:
        c.reset()
    E = [torch.empty(3 * int(np.prod(n)), dtype=torch.float64, device="cuda") for n in shapes]
    Jb = [torch.empty_like(e) for e in E]
    Js = [torch.empty_like(e) for e in E]
    for k in range(12):
        t = (70 + k) * alpha / math.sqrt(3.0)
        for c, p, e in zip(single, pulses, E):
            c.excitation(p, t, e)
        torch.cuda.synchronize()
        status, stats = gpu_lib.step_batch(batch, E, Jb, tol=1e-6)
        assert status == [0, 0, 0, 0]
        for c, e, j in zip(single, E, Js):
            c.step(e, j, tol=1e-6)
        torch.cuda.synchronize()
        for a, b in zip(Jb, Js):
            assert torch.equal(a, b)


def test_initial_guess_keeps_the_march(gpu_lib):
    # the refined solve started from the least-squares guess over earlier
    # solutions meets the same residual test: the currents agree with the
    # zero-start march to the solver tolerance, in fewer iterations
    import torch
    n, alpha = (16, 16, 16), 4
    eps = _eps(n)
    cs = [_ctx(gpu_lib, n, alpha, "f32_refined", eps=eps) for _ in range(2)]
    cs[0].set_predictor(8)
    for c in cs:
        c.reset()
    p = W.pulse(20)
    N = int(np.prod(n))
    e = torch.empty(3 * N, dtype=torch.float64, device="cuda")
    J = [torch.empty(3 * N, dtype=torch.float64, device="cuda") for _ in range(2)]
    its = [0, 0]
    err, ref = 0.0, 0.0
    for k in range(40):
        cs[0].excitation(p, (40 + k) * alpha / math.sqrt(3.0), e)
        for i in range(2):
            st = cs[i].step(e, J[i], tol=1e-6)[1]
            assert st["relres"] <= 1e-6
            its[i] += st["iters"]
        err = max(err, float(torch.linalg.vector_norm(J[0] - J[1])))
        ref = max(ref, float(torch.linalg.vector_norm(J[1])))
    assert err <= 2e-5 * ref, err / ref
    assert its[0] < its[1], its
    with pytest.raises(gpu_lib.MotError):
        _ctx(gpu_lib, (8, 4, 4), 2, "f64").set_predictor(2)
