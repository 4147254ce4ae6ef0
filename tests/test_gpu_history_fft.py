"""The history right-hand side with the far lags applied by FFTs in time
(history scheme 2), against the FP64 oracle's direct sums.

The scheme groups the steps in blocks of 32 and applies, at the first push of
a block, the lags reaching into every earlier block as products of length-64
transforms in time; the lags inside the current block stay with the blocked
per-lag pass.  The sums are the plain ones of the recursion (Eq. 3) in another
order, so the bar is the FP32 one of the history products (relative 1e-5).
"""

import functools
import math

import numpy as np
import pytest

import workloads as W
from oracle import basis, green, masks, operators

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def og(n, k, alpha):
    return green.green_octant(*n, k, alpha=alpha)


def _t(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to("cuda", dtype=dtype) if dtype is not None else t.to("cuda")


def _np(t):
    return t.detach().cpu().numpy()


def _ctx(native, n, alpha, prec, eps):
    c = native.Context(*n, alpha=alpha, precision=prec)
    c.set_material(_t(eps.ravel()))
    c.build_green_spectra()
    return c


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# pushes after which the right-hand side is checked: block starts (n a
# multiple of 32, where the far parts are formed), the steps after them, the
# second level of an 8-step block (its fifth step), the last steps of a time
# block, and pushes past 64 and 96 (two and three earlier blocks in reach)
CHECKS = (1, 2, 8, 9, 13, 32, 33, 34, 38, 41, 63, 64, 65, 66, 69, 72, 89, 96, 97, 100, 105, 110)


@pytest.mark.parametrize("prec,switch", [("f32", False), ("f32_refined", False), ("f32", True)])
def test_history_fft_time_vs_oracle(gpu_lib, prec, switch):
    # h_{n+1} = -(eps/2) J_n + (eps-1) sum_k G_k * J_{n+1-k}; ell = 49 (two
    # lag segments of 32), 110 pushes wrap the ring twice.  With switch the
    # scheme goes to the per-lag pass at push 70 (inside a time block) and
    # back at push 80: the block then in progress finishes with the per-lag
    # pass and the next one starts with FFTs in time.
    import torch
    n, alpha = (24, 12, 6), 1
    eps = W.eps_iid(n, 1.5, 6.0, seed=31)
    c = _ctx(gpu_lib, n, alpha, prec, eps)
    nl = c.info()["nlags"]
    assert nl >= 33
    c.set_history_scheme("fft_time")
    assert c.info()["history_scheme"] == 2
    Gs = [None] + [og(n, k, alpha) for k in range(1, nl + 1)]
    hist = []
    out = torch.empty(3 * math.prod(n), dtype=torch.float64, device="cuda")
    worst = 0.0
    for s in range(max(CHECKS)):
        if switch and s == 70:
            c.set_history_scheme("blocked")
            assert c.info()["history_scheme"] == 1
        if switch and s == 80:
            c.set_history_scheme("fft_time")
        J = W.random_current(n, seed=300 + s)
        hist.insert(0, J)
        c.history_update(_t(J.ravel()))
        if s + 1 not in CHECKS:
            continue
        c.history_rhs(out)
        acc = np.zeros_like(J)
        for k in range(1, nl + 1):
            if k - 1 < len(hist):
                acc += operators.gconv_fft(Gs[k], hist[k - 1])
        ref = -0.5 * eps[None] * J + (eps[None] - 1.0) * acc
        err = _rel(_np(out).reshape(J.shape), ref)
        worst = max(worst, err)
        assert err <= 1e-5, (s, err)
    print(f"[history fft_time] {prec} switch={switch}: worst relative error {worst:.2e} over {len(CHECKS)} checks")
    c.close()


def test_history_fft_time_is_the_default_for_long_histories(gpu_lib):
    # ell >= 128 on an FP32 ring: FFTs in time unless asked otherwise; shorter
    # histories keep the per-lag pass; an FP64 ring cannot use them
    c = gpu_lib.Context(32, 16, 8, alpha=1, precision="f32")
    assert 32 <= c.info()["nlags"] < 128 and c.info()["history_scheme"] == 1
    c.close()
    n = (80, 32, 16)
    c = gpu_lib.Context(*n, alpha=1, precision="f32")
    assert c.info()["nlags"] >= 128 and c.info()["history_scheme"] == 2
    c.set_history_scheme("blocked")
    assert c.info()["history_scheme"] == 1
    c.set_history_scheme("auto")
    assert c.info()["history_scheme"] == 2
    c.close()
    c = gpu_lib.Context(*n, alpha=1, precision="f64")
    assert c.info()["history_scheme"] == 1
    with pytest.raises(gpu_lib.MotError) as ei:
        c.set_history_scheme("fft_time")
    assert ei.value.status == gpu_lib.MOT_EINVAL
    c.close()


def _g_at(offs, k, alpha):
    """3x3 blocks G_k(d) for signed integer offsets d = (dz, dy, dx), (len, 3, 3)."""
    offs = np.asarray(offs, dtype=np.int64)
    az, ay, ax = np.abs(offs[:, 0]), np.abs(offs[:, 1]), np.abs(offs[:, 2])
    L = basis.cdt_from_alpha(alpha)
    v = green.dyad_at(ax, ay, az, np.asarray(k, dtype=np.float64), L)
    m = masks.mask(ax, ay, az, k, alpha=alpha) if np.ndim(k) == 0 else np.array(
        [masks.mask(ax[i], ay[i], az[i], int(k[i]), alpha=alpha) for i in range(len(ax))])
    v = v * m[None, :]
    sg = np.stack([np.where(offs[:, 2] < 0, -1.0, 1.0), np.where(offs[:, 1] < 0, -1.0, 1.0),
                   np.where(offs[:, 0] < 0, -1.0, 1.0)])  # x, y, z reflection signs
    B = np.zeros((len(offs), 3, 3))
    for cc, (p, q) in enumerate(green.PAIR):
        val = v[cc] * (sg[p] * sg[q] if p != q else 1.0)
        B[:, p, q] = val
        B[:, q, p] = val
    return B


def test_history_fft_time_pillars_full_size(gpu_lib):
    # The benchmarked array (320 x 320 x 48, ell = 52, a 640 x 640 x 96
    # embedding) with FFTs in time, 70 pushes of point currents (two voxels
    # per step): the right-hand side after push 65 (a time-block start, with
    # two earlier blocks in reach) and push 70, on sampled voxels against the
    # oracle's G_k evaluated at the source-observer offsets.
    import torch
    w = W.PILLARS
    n, alpha = w.n, w.alpha
    nx, ny, nz = n
    N = nx * ny * nz
    eps = w.eps()
    c = _ctx(gpu_lib, n, alpha, "f32", eps)
    d0, d1, d2 = W.regularization_for(alpha)
    c.set_regularization((d0, d1, d2))
    c.set_history_scheme("fft_time")
    c.reset()
    nl = c.info()["nlags"]
    rng = np.random.default_rng(77)
    srcs = []  # per push: list of ((z, y, x), amplitude 3-vector)
    J = torch.zeros(3 * N, dtype=torch.float64, device="cuda")
    h = torch.empty(3 * N, dtype=torch.float64, device="cuda")
    mat = np.argwhere(eps != 1.0)
    worst = 0.0
    for s in range(70):
        J.zero_()
        pts = []
        for _ in range(2):
            z, yy, x = (int(rng.integers(0, v)) for v in (nz, ny, nx))
            amp = rng.standard_normal(3)
            pts.append(((z, yy, x), amp))
            for q in range(3):
                J[q * N + (z * ny + yy) * nx + x] += float(amp[q])
        srcs.append(pts)
        c.history_update(J)
        if s + 1 not in (65, 70):
            continue
        c.history_rhs(h)
        got = _np(h).reshape(3, nz, ny, nx)
        pick = rng.choice(len(mat), size=24, replace=False)
        samples = [tuple(int(v) for v in mat[i]) for i in pick]
        # observers next to the newest sources too (short lags, strong fields)
        for (z, yy, x), _ in srcs[-1] + srcs[-2]:
            samples.append((z, yy, min(x + 1, nx - 1)))
        nn = s  # index of the newest push
        offs, ks, amps, obs = [], [], [], []
        for oi, (z, yy, x) in enumerate(samples):
            for k in range(1, nl + 1):
                t = nn + 1 - k
                if t < 0:
                    break
                for (sz_, sy_, sx_), amp in srcs[t]:
                    offs.append((z - sz_, yy - sy_, x - sx_))
                    ks.append(k)
                    amps.append(amp)
                    obs.append(oi)
        B = _g_at(np.array(offs), np.array(ks, dtype=np.float64), alpha)
        acc = np.zeros((len(samples), 3))
        np.add.at(acc, np.array(obs), np.einsum("mpq,mq->mp", B, np.array(amps)))
        err, scale = 0.0, 0.0
        for i, (z, yy, x) in enumerate(samples):
            e = eps[z, yy, x]
            jn = np.zeros(3)
            jp = np.zeros(3)
            for (p_, amp) in srcs[nn]:
                if p_ == (z, yy, x):
                    jn += amp
            for (p_, amp) in srcs[nn - 1]:
                if p_ == (z, yy, x):
                    jp += amp
            ref = -(0.5 + d1) * e * jn - d2 * e * jp + (e - 1.0) * acc[i]
            err = max(err, np.abs(got[:, z, yy, x] - ref).max())
            scale = max(scale, np.abs(ref).max())
        worst = max(worst, err / scale)
        assert err <= 1e-5 * scale, (s, err / scale)
    print(f"[history fft_time] pillars full size: worst relative error {worst:.2e}")
    c.close()


@pytest.mark.parametrize("scheme", ["blocked", "fft_time"])
def test_history_wide_offsets_bit_identical(gpu_lib, scheme):
    # the FP32 blocked multiply-accumulate takes 32-bit buffer offsets on
    # grids that allow them and 64-bit addresses otherwise; forced onto the
    # 64-bit form it must give the same right-hand sides bit for bit.  ell =
    # 49 and 110 pushes: block starts with every count of older slots from 1
    # to ell (every remainder of the pipelined loop), the second level of each
    # block, and with FFTs in time the partial blocks of 0..24 slots.
    import torch
    n, alpha = (24, 12, 6), 1
    eps = W.eps_iid(n, 1.5, 6.0, seed=31)
    cs = [_ctx(gpu_lib, n, alpha, "f32", eps) for _ in range(2)]
    cs[1].set_wide_offsets(True)
    assert gpu_lib.LIB.mot_set_wide_offsets(cs[0].h, 2) == gpu_lib.MOT_EINVAL
    for c in cs:
        c.set_history_scheme(scheme)
    N = math.prod(n)
    out = [torch.empty(3 * N, dtype=torch.float64, device="cuda") for _ in range(2)]
    for s in range(110):
        J = _t(W.random_current(n, seed=500 + s).ravel())
        for c, o in zip(cs, out):
            c.history_update(J)
            c.history_rhs(o)
        assert torch.equal(out[0], out[1]), s
    assert float(out[0].abs().max()) > 0.0
    for c in cs:
        c.close()
