"""Write the oracle's reference traces used by the GPU parity tests and the
benchmark's field-error figure.  Calls only ``oracle`` and the input recipes
of ``workloads``; run it on the CPU:

    python tests/golden/make_oracle_traces.py [cube32 | pillars80]

Each trace is an FP64 march of Eq. 3 from t = 0 with the regularized
operator of the workloads (workloads.regularization_for(alpha), Sec. II
delta-notation), TFQMR to 1e-10,
saved as an .npz (no pickles) holding: the step count, alpha, delta, the
per-step norm ||J_n||, the sampled voxel indices (flat, [z][y][x]) and J_n at
those voxels for every step, shape (steps, 3, nsamples).
"""

import concurrent.futures
import os
import sys
import time

import numpy as np
import scipy.fft

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import basis, green, march  # noqa: E402

CASES = {
    # a 32^3 cut of the 64^3 i.i.d. eps_r ~ U[2, 6] medium, dt = 8 dt_CFL, 300 steps
    "cube32": dict(eps=lambda: np.ascontiguousarray(W.CUBE64.eps()[:32, :32, :32]), alpha=8, steps=300,
                   ppw=W.CUBE64.ppw, nsamples=192, seed=11),
    # a 2x2-pillar cut (80 x 80 x 48) of the 8x8 pillar array, dt = 16 dt_CFL, 120 steps
    "pillars80": dict(eps=lambda: np.ascontiguousarray(W.PILLARS.eps()[:, :80, :80]), alpha=16, steps=120,
                      ppw=W.PILLARS.ppw, nsamples=192, seed=12),
}
# a 24^3 cut (indices 24..47 on every axis: the eps_r = 6 core and the 4 layer)
# of the 96^3 nested cube of the time-step sweep, over the sweep's window of
# 1600 dt_CFL for each alpha
for _a in (1, 2, 4, 8, 16):
    CASES[f"nested24_a{_a}"] = dict(eps=lambda: np.ascontiguousarray(W.CUBE96.eps()[24:48, 24:48, 24:48]),
                                    alpha=_a, steps=1600 // _a, ppw=W.CUBE96.ppw, nsamples=16, seed=13)


def _octant(a):
    nx, ny, nz, k, alpha = a
    return green.green_octant(nx, ny, nz, k, alpha=alpha)


def path(name):
    return os.path.join(HERE, f"oracle_trace_{name}.npz")


def make(name):
    cs = CASES[name]
    eps = cs["eps"]()
    nz, ny, nx = eps.shape
    alpha = cs["alpha"]
    delta = W.regularization_for(alpha)
    L = basis.cdt_from_alpha(alpha)
    nl = basis.nlags(nx, ny, nz, alpha=alpha)
    t0 = time.time()
    # the lags' tables are independent: one process per lag
    with concurrent.futures.ProcessPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        G = list(ex.map(_octant, [(nx, ny, nz, k, alpha) for k in range(nl + 1)]))
    print(f"{name}: {nx}x{ny}x{nz}, alpha {alpha}, ell {nl}, delta {delta}: Green {time.time() - t0:.0f}s", flush=True)
    rng = np.random.default_rng(cs["seed"])
    mat = np.flatnonzero(eps.ravel() != 1.0)
    idx = np.sort(rng.choice(mat, size=cs["nsamples"], replace=False))
    p = W.pulse(cs["ppw"])
    mot = march.Mot(eps, G, L, delta=delta)
    norms, samp = [], []
    for s in range(cs["steps"]):
        with scipy.fft.set_workers(os.cpu_count() or 1):
            J, res = mot.step(march.dt_einc(p, eps, s * L), tol=1e-10)
        norms.append(np.linalg.norm(J))
        samp.append(J.reshape(3, -1)[:, idx])
        if s % 10 == 0:
            print(f"  step {s}: |J| {norms[-1]:.4e}, {res.iterations} it, {time.time() - t0:.0f}s", flush=True)
    np.savez(path(name), steps=cs["steps"], alpha=alpha, delta=np.array(delta), shape=np.array([nx, ny, nz]),
             norms=np.array(norms), idx=idx, samples=np.array(samp))
    print(f"wrote {path(name)}", flush=True)


if __name__ == "__main__":
    for n in (sys.argv[1:] or list(CASES)):
        make(n)
