"""Throughput of the MOT-JVIE hot path on one MI355X.

Workload: 8x8 array of inhomogeneous dielectric pillars on a 320x320x48 voxel
grid (14,745,600 unknowns), dt = 16 dt_CFL (ell = 52 history lags), FP32 FFT
products with FP64 Krylov vectors and FP64 iterative refinement, TFQMR
tolerance 1e-6.  A "step" is one MOT step (Eq. 3): excitation, history
right-hand side, the Z0 solve and the history update.

Set-up (untimed): the Green spectra, then the autotuner picks the FFT tile
shape of each pass on this grid (mot_autotune; --no-autotune keeps the
defaults).

Timed region: K steps after W warm-up steps and B breakdown steps (one
history block, B = 8 for the FP32 ring), inputs
resident in HBM; the march starts at step ell with zero currents before it,
so the history ring counts as full and every timed step multiplies all ell
lags.  The breakdown steps (one history block, untimed) time every kernel and
name the dominant one; inside the timed region only that kernel carries HIP
timing events.  Prints one JSON line.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
ROOFLINE_KINDS = ("history_mac", "z_fused", "y_forward", "y_inverse")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(kind, n, t_bytes, io_bytes, nvalid, blk=1):
    """Minimal HBM bytes of one launch of a pass: each input and output
    array touched once (FP32 complex = 2 t_bytes, voxel vectors io_bytes)."""
    nx, ny, nz = n
    kx, py, pz = nx + 1, 2 * ny, 2 * nz
    N = nx * ny * nz
    c = 2 * t_bytes                       # one complex value
    a = 3 * nz * ny * kx * c              # after x pass
    b = 3 * nz * py * kx * c              # after y pass (z < nz)
    f = 3 * pz * py * kx * c              # full spectrum
    lam = 6 * (nz + 1) * (ny + 1) * kx * t_bytes
    return {
        "x_forward": 3 * N * io_bytes + a,
        "y_forward": a + b,
        "z_fused": b + lam + b,
        "y_inverse": b + a,
        "x_inverse_epilogue": a + 3 * N * io_bytes + N * 8 + 3 * N * io_bytes,
        "z_forward": b + f,
        "history_mac": nvalid * (f + lam) + blk * f,
        "z_inverse": f + b,
        # far lags by FFTs in time, at a block start with nvalid earlier
        # blocks of blk steps in reach: their currents, the lag-segment
        # spectra (blk + 1 frequencies of the 6 components, complex), and
        # the far parts of the next blk right-hand sides
        "history_far": nvalid * blk * f + nvalid * (blk + 1) * 2 * lam + blk * f,
    }.get(kind)


def cpu_baseline(w, eps, mv_per_step, nl, log_fn):
    """The FP64 oracle's MOT step rate at the benchmark size, from a bounded
    sample (a whole oracle step at this size needs its ell = 52 history
    spectra in complex FP64, about 100 GB of host memory, so it is not run):
    two oracle Z0 products, one spectral lag multiply-accumulate and the two
    transforms of one step, each timed once, first with the oracle's
    transforms on one thread, then on every host core (scipy.fft workers).  A
    step of the oracle's march is mv_per_step Z0 products (the count the GPU
    run measured) plus nl lag multiply-accumulates, one inverse and one
    forward transform of the history (oracle.march.Mot.step)."""
    import numpy as np
    import scipy.fft
    import workloads as W
    from oracle import green, march
    log_fn("cpu baseline: oracle spectra of G_0 (untimed set-up)")
    g0 = green.green_octant(*w.n, 0, alpha=w.alpha)
    mot = march.Mot(eps, [g0], w.alpha / math.sqrt(3.0))
    J = W.random_current(w.n, seed=1)
    cores = os.cpu_count() or 1

    def sample(workers):
        with scipy.fft.set_workers(workers):
            t = time.perf_counter()
            mot.z0(J)
            mot.z0(J)
            t_z0 = (time.perf_counter() - t) / 2
            t = time.perf_counter()
            Jh = mot._spec(J)
            t_spec = time.perf_counter() - t
            t = time.perf_counter()
            S = mot._apply_spec(mot.lams[0], Jh)
            t_mac = time.perf_counter() - t
            t = time.perf_counter()
            mot._back(S)
            t_back = time.perf_counter() - t
        t_step = mv_per_step * t_z0 + nl * t_mac + t_back + t_spec
        return {"z0_s": t_z0, "mac_s": t_mac, "fwd_s": t_spec, "inv_s": t_back, "step_s": t_step,
                "sample_s": 2 * t_z0 + t_spec + t_mac + t_back}

    log_fn("cpu baseline: timing the oracle sample on one thread")
    one = sample(1)
    log_fn(f"cpu baseline: timing the oracle sample with {cores} FFT workers")
    many = sample(cores)
    best = many if many["step_s"] < one["step_s"] else one

    def text(r, th):
        return (f"{th}: 2 Z0 products ({r['z0_s']:.2f} s each), one lag multiply-accumulate ({r['mac_s']:.2f} s), "
                f"forward and inverse transforms ({r['fwd_s']:.2f} s, {r['inv_s']:.2f} s), {r['sample_s']:.1f} s "
                f"in all; scaled to a step = {mv_per_step:.1f} Z0 products + {nl} lag MACs + 2 transforms = "
                f"{r['step_s']:.0f} s")
    return {"value": 1.0 / best["step_s"], "unit": "MOT steps/s", "cores": cores if best is many else 1,
            "kind": "oracle",
            "sample": f"oracle FP64 (NumPy/SciPy) at {w.n[0]}x{w.n[1]}x{w.n[2]}, a scaled sample, not a whole "
                      f"step; " + text(one, "one thread") + "; " + text(many, f"{cores} FFT workers")
                      + "; the lag multiply-accumulate is NumPy elementwise work on one thread in both",
            "single_thread": {"value": 1.0 / one["step_s"], "z0_matvecs_per_s": 1.0 / one["z0_s"]},
            "all_cores": {"value": 1.0 / many["step_s"], "z0_matvecs_per_s": 1.0 / many["z0_s"], "workers": cores},
            "z0_matvecs_per_s": 1.0 / best["z0_s"], "cpu": _cpu_name(), "host_cpu_count": cores}


def f64_march(args, w, eps, pulse, L, Js, n_keep, log_fn):
    """The same march in FP64 (FP64 FFT products and Krylov vectors) from the
    same state: steps/s over its last f64_steps steps, and the field error of
    the main run, max_n |J_n - J64_n| / max_n |J64_n| over the kept steps."""
    import torch
    import workloads as W
    from paper_2607_28309_amd import native
    n = w.n
    N = n[0] * n[1] * n[2]
    c = native.Context(*n, alpha=w.alpha, precision="f64")
    c.set_material(torch.from_numpy(eps.ravel()).cuda())
    c.build_green_spectra()
    c.set_regularization(W.regularization_for(w.alpha))
    if not args.no_autotune:
        c.autotune()
    nl = c.info()["nlags"]
    c.reset()
    c.set_step(nl)
    J64 = torch.empty(3 * N, dtype=torch.float64, device="cuda")
    einc = torch.empty(3 * N, dtype=torch.float64, device="cuda")
    err_num, ref_max, st64 = 0.0, 0.0, []
    t = None
    k = min(args.steps, args.f64_steps)
    for s in range(n_keep):
        if s == n_keep - k:
            torch.cuda.synchronize()
            t = time.perf_counter()
        c.excitation(pulse, (args.start_step + s) * L, einc)
        st = c.step(einc, J64, tol=args.tol, stats=True)[1]
        if s >= n_keep - k:
            st64.append(st)
        err_num = max(err_num, float(torch.linalg.vector_norm(Js[s] - J64)))
        ref_max = max(ref_max, float(torch.linalg.vector_norm(J64)))
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    c.close()
    res = {"mot_steps_per_s_f64": k / el, "ms_per_step_f64": 1e3 * el / k,
           "iters_per_step_f64": sum(x["iters"] for x in st64) / k,
           "field_err_vs_f64": err_num / ref_max if ref_max > 0 else 0.0,
           "field_err_steps": n_keep}
    log_fn(f"FP64 march: {res['ms_per_step_f64']:.1f} ms/step, field error of {args.precision} vs FP64 "
           f"{res['field_err_vs_f64']:.2e} over {n_keep} steps")
    return res


def batch_leg(args, log_fn):
    """Batch of 32 independent cubes (sides 24..80, alpha = 4, each with its own
    incidence), every context on its own stream: batch steps/s with the
    library's thread pool (mot_step_batch) and one context after another."""
    import torch
    import workloads as W
    from paper_2607_28309_amd import native
    sc = W.cube_batch()
    alpha = W.BATCH_ALPHA
    L = alpha / math.sqrt(3.0)
    t0 = time.perf_counter()
    ctxs = []
    for s_ in sc:
        c = native.Context(*s_.n, alpha=alpha, precision=args.precision, stream=torch.cuda.Stream())
        c.set_material(torch.from_numpy(s_.eps.ravel()).cuda())
        c.build_green_spectra()
        c.set_regularization(W.regularization_for(alpha))
        if not args.no_autotune:
            c.autotune(reps=5)
        c.reset()
        c.set_step(c.info()["nlags"])
        ctxs.append(c)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    pulses = [W.pulse(W.BATCH_PPW, k_hat=s_.k_hat, e_hat=s_.e_hat) for s_ in sc]
    E = [torch.empty(3 * c.N, dtype=torch.float64, device="cuda") for c in ctxs]
    J = [torch.empty_like(e) for e in E]
    start = 100

    def excite(k):
        for c, p_, e in zip(ctxs, pulses, E):
            c.excitation(p_, (start + k) * L, e)

    for k in range(2):
        excite(k)
        native.step_batch(ctxs, E, J, tol=args.tol)
    torch.cuda.synchronize()
    K = args.batch_steps
    t = time.perf_counter()
    its = 0
    for k in range(K):
        excite(2 + k)
        st = native.step_batch(ctxs, E, J, tol=args.tol)[1]
        its += sum(x["iters"] for x in st)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t
    t = time.perf_counter()
    for k in range(K):
        excite(2 + K + k)
        for c, e, j in zip(ctxs, E, J):
            c.step(e, j, tol=args.tol, stats=False)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t
    res = {"workload": "cubes32_sides24to80_a4", "scatterers": len(ctxs),
           "unknowns": sum(3 * c.N for c in ctxs), "nlags": [c.info()["nlags"] for c in ctxs],
           "precision": args.precision, "steps": K, "setup_s": setup,
           "batch_steps_per_s": K / tb, "sequential_steps_per_s": K / ts, "speedup": ts / tb,
           "iters_per_scatterer_step": its / (K * len(ctxs))}
    log_fn(f"batch of {len(ctxs)} cubes: {1e3 * tb / K:.1f} ms per batch step with the thread pool, "
           f"{1e3 * ts / K:.1f} ms one after another")
    for c in ctxs:
        c.close()
    return res


def adjoint_leg(args, log_fn):
    """Gradient of the far-field energy W with respect to eps_r by the adjoint
    march, on the first cube of the batch workload with a side of at most 48
    (alpha = 4, 150 steps from t = 0, its own incidence): the times of the
    recorded forward march and of the adjoint march, and one directional
    central difference of W checking <grad W, v>."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2607_28309_amd import adjoint as A
    from paper_2607_28309_amd import native
    sc = next(s_ for s_ in W.cube_batch() if s_.n[0] <= 48)
    alpha, nt, tol = W.BATCH_ALPHA, W.BATCH_STEPS, 1e-10
    c = native.Context(*sc.n, alpha=alpha, precision="f64")
    eps0 = torch.from_numpy(sc.eps.ravel()).cuda()
    c.set_material(eps0)
    c.build_green_spectra()
    c.set_regularization(W.regularization_for(alpha))
    pulse = W.pulse(W.BATCH_PPW, k_hat=sc.k_hat, e_hat=sc.e_hat)
    rhat = [-v for v in sc.k_hat]  # backscatter
    march = A.FarFieldMarch(c, pulse, nt, rhat, tol=tol)
    e_t = eps0.clone().requires_grad_(True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    Wt = A.far_field_energy(e_t, march)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t
    t = time.perf_counter()
    Wt.backward()
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t
    g = e_t.grad.detach()
    # direction: seeded, unit norm; step h in eps_r
    v = torch.from_numpy(np.random.default_rng(7).standard_normal(c.N)).cuda()
    v /= torch.linalg.norm(v)
    h = 1e-3
    fd = (march.forward(eps0 + h * v) - march.forward(eps0 - h * v)) / (2 * h)
    ad = float(torch.dot(g, v))
    res = {"workload": f"cube{sc.n[0]}_a{alpha}_{nt}steps_backscatter", "unknowns": 3 * c.N,
           "nlags": c.info()["nlags"], "precision": "f64", "tol": tol, "W": float(Wt.item()),
           "forward_march_s": t_fwd, "adjoint_march_s": t_bwd, "grad_norm": float(torch.linalg.norm(g)),
           "directional_check": {"h": h, "central_difference": fd, "adjoint": ad,
                                 "rel_err": abs(fd - ad) / max(abs(ad), 1e-300)}}
    log_fn(f"adjoint gradient on {res['workload']}: forward {t_fwd:.2f} s, adjoint {t_bwd:.2f} s, "
           f"<grad, v> {ad:.6e} against central difference {fd:.6e}")
    c.close()
    return res


def _trace_march(args, name, eps_full_cut, ppw, log_fn):
    """The march of the workload of a stored oracle trace (tests/golden/
    oracle_trace_<name>.npz: the oracle's FP64 march from t = 0, TFQMR to
    1e-10) in the benchmark's precision: max_n ||J_n - J_n^ref|| /
    max_n ||J_n^ref|| on the trace's sampled voxels, and the largest relative
    difference of the full norms ||J_n||."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2607_28309_amd import native
    path = os.path.join(ROOT, "tests", "golden", f"oracle_trace_{name}.npz")
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        tr = {k: z[k] for k in z.files}
    nx, ny, nz = (int(v) for v in tr["shape"])
    alpha, steps = int(tr["alpha"]), int(tr["steps"])
    eps = np.ascontiguousarray(eps_full_cut)
    c = native.Context(nx, ny, nz, alpha=alpha, precision=args.precision)
    c.set_material(torch.from_numpy(eps.ravel()).cuda())
    c.build_green_spectra()
    dl = tuple(float(v) for v in np.atleast_1d(tr["delta"]))
    c.set_regularization(dl if len(dl) == 3 else dl[0])
    c.reset()
    p = W.pulse(ppw)
    L = alpha / math.sqrt(3.0)
    N3 = 3 * nx * ny * nz
    einc = torch.empty(N3, dtype=torch.float64, device="cuda")
    J = torch.empty(N3, dtype=torch.float64, device="cuda")
    idx = torch.from_numpy(tr["idx"].astype(np.int64)).cuda()
    ref = torch.from_numpy(tr["samples"]).cuda()
    num = den = nerr = 0.0
    for s in range(steps):
        c.excitation(p, s * L, einc)
        c.step(einc, J, tol=args.tol, stats=False)
        sub = J.view(3, -1)[:, idx]
        num = max(num, float(torch.linalg.vector_norm(sub - ref[s])))
        den = max(den, float(torch.linalg.vector_norm(ref[s])))
        nerr = max(nerr, abs(float(torch.linalg.vector_norm(J)) - float(tr["norms"][s])))
    c.close()
    res = {"value": num / den, "norms": nerr / float(tr["norms"].max()), "grid": [nx, ny, nz], "alpha": alpha,
           "steps": steps, "samples": int(len(tr["idx"])), "precision": args.precision, "tol": args.tol,
           "delta": [float(v) for v in np.atleast_1d(tr["delta"])]}
    log_fn(f"field error vs the FP64 oracle, {name} ({nx}x{ny}x{nz}, alpha {alpha}, {steps} steps): "
           f"{res['value']:.2e} (sampled voxels), {res['norms']:.2e} (norms)")
    return res


def oracle_trace_leg(args, log_fn):
    """Field error against the FP64 oracle on a 2x2-pillar cut (80 x 80 x 48)
    of the benchmarked array, dt = 16 dt_CFL, 120 steps from t = 0."""
    import workloads as W
    res = _trace_march(args, "pillars80", W.PILLARS.eps()[:, :80, :80], W.PILLARS.ppw, log_fn)
    if res is not None:
        res["workload"] = "pillars2x2_80x80x48_a16"
    return res


# a march whose current passes this magnitude has left the physical range (the
# incident field and the currents it drives are of order one) and is stopped
GROWTH_LIMIT = 1e6


def sweep_leg(args, log_fn):
    """Large-time-step sweep on the 96^3 nested cube (layers 6 / 4 / 2.5 by
    Chebyshev distance, +-5 % seeded noise, seed 3): dt = alpha * dt_CFL over
    one physical window of `--sweep-window` dt_CFL (window / alpha steps from
    t = 0), every step with its statistics.  Per alpha: lags (Eq. 4), Z0
    nonzeros from the mask, TFQMR iterations and products per step, solve
    (LHS) against right-hand-side (history) time per step, wall time of the
    window, the largest |J| per quarter of the window, the step at which the
    march left the physical range (|J| > GROWTH_LIMIT or a non-finite
    residual; the run of that alpha stops there), and the x current at the
    central voxel at the times all runs share, compared with that of the
    smallest alpha whose march stayed bounded."""
    import torch
    import workloads as W
    from paper_2607_28309_amd import native
    w = W.CUBE96
    n = w.n
    N = n[0] * n[1] * n[2]
    eps = torch.from_numpy(w.eps().ravel()).cuda()
    p = W.pulse(w.ppw)
    probe = n[0] // 2 + n[0] * (n[1] // 2 + n[1] * (n[2] // 2))   # x component, central voxel
    common = math.lcm(*args.sweep_alphas)
    rows, probes = [], {}

    def march(alpha, scheme):
        steps = args.sweep_window // alpha
        L = alpha / math.sqrt(3.0)
        t0 = time.perf_counter()
        c = native.Context(*n, alpha=alpha, precision=args.precision)
        c.set_material(eps)
        c.build_green_spectra()
        c.set_regularization(W.regularization_for(alpha))
        c.set_history_scheme(scheme)
        if not args.no_autotune:
            c.autotune(reps=5)
        c.reset()
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        info = c.info()
        E = torch.empty(3 * N, dtype=torch.float64, device="cuda")
        J = torch.empty_like(E)
        st, pr, amax = [], [], []
        diverged = None
        t = time.perf_counter()
        for k in range(steps):
            c.excitation(p, k * L, E)
            rc, s_ = c.step(E, J, tol=args.tol, allow=(native.MOT_ENONFINITE, native.MOT_ENOCONV))
            if rc != 0:
                diverged = k
                break
            st.append(s_)
            amax.append(float(J.abs().max()))
            if amax[-1] > GROWTH_LIMIT:
                diverged = k
                break
            if (k * alpha) % common == 0:
                pr.append(float(J[probe]))
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        done = len(st)
        mv = sum(s_["matvecs"] for s_ in st)
        q = max(steps // 4, 1)
        quarters = [max(amax[i:i + q], default=None) for i in range(0, steps, q)][:4]
        # bounded: ran the whole window and the last quarter stays below the
        # peak of the earlier ones (ringing after the pulse, no growth)
        bounded = diverged is None and len(quarters) == 4 and quarters[-1] <= max(quarters[:3])
        row = {"alpha": alpha, "delta": list(W.regularization_for(alpha)), "steps": steps, "steps_done": done,
               "history_scheme": {1: "blocked", 2: "fft_time"}[info["history_scheme"]],
               "diverged_at_step": diverged,
               "bounded": bounded, "max_abs_J_per_quarter": quarters,
               "nlags": info["nlags"], "z0_nnz": native.zk_nnz(*n, k=0, alpha=alpha),
               "history_block": info["history_block"], "device_bytes": info["bytes"], "setup_s": setup,
               "window_s": el, "steps_per_s": done / el,
               "iters_per_step": {"mean": sum(s_["iters"] for s_ in st) / max(done, 1),
                                  "max": max((s_["iters"] for s_ in st), default=0)},
               "matvecs_per_step": mv / max(done, 1),
               "ms_lhs_per_step": sum(s_["ms_lhs"] for s_ in st) / max(done, 1),
               "ms_rhs_per_step": sum(s_["ms_rhs"] for s_ in st) / max(done, 1),
               "ms_per_matvec_in_solve": sum(s_["ms_lhs"] for s_ in st) / max(mv, 1),
               "relres_max": max((s_["relres"] for s_ in st), default=None)}
        log_fn(f"sweep alpha {alpha} ({row['history_scheme']}): {done} of {steps} steps in {el:.2f} s "
               f"(diverged at {diverged}), ell {info['nlags']}, "
               f"{row['iters_per_step']['mean']:.2f} iterations/step, LHS {row['ms_lhs_per_step']:.2f} ms/step, "
               f"RHS {row['ms_rhs_per_step']:.2f} ms/step")
        c.close()
        del c
        torch.cuda.empty_cache()
        return row, pr

    for alpha in args.sweep_alphas:
        # the library's history scheme, then (--sweep-history both) the other
        # one where an FP32 ring of >= 32 lags allows both
        row, pr = march(alpha, args.sweep_history if args.sweep_history != "both" else "auto")
        row["default_scheme"] = args.sweep_history in ("auto", "both")
        rows.append(row)
        probes[alpha] = pr
        if args.sweep_history == "both" and args.precision != "f64" and row["nlags"] >= 32:
            other = "blocked" if row["history_scheme"] == "fft_time" else "fft_time"
            alt, _ = march(alpha, other)
            alt["default_scheme"] = False
            rows.append(alt)
    # the march's own time-step convergence, against the smallest alpha whose
    # current stayed bounded over the whole window
    main = [r for r in rows if r["default_scheme"]]
    ok = [r["alpha"] for r in main if r["bounded"]]
    a0 = min(ok) if ok else None
    if a0 is not None:
        ref = probes[a0]
        scale = max(abs(v) for v in ref) or 1.0
        for row in main:
            pr = probes[row["alpha"]]
            m = min(len(pr), len(ref))
            row["probe_diff_vs_ref"] = (max(abs(a - b) for a, b in zip(pr[:m], ref[:m])) / scale) if m else None
            h = min(m, len(ref) // 2)   # first half of the window: the pulse itself, before the ringing
            row["probe_diff_vs_ref_first_half"] = (max(abs(a - b) for a, b in zip(pr[:h], ref[:h])) /
                                                   (max(abs(v) for v in ref[:h]) or 1.0)) if h else None
    # the same sweep on a 24^3 cut of this medium against the FP64 oracle
    cut = w.eps()[24:48, 24:48, 24:48]
    for row in main:
        row["cut24_field_err_vs_oracle"] = _trace_march(args, f"nested24_a{row['alpha']}", cut, w.ppw, log_fn)
    return {"workload": "nested_cube_96x96x96_fixed_window", "precision": args.precision,
            "tol": args.tol, "window_dt_cfl": args.sweep_window, "probe": "J_x at voxel (48, 48, 48)",
            "probe_ref_alpha": a0, "rows": rows}


def sources_sha256(paths):
    """sha256 over the concatenated contents of the given repository files."""
    import hashlib
    h = hashlib.sha256()
    for rel in paths:
        h.update(open(os.path.join(ROOT, rel), "rb").read())
    return h.hexdigest()


def measured_traffic(kernel, variant=0):
    """HBM bytes per launch from the committed counter runs (entry
    "<kernel>/v<variant>"), or None when the kernel's sources changed since
    they were taken or none were taken for that tile variant."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(f"{kernel}/v{variant}")
    if not rec or rec.get("tile_variant", 0) != variant:
        return None
    if sources_sha256(rec["sources"]) != rec["sources_sha256"]:
        return None
    return rec["bytes_per_launch"]


def _cpu_name():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def counter_summary(path, counter):
    """Per-kernel averages of one rocprofv3 --pmc counter (KiB per dispatch)
    from the counter_collection.csv files under path, keyed "name|grid size"
    (one kernel runs on the grids of several workloads).  Dispatches launched
    behind a closed convergence gate end at once and move almost nothing:
    a dispatch counts when its value exceeds 20 % of the kernel's median."""
    import csv
    import glob
    import statistics
    files = glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True)
    per = {}
    for f in files:
        for r in csv.DictReader(open(f)):
            if r.get("Counter_Name") == counter:
                key = f'{r["Kernel_Name"]}|{r.get("Grid_Size", "")}'
                per.setdefault(key, []).append(float(r["Counter_Value"]))
    out = {}
    for k, vs in per.items():
        med = statistics.median(vs)
        kept = [v for v in vs if v > 0.2 * med] or vs
        out[k] = {"kib": statistics.mean(kept), "dispatches": len(kept), "all_dispatches": len(vs)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16,
                    help="timed steps (a multiple of the history block, 8, times whole blocks)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="f32_refined", choices=["f32_refined", "f64", "f32"])
    ap.add_argument("--matvec-reps", type=int, default=60, help="timed Z0 products per precision (median reported)")
    ap.add_argument("--f64-steps", type=int, default=8,
                    help="steps of the FP64 march timed after the main run (0 = skip; 8 = one whole history "
                         "block); its currents also give the field error of the main run against FP64")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--start-step", type=int, default=22, help="pulse time index of the first warm-up step")
    ap.add_argument("--graphs", type=int, default=0, choices=[0, 1, 2],
                    help="1: replay TFQMR iterations from HIP graphs; 2: the first refinement sweep of each step as "
                         "one graph (timing events stay off in the steps that replay it)")
    ap.add_argument("--history", default="auto", choices=["auto", "blocked", "fft_time"],
                    help="history scheme of the benchmarked march (auto: the library's choice)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batch of 32 independent cubes (sides 24..80, alpha 4) stepped together")
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint leg (gradient of the far-field energy on one cube of the batch, "
                         "with a directional central-difference check)")
    ap.add_argument("--sweep", action="store_true",
                    help="also run the time-step sweep on the 96^3 nested cube (alpha 1..16, one physical window)")
    ap.add_argument("--sweep-only", action="store_true", help="run only the time-step sweep and print its JSON line")
    ap.add_argument("--sweep-alphas", type=int, nargs="+", default=[1, 2, 4, 8, 16])
    ap.add_argument("--sweep-window", type=int, default=1600, help="window length in dt_CFL")
    ap.add_argument("--sweep-history", default="both", choices=["auto", "blocked", "fft_time", "both"],
                    help="history scheme of the sweep's marches (both: the library's choice, then the other one "
                         "where both are possible)")
    ap.add_argument("--time-every", type=int, default=4,
                    help="timed steps whose launches of the dominant kernel carry timing events: every n-th")
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="no timing events in the timed region (the roofline then uses the breakdown steps)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default FFT tile shapes instead of timing both variants per pass first")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy kernel three times "
                         "(reference for the HBM traffic counters) and exit")
    ap.add_argument("--counter-summary", nargs=3, metavar=("DIR", "COUNTER", "OUT"),
                    help="reduce the rocprofv3 --pmc csv output under DIR to per-kernel averages of COUNTER "
                         "(KiB per dispatch), write them to OUT as JSON and exit (no GPU)")
    args = ap.parse_args()
    if args.counter_summary:
        d, cnt, out = args.counter_summary
        json.dump(counter_summary(d, cnt), open(out, "w"), indent=1)
        return
    if args.gpus != 1:
        print(f"bench.py runs the single-GPU path only; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as W
    from paper_2607_28309_amd import native

    if args.copy_calibration:
        a = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 4, "launches": 3}))
        return

    torch.cuda.set_device(0)
    if args.sweep_only:
        print(json.dumps({"sweep": sweep_leg(args, log)}), flush=True)
        return

    w = W.PILLARS
    n = w.n
    eps = w.eps()
    N = n[0] * n[1] * n[2]
    t0 = time.perf_counter()
    ctx = native.Context(*n, alpha=w.alpha, precision=args.precision)
    ctx.set_material(torch.from_numpy(eps.ravel()).cuda())
    log(f"context: {ctx.info()}")
    imag = ctx.build_green_spectra()
    ctx.set_regularization(W.regularization_for(w.alpha))
    ctx.set_history_scheme(args.history)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    info = ctx.info()
    nl = info["nlags"]
    log(f"spectra built in {setup_s:.1f} s (ell = {nl}, max |Im| = {imag:.2e})")
    tune_ms, tune_s = None, 0.0
    if not args.no_autotune:
        t0 = time.perf_counter()
        tune_ms = ctx.autotune()
        tune_s = time.perf_counter() - t0
        log(f"autotuned tile variants in {tune_s:.2f} s: {ctx.variants()}")
    variants = ctx.variants()

    # start the march at step ell with J_m = 0 before it: every step multiplies all ell lags
    ctx.reset()
    ctx.set_step(nl)
    p = W.pulse(w.ppw)
    L = w.alpha / math.sqrt(3.0)
    einc = torch.empty(3 * N, dtype=torch.float64, device="cuda")
    # step sequence: warm-up, breakdown (untimed, every kernel timed), timed region
    nbd = info["history_block"]  # one history block: exactly one block-start step
    first_timed = args.warmup + nbd
    # one output vector per step, so that the currents can be compared with an FP64 march afterwards
    n_keep = first_timed + min(args.steps, args.f64_steps)
    Js = [torch.empty(3 * N, dtype=torch.float64, device="cuda") for _ in range(n_keep)]
    J_spare = torch.empty(3 * N, dtype=torch.float64, device="cuda")

    def one_step(c, s, wait=True):
        """One step; wait=False: no device wait at its end (the statistics
        then carry no LHS/RHS times)."""
        c.excitation(p, (args.start_step + s) * L, einc)
        st = c.step(einc, Js[s] if s < n_keep else J_spare, tol=args.tol, stats=wait)[1]
        return st if wait else c.last_stats()

    for s in range(args.warmup):
        st = one_step(ctx, s)
        log(f"warm-up step {s}: {st['iters']} iterations, relres {st['relres']:.2e}")
    # breakdown over one history block (B = 8 steps for an FP32 ring): every
    # kernel timed; it names the dominant single kernel
    ctx.profile_kinds(None)
    ctx.profile(True)
    ctx.profile_read()
    bd_stats = [one_step(ctx, args.warmup + s) for s in range(nbd)]
    breakdown = ctx.profile_read()
    ctx.profile(False)
    dom = max(((k, pr, ms, cnt) for (k, pr), (ms, cnt) in breakdown.items() if k in ROOFLINE_KINDS),
              key=lambda r: r[2])
    log(f"dominant kernel over {nbd} steps: {dom[0]}.{dom[1]} ({dom[2] / nbd:.2f} ms/step)")
    if args.graphs:
        ctx.set_graphs(args.graphs)
    # inside the timed region only the dominant kernel carries timing events,
    # in every `--time-every`-th step (an event pair leaves the device idle
    # for a few microseconds on each side of the launch it brackets)
    sampled = [s for s in range(args.steps) if s % max(args.time_every, 1) == 0]
    ctx.profile_kinds([])
    ctx.profile(not args.no_kernel_timing)
    ctx.profile_read()
    torch.cuda.synchronize()
    t = time.perf_counter()
    stats = []
    # the timed steps do not wait for each other: each returns with its
    # history update in flight, and the next one's launches queue behind it
    for s in range(args.steps):
        ctx.profile_kinds([dom[0]] if s in sampled else [])
        stats.append(one_step(ctx, first_timed + s, wait=False))
        log(f"step {s}: {stats[-1]['iters']} it, {stats[-1]['matvecs']} mv "
            f"({stats[-1]['matvecs_f64']} f64), relres {stats[-1]['relres']:.2e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t
    prof = ctx.profile_read()
    ctx.profile(False)
    ms_per_step = 1e3 * elapsed / args.steps

    # Z0 product throughput (FP32 and FP64) on the context's stream (torch's
    # current stream): five rounds of reps products back to back between one
    # event pair, as the solver issues them (ms = the median round's average;
    # the first round after the march runs at lower clocks); then one event
    # pair per product (median)
    mv = {}
    reps = max(args.matvec_reps, 1)
    for dt_name, tdt in (("f32", torch.float32), ("f64", torch.float64)):
        Jm = torch.randn(3 * N, dtype=tdt, device="cuda")
        ym = torch.empty_like(Jm)
        for _ in range(10):
            ctx.z0_matvec(Jm, ym, dt_name)
        rounds = []
        for _ in range(5):
            s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s0.record()
            for _ in range(reps):
                ctx.z0_matvec(Jm, ym, dt_name)
            s1.record()
            rounds.append((s0, s1))
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for e0, e1 in ev:
            e0.record()
            ctx.z0_matvec(Jm, ym, dt_name)
            e1.record()
        torch.cuda.synchronize()
        ms = sorted(a.elapsed_time(b) / reps for a, b in rounds)[len(rounds) // 2]
        times = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
        mv[dt_name] = {"ms": ms, "per_s": 1e3 / ms, "reps": reps, "ms_event_pairs_median": times[len(times) // 2]}
        log(f"z0_matvec {dt_name}: {ms:.4f} ms back to back over {reps} "
            f"(one event pair per product: median {times[len(times) // 2]:.4f} ms)")
        del Jm, ym

    # roofline of the dominant kernel (the largest share of a history block
    # among the passes whose launches are all the same kernel), timed live in
    # the timed region
    ring_t = 8 if args.precision == "f64" else 4
    kernels = {}
    for (kind, prec), (ms, cnt) in breakdown.items():
        # enqueued launches include those behind a closed convergence gate
        kernels[f"{kind}.{prec}"] = {"ms_per_step": round(ms / nbd, 3), "enqueued_per_step": cnt / nbd}
    if args.no_kernel_timing:
        kind, prec, ms, cnt = dom
        steps_counted, st_counted = nbd, None
    else:
        (kind, prec), (ms, cnt) = max(((k, v) for k, v in prof.items() if k[0] == dom[0]), key=lambda r: r[1][0])
        steps_counted, st_counted = len(sampled), [stats[s] for s in sampled]
    # Launches of the product passes behind a closed convergence gate end at
    # once; the device counts the products that ran (one launch of each pass
    # each), so the average is the class's whole time over those.
    if st_counted is not None and kind in ("z_fused", "y_forward", "y_inverse"):
        ran = sum(x["matvecs_f64"] if prec == "f64" else x["matvecs"] - x["matvecs_f64"] for x in st_counted)
        if kind != "z_fused":
            ran += steps_counted  # the history update's pass (never gated)
        if 0 < ran <= cnt:
            cnt = ran
    tb = 8 if prec == "f64" else 4
    if kind == "history_mac":
        tb = ring_t
    # the history pass at a block start writes the partial sums of the B steps of a block
    alg = algorithmic_bytes(kind, n, tb, tb, nl, blk=info["history_block"])
    avg_s = ms / cnt / 1e3
    achieved = alg / avg_s / 1e9
    knob = {"z_fused": "z_fused", "y_forward": "y", "y_inverse": "y"}.get(kind)
    var = variants[prec][knob] if knob else 0
    roofline = {"bound": "hbm", "kernel": f"{kind}.{prec}", "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": measured_traffic(f"{kind}.{prec}", var),
                "algorithmic_bytes_per_launch": alg, "avg_launch_ms": ms / cnt, "tile_variant": var,
                "launches_timed": cnt,
                "timed_steps": (f"{len(sampled)} of the {args.steps} timed steps (every {args.time_every}-th)"
                                if not args.no_kernel_timing else f"the {nbd} breakdown steps")}
    # Z0 pipeline as a whole (five passes)
    pipe_bytes = sum(algorithmic_bytes(k, n, 4, 4, nl) for k in
                     ("x_forward", "y_forward", "z_fused", "y_inverse", "x_inverse_epilogue"))

    its = [s["iters"] for s in stats]
    out = {
        "metric": "Z0 FFT-matvecs/s + MOT steps/s at 15M unknowns; achieved HBM GB/s vs peak",
        "value": args.steps / elapsed,
        "unit": "MOT steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision != "f64" else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "grid": list(n), "unknowns": 3 * N, "alpha": w.alpha, "nlags": nl,
                   "delta": list(W.regularization_for(w.alpha)), "precision": args.precision, "tol": args.tol,
                   "history_scheme": {1: "blocked", 2: "fft_time"}[info["history_scheme"]],
                   "parallelism": "single GPU"},
        "z0_matvecs_per_s": {k: v["per_s"] for k, v in mv.items()},
        "z0_matvec_ms": {k: v["ms"] for k, v in mv.items()},
        "z0_matvec_ms_event_pairs": {k: v["ms_event_pairs_median"] for k, v in mv.items()},
        "z0_pipeline_gbs_f32": pipe_bytes / (mv["f32"]["ms"] / 1e3) / 1e9,
        "z0_pipeline_frac_f32": pipe_bytes / (mv["f32"]["ms"] / 1e3) / 8e12,
        "iters_per_step": {"min": min(its), "max": max(its), "mean": sum(its) / len(its)},
        "matvecs_per_step": sum(s["matvecs"] for s in stats) / len(stats),
        "relres_max": max(s["relres"] for s in stats),
        # LHS and RHS times of Eq. 6 from the breakdown steps (one history block)
        "ms_lhs_mean": sum(s["ms_lhs"] for s in bd_stats) / len(bd_stats),
        "ms_rhs_mean": sum(s["ms_rhs"] for s in bd_stats) / len(bd_stats),
        "setup_s": setup_s,
        "autotune_s": tune_s,
        "tile_variants": variants,
        "autotune_ms": tune_ms,
        "roofline": roofline,
        "kernels": kernels,
    }
    ctx.close()
    del ctx
    if args.f64_steps > 0:
        out.update(f64_march(args, w, eps, p, L, Js, n_keep, log))
    out["field_err_vs_oracle"] = oracle_trace_leg(args, log)
    if not args.no_batch:
        out["batch"] = batch_leg(args, log)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_leg(args, log)
    if args.sweep:
        out["sweep"] = sweep_leg(args, log)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, eps, out["matvecs_per_step"], nl, log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
