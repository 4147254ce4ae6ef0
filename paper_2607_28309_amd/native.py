"""ctypes binding of libmotjvie.so (argument marshalling only).

Every computation runs in the HIP library; this module converts torch
tensors to device pointers and the library's status codes to exceptions.
Importing it loads the library and fails loudly if it is missing: there is
no CPU fallback.
"""

import ctypes
import os

# torch ships its own HIP runtime: load it before the library so that the
# library binds to that runtime (loading the library first would pull in a
# second copy from the system ROCm, whose device memory and streams are not
# torch's)
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmotjvie.so")

MOT_OK, MOT_EINVAL, MOT_ENOMEM, MOT_EHIP, MOT_ENOCONV, MOT_EBREAKDOWN, MOT_ENONFINITE, MOT_ESTATE = (
    0, -1, -2, -3, -4, -5, -6, -7)
MOT_F64, MOT_F32, MOT_F32_REFINED = 0, 1, 2
PRECISIONS = {"f64": MOT_F64, "f32": MOT_F32, "f32_refined": MOT_F32_REFINED}

EXPORTS = (
    "mot_create", "mot_destroy", "mot_info", "build_green_spectra", "mot_spectra_imag",
    "mot_set_material", "z0_matvec", "gk_matvec", "history_update", "mot_get_history_rhs",
    "mot_excitation", "mot_step", "mot_reset", "mot_green_table", "mot_nlags", "mot_zk_nnz",
    "mot_length_supported", "mot_strerror", "mot_last_error", "mot_profile", "mot_profile_read",
    "mot_set_step", "mot_set_adjoint", "z0t_matvec", "mot_history_gfield", "mot_farfield",
    "mot_farfield_adjoint", "mot_adjoint_gradient", "mot_profile_kinds", "mot_set_graphs", "mot_step_batch",
    "mot_set_variants", "mot_get_variants", "mot_autotune", "mot_set_predictor", "mot_set_regularization",
    "mot_farfield_static", "mot_set_history_scheme", "mot_set_wide_offsets", "mot_set_breakdown_tolerance", "mot_last_stats",
)
TUNE_KNOBS = ("x", "y", "z_history", "z_fused")
PROF_NCLASS = 24
PROF_KINDS = ("x_forward", "y_forward", "z_fused", "y_inverse", "x_inverse_epilogue", "z_forward",
              "history_mac", "z_inverse", "krylov", "excitation", "history_mac_recent", "history_far")


class MotGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("alpha", ctypes.c_int32), ("cdt", ctypes.c_double), ("nlags", ctypes.c_int32),
                ("quad", ctypes.c_int32)]


class MotStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("matvecs", ctypes.c_int32), ("matvecs_f64", ctypes.c_int32),
                ("refinements", ctypes.c_int32), ("relres", ctypes.c_double), ("ms_lhs", ctypes.c_double),
                ("ms_rhs", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class MotPulse(ctypes.Structure):
    _fields_ = [("e", ctypes.c_double * 3), ("k", ctypes.c_double * 3), ("f0", ctypes.c_double),
                ("sigma", ctypes.c_double), ("t0", ctypes.c_double), ("amp", ctypes.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2607_28309_amd/build.py (or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "mot_create": (ctypes.c_int, [ctypes.POINTER(MotGrid), ctypes.c_int, vp, ctypes.POINTER(vp)]),
        "mot_destroy": (ctypes.c_int, [vp]),
        "mot_info": (ctypes.c_int, [vp, ctypes.POINTER(i64), i32]),
        "build_green_spectra": (ctypes.c_int, [vp]),
        "mot_spectra_imag": (dbl, [vp]),
        "mot_set_material": (ctypes.c_int, [vp, vp]),
        "z0_matvec": (ctypes.c_int, [vp, vp, vp, ctypes.c_int]),
        "gk_matvec": (ctypes.c_int, [vp, i32, vp, vp, ctypes.c_int]),
        "history_update": (ctypes.c_int, [vp, vp]),
        "mot_get_history_rhs": (ctypes.c_int, [vp, vp]),
        "mot_excitation": (ctypes.c_int, [vp, ctypes.POINTER(MotPulse), dbl, vp]),
        "mot_step": (ctypes.c_int, [vp, vp, vp, dbl, i32, ctypes.POINTER(MotStats)]),
        "mot_last_stats": (ctypes.c_int, [vp, ctypes.POINTER(MotStats)]),
        "mot_reset": (ctypes.c_int, [vp]),
        "mot_set_step": (ctypes.c_int, [vp, i64]),
        "mot_green_table": (ctypes.c_int, [vp, i32, vp]),
        "mot_nlags": (i32, [ctypes.POINTER(MotGrid)]),
        "mot_zk_nnz": (i64, [ctypes.POINTER(MotGrid), i32]),
        "mot_length_supported": (i32, [i32]),
        "mot_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "mot_profile": (ctypes.c_int, [vp, i32]),
        "mot_profile_read": (ctypes.c_int, [vp, ctypes.POINTER(dbl), ctypes.POINTER(i64), i32]),
        "mot_last_error": (ctypes.c_char_p, [vp]),
        "mot_set_adjoint": (ctypes.c_int, [vp, i32]),
        "mot_profile_kinds": (ctypes.c_int, [vp, i32]),
        "mot_set_graphs": (ctypes.c_int, [vp, i32]),
        "mot_step_batch": (ctypes.c_int, [ctypes.POINTER(vp), i32, ctypes.POINTER(vp), ctypes.POINTER(vp), dbl, i32,
                                          ctypes.POINTER(MotStats), ctypes.POINTER(i32), i32]),
        "z0t_matvec": (ctypes.c_int, [vp, vp, vp, ctypes.c_int]),
        "mot_history_gfield": (ctypes.c_int, [vp, vp]),
        "mot_farfield": (ctypes.c_int, [vp, vp, i32, ctypes.POINTER(dbl), i32, i32, vp, vp]),
        "mot_farfield_static": (ctypes.c_int, [vp, vp, i32, ctypes.POINTER(dbl), i32, i32, vp, vp]),
        "mot_farfield_adjoint": (ctypes.c_int, [vp, vp, i32, i32, ctypes.POINTER(dbl), dbl, i64, vp]),
        "mot_adjoint_gradient": (ctypes.c_int, [vp, ctypes.POINTER(MotPulse), dbl, vp, vp, vp, vp, vp, vp, vp]),
        "mot_set_variants": (ctypes.c_int, [vp, ctypes.POINTER(i32)]),
        "mot_get_variants": (ctypes.c_int, [vp, ctypes.POINTER(i32)]),
        "mot_autotune": (ctypes.c_int, [vp, i32, ctypes.POINTER(dbl)]),
        "mot_set_predictor": (ctypes.c_int, [vp, i32]),
        "mot_set_regularization": (ctypes.c_int, [vp, dbl, dbl, dbl]),
        "mot_set_history_scheme": (ctypes.c_int, [vp, i32]),
        "mot_set_wide_offsets": (ctypes.c_int, [vp, i32]),
        "mot_set_breakdown_tolerance": (ctypes.c_int, [vp, dbl]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


LIB = _load()


def step_batch(contexts, eincs, Js, tol=1e-6, max_iter=1000, threads=None, allow=()):
    """One MOT step of every context (each on its own stream) by a pool of host
    threads inside the library (default min(contexts, 8): more threads than
    that contend for the device's few hardware queues); returns (statuses,
    stats dicts)."""
    import torch
    n = len(contexts)
    if not (len(eincs) == len(Js) == n) or n == 0:
        raise ValueError("one excitation and one current vector per context")
    ctxs = (ctypes.c_void_p * n)(*[c.h for c in contexts])
    e = (ctypes.c_void_p * n)(*[_ptr(x, torch.float64, 3 * c.N) for x, c in zip(eincs, contexts)])
    j = (ctypes.c_void_p * n)(*[_ptr(x, torch.float64, 3 * c.N) for x, c in zip(Js, contexts)])
    st = (MotStats * n)()
    status = (ctypes.c_int32 * n)()
    rc = LIB.mot_step_batch(ctxs, n, e, j, float(tol), int(max_iter), st, status, int(threads or min(n, 8)))
    if rc != MOT_OK and rc not in allow:
        bad = [i for i in range(n) if status[i] != MOT_OK and status[i] not in allow]
        if bad:
            i = bad[0]
            raise MotError(status[i], f"mot_step_batch, context {i}: {LIB.mot_last_error(contexts[i].h).decode()}")
    return list(status), [s.as_dict() for s in st]


class MotError(RuntimeError):
    def __init__(self, status, detail):
        self.status = status
        super().__init__(f"{LIB.mot_strerror(status).decode()} ({status}): {detail}")


def make_pulse(pulse):
    """MotPulse from a dict with keys e, k, f0, sigma, t0 (and amp, default 1)."""
    return MotPulse((ctypes.c_double * 3)(*[float(v) for v in pulse["e"]]),
                    (ctypes.c_double * 3)(*[float(v) for v in pulse["k"]]),
                    float(pulse["f0"]), float(pulse["sigma"]), float(pulse["t0"]), float(pulse.get("amp", 1.0)))


def make_grid(nx, ny, nz, alpha=0, cdt=0.0, nlags=0, quad=0):
    return MotGrid(int(nx), int(ny), int(nz), int(alpha), float(cdt), int(nlags), int(quad))


def nlags(nx, ny, nz, alpha=0, cdt=0.0):
    return int(LIB.mot_nlags(ctypes.byref(make_grid(nx, ny, nz, alpha, cdt))))


def zk_nnz(nx, ny, nz, k=0, alpha=0, cdt=0.0):
    return int(LIB.mot_zk_nnz(ctypes.byref(make_grid(nx, ny, nz, alpha, cdt)), int(k)))


def length_supported(n):
    return bool(LIB.mot_length_supported(int(n)))


def _ptr(t, dtype, numel):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("expected a device tensor")
    if t.dtype != dtype or not t.is_contiguous() or t.numel() != numel:
        raise ValueError(f"expected a contiguous {dtype} tensor of {numel} elements, got {t.dtype} "
                         f"{tuple(t.shape)} contiguous={t.is_contiguous()}")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """One solver context on one stream (torch's current stream by default)."""

    def __init__(self, nx, ny, nz, alpha=0, cdt=0.0, precision="f64", nlags=0, quad=0, stream=None):
        import torch
        self.shape = (int(nx), int(ny), int(nz))
        self.precision = precision
        self.grid = make_grid(nx, ny, nz, alpha, cdt, nlags, quad)
        self.N = self.shape[0] * self.shape[1] * self.shape[2]
        s = stream if stream is not None else torch.cuda.current_stream()
        self.stream = s
        h = ctypes.c_void_p()
        rc = LIB.mot_create(ctypes.byref(self.grid), PRECISIONS[precision], ctypes.c_void_p(s.cuda_stream),
                            ctypes.byref(h))
        if rc != MOT_OK:
            raise MotError(rc, "mot_create")
        self.h = h

    def _check(self, rc, what, allow=()):
        if rc != MOT_OK and rc not in allow:
            raise MotError(rc, f"{what}: {LIB.mot_last_error(self.h).decode()}")
        return rc

    def close(self):
        if getattr(self, "h", None):
            LIB.mot_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        out = (ctypes.c_int64 * 9)()
        self._check(LIB.mot_info(self.h, out, 9), "mot_info")
        keys = ("nlags", "px", "py", "pz", "kxs", "bytes", "steps", "history_block", "history_scheme")
        return dict(zip(keys, list(out)))

    def build_green_spectra(self):
        self._check(LIB.build_green_spectra(self.h), "build_green_spectra")
        return float(LIB.mot_spectra_imag(self.h))

    def set_material(self, eps):
        import torch
        self._check(LIB.mot_set_material(self.h, _ptr(eps, torch.float64, self.N)), "mot_set_material")

    def z0_matvec(self, J, y, dtype="f64"):
        import torch
        tdt = torch.float32 if dtype == "f32" else torch.float64
        self._check(LIB.z0_matvec(self.h, _ptr(J, tdt, 3 * self.N), _ptr(y, tdt, 3 * self.N), PRECISIONS[dtype]),
                    "z0_matvec")

    def gk_matvec(self, k, J, y, dtype="f64"):
        import torch
        tdt = torch.float32 if dtype == "f32" else torch.float64
        self._check(LIB.gk_matvec(self.h, int(k), _ptr(J, tdt, 3 * self.N), _ptr(y, tdt, 3 * self.N),
                                  PRECISIONS[dtype]), "gk_matvec")

    def history_update(self, J):
        import torch
        self._check(LIB.history_update(self.h, _ptr(J, torch.float64, 3 * self.N)), "history_update")

    def history_rhs(self, out):
        import torch
        self._check(LIB.mot_get_history_rhs(self.h, _ptr(out, torch.float64, 3 * self.N)), "mot_get_history_rhs")

    def excitation(self, pulse, t, out):
        import torch
        p = make_pulse(pulse)
        self._check(LIB.mot_excitation(self.h, ctypes.byref(p), float(t), _ptr(out, torch.float64, 3 * self.N)),
                    "mot_excitation")

    def set_graphs(self, on=True):
        """on: False/0 stream launches, True/1 TFQMR iterations from graphs,
        2 the refined solve's first sweep as one graph per step."""
        mode = int(on) if not isinstance(on, bool) else (1 if on else 0)
        self._check(LIB.mot_set_graphs(self.h, mode), "mot_set_graphs")

    def set_adjoint(self, on=True):
        self._check(LIB.mot_set_adjoint(self.h, 1 if on else 0), "mot_set_adjoint")

    def set_regularization(self, delta):
        """Regularization (d_0, d_1, d_2) of Z_0, Z_1, Z_2, or a number d for (d, -d, 0)
        (0 = the unregularized operator)."""
        import numpy as np
        d = (float(delta), -float(delta), 0.0) if np.ndim(delta) == 0 else tuple(float(v) for v in delta)
        if len(d) != 3:
            raise ValueError("delta: a number or (d_0, d_1, d_2)")
        self._check(LIB.mot_set_regularization(self.h, *d), "mot_set_regularization")

    def set_history_scheme(self, scheme):
        """History sums: "auto" (0), "blocked" (1, per-lag multiply-accumulate) or
        "fft_time" (2, far lags by FFTs in time over blocks of 32 steps)."""
        code = {"auto": 0, "blocked": 1, "fft_time": 2}.get(scheme, scheme)
        self._check(LIB.mot_set_history_scheme(self.h, int(code)), "mot_set_history_scheme")

    def set_wide_offsets(self, on):
        """Force (True) or release (False) the 64-bit address form of the FP32
        blocked history multiply-accumulate; both give the same sums bit for bit."""
        self._check(LIB.mot_set_wide_offsets(self.h, int(bool(on))), "mot_set_wide_offsets")

    def set_breakdown_tolerance(self, t):
        """TFQMR stops as broken down when |rho| or |sigma| <= t |b|^2 (0: exact zero only)."""
        self._check(LIB.mot_set_breakdown_tolerance(self.h, float(t)), "mot_set_breakdown_tolerance")

    def set_predictor(self, k):
        """Initial guess of the refined solve from the last k solutions (0 = off)."""
        self._check(LIB.mot_set_predictor(self.h, int(k)), "mot_set_predictor")

    def variants(self):
        """{"f32": {knob: 0|1}, "f64": {...}} of the FFT pass tile shapes."""
        v = (ctypes.c_int32 * 8)()
        self._check(LIB.mot_get_variants(self.h, v), "mot_get_variants")
        return {p: {k: int(v[4 * i + j]) for j, k in enumerate(TUNE_KNOBS)} for i, p in enumerate(("f32", "f64"))}

    def set_variants(self, variants):
        """variants: 8 ints ([FP32 knobs, FP64 knobs], knob order TUNE_KNOBS)
        or a dict as returned by ``variants``."""
        if isinstance(variants, dict):
            variants = [variants[p][k] for p in ("f32", "f64") for k in TUNE_KNOBS]
        if len(variants) != 8:
            raise ValueError("8 variants: 4 knobs for FP32 and 4 for FP64")
        v = (ctypes.c_int32 * 8)(*[int(x) for x in variants])
        self._check(LIB.mot_set_variants(self.h, v), "mot_set_variants")

    def autotune(self, reps=0):
        """Time both tile variants of every knob on this grid and keep the
        faster; returns {"f32"|"f64": {knob: [ms variant 0, ms variant 1] or None}}."""
        ms = (ctypes.c_double * 16)()
        self._check(LIB.mot_autotune(self.h, int(reps), ms), "mot_autotune")
        out = {}
        for i, p in enumerate(("f32", "f64")):
            out[p] = {}
            for j, k in enumerate(TUNE_KNOBS):
                a, b = ms[2 * (4 * i + j)], ms[2 * (4 * i + j) + 1]
                out[p][k] = [a, b] if a >= 0 else None
        return out

    def z0t_matvec(self, v, y, dtype="f64"):
        import torch
        tdt = torch.float32 if dtype == "f32" else torch.float64
        self._check(LIB.z0t_matvec(self.h, _ptr(v, tdt, 3 * self.N), _ptr(y, tdt, 3 * self.N), PRECISIONS[dtype]),
                    "z0t_matvec")

    def history_gfield(self, out):
        import torch
        self._check(LIB.mot_history_gfield(self.h, _ptr(out, torch.float64, 3 * self.N)), "mot_history_gfield")

    def farfield(self, Jhist, rhat, j0, nj, e, energy=None):
        import torch
        nsteps = Jhist.numel() // (3 * self.N)
        r = (ctypes.c_double * 3)(*[float(v) for v in rhat])
        en = _ptr(energy, torch.float64, 1) if energy is not None else None
        self._check(LIB.mot_farfield(self.h, _ptr(Jhist, torch.float64, nsteps * 3 * self.N), int(nsteps), r,
                                     int(j0), int(nj), _ptr(e, torch.float64, 3 * int(nj)), en), "mot_farfield")

    def farfield_static(self, Jhist, rhat, j0, nj, e, energy=None):
        """mot_farfield without any device allocation (partials in the library's static array)."""
        import torch
        nsteps = Jhist.numel() // (3 * self.N)
        r = (ctypes.c_double * 3)(*[float(v) for v in rhat])
        en = _ptr(energy, torch.float64, 1) if energy is not None else None
        self._check(LIB.mot_farfield_static(self.h, _ptr(Jhist, torch.float64, nsteps * 3 * self.N), int(nsteps),
                                            r, int(j0), int(nj), _ptr(e, torch.float64, 3 * int(nj)), en),
                    "mot_farfield_static")

    def farfield_adjoint(self, w, j0, rhat, n, g_n, scale=1.0):
        import torch
        nj = w.numel() // 3
        r = (ctypes.c_double * 3)(*[float(v) for v in rhat])
        self._check(LIB.mot_farfield_adjoint(self.h, _ptr(w, torch.float64, 3 * nj), int(j0), int(nj), r,
                                             float(scale), int(n), _ptr(g_n, torch.float64, 3 * self.N)),
                    "mot_farfield_adjoint")

    def adjoint_gradient(self, pulse, t, lam_n, J_n, J_prev, uh_n, u0_n, grad, J_prev2=None):
        import torch
        p = make_pulse(pulse)
        v3 = 3 * self.N
        jp = _ptr(J_prev, torch.float64, v3) if J_prev is not None else None
        jp2 = _ptr(J_prev2, torch.float64, v3) if J_prev2 is not None else None
        self._check(LIB.mot_adjoint_gradient(self.h, ctypes.byref(p), float(t), _ptr(lam_n, torch.float64, v3),
                                             _ptr(J_n, torch.float64, v3), jp, jp2, _ptr(uh_n, torch.float64, v3),
                                             _ptr(u0_n, torch.float64, v3), _ptr(grad, torch.float64, self.N)),
                    "mot_adjoint_gradient")

    def step(self, einc, J, tol=1e-6, max_iter=1000, stats=True, allow=()):
        """One MOT step; returns (status, stats dict or None)."""
        import torch
        st = MotStats() if stats else None
        rc = LIB.mot_step(self.h, _ptr(einc, torch.float64, 3 * self.N), _ptr(J, torch.float64, 3 * self.N),
                          float(tol), int(max_iter), ctypes.byref(st) if st is not None else None)
        self._check(rc, "mot_step", allow=allow)
        return rc, (st.as_dict() if st is not None else None)

    def last_stats(self):
        """Statistics of the last step (no device wait; ms_lhs and ms_rhs are
        -1 when it ran without stats)."""
        st = MotStats()
        self._check(LIB.mot_last_stats(self.h, ctypes.byref(st)), "mot_last_stats")
        return st.as_dict()

    def reset(self):
        self._check(LIB.mot_reset(self.h), "mot_reset")

    def set_step(self, n):
        self._check(LIB.mot_set_step(self.h, int(n)), "mot_set_step")

    def profile(self, enable=True):
        self._check(LIB.mot_profile(self.h, 1 if enable else 0), "mot_profile")

    def profile_kinds(self, kinds=None):
        """Time only the given kinds (names of PROF_KINDS); None = all."""
        mask = (1 << len(PROF_KINDS)) - 1 if kinds is None else sum(1 << PROF_KINDS.index(k) for k in kinds)
        self._check(LIB.mot_profile_kinds(self.h, int(mask)), "mot_profile_kinds")

    def profile_read(self):
        """{(kind, 'f32'|'f64'): (ms, launches)} accumulated since the last read."""
        ms = (ctypes.c_double * PROF_NCLASS)()
        cnt = (ctypes.c_int64 * PROF_NCLASS)()
        self._check(LIB.mot_profile_read(self.h, ms, cnt, PROF_NCLASS), "mot_profile_read")
        out = {}
        for i in range(PROF_NCLASS):
            if cnt[i]:
                out[(PROF_KINDS[i // 2], "f64" if i % 2 else "f32")] = (float(ms[i]), int(cnt[i]))
        return out

    def green_table(self, k, out):
        import torch
        self._check(LIB.mot_green_table(self.h, int(k), _ptr(out, torch.float64, 6 * self.N)), "mot_green_table")
