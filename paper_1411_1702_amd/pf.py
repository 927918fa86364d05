"""Python binding of the C ABI in include/pf.h and include/pf_test.h.

Argument marshalling only: every step of the filter runs in the HIP library.
The library must be built (paper_1411_1702_amd/build.py); loading fails
loudly otherwise -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpf_hip.so")

PF_OK, PF_EINVAL, PF_ENOMEM, PF_EADMIT, PF_EDEGENERATE = 0, 1, 2, 3, 4
PF_ENONFINITE, PF_EDEVICE, PF_EBUSY, PF_EORDER = 5, 6, 7, 8
PF_MODEL_ROBERTSON, PF_MODEL_CHAIN16, PF_MODEL_ADVDIFF = 1, 2, 3
PF_LMM_BDF, PF_LMM_AM, PF_LMM_BDF_SDIRK = 0, 1, 2
PF_PREC_FP64, PF_PREC_FP32_PROP = 0, 1
PF_RESAMPLE_SYSTEMATIC, PF_RESAMPLE_MULTINOMIAL = 0, 1
PF_TIME_STEP, PF_TIME_PREDICT, PF_TIME_RESAMPLE, PF_TIME_UPDATE, PF_TIME_MOMENTS = 0, 1, 2, 3, 4

EXPORTS = [
    "pf_context_create", "pf_context_destroy", "pf_filter_bytes", "pf_context_memory",
    "pf_create", "pf_assimilate", "pf_assimilate_async", "pf_wait", "pf_assimilate_batch",
    "pf_posterior", "pf_stats", "pf_destroy", "pf_status_str", "pf_last_error",
    "pf_context_profile", "pf_context_kernel_time", "pf_context_autotune", "pf_context_launch_grid", "pf_query",
    "pf_server_create", "pf_server_open", "pf_server_submit", "pf_server_poll", "pf_server_posterior",
    "pf_server_close", "pf_server_drain", "pf_server_stats", "pf_server_destroy", "pf_resample_noalloc",
    "pf_test_philox", "pf_test_normals", "pf_test_propagate", "pf_test_resample", "pf_test_resample_multinomial",
    "pf_test_get_ensemble", "pf_test_set_ensemble", "pf_test_last_ancestors", "pf_test_moments",
]


class PfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class pf_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


class pf_config(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("model", C.c_int), ("d", C.c_uint32), ("p", C.c_uint32),
        ("m", C.c_uint32), ("obs_index", C.POINTER(C.c_uint32)),
        ("model_consts", C.POINTER(C.c_double)), ("n_model_consts", C.c_uint32),
        ("rates_fixed", C.POINTER(C.c_double)), ("n_rates_fixed", C.c_uint32),
        ("n_particles", C.c_uint64), ("seed", C.c_uint64), ("t0", C.c_double),
        ("x0", C.POINTER(C.c_double)), ("prior_mean", C.POINTER(C.c_double)),
        ("prior_sd", C.POINTER(C.c_double)), ("shrink_a", C.c_double), ("lmm", C.c_int),
        ("order", C.c_uint32), ("substeps", C.c_uint32), ("newton_max_iter", C.c_uint32),
        ("newton_rtol", C.c_double), ("state_floor", C.POINTER(C.c_double)),
        ("precision", C.c_int), ("resampling", C.c_int),
    ]


class pf_server_config(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("max_inflight", C.c_uint32), ("max_batch", C.c_uint32),
                ("reserved", C.c_uint32)]


class pf_server_report(C.Structure):
    _fields_ = [("streams_opened", C.c_uint64), ("streams_admitted", C.c_uint64),
                ("streams_closed", C.c_uint64), ("ticks", C.c_uint64), ("steps_completed", C.c_uint64),
                ("steps_skipped", C.c_uint64), ("particle_steps", C.c_uint64),
                ("latency_p50_ms", C.c_double), ("latency_p99_ms", C.c_double), ("latency_max_ms", C.c_double),
                ("admit_wait_p50_ms", C.c_double), ("admit_wait_p99_ms", C.c_double),
                ("mean_batch", C.c_double), ("busy_s", C.c_double)]


_lib = None


def lib():
    """Load the HIP library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"HIP library not built: {LIB_PATH} (run paper_1411_1702_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        vp, dp, u64 = C.c_void_p, C.POINTER(C.c_double), C.c_uint64
        L.pf_context_create.argtypes = [C.c_int, u64, C.POINTER(pf_allocator), vp, C.POINTER(vp)]
        L.pf_context_destroy.argtypes = [vp]
        L.pf_context_destroy.restype = None
        L.pf_filter_bytes.argtypes = [C.POINTER(pf_config)]
        L.pf_filter_bytes.restype = u64
        L.pf_context_memory.argtypes = [vp, C.POINTER(u64), C.POINTER(u64)]
        L.pf_create.argtypes = [vp, C.POINTER(pf_config), C.POINTER(vp)]
        L.pf_assimilate.argtypes = [vp, C.c_double, dp, dp]
        L.pf_assimilate_async.argtypes = [vp, C.c_double, dp, dp, C.POINTER(u64)]
        L.pf_wait.argtypes = [vp, u64]
        L.pf_assimilate_batch.argtypes = [vp, C.c_uint32, C.POINTER(vp), dp, dp, dp, C.POINTER(u64)]
        L.pf_posterior.argtypes = [vp, dp, dp, dp, dp, C.POINTER(u64)]
        L.pf_stats.argtypes = [vp, C.POINTER(u64), C.c_uint32]
        L.pf_context_profile.argtypes = [vp, C.c_int]
        L.pf_context_kernel_time.argtypes = [vp, C.c_int, C.POINTER(u64), C.POINTER(C.c_double)]
        L.pf_context_autotune.argtypes = [vp, C.c_int]
        L.pf_context_launch_grid.argtypes = [vp, C.c_int, C.c_uint32, C.POINTER(C.c_uint32), C.POINTER(C.c_int)]
        L.pf_destroy.argtypes = [vp]
        L.pf_destroy.restype = None
        L.pf_status_str.argtypes = [C.c_int]
        L.pf_status_str.restype = C.c_char_p
        L.pf_last_error.restype = C.c_char_p
        L.pf_test_philox.argtypes = [u64, vp, vp, vp, vp]
        L.pf_test_normals.argtypes = [u64, u64, u64, u64, C.c_uint32, vp, vp]
        L.pf_test_propagate.argtypes = [C.POINTER(pf_config), u64, vp, vp, C.c_double, C.c_int, vp, vp,
                                        vp, vp]
        L.pf_test_resample.argtypes = [u64, vp, u64, vp, vp]
        L.pf_test_resample_multinomial.argtypes = [u64, vp, u64, u64, vp, vp]
        L.pf_resample_noalloc.argtypes = [u64, vp, u64, vp, vp]
        L.pf_test_moments.argtypes = [u64, C.c_uint32, vp, vp, dp, dp, dp, dp, vp]
        L.pf_test_get_ensemble.argtypes = [vp, vp, vp, vp]
        L.pf_test_set_ensemble.argtypes = [vp, vp, vp, vp, dp, dp, u64, C.c_double]
        L.pf_test_last_ancestors.argtypes = [vp, vp]
        L.pf_query.argtypes = [vp, u64]
        L.pf_server_create.argtypes = [vp, C.POINTER(pf_server_config), C.POINTER(vp)]
        L.pf_server_open.argtypes = [vp, C.POINTER(pf_config), C.POINTER(u64)]
        L.pf_server_submit.argtypes = [vp, u64, C.c_double, dp, dp, C.POINTER(u64)]
        L.pf_server_poll.argtypes = [vp, u64, u64, dp]
        L.pf_server_posterior.argtypes = [vp, u64, dp, dp, dp, C.POINTER(u64)]
        L.pf_server_close.argtypes = [vp, u64]
        L.pf_server_drain.argtypes = [vp]
        L.pf_server_stats.argtypes = [vp, C.POINTER(pf_server_report)]
        L.pf_server_destroy.argtypes = [vp]
        L.pf_server_destroy.restype = None
        _lib = L
    return _lib


def check(status, what=""):
    if status != PF_OK:
        raise PfError(status, f"{what}: {lib().pf_last_error().decode()}")


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Config:
    """pf_config plus the host arrays it points to (kept alive here)."""

    def __init__(self, prob, precision=PF_PREC_FP32_PROP, n_particles=None, seed=None,
                 newton_rtol=None, resampling=None):
        self.prob = prob
        f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
        self.obs = np.ascontiguousarray(prob.obs_index, dtype=np.uint32)
        self.mc = f64(prob.model_consts if len(prob.model_consts) else np.zeros(1))
        self.rf = f64(prob.rates_fixed if len(prob.rates_fixed) else np.zeros(1))
        self.x0 = f64(prob.x0)
        self.pm = f64(prob.prior_mean)
        self.ps = f64(prob.prior_sd)
        self.fl = f64(prob.state_floor)
        c = pf_config()
        c.struct_size = C.sizeof(pf_config)
        c.model = int(prob.model)
        c.d, c.p, c.m = prob.d, prob.p, prob.m
        c.obs_index = self.obs.ctypes.data_as(C.POINTER(C.c_uint32))
        chain = prob.model == PF_MODEL_CHAIN16
        consts = chain or prob.model == PF_MODEL_ADVDIFF
        c.model_consts = _dp(self.mc) if consts else None
        c.n_model_consts = len(prob.model_consts) if consts else 0
        c.rates_fixed = _dp(self.rf) if chain else None
        c.n_rates_fixed = len(prob.rates_fixed) if chain else 0
        c.n_particles = int(prob.n_particles if n_particles is None else n_particles)
        c.seed = int(prob.seed if seed is None else seed)
        c.t0 = float(prob.t0)
        c.x0, c.prior_mean, c.prior_sd = _dp(self.x0), _dp(self.pm), _dp(self.ps)
        c.shrink_a = float(prob.shrink_a)
        c.lmm = int(getattr(prob, "lmm", PF_LMM_BDF))
        c.order, c.substeps = int(prob.order), int(prob.substeps)
        c.newton_max_iter = int(prob.newton_max_iter)
        if newton_rtol is None:
            newton_rtol = prob.newton_rtol_fp32 if precision == PF_PREC_FP32_PROP else prob.newton_rtol_fp64
        c.newton_rtol = float(newton_rtol)
        c.resampling = int(getattr(prob, "resampling", 0) if resampling is None else resampling)
        c.state_floor = _dp(self.fl)
        c.precision = int(precision)
        self.c = c

    def ptr(self):
        return C.byref(self.c)


class Context:
    def __init__(self, device=0, pool_bytes=0, stream=None, allocator=None):
        """allocator: optional (alloc(bytes, stream) -> device pointer, free(ptr, stream))
        pair of Python callables that provide the context's device pool."""
        h = C.c_void_p()
        self._alloc = None
        if allocator is not None:
            fa, ff = allocator
            # the ctypes callbacks must outlive the context
            self._alloc = pf_allocator(ALLOC_FN(lambda user, n, st: fa(int(n), st)),
                                       FREE_FN(lambda user, p, st: ff(p, st)), None)
        check(lib().pf_context_create(device, int(pool_bytes), C.byref(self._alloc) if self._alloc else None,
                                      stream, C.byref(h)), "pf_context_create")
        self.h = h

    def memory(self):
        u, c = C.c_uint64(), C.c_uint64()
        check(lib().pf_context_memory(self.h, C.byref(u), C.byref(c)), "pf_context_memory")
        return u.value, c.value

    def assimilate_batch(self, filters, t_obs, y, sigma):
        n = len(filters)
        hs = (C.c_void_p * n)(*[f.h.value for f in filters])
        t = np.ascontiguousarray(t_obs, dtype=np.float64)
        # rows of 4 observations (the library refuses a filter with m > 4)
        yy = np.zeros((n, 4))
        ss = np.ones((n, 4))
        for i, f in enumerate(filters):
            k = min(f.m, 4)
            yy[i, :k] = y[i][:k]
            ss[i, :k] = sigma[i][:k]
        tk = (C.c_uint64 * n)()
        check(lib().pf_assimilate_batch(self.h, n, hs, _dp(t), _dp(yy), _dp(ss), tk), "pf_assimilate_batch")
        return list(tk)

    def profile(self, enable=True):
        check(lib().pf_context_profile(self.h, int(enable)), "pf_context_profile")

    def kernel_time(self, which):
        """(timed submissions, total ms) for PF_TIME_* group `which`."""
        n, ms = C.c_uint64(), C.c_double()
        check(lib().pf_context_kernel_time(self.h, int(which), C.byref(n), C.byref(ms)), "kernel_time")
        return n.value, ms.value

    def autotune(self, enable=True):
        check(lib().pf_context_autotune(self.h, int(enable)), "pf_context_autotune")

    def launch_grid(self, group, items):
        """(grid, tuned) of a multi-filter submission's launch group (0 predictor,
        1 resampling, 2 update) over `items` tiles."""
        g, t = C.c_uint32(), C.c_int()
        check(lib().pf_context_launch_grid(self.h, int(group), int(items), C.byref(g), C.byref(t)),
              "pf_context_launch_grid")
        return g.value, bool(t.value)

    def close(self):
        if self.h:
            lib().pf_context_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Filter:
    def __init__(self, ctx: Context, cfg: Config):
        self.ctx, self.cfg = ctx, cfg
        self.d, self.p, self.m = cfg.c.d, cfg.c.p, cfg.c.m
        self.N = cfg.c.n_particles
        h = C.c_void_p()
        check(lib().pf_create(ctx.h, cfg.ptr(), C.byref(h)), "pf_create")
        self.h = h
        # y and sigma of a step go through two small ctypes buffers of this
        # filter (the library copies them during the call): converting numpy
        # arrays to pointers costs a few microseconds per call, per array
        n = max(4, self.m)
        self._y = (C.c_double * n)()
        self._s = (C.c_double * n)(*([1.0] * n))
        self._tk = C.c_uint64()

    def _load(self, y, sigma):
        for i in range(self.m):
            self._y[i] = y[i]
            self._s[i] = sigma[i]

    def assimilate(self, t, y, sigma):
        """Returns the step's status (PF_OK or PF_EDEGENERATE); raises on other errors."""
        self._load(y, sigma)
        st = lib().pf_assimilate(self.h, float(t), self._y, self._s)
        if st not in (PF_OK, PF_EDEGENERATE):
            check(st, "pf_assimilate")
        return st

    def assimilate_async(self, t, y, sigma):
        self._load(y, sigma)
        check(lib().pf_assimilate_async(self.h, float(t), self._y, self._s, C.byref(self._tk)),
              "pf_assimilate_async")
        return self._tk.value

    def wait(self, ticket):
        return lib().pf_wait(self.h, int(ticket))

    def posterior(self):
        mean = np.zeros(self.p)
        cov = np.zeros(self.p * self.p)
        xm = np.zeros(self.d)
        ess = C.c_double()
        step = C.c_uint64()
        check(lib().pf_posterior(self.h, _dp(mean), _dp(cov), _dp(xm), C.byref(ess), C.byref(step)),
              "pf_posterior")
        return {"mean": mean, "cov": cov.reshape(self.p, self.p), "state_mean": xm, "ess": ess.value,
                "step": step.value}

    def stats(self):
        names = ["newton_predict", "newton_update", "newton_fails", "nonfinite", "jitters", "negative_states"]
        v = (C.c_uint64 * len(names))()
        check(lib().pf_stats(self.h, v, len(names)), "pf_stats")
        return dict(zip(names, list(v)))

    def close(self):
        if self.h:
            lib().pf_destroy(self.h)
            self.h = None


class Server:
    """Continuous-batching server over a context (pf_server_* of the C ABI)."""

    def __init__(self, ctx: Context, max_inflight=3, max_batch=4096):
        cfg = pf_server_config(C.sizeof(pf_server_config), int(max_inflight), int(max_batch), 0)
        h = C.c_void_p()
        check(lib().pf_server_create(ctx.h, C.byref(cfg), C.byref(h)), "pf_server_create")
        self.h = h
        self.m = {}

    def open(self, cfg: Config) -> int:
        sid = C.c_uint64()
        check(lib().pf_server_open(self.h, cfg.ptr(), C.byref(sid)), "pf_server_open")
        self.m[sid.value] = cfg.c.m
        return sid.value

    def submit(self, sid, t, y, sigma) -> int:
        m = self.m[sid]
        yy = np.zeros(4)
        ss = np.ones(4)
        yy[:m] = y[:m]
        ss[:m] = sigma[:m]
        tk = C.c_uint64()
        check(lib().pf_server_submit(self.h, sid, float(t), _dp(yy), _dp(ss), C.byref(tk)), "pf_server_submit")
        return tk.value

    def poll(self, sid, ticket):
        """(status, latency_ms); status PF_EBUSY while pending."""
        lat = C.c_double()
        st = lib().pf_server_poll(self.h, sid, ticket, C.byref(lat))
        return st, lat.value

    def posterior(self, sid, p):
        mean = np.zeros(p)
        cov = np.zeros(p * p)
        ess = C.c_double()
        step = C.c_uint64()
        check(lib().pf_server_posterior(self.h, sid, _dp(mean), _dp(cov), C.byref(ess), C.byref(step)),
              "pf_server_posterior")
        return {"mean": mean, "cov": cov.reshape(p, p), "ess": ess.value, "step": step.value}

    def close(self, sid):
        check(lib().pf_server_close(self.h, sid), "pf_server_close")

    def drain(self):
        check(lib().pf_server_drain(self.h), "pf_server_drain")

    def stats(self):
        r = pf_server_report()
        check(lib().pf_server_stats(self.h, C.byref(r)), "pf_server_stats")
        return {name: getattr(r, name) for name, _ in pf_server_report._fields_}

    def destroy(self):
        if self.h:
            lib().pf_server_destroy(self.h)
            self.h = None


def run_filter(ctx, prob, precision=PF_PREC_FP32_PROP, T=None, n_particles=None, seed=None):
    """Assimilate the first T observations; returns per-step posterior means, sds, ess."""
    cfg = Config(prob, precision, n_particles=n_particles, seed=seed)
    f = Filter(ctx, cfg)
    T = prob.T if T is None else int(T)
    means, sds, ess = [], [], []
    try:
        for j in range(T):
            st = f.assimilate(prob.times[j], prob.y[j], prob.sigma[j])
            post = f.posterior()   # a skipped (degenerate) step leaves the ensemble as it was
            means.append(post["mean"])
            sds.append(np.sqrt(np.diag(post["cov"])))
            ess.append(post["ess"] if st == PF_OK else np.nan)
    finally:
        f.close()
    return np.array(means), np.array(sds), np.array(ess)
