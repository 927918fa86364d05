"""ctypes wrapper of the FP64 CPU oracle (pf_oracle.c).

TEST INFRASTRUCTURE ONLY: the oracle is what the GPU path is checked against.
Only the tests, the smoke check and the benchmark's CPU-baseline leg use it;
the product library never loads it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pf_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
# another build of the same source (e.g. with sanitizers) can be loaded instead
LIB_OVERRIDE = os.environ.get("PF_ORACLE_LIB")

OK, EINVAL, EDEGENERATE = 0, 1, 4
PUR_PRIOR, PUR_RESAMPLE, PUR_PROLIF, PUR_INNOV = 1, 2, 3, 4
MODEL_DECAY, MODEL_ROBERTSON, MODEL_CHAIN, MODEL_ADVDIFF = 0, 1, 2, 3
DMAX, PMAX, MMAX = 1521, 12, 32


CFLAGS = ["-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall"]


def compile_to(src: str, out: str, extra=()) -> str:
    """gcc one oracle source into a shared library at `out`."""
    tmp = out + ".tmp"
    subprocess.check_call(["gcc"] + CFLAGS + list(extra) + ["-o", tmp, src, "-lm"])
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP over particles)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        compile_to(SRC, LIB)
    return LIB


class _Cfg(C.Structure):
    _fields_ = [("model", C.c_int), ("d", C.c_int), ("p", C.c_int), ("m", C.c_int),
                ("obs", C.c_int * MMAX),
                ("mc", C.POINTER(C.c_double)), ("rates_fixed", C.POINTER(C.c_double)),
                ("N", C.c_long), ("seed", C.c_uint64), ("a", C.c_double),
                ("order", C.c_int), ("substeps", C.c_int),
                ("kmax", C.c_int), ("rtol", C.c_double),
                ("floor_", C.c_double * DMAX), ("x0", C.c_double * DMAX),
                ("prior_mean", C.c_double * PMAX), ("prior_sd", C.c_double * PMAX),
                ("resampling", C.c_int), ("lmm", C.c_int)]


class _State(C.Structure):
    _fields_ = [("j", C.c_uint64), ("t", C.c_double),
                ("x", C.POINTER(C.c_double)), ("theta", C.POINTER(C.c_double)),
                ("logw", C.POINTER(C.c_double)),
                ("theta_bar", C.c_double * PMAX), ("C", C.c_double * (PMAX * PMAX)),
                ("L", C.c_double * (PMAX * PMAX))]


class _Diag(C.Structure):
    _fields_ = [("ess", C.c_double), ("state_mean", C.c_double * DMAX),
                ("newton_iters", C.c_long), ("newton_fails", C.c_long), ("lu_fails", C.c_long),
                ("nonfinite", C.c_long), ("jitters", C.c_int), ("first_anc", C.c_int32)]


class _PsiStats(C.Structure):
    _fields_ = [("newton_iters", C.c_long), ("newton_fails", C.c_long), ("lu_fails", C.c_long)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if LIB_OVERRIDE:
            L = C.CDLL(LIB_OVERRIDE)
        else:
            if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
                build(force=True)
            L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        up = C.POINTER(C.c_uint64)
        L.or_philox4x64.argtypes = [up, up, up]
        L.or_u01.argtypes = [C.c_uint64]
        L.or_u01.restype = C.c_double
        L.or_normals.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint64, C.c_int, dp]
        L.or_bdf.argtypes = [C.c_int, dp, dp, dp]
        L.or_am.argtypes = [C.c_int, dp, dp]
        L.or_sdirk.argtypes = [C.c_int, dp, C.POINTER(C.c_int)]
        L.or_psi_lmm.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, dp, dp, dp, dp, C.c_double, C.c_int,
                                 C.c_int, C.c_int, C.c_double, C.c_int, dp, dp, C.c_int, dp, dp,
                                 C.POINTER(_PsiStats)]
        L.or_rhs.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, dp, dp, dp, dp]
        L.or_lu_solve.argtypes = [C.c_int, dp, dp]
        L.or_psi.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, dp, dp, C.c_double, C.c_int,
                             C.c_int, C.c_int, C.c_double, C.c_int, dp, dp, C.c_int, dp, dp,
                             C.POINTER(_PsiStats)]
        L.or_loglik.argtypes = [C.c_int, C.POINTER(C.c_int), dp, dp, dp]
        L.or_loglik.restype = C.c_double
        L.or_normalise.argtypes = [C.c_long, dp, dp]
        L.or_normalise.restype = C.c_double
        L.or_resample_shift.argtypes = [C.c_long]
        L.or_resample_int.argtypes = [C.c_long, up, C.c_uint64, C.POINTER(C.c_int32)]
        L.or_resample.argtypes = [C.c_long, dp, C.c_uint64, C.POINTER(C.c_int32)]
        L.or_resample_multinomial_int.argtypes = [C.c_long, up, up, C.POINTER(C.c_int32)]
        L.or_resample_multinomial.argtypes = [C.c_long, dp, C.c_uint64, C.c_uint64, C.POINTER(C.c_int32)]
        L.or_moments.argtypes = [C.c_long, C.c_int, dp, dp, dp, dp]
        L.or_cholesky.argtypes = [C.c_int, dp, dp, C.POINTER(C.c_int)]
        L.or_filter_init.argtypes = [C.POINTER(_Cfg), C.c_double, C.POINTER(_State)]
        L.or_filter_step.argtypes = [C.POINTER(_Cfg), C.POINTER(_State), C.c_double, dp, dp,
                                     C.POINTER(_Diag)]
        L.or_filter_stage1.argtypes = [C.POINTER(_Cfg), C.POINTER(_State), C.c_double, dp, dp,
                                       dp, C.POINTER(C.c_int32)]
        L.or_filter_step_given.argtypes = [C.POINTER(_Cfg), C.POINTER(_State), C.c_double, dp, dp,
                                           C.POINTER(C.c_int32), C.POINTER(_Diag)]
        L.or_num_threads.restype = C.c_int
        L.or_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# RNG
# --------------------------------------------------------------------------
def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    up = C.POINTER(C.c_uint64)
    lib().or_philox4x64(c.ctypes.data_as(up), k.ctypes.data_as(up), out.ctypes.data_as(up))
    return out


def u01(w: int) -> float:
    return lib().or_u01(C.c_uint64(int(w)))


def normals(seed, step, particle, purpose, count):
    out = np.zeros(max(count, 1))
    lib().or_normals(seed, step, particle, purpose, count, _dp(out))
    return out[:count]


# --------------------------------------------------------------------------
# integrator pieces
# --------------------------------------------------------------------------
def bdf(q):
    alpha = np.zeros(4)
    beta = np.zeros(1)
    errc = np.zeros(1)
    st = lib().or_bdf(q, _dp(alpha), _dp(beta), _dp(errc))
    if st:
        raise ValueError(q)
    return alpha[: q + 1], float(beta[0]), float(errc[0])


def rhs(model, x, theta, mc=None, rates_fixed=None, d=None, p=None):
    x = _f64(x)
    theta = _f64(theta)
    d = len(x) if d is None else d
    p = len(theta) if p is None else p
    if not 1 <= d <= DMAX:
        raise ValueError(f"state dimension {d} outside 1..{DMAX}")
    mc = _f64(mc if mc is not None else np.zeros(1))
    rf = _f64(rates_fixed if rates_fixed is not None and len(rates_fixed) else np.zeros(1))
    f = np.zeros(d)
    J = np.zeros(d * d)
    lib().or_rhs(model, d, p, _dp(mc), _dp(rf), _dp(x), _dp(theta), _dp(f), _dp(J))
    return f, J.reshape(d, d)


def lu_solve(A, b):
    A = _f64(A).copy()
    b = _f64(b).copy()
    st = lib().or_lu_solve(len(b), _dp(A), _dp(b))
    if st:
        raise np.linalg.LinAlgError("singular")
    return b


def am(q):
    """Adams-Moulton q-step coefficients (beta_0..beta_3) and |error constant|."""
    beta = np.zeros(4)
    e = np.zeros(1)
    rc = lib().or_am(int(q), _dp(beta), _dp(e))
    if rc:
        raise ValueError(q)
    return beta, float(e[0])


def sdirk(k):
    """Butcher matrix (3x3, zero padded) and stage count of the start-up SDIRK of order k."""
    A = np.zeros(9)
    ns = C.c_int(0)
    if lib().or_sdirk(int(k), _dp(A), C.byref(ns)):
        raise ValueError(k)
    n = ns.value
    return A.reshape(3, 3)[:n, :n].copy(), n


def psi(model, x0, theta, h, M, k, lte=False, rtol=1e-12, kmax=10, floor=None,
        mc=None, rates_fixed=None, hist=None, lmm=0):
    """One particle over one interval; returns (x, gamma, stats dict).
    lmm: 0 BDF (order k), 1 Adams-Moulton (k steps), 2 BDF with the SDIRK start-up."""
    x0 = _f64(x0)
    theta = _f64(theta)
    d, p = len(x0), len(theta)
    floor = _f64(floor if floor is not None else np.full(d, 1e-300))
    mc = _f64(mc if mc is not None and len(mc) else np.zeros(1))
    rf = _f64(rates_fixed if rates_fixed is not None and len(rates_fixed) else np.zeros(1))
    xo = np.zeros(d)
    go = np.zeros(d)
    st = _PsiStats()
    if hist is not None:
        hh = _f64(np.atleast_2d(hist))
        hptr, nq = _dp(hh), hh.shape[0]
    else:
        hptr, nq = None, 0
    rc = lib().or_psi_lmm(int(lmm), model, d, p, _dp(mc), _dp(rf), _dp(x0), _dp(theta), float(h), int(M),
                          int(k), 1 if lte else 0, float(rtol), int(kmax), _dp(floor), hptr, nq, _dp(xo),
                          _dp(go), C.byref(st))
    if rc:
        raise ValueError(f"oracle psi rejected its arguments (status {rc})")
    return xo, go, {"newton_iters": st.newton_iters, "newton_fails": st.newton_fails,
                    "lu_fails": st.lu_fails}


# --------------------------------------------------------------------------
# weights, resampling, moments
# --------------------------------------------------------------------------
def loglik(x, y, sigma, obs):
    obs_c = np.ascontiguousarray(obs, dtype=np.int32)
    return lib().or_loglik(len(obs_c), obs_c.ctypes.data_as(C.POINTER(C.c_int)), _dp(_f64(y)),
                           _dp(_f64(sigma)), _dp(_f64(x)))


def normalise(l):
    l = _f64(l)
    w = np.zeros(len(l))
    lz = lib().or_normalise(len(l), _dp(l), _dp(w))
    return w, lz


def resample_shift(N):
    return lib().or_resample_shift(int(N))


def resample_int(q, V):
    q = np.ascontiguousarray(q, dtype=np.uint64)
    anc = np.zeros(len(q), dtype=np.int32)
    st = lib().or_resample_int(len(q), q.ctypes.data_as(C.POINTER(C.c_uint64)), C.c_uint64(int(V)),
                               anc.ctypes.data_as(C.POINTER(C.c_int32)))
    return st, anc


def resample(g, r):
    g = _f64(g)
    anc = np.zeros(len(g), dtype=np.int32)
    st = lib().or_resample(len(g), _dp(g), C.c_uint64(int(r)), anc.ctypes.data_as(C.POINTER(C.c_int32)))
    return st, anc


def resample_multinomial_int(q, r):
    """Multinomial draw on integer weights q with one uniform word per slot."""
    q = np.ascontiguousarray(q, dtype=np.uint64)
    r = np.ascontiguousarray(r, dtype=np.uint64)
    anc = np.zeros(len(q), dtype=np.int32)
    st = lib().or_resample_multinomial_int(len(q), q.ctypes.data_as(C.POINTER(C.c_uint64)),
                                           r.ctypes.data_as(C.POINTER(C.c_uint64)),
                                           anc.ctypes.data_as(C.POINTER(C.c_int32)))
    return st, anc


def resample_multinomial(g, seed, step):
    """Multinomial draw on the weights g with the RESAMPLE words of (seed, step)."""
    g = _f64(g)
    anc = np.zeros(len(g), dtype=np.int32)
    st = lib().or_resample_multinomial(len(g), _dp(g), C.c_uint64(int(seed)), C.c_uint64(int(step)),
                                       anc.ctypes.data_as(C.POINTER(C.c_int32)))
    return st, anc


def moments(theta, w):
    theta = _f64(theta)
    N, p = theta.shape
    mean = np.zeros(p)
    cov = np.zeros(p * p)
    lib().or_moments(N, p, _dp(theta), _dp(_f64(w)), _dp(mean), _dp(cov))
    return mean, cov.reshape(p, p)


def cholesky(Cm):
    Cm = _f64(Cm)
    p = Cm.shape[0]
    L = np.zeros(p * p)
    jit = C.c_int(0)
    st = lib().or_cholesky(p, _dp(Cm), _dp(L), C.byref(jit))
    return st, L.reshape(p, p), jit.value


def set_threads(n):
    lib().or_set_num_threads(int(n))


def num_threads():
    return lib().or_num_threads()


# --------------------------------------------------------------------------
# the filter
# --------------------------------------------------------------------------
class Filter:
    """Algorithm 1 on the CPU.  `prob` is an inputs.Problem (or any object with
    the same fields)."""

    def __init__(self, prob, n_particles=None, seed=None, rtol=None, resampling=None):
        self.prob = prob
        N = int(prob.n_particles if n_particles is None else n_particles)
        d, p, m = prob.d, prob.p, prob.m
        self.N, self.d, self.p, self.m = N, d, p, m
        self._mc = _f64(prob.model_consts if len(prob.model_consts) else np.zeros(1))
        self._rf = _f64(prob.rates_fixed if len(prob.rates_fixed) else np.zeros(1))
        cfg = _Cfg()
        cfg.model, cfg.d, cfg.p, cfg.m = prob.model, d, p, m
        for i, o in enumerate(prob.obs_index):
            cfg.obs[i] = int(o)
        cfg.mc = _dp(self._mc)
        cfg.rates_fixed = _dp(self._rf)
        cfg.N = N
        cfg.seed = int(prob.seed if seed is None else seed)
        cfg.a = float(prob.shrink_a)
        cfg.order, cfg.substeps = int(prob.order), int(prob.substeps)
        cfg.kmax = int(prob.newton_max_iter)
        cfg.rtol = float(prob.newton_rtol_fp64 if rtol is None else rtol)
        cfg.resampling = int(getattr(prob, "resampling", 0) if resampling is None else resampling)
        cfg.lmm = int(getattr(prob, "lmm", 0))
        for i in range(d):
            cfg.floor_[i] = float(prob.state_floor[i])
            cfg.x0[i] = float(prob.x0[i])
        for i in range(p):
            cfg.prior_mean[i] = float(prob.prior_mean[i])
            cfg.prior_sd[i] = float(prob.prior_sd[i])
        self.cfg = cfg
        self.x = np.zeros((N, d))
        self.theta = np.zeros((N, p))
        self.logw = np.zeros(N)
        st = _State()
        st.x, st.theta, st.logw = _dp(self.x), _dp(self.theta), _dp(self.logw)
        self.st = st
        rc = lib().or_filter_init(C.byref(cfg), float(prob.t0), C.byref(st))
        if rc:
            raise RuntimeError(f"oracle init failed: {rc}")

    # ensemble access -----------------------------------------------------
    @property
    def j(self):
        return int(self.st.j)

    @property
    def t(self):
        return float(self.st.t)

    def moments(self):
        p = self.p
        mean = np.array(self.st.theta_bar[:p])
        cov = np.array(self.st.C[: PMAX * PMAX])[: p * p].reshape(p, p)
        return mean, cov

    def chol(self):
        p = self.p
        return np.array(self.st.L[: PMAX * PMAX])[: p * p].reshape(p, p)

    def set_ensemble(self, x, theta, logw, theta_bar, C_, L, j, t):
        self.x[...] = x
        self.theta[...] = theta
        self.logw[...] = logw
        p = self.p
        for i in range(p):
            self.st.theta_bar[i] = float(theta_bar[i])
        for i in range(p * p):
            self.st.C[i] = float(np.asarray(C_).ravel()[i])
            self.st.L[i] = float(np.asarray(L).ravel()[i])
        self.st.j = int(j)
        self.st.t = float(t)

    # steps -----------------------------------------------------------------
    def step(self, t_next, y, sigma):
        dg = _Diag()
        rc = lib().or_filter_step(C.byref(self.cfg), C.byref(self.st), float(t_next),
                                  _dp(_f64(y)), _dp(_f64(sigma)), C.byref(dg))
        out = {"status": rc, "ess": dg.ess, "state_mean": np.array(dg.state_mean[: self.d]),
               "newton_iters": dg.newton_iters, "newton_fails": dg.newton_fails,
               "lu_fails": dg.lu_fails, "nonfinite": dg.nonfinite, "jitters": dg.jitters}
        return out

    def step_given(self, t_next, y, sigma, anc):
        """The step with these N ancestors in place of its own index draw of
        step 3(b) (test use: the rest of the step for another implementation's
        draw); returns the status."""
        a = np.ascontiguousarray(anc, dtype=np.int32)
        assert a.shape == (self.N,)
        dg = _Diag()
        return lib().or_filter_step_given(C.byref(self.cfg), C.byref(self.st), float(t_next),
                                          _dp(_f64(y)), _dp(_f64(sigma)),
                                          a.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(dg))

    def stage1(self, t_next, y, sigma):
        g = np.zeros(self.N)
        anc = np.zeros(self.N, dtype=np.int32)
        rc = lib().or_filter_stage1(C.byref(self.cfg), C.byref(self.st), float(t_next),
                                    _dp(_f64(y)), _dp(_f64(sigma)), _dp(g),
                                    anc.ctypes.data_as(C.POINTER(C.c_int32)))
        return rc, g, anc

    def run(self, T=None, callback=None):
        """Assimilate the first T observations; returns per-step mean, sd, ess."""
        prob = self.prob
        T = prob.T if T is None else int(T)
        means, sds, ess = [], [], []
        for j in range(T):
            out = self.step(prob.times[j], prob.y[j], prob.sigma[j])
            if out["status"] not in (OK, EDEGENERATE):
                raise RuntimeError(f"oracle step {j} failed: {out['status']}")
            # a degenerate step is skipped: the ensemble and its moments stay
            mean, cov = self.moments()
            means.append(mean)
            sds.append(np.sqrt(np.diag(cov)))
            ess.append(out["ess"] if out["status"] == OK else np.nan)
            if callback:
                callback(j, out)
        return np.array(means), np.array(sds), np.array(ess)
