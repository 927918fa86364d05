"""Seeded synthetic workloads for the LMM PF-SMC sampler.

This module only *generates inputs*: problem definitions (model constants,
priors, observation times), true trajectories and noisy observations.  It
holds none of the filter's arithmetic.  Both the GPU library and the CPU
oracle consume what it produces, so it must not import either of them.

The paper's own test problems cannot be rebuilt from its text (the
Michaelis-Menten system of Sec. 2.1 prints no constants), so the workloads are:

* Robertson stiff kinetics, 3 states, log-rates estimated;
* a 16-compartment chain with Michaelis-Menten losses, 12 log-rates estimated;
* the 2D periodic advection-diffusion problem of Sec. 4 (six-plume initial
  field of Table 3, fixed parameters K and c of Sec. 4, 20 fixed observation
  sites), 5 parameters estimated;
* mixes of the first two for many independent filters (batched and served
  forms).

True trajectories come from scipy's Radau integrator at tight tolerance (the
kinetic models) or from the exact matrix exponential of the discretised
operator (advection-diffusion); the model right-hand sides below exist only
for that purpose.  Observation noise,
chain constants and the mixes are drawn from numpy's Philox4x64-10 streams
keyed by (seed, purpose).
"""
from __future__ import annotations

import dataclasses
import functools

import numpy as np

MODEL_ROBERTSON = 1
MODEL_CHAIN = 2
MODEL_ADVDIFF = 3

# RNG purposes (second key word of the input streams)
PURPOSE_DATA = 5
PURPOSE_MODEL = 6
PURPOSE_MIX = 7
PURPOSE_ARRIVAL = 8

ROBERTSON_TRUE_K = (0.04, 3.0e7, 1.0e4)
CHAIN_D = 16
CHAIN_P = 12


def _stream(seed: int, purpose: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=[int(seed), int(purpose)]))


@dataclasses.dataclass
class Problem:
    """One filtering problem: model, prior, observation schedule and data."""

    name: str
    model: int
    d: int
    p: int
    m: int
    obs_index: np.ndarray        # (m,) observed state components
    model_consts: np.ndarray     # chain: [V(d), K(d)]; advection-diffusion: [grid side]; Robertson: empty
    rates_fixed: np.ndarray      # chain: all d rates (first p are estimated); Robertson: empty
    x0: np.ndarray               # (d,)
    prior_mean: np.ndarray       # (p,) Gaussian prior on the parameters (log-rates for the kinetic models)
    prior_sd: np.ndarray         # (p,)
    theta_true: np.ndarray       # (p,)
    t0: float
    times: np.ndarray            # (T,) observation times, increasing, > t0
    x_true: np.ndarray           # (T, d)
    y: np.ndarray                # (T, m)
    sigma: np.ndarray            # (T, m)
    order: int                   # BDF order k
    substeps: int                # fixed LMM steps per observation interval M
    n_particles: int
    seed: int
    shrink_a: float = 0.98
    newton_max_iter: int = 10
    newton_rtol_fp64: float = 1e-12
    newton_rtol_fp32: float = 2e-6
    state_floor: np.ndarray = None   # (d,) scale floors (Newton test, parity)
    resampling: int = 0              # step 3(b): 0 systematic, 1 multinomial
    lmm: int = 0                     # 0 BDF (order k), 1 Adams-Moulton (k steps), 2 BDF + SDIRK start-up

    @property
    def T(self) -> int:
        return len(self.times)

    def with_particles(self, n: int) -> "Problem":
        return dataclasses.replace(self, n_particles=int(n))

    def truncated(self, T: int) -> "Problem":
        return dataclasses.replace(self, times=self.times[:T], x_true=self.x_true[:T],
                                   y=self.y[:T], sigma=self.sigma[:T])


# --------------------------------------------------------------------------
# true trajectories (Radau, tight tolerance)
# --------------------------------------------------------------------------
def _robertson_rhs(k):
    k1, k2, k3 = k

    def f(t, x):
        return [-k1 * x[0] + k3 * x[1] * x[2],
                k1 * x[0] - k2 * x[1] ** 2 - k3 * x[1] * x[2],
                k2 * x[1] ** 2]

    def jac(t, x):
        return [[-k1, k3 * x[2], k3 * x[1]],
                [k1, -2 * k2 * x[1] - k3 * x[2], -k3 * x[1]],
                [0.0, 2 * k2 * x[1], 0.0]]
    return f, jac


def _chain_rhs(k, V, K):
    k = np.asarray(k, float)
    V = np.asarray(V, float)
    K = np.asarray(K, float)

    def f(t, x):
        inflow = np.concatenate([[1.0], k[:-1] * x[:-1]])
        return inflow - k * x - V * x / (K + x)

    def jac(t, x):
        return np.diag(-k - V * K / (K + x) ** 2) + np.diag(k[:-1], -1)
    return f, jac


def _truth(f, jac, x0, times, atol):
    from scipy.integrate import solve_ivp
    sol = solve_ivp(f, (0.0, float(times[-1])), np.asarray(x0, float), method="Radau",
                    rtol=1e-12, atol=atol, jac=jac, t_eval=np.asarray(times, float))
    if sol.status != 0:
        raise RuntimeError(f"truth integration failed: {sol.message}")
    return sol.y.T.copy()


def _noise(x_true, obs, seed):
    """2% of signal, with a floor at 1e-3 of the component's largest value."""
    sig_src = np.abs(x_true[:, obs])
    floor = 1e-3 * sig_src.max(axis=0)
    sigma = 0.02 * np.maximum(sig_src, floor)
    eps = _stream(seed, PURPOSE_DATA).standard_normal(sigma.shape)
    return x_true[:, obs] + sigma * eps, sigma


# --------------------------------------------------------------------------
# problems
# --------------------------------------------------------------------------
@functools.lru_cache(maxsize=64)
def _robertson_truth(T: int):
    times = np.logspace(-3.0, 3.0, T)
    f, jac = _robertson_rhs(ROBERTSON_TRUE_K)
    x_true = _truth(f, jac, [1.0, 0.0, 0.0], times, atol=1e-20)
    return times, x_true


def robertson(n_particles: int = 1000, T: int = 50, seed: int = 0, substeps: int = 20,
              order: int = 2) -> Problem:
    """Robertson kinetics, observe x2 at T log-spaced times in [1e-3, 1e3]."""
    times, x_true = _robertson_truth(int(T))
    obs = np.array([1], dtype=np.int32)
    y, sigma = _noise(x_true, obs, seed)
    theta = np.log(np.array(ROBERTSON_TRUE_K))
    scale = np.maximum(np.abs(x_true).max(axis=0), np.array([1.0, 0.0, 0.0]))
    return Problem(
        name=f"robertson_N{n_particles}_T{T}", model=MODEL_ROBERTSON, d=3, p=3, m=1,
        obs_index=obs, model_consts=np.zeros(0), rates_fixed=np.zeros(0),
        x0=np.array([1.0, 0.0, 0.0]), prior_mean=theta.copy(), prior_sd=np.full(3, 0.5),
        theta_true=theta, t0=0.0, times=times, x_true=x_true, y=y, sigma=sigma,
        order=order, substeps=substeps, n_particles=int(n_particles), seed=int(seed),
        state_floor=1e-6 * scale)


def chain_constants(model_seed: int):
    """Chain constants: rates k_i and maximal rates V_i log-uniform on
    [1e-2, 1e4]; affinities K_i log-uniform on [1e-1, 1e1]."""
    g = _stream(model_seed, PURPOSE_MODEL)
    k = 10.0 ** g.uniform(-2.0, 4.0, CHAIN_D)
    V = 10.0 ** g.uniform(-2.0, 4.0, CHAIN_D)
    K = 10.0 ** g.uniform(-1.0, 1.0, CHAIN_D)
    return k, V, K


CHAIN_X0 = 0.1   # every compartment starts at 0.1


@functools.lru_cache(maxsize=64)
def _chain_truth(model_seed: int, T: int, dt: float):
    k, V, K = chain_constants(model_seed)
    times = dt * np.arange(1, T + 1)
    f, jac = _chain_rhs(k, V, K)
    x_true = _truth(f, jac, np.full(CHAIN_D, CHAIN_X0), times, atol=1e-30)
    return times, x_true


def chain16(n_particles: int = 65536, T: int = 100, seed: int = 0, model_seed: int = 0,
            substeps: int = 40, order: int = 3) -> Problem:
    """16-compartment chain, observe x8 and x16 every 0.1 time units."""
    k, V, K = chain_constants(model_seed)
    times, x_true = _chain_truth(int(model_seed), int(T), 0.1)
    obs = np.array([7, 15], dtype=np.int32)
    y, sigma = _noise(x_true, obs, seed)
    theta = np.log(k[:CHAIN_P])
    scale = np.abs(x_true).max(axis=0)
    return Problem(
        name=f"chain16_N{n_particles}_T{T}", model=MODEL_CHAIN, d=CHAIN_D, p=CHAIN_P, m=2,
        obs_index=obs, model_consts=np.concatenate([V, K]), rates_fixed=k.copy(),
        x0=np.full(CHAIN_D, CHAIN_X0), prior_mean=theta.copy(), prior_sd=np.full(CHAIN_P, 0.5),
        theta_true=theta, t0=0.0, times=times, x_true=x_true, y=y, sigma=sigma,
        order=order, substeps=substeps, n_particles=int(n_particles), seed=int(seed),
        state_floor=1e-6 * scale)


# --------------------------------------------------------------------------
# 2D periodic advection-diffusion (Sec. 4)
# --------------------------------------------------------------------------
# Table 3: plume standard deviations and centres
PLUME_GAMMA = (0.04, 0.08, 0.07, 0.10, 0.05, 0.06)
PLUME_XC = (0.20, 0.30, 0.40, 0.50, 0.50, 0.70)
PLUME_YC = (0.80, 0.40, 0.40, 0.50, 0.60, 0.50)
# the fixed parameters that generate the data: K = [[k1, k3], [0, k2]] =
# [[9, 6], [0, 4]], c = (2.5, -1.5); theta = (k1, k2, k3, c1, c2)
ADVDIFF_THETA = (9.0, 4.0, 6.0, 2.5, -1.5)
ADVDIFF_P = 5


def advdiff_initial(n: int) -> np.ndarray:
    """Six Gaussian plumes on the periodic (n-1) x (n-1) grid of [0, 1)^2,
    x_i = i / (n - 1), stacked with x fastest: u[iy * (n-1) + ix]."""
    nt = n - 1
    g = np.arange(nt) / nt
    X, Y = np.meshgrid(g, g)            # X[iy, ix] = x_ix, Y[iy, ix] = y_iy
    u = np.zeros((nt, nt))
    for gam, xc, yc in zip(PLUME_GAMMA, PLUME_XC, PLUME_YC):
        u += np.exp(-((X - xc) ** 2 + (Y - yc) ** 2) / (2 * gam * gam)) / (gam * np.sqrt(2 * np.pi))
    return u.reshape(-1)


def _advdiff_operator(nt: int, theta):
    """Sparse L(theta) of the semi-discrete system dU/dt = L U (Sec. 4), for
    the truth only: B1 = I (x) l, B2 = l (x) I with the periodic backward
    difference l."""
    import scipy.sparse as sp
    k1, k2, k3, c1, c2 = theta
    ell = sp.eye(nt, format="csr") - sp.eye(nt, k=-1, format="csr") - sp.eye(nt, k=nt - 1, format="csr")
    I = sp.eye(nt, format="csr")
    B1 = sp.kron(I, ell, format="csr")
    B2 = sp.kron(ell, I, format="csr")
    return (-(k1 * k1 * (B1.T @ B1) + k1 * k3 * (B1.T @ B2 + B2.T @ B1) + (k2 * k2 + k3 * k3) * (B2.T @ B2))
            + c1 * B1 + c2 * B2).tocsc()


@functools.lru_cache(maxsize=16)
def _advdiff_truth(n: int, T: int, dt: float):
    from scipy.sparse.linalg import expm_multiply
    nt = n - 1
    L = _advdiff_operator(nt, ADVDIFF_THETA)
    u0 = advdiff_initial(n)
    times = dt * np.arange(1, T + 1)
    x_true = expm_multiply(L, u0, start=dt, stop=dt * T, num=T, endpoint=True)
    return times, np.asarray(x_true)


def advdiff(n_particles: int = 5000, T: int = 30, seed: int = 0, n: int = 20, sites: int = 20,
            substeps: int = 10, order: int = 2, prior_sd: float = 1.0) -> Problem:
    """The advection-diffusion workload of Sec. 4 on an n x n grid ((n-1)^2
    states): observe the field at `sites` fixed grid points drawn without
    replacement, every time unit (T observations); noise sd = the largest
    initial value at the sites / 50.  BDF2 with h = 0.1 (10 steps per unit).
    theta = (k1, k2, k3, c1, c2) with a Gaussian prior N(truth, prior_sd^2 I)."""
    nt = n - 1
    d = nt * nt
    times, x_true = _advdiff_truth(int(n), int(T), 1.0)
    u0 = advdiff_initial(n)
    obs = np.sort(_stream(seed, PURPOSE_MODEL).choice(d, size=min(sites, d), replace=False)).astype(np.int32)
    sd = np.abs(u0[obs]).max() / 50.0
    sigma = np.full((len(times), len(obs)), sd)
    y = x_true[:, obs] + sigma * _stream(seed, PURPOSE_DATA).standard_normal(sigma.shape)
    theta = np.array(ADVDIFF_THETA)
    return Problem(
        name=f"advdiff_n{n}_N{n_particles}_T{T}", model=MODEL_ADVDIFF, d=d, p=ADVDIFF_P, m=len(obs),
        obs_index=obs, model_consts=np.array([float(nt)]), rates_fixed=np.zeros(0),
        x0=u0, prior_mean=theta.copy(), prior_sd=np.full(ADVDIFF_P, prior_sd),
        theta_true=theta, t0=0.0, times=times, x_true=x_true, y=y, sigma=sigma,
        order=order, substeps=substeps, n_particles=int(n_particles), seed=int(seed),
        state_floor=np.full(d, 1e-6 * np.abs(u0).max()))


def decay_consts():
    return np.zeros(0)


# --------------------------------------------------------------------------
# configurations of the study
# --------------------------------------------------------------------------
def config_small() -> Problem:
    """Robertson, N = 1000, 50 observations, BDF2 with 20 steps, seed 0."""
    return robertson(1000, 50, seed=0)


def config_robertson_large() -> Problem:
    """Robertson, N = 2^17, 200 observations log-spaced in [1e-3, 1e3]."""
    return robertson(1 << 17, 200, seed=0)


def config_chain() -> Problem:
    """16-state chain, N = 2^16, 100 observations, BDF3 with 40 steps."""
    return chain16(1 << 16, 100, seed=0)


def config_advdiff(n: int = 20) -> Problem:
    """Advection-diffusion of Sec. 4 on the n x n grid (n = 20: 361 states;
    n = 40: 1521), N = 5000, 30 observations at 20 sites, BDF2 with h = 0.1."""
    return advdiff(5000, 30, seed=0, n=n)


# Constant sets of the chain used by the many-filter mixes.  A random draw of
# the 48 rates/affinities often gives observed compartments so small or so
# sharply informative that a few hundred particles collapse onto one at the
# first observation; these seeds were kept because a 512-particle FP64
# reference filter assimilates their first 10 observations without a
# skipped step.
CHAIN_INSTANCES = (0, 3, 8, 9, 10, 11, 12, 15)
N_CHAIN_INSTANCES = len(CHAIN_INSTANCES)


def batched_mix(n_filters: int = 256, seed: int = 0, n_min: int = 512, n_max: int = 65536,
                chain_fraction: float = 0.5):
    """Independent filters for the batched step: model chosen with
    probability `chain_fraction`, N log-uniform on [n_min, n_max], filter f
    uses data seed f.  Chain instances reuse a few constant sets (their data
    and filter seeds still differ)."""
    g = _stream(seed, PURPOSE_MIX)
    probs = []
    lo, hi = np.log2(n_min), np.log2(n_max)
    for f in range(n_filters):
        is_chain = g.uniform() < chain_fraction
        n = int(round(2.0 ** (lo + (hi - lo) * g.uniform())))
        if is_chain:
            probs.append(chain16(n, 100, seed=f, model_seed=CHAIN_INSTANCES[f % N_CHAIN_INSTANCES]))
        else:
            probs.append(robertson(n, 50, seed=f))
    return probs


@dataclasses.dataclass
class StreamRequest:
    stream_id: int
    arrival: float             # seconds after start
    problem: Problem
    obs_offsets: np.ndarray    # (T,) wall-clock offsets of each observation after arrival


def serving_trace(n_streams: int = 2000, rate: float = 200.0, seed: int = 0,
                  chain_fraction: float = 0.3, sizes=(4096, 16384, 65536),
                  obs_gap_mean: float = 0.010):
    """Poisson arrivals of filtering streams; each stream then delivers its
    observations with exponential wall-clock gaps."""
    g = _stream(seed, PURPOSE_ARRIVAL)
    t = 0.0
    out = []
    for s in range(n_streams):
        t += g.exponential(1.0 / rate)
        is_chain = g.uniform() < chain_fraction
        n = int(sizes[int(g.integers(len(sizes)))])
        if is_chain:
            prob = chain16(n, 100, seed=1000 + s, model_seed=CHAIN_INSTANCES[s % N_CHAIN_INSTANCES])
        else:
            prob = robertson(n, 50, seed=1000 + s)
        gaps = g.exponential(obs_gap_mean, prob.T)
        out.append(StreamRequest(s, t, prob, np.cumsum(gaps)))
    return out
