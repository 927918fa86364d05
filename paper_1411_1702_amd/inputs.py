"""Seeded synthetic workloads for the LMM PF-SMC sampler.

This module only *generates inputs*: problem definitions (model constants,
priors, observation times), true trajectories and noisy observations.  It
holds none of the filter's arithmetic.  Both the GPU library and the CPU
oracle consume what it produces, so it must not import either of them.

The paper's own test problems cannot be rebuilt from its text (the
Michaelis-Menten system of Sec. 2.1 prints no constants), so the workloads are:

* Robertson stiff kinetics, 3 states, log-rates estimated;
* a 16-compartment chain with Michaelis-Menten losses, 12 log-rates estimated;
* mixes of the two for many independent filters (batched and served forms).

True trajectories come from scipy's Radau integrator at tight tolerance; the
model right-hand sides below exist only for that purpose.  Observation noise,
chain constants and the mixes are drawn from numpy's Philox4x64-10 streams
keyed by (seed, purpose).
"""
from __future__ import annotations

import dataclasses
import functools

import numpy as np

MODEL_ROBERTSON = 1
MODEL_CHAIN = 2

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
    model_consts: np.ndarray     # chain: [V(d), K(d)]; Robertson: empty
    rates_fixed: np.ndarray      # chain: all d rates (first p are estimated); Robertson: empty
    x0: np.ndarray               # (d,)
    prior_mean: np.ndarray       # (p,) Gaussian prior on log-parameters
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
    lmm: int = 0                     # 0 BDF (order k), 1 Adams-Moulton (k steps)

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
