"""Pins of the oracle's multinomial resampling (the literal draw of Algorithm 1
step 3(b): every output slot an independent index drawn with probability
g_k), on the same integer weights q_k = floor(g_k 2^S) as the systematic
scheme: slot i takes the first k with C_k > floor(r_i T / 2^64).

Pinned against numpy.searchsorted on exact integer targets, the binomial
mean and variance of the offspring counts, the chi-square law of the draws,
numpy's independent Philox for the per-slot words, and the degenerate cases.
"""
import numpy as np
import pytest
from scipy import stats

from test_oracle_philox import _numpy_block

PUR_RESAMPLE = 2


def _targets(q, r):
    T = int(sum(int(v) for v in q))
    return [(int(ri) * T) >> 64 for ri in r], T


def test_multinomial_int_is_searchsorted(oracle):
    rng = np.random.default_rng(3)
    for N in (1, 2, 7, 64, 1000):
        q = rng.integers(0, 2**40, size=N, dtype=np.uint64)
        q[rng.random(N) < 0.3] = 0
        if q.sum() == 0:
            q[0] = 1
        r = rng.integers(0, 2**63, size=N, dtype=np.uint64) * 2 + rng.integers(0, 2, size=N, dtype=np.uint64)
        st, anc = oracle.resample_multinomial_int(q, r)
        assert st == 0
        tau, T = _targets(q, r)
        C = np.cumsum([int(v) for v in q], dtype=object)
        ref = np.searchsorted(np.array(C, dtype=np.float64), np.array(tau, dtype=np.float64), side="right")
        # the float search is exact here only when the values fit 53 bits; check by integers instead
        ref_int = [next(k for k in range(N) if C[k] > t) for t in tau]
        assert list(anc) == ref_int
        if T < 2**53:
            assert list(anc) == list(ref)
        # every chosen particle has weight
        assert all(q[k] > 0 for k in anc)


def test_multinomial_hand_example(oracle):
    # q = (1, 0, 3, 4), T = 8, C = (1, 1, 4, 8)
    q = np.array([1, 0, 3, 4], dtype=np.uint64)
    r = np.array([0, 2**62, 2**63, 2**64 - 1], dtype=np.uint64)   # tau = 0, 2, 4, 7
    st, anc = oracle.resample_multinomial_int(q, r)
    assert st == 0 and list(anc) == [0, 2, 3, 3]


def test_multinomial_counts_binomial_moments(oracle):
    # offspring count of particle k over many independent steps: Binomial(N, g_k)
    N, reps = 16, 4000
    g = np.array([0.3, 0.2, 0.15, 0.1, 0.1, 0.05, 0.05, 0.05] + [0.0] * 8)
    counts = np.zeros((reps, N))
    for s in range(reps):
        st, anc = oracle.resample_multinomial(g, seed=11, step=s + 1)
        assert st == 0
        counts[s] = np.bincount(anc, minlength=N)
    mean, var = counts.mean(0), counts.var(0, ddof=1)
    se_mean = np.sqrt(N * g * (1 - g) / reps)
    assert np.all(np.abs(mean - N * g) <= 4 * se_mean + 1e-12)
    nz = g > 0
    # sample variance of a binomial: relative s.e. ~ sqrt(2/reps) (+ kurtosis), allow 15%
    assert np.all(np.abs(var[nz] / (N * g[nz] * (1 - g[nz])) - 1) < 0.15)
    assert np.all(counts[:, ~nz] == 0)


def test_multinomial_chi_square(oracle):
    N = 200000
    g = np.array([0.5, 0.25, 0.125, 0.0625, 0.0625])
    gg = np.zeros(N)
    gg[:5] = g
    st, anc = oracle.resample_multinomial(gg, seed=5, step=7)
    assert st == 0
    obs = np.bincount(anc, minlength=5)[:5]
    assert obs.sum() == N
    chi2, p = stats.chisquare(obs, N * g)
    assert p > 1e-4


def test_multinomial_words_are_philox_per_slot(oracle):
    # slot i's word is Philox(seed; step, i, RESAMPLE, 0)[0], from numpy's Philox
    N, seed, step = 37, 123, 9
    rng = np.random.default_rng(8)
    g = rng.random(N)
    g /= g.sum()
    st, anc = oracle.resample_multinomial(g, seed=seed, step=step)
    assert st == 0
    S = oracle.resample_shift(N)
    q = np.array([int(np.floor(np.ldexp(v, S))) for v in g], dtype=object)
    r = [int(_numpy_block([step, i, PUR_RESAMPLE, 0], [seed, 0])[0]) for i in range(N)]
    T = int(sum(q))
    C = np.cumsum(q)
    ref = [next(k for k in range(N) if C[k] > (ri * T) >> 64) for ri in r]
    assert list(anc) == ref


def test_multinomial_degenerate_and_single(oracle):
    st, _ = oracle.resample_multinomial_int(np.zeros(5, dtype=np.uint64), np.arange(5, dtype=np.uint64))
    assert st != 0
    q = np.zeros(9, dtype=np.uint64)
    q[4] = 7
    st, anc = oracle.resample_multinomial_int(q, np.array([0, 1, 2**63, 2**64 - 1] * 2 + [5], dtype=np.uint64))
    assert st == 0 and np.all(anc == 4)


def test_filter_with_multinomial_keeps_prior_under_flat_data(oracle):
    # uninformative observations (huge sigma): the posterior stays at the prior
    # (mean within Monte Carlo error, a^2 + s^2 = 1 keeps the spread)
    from paper_1411_1702_amd import inputs
    prob = inputs.robertson(4000, 6, seed=2)
    prob.sigma[:] = 1e12
    F = oracle.Filter(prob, resampling=1)
    for j in range(6):
        out = F.step(prob.times[j], prob.y[j], prob.sigma[j])
        assert out["status"] == 0
    mean, cov = F.moments()
    sd = np.asarray(prob.prior_sd)
    assert np.all(np.abs(mean - np.asarray(prob.prior_mean)) < 5 * sd / np.sqrt(4000) * 3)
    assert np.all(np.abs(np.sqrt(np.diag(cov)) / sd - 1) < 0.15)
