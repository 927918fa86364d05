"""Pins of the oracle's weights, systematic resampling, moments and
Cholesky factor (Algorithm 1 steps 1, 3, 5 and 6)."""
from fractions import Fraction
import itertools

import numpy as np
import pytest
from scipy import stats


# ---------------------------------------------------------------- likelihood
def test_loglik_is_gaussian_up_to_constants(oracle):
    rng = np.random.default_rng(1)
    obs = [1, 2]
    for _ in range(10):
        x = rng.standard_normal(3)
        x2 = rng.standard_normal(3)
        y = rng.standard_normal(2)
        sig = rng.uniform(0.1, 2.0, 2)
        d_or = oracle.loglik(x, y, sig, obs) - oracle.loglik(x2, y, sig, obs)
        d_sp = (stats.norm.logpdf(y, x[obs], sig).sum() - stats.norm.logpdf(y, x2[obs], sig).sum())
        assert d_or == pytest.approx(d_sp, rel=1e-12, abs=1e-12)
    assert oracle.loglik(x, y, sig, obs) <= 0.0


def test_loglik_nonfinite_state(oracle):
    assert oracle.loglik(np.array([0.0, np.nan, 1.0]), [0.0], [1.0], [1]) == -np.inf
    assert oracle.loglik(np.array([0.0, np.inf, 1.0]), [0.0], [1.0], [1]) == -np.inf
    # a non-finite unobserved component does not matter
    assert np.isfinite(oracle.loglik(np.array([np.nan, 0.5, 1.0]), [0.0], [1.0], [1]))


# ---------------------------------------------------------------- normalisation
def test_normalise_sums_to_one_and_shift_invariant(oracle):
    rng = np.random.default_rng(2)
    for N in (1, 7, 1000, 100000):
        l = rng.standard_normal(N) * 30
        w, lz = oracle.normalise(l)
        assert abs(w.sum() - 1) < 4 * N * 2.0**-53 + 1e-15
        w2, lz2 = oracle.normalise(l + 1234.5)
        assert np.allclose(w, w2, rtol=1e-9, atol=0)
        assert lz2 - lz == pytest.approx(1234.5, rel=1e-12)
        assert lz == pytest.approx(np.logaddexp.reduce(l), rel=1e-12)


def test_normalise_degenerate(oracle):
    w, lz = oracle.normalise(np.array([-np.inf, -np.inf, np.nan]))
    assert lz == -np.inf and not w.any()
    w, lz = oracle.normalise(np.array([-np.inf, 0.0, np.nan]))
    assert w.tolist() == [0.0, 1.0, 0.0]


# ---------------------------------------------------------------- resampling
def _systematic_rational(q, V):
    """Systematic resampling written with exact rationals: u_i = (i + U)/N with
    U = V/T, ancestor of slot i = first k with C_k / T > u_i."""
    N, T = len(q), sum(q)
    C = list(itertools.accumulate(q))
    U = Fraction(V, T)
    out = []
    for i in range(N):
        u = (i + U) / N
        out.append(next(k for k in range(N) if Fraction(C[k], T) > u))
    return np.array(out)


def test_resample_int_brute_force_small(oracle):
    rng = np.random.default_rng(4)
    for N in range(1, 9):
        for _ in range(40):
            q = rng.integers(0, 6, N).astype(np.uint64)
            if q.sum() == 0:
                q[rng.integers(N)] = 1
            T = int(q.sum())
            for V in sorted({0, T - 1, int(rng.integers(T))}):
                st, anc = oracle.resample_int(q, V)
                assert st == 0
                assert np.array_equal(anc, _systematic_rational([int(v) for v in q], V))


def test_resample_exact_expectation(oracle):
    # over all offsets V in [0, T) each particle is copied exactly N q_k times
    rng = np.random.default_rng(5)
    for N in (1, 2, 3, 5, 8):
        for _ in range(10):
            q = rng.integers(0, 5, N).astype(np.uint64)
            q[0] += 1
            T = int(q.sum())
            total = np.zeros(N, dtype=np.int64)
            for V in range(T):
                st, anc = oracle.resample_int(q, V)
                total += np.bincount(anc, minlength=N)
            assert np.array_equal(total, N * q.astype(np.int64))


def test_resample_counts_floor_or_ceil(oracle):
    rng = np.random.default_rng(6)
    for N in (2, 5, 8, 100, 4096):
        g = rng.exponential(size=N) ** 3
        g[rng.integers(N)] = 0.0
        g /= g.sum()
        for r in rng.integers(0, 2**63, 5, dtype=np.int64):
            st, anc = oracle.resample(g, int(r) * 2 + 1)
            assert st == 0
            assert np.all(np.diff(anc) >= 0)
            cnt = np.bincount(anc, minlength=N)
            S = oracle.resample_shift(N)
            q = np.floor(np.ldexp(g, S))
            share = N * q / q.sum()
            assert np.all(cnt >= np.floor(share)) and np.all(cnt <= np.floor(share) + 1)
            assert np.all(cnt[g == 0] == 0)


def test_resample_shift_keeps_products_below_2_63(oracle):
    for N in (1, 2, 3, 1000, 1024, 1025, 1 << 17, (1 << 24) - 3):
        S = oracle.resample_shift(N)
        assert (1 << (62 - S)) >= N
        assert 2 * (1 << S) * N <= 1 << 63


def test_resample_equal_weights_is_identity(oracle):
    for N in (1, 10, 1000, 4097):
        for r in (0, 12345, 2**64 - 1):
            st, anc = oracle.resample(np.full(N, 1.0 / N), r)
            assert np.array_equal(anc, np.arange(N))


def test_resample_degenerate(oracle):
    st, _ = oracle.resample(np.zeros(4), 7)
    assert st == oracle.EDEGENERATE


# ---------------------------------------------------------------- moments
def test_moments_match_numpy(oracle):
    rng = np.random.default_rng(7)
    for N, p in ((10, 3), (1000, 12), (5, 1)):
        th = rng.standard_normal((N, p)) * rng.uniform(0.1, 3, p) + rng.standard_normal(p)
        w = rng.exponential(size=N)
        w /= w.sum()
        mean, cov = oracle.moments(th, w)
        assert np.allclose(mean, np.average(th, axis=0, weights=w), rtol=1e-12, atol=1e-14)
        want = np.atleast_2d(np.cov(th.T, aweights=w, bias=True))
        assert np.allclose(cov, want, rtol=1e-10, atol=1e-14)


def test_cholesky_matches_numpy(oracle):
    rng = np.random.default_rng(8)
    for p in (1, 3, 12):
        A = rng.standard_normal((p, p + 3))
        Cm = A @ A.T
        st, L, jit = oracle.cholesky(Cm)
        assert st == 0 and jit == 0
        assert np.allclose(L, np.linalg.cholesky(Cm), rtol=1e-10, atol=1e-12)


def test_cholesky_jitter_rule(oracle):
    # rank-deficient but non-zero trace: the first jitter 1e-10 tr/p succeeds
    v = np.array([1.0, 2.0, 3.0])
    Cm = np.outer(v, v)
    st, L, jit = oracle.cholesky(Cm)
    assert st == 0 and jit >= 1
    assert np.allclose(L @ L.T, Cm, atol=1e-8)
    st, _, _ = oracle.cholesky(np.zeros((3, 3)))
    assert st == oracle.EDEGENERATE
