"""Pins of the oracle's Adams-Moulton propagation (the paper's other implicit
LMM family; AMk read as the k-step formula of order k + 1, AM1 the
trapezoidal rule) against exact rational order conditions, closed forms,
convergence orders under step halving, the true one-step error, a linear
invariant and the Radau truth."""
from fractions import Fraction
from math import factorial

import numpy as np
import pytest

from paper_1411_1702_amd import inputs


@pytest.mark.parametrize("q", [1, 2, 3])
def test_am_order_conditions_exact(oracle, q):
    beta, errc = oracle.am(q)
    B = [Fraction(b).limit_denominator(10000) for b in beta]
    E = Fraction(errc).limit_denominator(10000)
    assert [float(b) for b in B] == list(beta) and float(E) == errc
    # x(t) = t^r, t_m = 0, h = 1: x_m - x_{m-1} = -(-1)^r, f_{m-i} = r (-i)^(r-1)
    def residual(r):
        lhs = Fraction(0) ** r - Fraction(-1) ** r
        rhs = sum(B[i] * r * Fraction(-i) ** (r - 1) for i in range(q + 1)) if r > 0 else Fraction(0)
        return lhs - rhs
    for r in range(q + 2):
        assert residual(r) == 0, (q, r)           # order q + 1
    assert abs(residual(q + 2)) / factorial(q + 2) == E
    assert residual(q + 2) != 0


def _decay(oracle, lam, x0, T, M, k, hist=None, lte=False, rtol=1e-14):
    theta = np.log(np.atleast_1d(lam))
    return oracle.psi(0, np.atleast_1d(x0), theta, T / M, M, k, lte=lte, rtol=rtol,
                      floor=np.full(len(theta), 1e-300), hist=hist, lmm=1)


def _slope(errs):
    return np.log2(errs[:-1] / errs[1:])


def test_am1_trapezoid_closed_form(oracle):
    for lam, T, M in ((2.0, 1.0, 10), (50.0, 0.3, 7), (1e4, 1.0, 5)):
        z = lam * T / M
        x, _, _ = _decay(oracle, lam, 1.0, T, M, 1)
        assert x[0] == pytest.approx(((1 - z / 2) / (1 + z / 2)) ** M, rel=1e-12, abs=1e-300)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_am_full_order_with_exact_history(oracle, k):
    lam, T = 2.0, 1.0
    errs = []
    for M in (20, 40, 80, 160):
        h = T / M
        hist = np.array([[np.exp(lam * h * r)] for r in range(1, k + 2)])
        x, _, _ = _decay(oracle, lam, 1.0, T, M, k, hist=hist)
        errs.append(abs(x[0] - np.exp(-lam * T)))
    assert np.allclose(_slope(np.array(errs)), k + 1, atol=0.12), _slope(np.array(errs))


@pytest.mark.parametrize("k", [1, 2, 3])
def test_am_restarted_at_least_second_order(oracle, k):
    # restart from one value each interval: the first step is the trapezoidal
    # rule and every later step is at least second order, so the interval is
    # at least second order (on this linear problem the startup error of the
    # two- and three-step formulas even decays faster than h^3)
    lam, T = 2.0, 1.0
    errs = np.array([abs(_decay(oracle, lam, 1.0, T, M, k)[0][0] - np.exp(-lam * T))
                     for M in (20, 40, 80, 160)])
    assert np.all(_slope(errs) > 1.9), _slope(errs)
    if k == 1:
        assert np.allclose(_slope(errs), 2.0, atol=0.05)


def test_am_stiff_stability(oracle):
    # x' = -lambda x with h lambda = 10: the trapezoidal rule (A-stable) decays,
    # the two- and three-step formulas (real stability interval about
    # [-6, 0] and [-3, 0]) grow -- why the stiff workloads use AM1
    lam, T, M = 200.0, 1.0, 20
    x1, _, _ = _decay(oracle, lam, 1.0, T, M, 1)
    x2, _, _ = _decay(oracle, lam, 1.0, T, M, 2)
    x3, _, _ = _decay(oracle, lam, 1.0, T, M, 3)
    assert abs(x1[0]) < 1.0
    assert abs(x2[0]) > 1.0 and abs(x3[0]) > 1.0


@pytest.mark.parametrize("k,hs", [(1, (1e-2, 1e-3, 1e-4)), (2, (3e-2, 1e-2, 3e-3))])
def test_am_lte_estimate_matches_true_one_step_error(oracle, k, hs):
    # one step from exact history (enough for the full-order comparison
    # value): the Milne estimate -> the true local error as h -> 0
    lam = 3.0
    dev = []
    for h in hs:
        hist = np.array([[np.exp(lam * h * r)] for r in range(1, k + 2)])
        x, gam, _ = _decay(oracle, lam, 1.0, h, 1, k, hist=hist, lte=True)
        ratio = np.sqrt(gam[0]) / abs(np.exp(-lam * h) - x[0])
        dev.append(abs(ratio - 1))
        assert dev[-1] < 10 * lam * h
    assert dev[-1] < dev[0]


def test_am_robertson_linear_invariant(oracle):
    pr = inputs.robertson(10, 50)
    rng = np.random.default_rng(1)
    # AM1 (A-stable) on every interval; AM2, AM3 where h keeps the stiff
    # eigenvalue inside their stability intervals (the first interval)
    for j in (0, 10, 30, 49):
        x0 = pr.x_true[j - 1] if j else pr.x0
        t0 = pr.times[j - 1] if j else 0.0
        for k in ((1, 2, 3) if j == 0 else (1,)):
            th = pr.theta_true + 0.5 * rng.standard_normal(3)
            x, _, _ = oracle.psi(1, x0, th, (pr.times[j] - t0) / 20, 20, k, rtol=1e-12,
                                 floor=pr.state_floor, lmm=1)
            assert abs(x.sum() - x0.sum()) < 5e-15


def test_am_robertson_global_error_vs_radau(oracle):
    # x_true holds the Radau solution at the observation times; AM1 is second
    # order on the stiff problem
    pr = inputs.robertson(10, 50)
    j = 20
    x0, t0, t1 = pr.x_true[j - 1], pr.times[j - 1], pr.times[j]
    errs = []
    for M in (20, 40, 80, 160):
        x, _, _ = oracle.psi(1, x0, pr.theta_true, (t1 - t0) / M, M, 1, rtol=1e-13,
                             floor=pr.state_floor, lmm=1)
        errs.append(np.max(np.abs(x - pr.x_true[j]) / np.maximum(np.abs(pr.x_true[j]), pr.state_floor)))
    errs = np.array(errs)
    assert errs[-1] < 1e-5
    assert np.all(_slope(errs) > 1.7), _slope(errs)


def test_am_filter_posterior_contracts(oracle):
    pr = inputs.config_small()
    pr.lmm, pr.order = 1, 1      # the trapezoidal rule: A-stable on the stiff problem
    F = oracle.Filter(pr)
    means, sds, ess = F.run()
    assert np.all(ess > 10)
    assert np.all(sds[-1] < pr.prior_sd / 5)
    assert np.all(np.abs(means[-1] - pr.theta_true) < 4 * sds[-1] + 0.05)
