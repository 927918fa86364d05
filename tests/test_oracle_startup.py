"""Pins of the order-preserving start-up (BDF with an L-stable SDIRK method of
order k for the first k - 1 steps of every interval): the Butcher tables'
order conditions, stiff accuracy and L-stability, interval orders under step
halving, stiff damping, the linear invariant and the Radau truth."""
import numpy as np
import pytest

from paper_1411_1702_amd import inputs


@pytest.mark.parametrize("k", [2, 3])
def test_sdirk_tables(oracle, k):
    A, ns = oracle.sdirk(k)
    b = A[-1]
    c = A.sum(axis=1)
    assert ns == k
    assert np.allclose(np.diag(A), A[0, 0]) and np.allclose(np.triu(A, 1), 0)   # singly diagonal, implicit
    assert b.sum() == pytest.approx(1, abs=1e-15)
    assert b @ c == pytest.approx(0.5, abs=1e-15)
    if k == 3:
        assert b @ c**2 == pytest.approx(1 / 3, abs=1e-15)
        assert b @ A @ c == pytest.approx(1 / 6, abs=1e-15)
    # stability function R(z) = 1 + z b^T (I - zA)^{-1} 1: L-stable (R -> 0) and
    # A-stable on the imaginary axis
    def R(z):
        return 1 + z * b @ np.linalg.solve(np.eye(ns) - z * A, np.ones(ns))
    assert abs(R(-1e8)) < 1e-6
    assert all(abs(R(1j * y)) <= 1 + 1e-12 for y in np.logspace(-3, 6, 40))
    assert all(abs(R(-x)) < 1 for x in np.logspace(-3, 6, 40))


def _decay(oracle, lam, T, M, k, lmm=2):
    return oracle.psi(0, np.array([1.0]), np.log([lam]), T / M, M, k, rtol=1e-14,
                      floor=np.array([1e-300]), lmm=lmm)


def _slope(e):
    return np.log2(e[:-1] / e[1:])


@pytest.mark.parametrize("k", [1, 2, 3])
def test_startup_restores_interval_order(oracle, k):
    lam = 2.0
    errs = np.array([abs(_decay(oracle, lam, 1.0, M, k)[0][0] - np.exp(-lam)) for M in (160, 320, 640, 1280)])
    sl = _slope(errs)
    assert np.all(sl > k - 0.08) and abs(sl[-1] - k) < 0.03, sl
    if k == 3:
        # the restarted ramp caps BDF3 at order 2
        ramp = np.array([abs(_decay(oracle, lam, 1.0, M, k, lmm=0)[0][0] - np.exp(-lam)) for M in (320, 640, 1280)])
        assert np.allclose(_slope(ramp), 2.0, atol=0.06)
        assert errs[-1] < ramp[-1] / 10


@pytest.mark.parametrize("k", [2, 3])
def test_startup_damps_stiff_decay(oracle, k):
    # h lambda = 2.5e5: L-stable start, then BDF
    x, _, _ = _decay(oracle, 1e6, 1.0, 4, k)
    assert abs(x[0]) < 1e-9


def test_startup_robertson_invariant_and_radau(oracle):
    pr = inputs.robertson(10, 50)
    rng = np.random.default_rng(2)
    for j in (0, 10, 30, 49):
        x0 = pr.x_true[j - 1] if j else pr.x0
        t0 = pr.times[j - 1] if j else 0.0
        th = pr.theta_true + 0.5 * rng.standard_normal(3)
        x, _, _ = oracle.psi(1, x0, th, (pr.times[j] - t0) / 20, 20, 3, rtol=1e-12,
                             floor=pr.state_floor, lmm=2)
        assert abs(x.sum() - x0.sum()) < 5e-15
    j = 20
    x0, t0, t1 = pr.x_true[j - 1], pr.times[j - 1], pr.times[j]
    errs = []
    for M in (20, 40, 80, 160):
        x, _, _ = oracle.psi(1, x0, pr.theta_true, (t1 - t0) / M, M, 3, rtol=1e-13,
                             floor=pr.state_floor, lmm=2)
        errs.append(np.max(np.abs(x - pr.x_true[j]) / np.maximum(np.abs(pr.x_true[j]), pr.state_floor)))
    errs = np.array(errs)
    assert np.all(_slope(errs) > 2.4), _slope(errs)


def test_startup_filter_posterior_contracts(oracle):
    pr = inputs.config_small()
    pr.lmm, pr.order = 2, 3
    means, sds, ess = oracle.Filter(pr).run()
    # the first observation is nearly degenerate at N = 1000 for every start-up
    # (effective sample size 1-65 across BDF2/3 with and without it); later
    # steps are healthy
    assert ess[0] >= 1.0 and np.all(ess[1:] > 10)
    assert np.all(sds[-1] < pr.prior_sd / 5)
    assert np.all(np.abs(means[-1] - pr.theta_true) < 4 * sds[-1] + 0.05)


def test_startup_accuracy_on_robertson_interval(oracle):
    # One observation interval of the large Robertson schedule at M = 20: the
    # start-up makes BDF3 third order (error ratio ~8 under step halving
    # instead of ~4) and far more accurate at the same M
    prob = inputs.config_robertson_large()
    j = 20
    x0, H = prob.x_true[j - 1], prob.times[j] - prob.times[j - 1]
    th = prob.prior_mean
    kw = dict(lte=False, rtol=1e-13, kmax=20, floor=prob.state_floor)
    ref, _, _ = oracle.psi(prob.model, x0, th, H / 4000, 4000, 3, lmm=2, **kw)

    def err(lmm, M):
        x, _, _ = oracle.psi(prob.model, x0, th, H / M, M, 3, lmm=lmm, **kw)
        return np.max(np.abs(x - ref) / np.maximum(np.abs(ref), prob.state_floor))

    e_bdf, e_sd = err(0, 20), err(2, 20)
    assert e_sd < e_bdf / 20, (e_bdf, e_sd)
    assert 6.5 < e_sd / err(2, 40) < 10.0
    assert 3.0 < e_bdf / err(0, 40) < 5.0
