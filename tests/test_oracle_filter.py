"""End-to-end pins of the oracle filter (Algorithm 1)."""
import dataclasses

import numpy as np
import pytest

from paper_1411_1702_amd import inputs


def _decay_problem(N, sigma=1e10, T=3, seed=0):
    """x' = -k x per component, d = p = 3, with (almost) uninformative data."""
    times = np.array([0.5, 1.0, 1.5, 2.0, 2.5])[:T]
    x0 = np.array([1.0, 2.0, 3.0])
    theta = np.log(np.array([0.5, 1.0, 2.0]))
    return inputs.Problem(
        name="decay", model=0, d=3, p=3, m=1, obs_index=np.array([0], dtype=np.int32),
        model_consts=np.zeros(0), rates_fixed=np.zeros(0), x0=x0,
        prior_mean=theta, prior_sd=np.array([0.3, 0.5, 0.2]), theta_true=theta, t0=0.0,
        times=times, x_true=np.zeros((T, 3)), y=np.zeros((T, 1)), sigma=np.full((T, 1), sigma),
        order=2, substeps=4, n_particles=N, seed=seed, state_floor=np.full(3, 1e-8))


def test_uninformative_step_preserves_mean_and_covariance(oracle):
    # equal weights: systematic resampling keeps every particle once, and the
    # shrink-then-jitter kernel with a^2 + s^2 = 1 keeps mean and covariance
    N = 200_000
    pr = _decay_problem(N)
    F = oracle.Filter(pr)
    m0, C0 = F.moments()
    rc, g, anc = F.stage1(pr.times[0], pr.y[0], pr.sigma[0])
    assert rc == 0 and np.array_equal(anc, np.arange(N))
    out = F.step(pr.times[0], pr.y[0], pr.sigma[0])
    assert out["status"] == 0
    m1, C1 = F.moments()
    sd0 = np.sqrt(np.diag(C0))
    assert np.all(np.abs(m1 - m0) < 4.5 * sd0 / np.sqrt(N))
    assert np.allclose(np.diag(C1), np.diag(C0), rtol=4.5 * np.sqrt(2.0 / N) * 1.5)
    assert abs(C1[0, 1]) < 4.5 * sd0[0] * sd0[1] / np.sqrt(N) * 1.5
    # the prior itself: mean and sd as configured
    assert np.allclose(sd0, pr.prior_sd, rtol=4.5 * np.sqrt(2.0 / N))


def test_uninformative_filter_stays_at_prior(oracle):
    N = 20_000
    pr = _decay_problem(N, T=5)
    F = oracle.Filter(pr)
    means, sds, ess = F.run()
    assert np.all(ess > 0.999 * N)
    assert np.all(np.abs(means - pr.prior_mean) < 5 * pr.prior_sd * np.sqrt(6.0 / N))
    assert np.allclose(sds, pr.prior_sd, rtol=0.05)


def test_small_robertson_posterior_contracts(oracle):
    pr = inputs.config_small()
    F = oracle.Filter(pr)
    means, sds, ess = F.run()
    assert np.all(ess > 10)
    assert np.all(sds[-1] < pr.prior_sd / 5)
    assert np.all(np.abs(means[-1] - pr.theta_true) < 4 * sds[-1] + 0.05)


def test_deterministic(oracle):
    pr = inputs.robertson(300, 10)
    a = oracle.Filter(pr).run()
    b = oracle.Filter(pr).run()
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    c = oracle.Filter(pr, seed=1).run()
    assert not np.array_equal(a[0], c[0])


def test_stage1_ancestors_consistent(oracle):
    pr = inputs.robertson(500, 10)
    F = oracle.Filter(pr)
    F.run(3)
    rc, g, anc = F.stage1(pr.times[3], pr.y[3], pr.sigma[3])
    assert rc == 0
    assert abs(g.sum() - 1) < 1e-12
    w = oracle.philox([4, 0, oracle.PUR_RESAMPLE, 0], [pr.seed, 0])[0]
    st, anc2 = oracle.resample(g, int(w))
    assert np.array_equal(anc, anc2)
    assert np.all(np.diff(anc) >= 0)


def test_step_given_own_ancestors_is_the_step(oracle):
    # the step with its own draw passed in computes exactly the plain step;
    # with a different valid draw the copies follow those ancestors
    pr = inputs.robertson(500, 10)
    A, B, C = oracle.Filter(pr), oracle.Filter(pr), oracle.Filter(pr)
    for F in (A, B, C):
        F.run(3)
    rc, _, anc = A.stage1(pr.times[3], pr.y[3], pr.sigma[3])
    assert rc == 0
    assert A.step(pr.times[3], pr.y[3], pr.sigma[3])["status"] == 0
    assert B.step_given(pr.times[3], pr.y[3], pr.sigma[3], anc) == 0
    assert np.array_equal(A.x, B.x) and np.array_equal(A.theta, B.theta)
    assert np.array_equal(A.logw, B.logw)
    shifted = np.roll(anc, 1)
    assert C.step_given(pr.times[3], pr.y[3], pr.sigma[3], shifted) == 0
    # slot n now repropagates ancestor shifted[n]: its parameters are that
    # ancestor's shrunk ones plus the slot's own jitter, so they differ
    assert not np.array_equal(C.theta, A.theta)
    bad = anc.copy()
    bad[0] = pr.n_particles
    D = oracle.Filter(pr)
    D.run(3)
    assert D.step_given(pr.times[3], pr.y[3], pr.sigma[3], bad) == oracle.EINVAL
    assert D.j == 3


def test_degenerate_observation_leaves_state_unchanged(oracle):
    pr = inputs.robertson(200, 5)
    F = oracle.Filter(pr)
    F.run(2)
    x, th, lw, mom = F.x.copy(), F.theta.copy(), F.logw.copy(), F.moments()
    out = F.step(pr.times[2], [1e200], [1e-200])
    assert out["status"] == oracle.EDEGENERATE
    assert np.array_equal(F.x, x) and np.array_equal(F.theta, th) and np.array_equal(F.logw, lw)
    assert F.j == 2
    out = F.step(pr.times[2], pr.y[2], pr.sigma[2])
    assert out["status"] == 0 and F.j == 3


def test_invalid_inputs(oracle):
    pr = inputs.robertson(50, 5)
    F = oracle.Filter(pr)
    assert F.step(pr.times[0], [np.nan], [1.0])["status"] == oracle.EINVAL
    assert F.step(pr.times[0], [1.0], [0.0])["status"] == oracle.EINVAL
    assert F.step(0.0, [1.0], [1.0])["status"] == oracle.EINVAL
    assert F.j == 0
