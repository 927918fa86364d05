"""Pins of the oracle's integrator Psi (BDF + Newton + local-error estimate)
against closed forms, exact rational order conditions, library routines and
the Radau truth (Algorithm 1 steps 2 and 4; Sec. 2.1)."""
from fractions import Fraction
from math import factorial

import numpy as np
import pytest
from scipy.linalg import expm

from paper_1411_1702_amd import inputs


# ---------------------------------------------------------------- coefficients
@pytest.mark.parametrize("q", [1, 2, 3])
def test_bdf_order_conditions_exact(oracle, q):
    alpha, beta, errc = oracle.bdf(q)
    A = [Fraction(a).limit_denominator(1000) for a in alpha]
    B = Fraction(beta).limit_denominator(1000)
    Cq = Fraction(errc).limit_denominator(1000)
    assert [float(a) for a in A] == list(alpha) and float(B) == beta and float(Cq) == errc
    # apply the formula to x(t) = t^r with t_m = 0, h = 1: residual
    #   sum_i alpha_i (-i)^r - beta * r * 0^(r-1)
    for r in range(q + 1):
        lhs = sum(A[i] * Fraction(-i) ** r for i in range(q + 1))
        rhs = B * r if r == 1 else Fraction(0)
        assert lhs == rhs, (q, r)
    # degree q+1 gives the error constant
    lead = sum(A[i] * Fraction(-i) ** (q + 1) for i in range(q + 1)) / factorial(q + 1)
    assert lead == Cq
    # general closed form of the BDF error constant: -1/((q+1) H_q)
    Hq = sum(Fraction(1, i) for i in range(1, q + 1))
    assert Cq == -1 / ((q + 1) * Hq)


# ---------------------------------------------------------------- x' = -lambda x
def _decay(oracle, lam, x0, T, M, k, hist=None, lte=False, rtol=1e-14):
    theta = np.log(np.atleast_1d(lam))
    return oracle.psi(0, np.atleast_1d(x0), theta, T / M, M, k, lte=lte, rtol=rtol,
                      floor=np.full(len(theta), 1e-300), hist=hist)


def test_bdf1_closed_form(oracle):
    for lam, T, M in [(1.0, 1.0, 10), (50.0, 0.3, 7), (1e4, 2.0, 20)]:
        x, _, st = _decay(oracle, lam, 2.0, T, M, 1)
        h = T / M
        assert x[0] == pytest.approx(2.0 / (1 + h * lam) ** M, rel=1e-13)
        assert st["newton_fails"] == 0


def test_diagonal_multi_component_matches_scalar(oracle):
    lams = np.array([0.5, 3.0, 40.0, 900.0])
    x0 = np.array([1.0, -2.0, 0.5, 3.0])
    x, _, _ = _decay(oracle, lams, x0, 1.5, 12, 2)
    for i in range(4):
        xi, _, _ = _decay(oracle, lams[i], x0[i], 1.5, 12, 2)
        assert x[i] == pytest.approx(xi[0], rel=1e-14)


def test_linear_newton_exact_after_one_iteration(oracle):
    # the first Newton update solves the linear step exactly: a loose and a
    # tight stopping tolerance give the same result
    a, _, _ = _decay(oracle, 7.0, 1.0, 1.0, 9, 3, rtol=1e-3)
    b, _, _ = _decay(oracle, 7.0, 1.0, 1.0, 9, 3, rtol=1e-15)
    assert a[0] == pytest.approx(b[0], rel=1e-14)


def _slope(errs):
    return np.log2(errs[:-1] / errs[1:])


@pytest.mark.parametrize("k,expected", [(1, 1.0), (2, 2.0), (3, 2.0)])
def test_restarted_order_under_step_halving(oracle, k, expected):
    # restart from one value each interval: order ramp 1,1,2,..,k; the two
    # first-order start steps cap the interval's order at 2
    lam, T = 2.0, 1.0
    errs = np.array([abs(_decay(oracle, lam, 1.0, T, M, k)[0][0] - np.exp(-lam * T))
                     for M in (40, 80, 160, 320)])
    assert np.allclose(_slope(errs), expected, atol=0.08), _slope(errs)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_full_order_with_exact_history(oracle, k):
    lam, T = 2.0, 1.0
    errs = []
    for M in (40, 80, 160, 320):
        h = T / M
        hist = np.array([[np.exp(lam * h * r)] for r in range(1, k)]) if k > 1 else None
        x, _, _ = _decay(oracle, lam, 1.0, T, M, k, hist=hist)
        errs.append(abs(x[0] - np.exp(-lam * T)))
    assert np.allclose(_slope(np.array(errs)), k, atol=0.08)


@pytest.mark.parametrize("k,hs", [(1, (1e-2, 1e-3, 1e-4)), (2, (1e-2, 1e-3, 1e-4)),
                                  (3, (3e-2, 1e-2, 3e-3))])
def test_lte_estimate_matches_true_one_step_error(oracle, k, hs):
    # one step from exact history: the estimate -> the true local error, with
    # a deviation of order lambda*h
    lam = 3.0
    dev = []
    for h in hs:
        hist = np.array([[np.exp(lam * h * r)] for r in range(1, k + 1)])
        x, gam, _ = _decay(oracle, lam, 1.0, h, 1, k, hist=hist, lte=True)
        ratio = np.sqrt(gam[0]) / abs(np.exp(-lam * h) - x[0])
        dev.append(abs(ratio - 1))
        assert dev[-1] < 10 * lam * h
    assert dev[-1] < dev[0]


def test_lte_estimate_start_step(oracle):
    # step 1 of an interval: BDF1 with the Euler comparison value
    lam = 3.0
    for h in (1e-3, 1e-5):
        x, gam, _ = _decay(oracle, lam, 1.0, h, 1, 2, lte=True)
        r = np.sqrt(gam[0]) / abs(np.exp(-lam * h) - x[0])
        assert abs(r - 1) < 10 * lam * h


def test_lte_filtered_for_stiff_components(oracle):
    # h*lambda = z >> 1.  Step 1 compares x1 = 1/(1+z) with the explicit Euler
    # value 1 - z: the distance z^2/(1+z), which the Newton matrix divides by
    # (1 + z) twice at this step, so the estimate is (1/2) z^2/(1+z)^3 ~
    # x0/(2z), of the order of the true local error 1/(1+z) - e^-z ~ x0/z
    # (one division would leave (1/2)(z/(1+z))^2 ~ x0/2).
    lam, h = 1e6, 0.25
    z = h * lam
    x, gam, _ = _decay(oracle, lam, 1.0, h, 1, 2, lte=True)
    assert np.sqrt(gam[0]) == pytest.approx(0.5 * z * z / (1 + z) ** 3, rel=1e-9)
    # over four steps every step adds O(1/z): 1/(2z) at step 1, 1/(3z) at
    # step 2 (q = 1), about 0.27/z at step 3 (q = 2), much less at step 4;
    # in quadrature about 0.66/z
    x, gam, _ = _decay(oracle, lam, 1.0, 4 * h, 4, 2, lte=True)
    assert 0.62 / z < np.sqrt(gam[0]) < 0.70 / z
    assert abs(x[0]) < 1e-10


def test_lte_start_step_tracks_true_error_at_every_stiffness(oracle):
    # one BDF1 step on x' = -lambda x from x0 = 1, z = h lambda from 1e-3 to
    # 1e5: the estimate stays within a factor 3 of the true local error
    # 1/(1+z) - e^-z (it tends to it as z -> 0 and to half of it as z -> inf)
    for z in np.logspace(-3, 5, 33):
        x, gam, _ = _decay(oracle, z, 1.0, 1.0, 1, 1, lte=True)
        ratio = np.sqrt(gam[0]) / abs(1 / (1 + z) - np.exp(-z))
        assert 0.33 < ratio < 1.01, (z, ratio)


# ---------------------------------------------------------------- LU
@pytest.mark.parametrize("d", [1, 3, 7, 16])
def test_lu_solve_matches_numpy(oracle, d):
    rng = np.random.default_rng(d)
    for _ in range(20):
        A = rng.standard_normal((d, d))
        A[0, 0] = 1e-14   # forces a row exchange
        b = rng.standard_normal(d)
        want = np.linalg.solve(A, b)
        got = oracle.lu_solve(A, b)
        assert np.allclose(got, want, rtol=1e-9, atol=1e-11 * np.abs(want).max())


def test_lu_solve_singular(oracle):
    with pytest.raises(np.linalg.LinAlgError):
        oracle.lu_solve(np.zeros((3, 3)), np.ones(3))


# ---------------------------------------------------------------- models
def _fd_jac(oracle, model, x, theta, mc, rf):
    d = len(x)
    J = np.zeros((d, d))
    for j in range(d):
        e = max(abs(x[j]), 1e-3) * 1e-6
        xp, xm = x.copy(), x.copy()
        xp[j] += e
        xm[j] -= e
        fp, _ = oracle.rhs(model, xp, theta, mc, rf)
        fm, _ = oracle.rhs(model, xm, theta, mc, rf)
        J[:, j] = (fp - fm) / (2 * e)
    return J


def test_robertson_jacobian_finite_difference(oracle):
    pr = inputs.robertson(10, 50)
    for x in (np.array([0.9, 3e-5, 0.1]), np.array([0.3, 2e-6, 0.7])):
        f, J = oracle.rhs(1, x, pr.theta_true)
        k1, k2, k3 = np.exp(pr.theta_true)
        assert f == pytest.approx([-k1 * x[0] + k3 * x[1] * x[2],
                                   k1 * x[0] - k2 * x[1] ** 2 - k3 * x[1] * x[2],
                                   k2 * x[1] ** 2], rel=1e-14)
        assert abs(f.sum()) < 1e-15 * np.abs(f).max() * 10
        assert np.allclose(J, _fd_jac(oracle, 1, x, pr.theta_true, None, None), rtol=1e-6, atol=1e-6)


def test_chain_jacobian_finite_difference(oracle):
    pr = inputs.chain16(10, 5)
    x = np.abs(pr.x_true[2]) + 0.01
    f, J = oracle.rhs(2, x, pr.theta_true, pr.model_consts, pr.rates_fixed)
    Jfd = _fd_jac(oracle, 2, x, pr.theta_true, pr.model_consts, pr.rates_fixed)
    assert np.allclose(J, Jfd, rtol=1e-5, atol=1e-6 * np.abs(J).max())
    assert np.count_nonzero(np.triu(J, 1)) == 0 and np.count_nonzero(np.tril(J, -2)) == 0


def test_robertson_linear_invariant(oracle):
    # the column sums of J vanish, so BDF + Newton keep sum(x) (= 1) exactly
    # up to rounding, whatever the parameters and the step
    pr = inputs.robertson(10, 50)
    rng = np.random.default_rng(0)
    for j in (0, 10, 30, 49):
        x0 = pr.x_true[j - 1] if j else pr.x0
        t0 = pr.times[j - 1] if j else 0.0
        for _ in range(3):
            th = pr.theta_true + 0.5 * rng.standard_normal(3)
            x, _, st = oracle.psi(1, x0, th, (pr.times[j] - t0) / 20, 20, 2,
                                  rtol=1e-12, floor=pr.state_floor)
            assert abs(x.sum() - x0.sum()) < 5e-15


def test_robertson_global_error_vs_radau(oracle):
    pr = inputs.robertson(10, 50)
    j = 20
    x0, t0, t1 = pr.x_true[j - 1], pr.times[j - 1], pr.times[j]
    errs = []
    for M in (20, 40, 80, 160):
        x, _, _ = oracle.psi(1, x0, pr.theta_true, (t1 - t0) / M, M, 2, rtol=1e-13,
                             floor=pr.state_floor)
        errs.append(np.max(np.abs(x - pr.x_true[j]) / np.maximum(np.abs(pr.x_true[j]), pr.state_floor)))
    errs = np.array(errs)
    assert errs[-1] < 1e-6
    assert np.all(_slope(errs) > 1.7), _slope(errs)


def test_chain_linear_case_closed_form(oracle):
    # V = 0 makes the chain linear: x' = B x + e1, solved by the exponential of
    # the augmented matrix
    pr = inputs.chain16(10, 5)
    d = 16
    mc = np.concatenate([np.zeros(d), pr.model_consts[d:]])
    k = pr.rates_fixed
    B = np.diag(-k) + np.diag(k[:-1], -1)
    Aug = np.zeros((d + 1, d + 1))
    Aug[:d, :d] = B
    Aug[0, d] = 1.0
    T = 0.1
    want = (expm(Aug * T) @ np.concatenate([np.ones(d), [1.0]]))[:d]
    errs = []
    for M in (160, 320, 640, 1280):
        x, _, _ = oracle.psi(2, np.ones(d), pr.theta_true, T / M, M, 3, rtol=1e-14,
                             floor=np.full(d, 1e-12), mc=mc, rates_fixed=pr.rates_fixed)
        errs.append(np.max(np.abs(x - want) / np.maximum(np.abs(want), 1e-6)))
    errs = np.array(errs)
    assert errs[-1] < 1e-5
    assert np.all(_slope(errs) > 1.8), _slope(errs)


def test_chain_full_model_vs_radau(oracle):
    # first interval: a fast initial transient (V/K up to 1e4), so the error
    # falls below the pre-asymptotic rate first
    pr = inputs.chain16(10, 5)
    errs = []
    for M in (640, 2560, 10240):
        x, _, st = oracle.psi(2, pr.x0, pr.theta_true, 0.1 / M, M, 3, rtol=1e-13,
                              floor=pr.state_floor, mc=pr.model_consts, rates_fixed=pr.rates_fixed)
        errs.append(np.max(np.abs(x - pr.x_true[0]) / np.maximum(np.abs(pr.x_true[0]), pr.state_floor)))
        assert st["newton_fails"] == 0
    assert errs[-1] < 1e-4 and errs[0] > errs[1] > errs[2]
    # a later interval starts on the slow manifold: full restarted order 2
    x0, t0, t1 = pr.x_true[2], pr.times[2], pr.times[3]
    errs = []
    for M in (160, 320, 640, 1280):
        x, _, _ = oracle.psi(2, x0, pr.theta_true, (t1 - t0) / M, M, 3, rtol=1e-13,
                             floor=pr.state_floor, mc=pr.model_consts, rates_fixed=pr.rates_fixed)
        errs.append(np.max(np.abs(x - pr.x_true[3]) / np.maximum(np.abs(pr.x_true[3]), pr.state_floor)))
    assert errs[-1] < 1e-5, errs
    assert np.all(_slope(np.array(errs)) > 1.8), errs
