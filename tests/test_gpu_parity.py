"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bars (from the method's precision split): RNG words and resampling indices
bit-exact given identical inputs; per-step states within 1e-10 relative in
FP64 and 1e-4 relative in FP32 propagation, relative to max(|x|, floor) with
floor = 1e-6 of each component's scale; normals within a few ulp (device vs
host libm).
"""
import numpy as np
import pytest

from paper_1411_1702_amd import inputs
import jitter_bound as JB

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {0: 1e-10, 1: 1e-4}   # by precision: FP64, FP32 propagation


@pytest.fixture(scope="module")
def pf():
    from paper_1411_1702_amd import pf as _pf
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _pf.lib()
    return _pf


@pytest.fixture(scope="module")
def ctx(pf):
    c = pf.Context(0, 1 << 30)
    yield c
    c.close()


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def relerr(a, b, floor):
    return np.abs(a - b) / np.maximum(np.abs(b), floor)


# ---------------------------------------------------------------- RNG
def test_philox_bitexact(pf, oracle):
    rng = np.random.default_rng(11)
    n = 3000
    ctr = rng.integers(0, 2**63, (n, 4), dtype=np.int64).astype(np.uint64) * np.uint64(2) + \
        rng.integers(0, 2, (n, 4), dtype=np.int64).astype(np.uint64)
    ctr[:10] = np.arange(40, dtype=np.uint64).reshape(10, 4)
    key = rng.integers(0, 2**63, (n, 2), dtype=np.int64).astype(np.uint64)
    c_d = torch.from_numpy(ctr.view(np.int64)).cuda()
    k_d = torch.from_numpy(key.view(np.int64)).cuda()
    o_d = torch.zeros((n, 4), dtype=torch.int64, device="cuda")
    pf.check(pf.lib().pf_test_philox(n, c_d.data_ptr(), k_d.data_ptr(), o_d.data_ptr(), None), "philox")
    got = o_d.cpu().numpy().view(np.uint64)
    for i in range(n):
        assert np.array_equal(got[i], oracle.philox(ctr[i], key[i])), i


@pytest.mark.parametrize("count,purpose", [(3, 3), (12, 3), (16, 4), (1, 2), (5, 1)])
def test_normals_match_oracle(pf, oracle, count, purpose):
    n, seed, step = 777, 12345, 17
    out = torch.zeros((n, count), dtype=torch.float64, device="cuda")
    pf.check(pf.lib().pf_test_normals(n, seed, step, purpose, count, out.data_ptr(), None), "normals")
    got = out.cpu().numpy()
    want = np.array([oracle.normals(seed, step, i, purpose, count) for i in range(n)])
    assert np.allclose(got, want, rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------- propagation
def _robertson_inputs(oracle, n=1000, j_list=(1, 10, 25, 45)):
    """(x_j, theta, h) sets from a short oracle run on the small Robertson config."""
    prob = inputs.robertson(n, 50)
    F = oracle.Filter(prob)
    out = []
    for j in range(max(j_list) + 1):
        if j in j_list:
            h = (prob.times[j] - F.t) / prob.substeps
            out.append((F.x.copy(), F.theta.copy(), h))
        F.step(prob.times[j], prob.y[j], prob.sigma[j])
    return prob, out


def _propagate_gpu(pf, prob, prec, x, theta, h, lte):
    n = x.shape[0]
    cfg = pf.Config(prob, prec)
    xi, ti = dev(x.T), dev(theta.T)
    xo = torch.zeros_like(xi)
    go = torch.zeros_like(xi)
    it = torch.zeros(1, dtype=torch.int64, device="cuda")
    pf.check(pf.lib().pf_test_propagate(cfg.ptr(), n, xi.data_ptr(), ti.data_ptr(), h, int(lte),
                                        xo.data_ptr(), go.data_ptr(), it.data_ptr(), None), "propagate")
    return xo.cpu().numpy().T, go.cpu().numpy().T, int(it.item())


def _propagate_oracle(oracle, prob, x, theta, h, lte, rtol):
    xs, gs, its = [], [], 0
    for i in range(x.shape[0]):
        xo, go, st = oracle.psi(prob.model, x[i], theta[i], h, prob.substeps, prob.order, lte=lte,
                                rtol=rtol, kmax=prob.newton_max_iter, floor=prob.state_floor,
                                mc=prob.model_consts, rates_fixed=prob.rates_fixed, lmm=prob.lmm)
        xs.append(xo)
        gs.append(go)
        its += st["newton_iters"]
    return np.array(xs), np.array(gs), its


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("lte", [False, True])
def test_propagate_robertson(pf, oracle, prec, lte):
    prob, sets = _robertson_inputs(oracle)
    rtol = prob.newton_rtol_fp64 if prec == 0 else prob.newton_rtol_fp32
    for x, th, h in sets:
        xg, gg, itg = _propagate_gpu(pf, prob, prec, x, th, h, lte)
        xo, go, ito = _propagate_oracle(oracle, prob, x, th, h, lte, rtol)
        err = relerr(xg, xo, prob.state_floor)
        assert err.max() < TOL[prec], (h, err.max())
        if lte:
            # FP32: a local error below the state's own resolution is seen as
            # rounding noise of order sqrt(M) ulp(x); bound it by that
            noise = 0.0 if prec == 0 else 4 * np.sqrt(prob.substeps) * 2.0**-23 * np.abs(xo)
            dev_ = np.abs(np.sqrt(gg) - np.sqrt(go))
            bound = (1e-7 if prec == 0 else 2e-3) * np.maximum(np.sqrt(go), prob.state_floor) + noise
            assert np.all(dev_ <= bound), (h, (dev_ / bound).max())
        if prec == 0:
            assert abs(itg - ito) <= 0.01 * ito + 5


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("lte", [False, True])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_propagate_robertson_am(pf, oracle, prec, lte, k):
    # Adams-Moulton k steps; AM2 and AM3 on the first interval only (their
    # stability intervals do not cover the stiff eigenvalue at later steps)
    prob, sets = _robertson_inputs(oracle, j_list=(1, 10, 25, 45) if k == 1 else (0,))
    prob.lmm, prob.order = 1, k
    rtol = prob.newton_rtol_fp64 if prec == 0 else prob.newton_rtol_fp32
    for x, th, h in sets:
        xg, gg, itg = _propagate_gpu(pf, prob, prec, x, th, h, lte)
        xo, go, ito = _propagate_oracle(oracle, prob, x, th, h, lte, rtol)
        err = relerr(xg, xo, prob.state_floor)
        assert err.max() < TOL[prec], (k, h, err.max())
        if lte:
            noise = 0.0 if prec == 0 else 4 * np.sqrt(prob.substeps) * 2.0**-23 * np.abs(xo)
            dev_ = np.abs(np.sqrt(gg) - np.sqrt(go))
            bound = (1e-7 if prec == 0 else 2e-3) * np.maximum(np.sqrt(go), prob.state_floor) + noise
            assert np.all(dev_ <= bound), (k, h, (dev_ / bound).max())
        if prec == 0:
            assert abs(itg - ito) <= 0.01 * ito + 5


# FP32 rounding of trapezoidal (AM1) steps, the error model of the bound
# below: each step adds rounding of a few units in the last place of the
# state's largest component (its sums run over all components through the
# chain's coupling), and the trapezoidal rule is A- but not L-stable -- it
# multiplies a stiff mode's error by |(1 + z/2)/(1 - z/2)| (0.67 at h k = 10,
# 0.85 at 25) per step instead of BDF's |1/(1 - z)| -- so a step's rounding in
# a stiff component is not forgotten within the next steps and can dominate
# a component that is small at the end (x_i of 1e-8 beside |x| of 600).
# Bound per component: the relative contract plus M steps of 10 units of
# 2^-24 of the state's largest component.  Measured on these inputs (h k up
# to 12): at most 9.4e-7 of the largest component, against 2.4e-5 allowed.
AM1_ULPS_PER_STEP = 10


@pytest.mark.parametrize("prec", [0, 1])
def test_propagate_chain_am1(pf, oracle, prec):
    prob, sets = _chain_inputs()
    prob.lmm, prob.order = 1, 1
    rtol = prob.newton_rtol_fp64 if prec == 0 else prob.newton_rtol_fp32
    for x, th, h in sets:
        xg, gg, _ = _propagate_gpu(pf, prob, prec, x, th, h, True)
        xo, go, _ = _propagate_oracle(oracle, prob, x, th, h, True, rtol)
        err = relerr(xg, xo, prob.state_floor)
        if prec == 0:
            assert err.max() < TOL[0], (h, err.max())
            continue
        big = np.abs(xo).max(axis=1, keepdims=True)
        allow = TOL[1] * np.maximum(np.abs(xo), prob.state_floor) + \
            prob.substeps * AM1_ULPS_PER_STEP * 2.0**-24 * big
        dev_ = np.abs(xg - xo)
        print("chain AM1 FP32: worst error / allowance %.3f, largest error / |x|_max %.2e"
              % ((dev_ / allow).max(), (dev_ / big).max()))
        assert np.all(dev_ <= allow), (h, (dev_ / allow).max())
        assert np.median(err) < 1e-5


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("lte", [False, True])
@pytest.mark.parametrize("k", [2, 3])
def test_propagate_robertson_sdirk(pf, oracle, prec, lte, k):
    # BDFk with the SDIRK start-up (k stages per start-up step, then BDFk)
    prob, sets = _robertson_inputs(oracle)
    prob.lmm, prob.order = pf.PF_LMM_BDF_SDIRK, k
    rtol = prob.newton_rtol_fp64 if prec == 0 else prob.newton_rtol_fp32
    for x, th, h in sets:
        xg, gg, itg = _propagate_gpu(pf, prob, prec, x, th, h, lte)
        xo, go, ito = _propagate_oracle(oracle, prob, x, th, h, lte, rtol)
        err = relerr(xg, xo, prob.state_floor)
        assert err.max() < TOL[prec], (k, h, err.max())
        if lte:
            noise = 0.0 if prec == 0 else 4 * np.sqrt(prob.substeps) * 2.0**-23 * np.abs(xo)
            dev_ = np.abs(np.sqrt(gg) - np.sqrt(go))
            bound = (1e-7 if prec == 0 else 2e-3) * np.maximum(np.sqrt(go), prob.state_floor) + noise
            assert np.all(dev_ <= bound), (k, h, (dev_ / bound).max())
        if prec == 0:
            assert abs(itg - ito) <= 0.01 * ito + 5


@pytest.mark.parametrize("prec", [0, 1])
def test_propagate_sdirk_order1_is_bdf1(pf, oracle, prec):
    # with k = 1 there is no start-up: the result is plain BDF1's, bit for bit
    prob, sets = _robertson_inputs(oracle, n=300, j_list=(10,))
    prob.order = 1
    x, th, h = sets[0]
    xa, ga, ia = _propagate_gpu(pf, prob, prec, x, th, h, True)
    prob.lmm = pf.PF_LMM_BDF_SDIRK
    xb, gb, ib = _propagate_gpu(pf, prob, prec, x, th, h, True)
    assert np.array_equal(xa, xb) and np.array_equal(ga, gb) and ia == ib


def _chain_inputs(n=600, seed=3):
    prob = inputs.chain16(n, 10)
    rng = np.random.default_rng(seed)
    sets = []
    for j in (0, 3, 8):
        x0 = prob.x0 if j == 0 else prob.x_true[j - 1]
        t0 = 0.0 if j == 0 else prob.times[j - 1]
        x = np.tile(x0, (n, 1)) * np.exp(0.01 * rng.standard_normal((n, prob.d)))
        th = prob.prior_mean + 0.3 * rng.standard_normal((n, prob.p))
        sets.append((x, th, (prob.times[j] - t0) / prob.substeps))
    return prob, sets


@pytest.mark.parametrize("prec", [0, 1])
def test_propagate_chain(pf, oracle, prec):
    prob, sets = _chain_inputs()
    rtol = prob.newton_rtol_fp64 if prec == 0 else prob.newton_rtol_fp32
    for x, th, h in sets:
        xg, gg, _ = _propagate_gpu(pf, prob, prec, x, th, h, True)
        xo, go, _ = _propagate_oracle(oracle, prob, x, th, h, True, rtol)
        err = relerr(xg, xo, prob.state_floor)
        assert err.max() < TOL[prec], (h, err.max())


# ---------------------------------------------------------------- moments
def _moments_gpu(pf, theta, logw):
    n, p = theta.shape
    th, lw = dev(theta.T), dev(logw)
    mean, cov, L = np.zeros(p), np.zeros(p * p), np.zeros(p * p)
    ess = np.zeros(1)
    st = pf.lib().pf_test_moments(n, p, th.data_ptr(), lw.data_ptr(), pf._dp(mean), pf._dp(cov), pf._dp(L),
                                  pf._dp(ess), None)
    return st, mean, cov.reshape(p, p), L.reshape(p, p), ess[0]


@pytest.mark.parametrize("p", [3, 5, 12])
@pytest.mark.parametrize("n", [1, 300, 4097, 65536 + 7, 1 << 17, (1 << 18) + 5])
def test_moments_match_oracle(pf, oracle, p, n):
    rng = np.random.default_rng(p * 1000 + n)
    theta = rng.standard_normal((n, p)) * rng.uniform(0.1, 3.0, p) + rng.uniform(-5, 5, p)
    logw = 3.0 * rng.standard_normal(n)
    logw[rng.uniform(size=n) < 0.1] = -np.inf
    if n == 1:
        logw[0] = 0.0
    st, mean, cov, L, ess = _moments_gpu(pf, theta, logw)
    w, _ = oracle.normalise(logw)
    om, oc = oracle.moments(theta, w)
    if n == 1:
        # one particle: zero covariance, no jitter makes it factorable
        assert st == pf.PF_EDEGENERATE
        return
    assert st == pf.PF_OK
    ost, oL, _ = oracle.cholesky(oc)
    assert ost == 0
    assert np.allclose(mean, om, rtol=1e-12, atol=1e-12)
    assert np.allclose(cov, oc, rtol=1e-10, atol=1e-13 * np.abs(oc).max())
    assert np.allclose(L, oL, rtol=1e-9, atol=1e-12 * np.abs(oL).max())
    assert ess == pytest.approx(1.0 / np.sum(w * w), rel=1e-10)


def test_moments_jitter_and_degenerate(pf, oracle):
    rng = np.random.default_rng(7)
    n, p = 2000, 5
    theta = rng.standard_normal((n, p))
    theta[:, 3] = theta[:, 1]          # rank deficient: the jitter rule decides
    logw = rng.standard_normal(n)
    st, mean, cov, L, ess = _moments_gpu(pf, theta, logw)
    w, _ = oracle.normalise(logw)
    om, oc = oracle.moments(theta, w)
    ost, oL, ojit = oracle.cholesky(oc)
    assert st == (pf.PF_OK if ost == 0 else pf.PF_EDEGENERATE)
    if ost == 0:
        # the factor's column for the dependent direction is rounding noise
        # over sqrt(delta) on both sides; the product L L^T = C + delta I is
        # what the jitter rule fixes, and the columns before it are determined
        assert np.allclose(L @ L.T, oL @ oL.T, rtol=0, atol=1e-8 * np.abs(oc).max())
        assert np.allclose(L[:, :3], oL[:, :3], rtol=1e-9, atol=1e-12)
    st, *_ = _moments_gpu(pf, theta, np.full(n, -np.inf))
    assert st == pf.PF_EDEGENERATE


# ---------------------------------------------------------------- resampling
@pytest.mark.parametrize("N", [1, 7, 256, 257, 1000, 4097, 65536 + 13])
def test_resample_bitexact(pf, oracle, N):
    rng = np.random.default_rng(N)
    for trial in range(3):
        g = rng.exponential(size=N) ** (1 + 2 * trial)
        g[rng.random(N) < 0.2] = 0.0
        if g.sum() == 0:
            g[0] = 1.0
        g /= g.sum()
        r = int(rng.integers(0, 2**63)) * 2 + trial
        gd = dev(g)
        ad = torch.zeros(N, dtype=torch.int32, device="cuda")
        pf.check(pf.lib().pf_test_resample(N, gd.data_ptr(), r, ad.data_ptr(), None), "resample")
        st, want = oracle.resample(g, r)
        assert st == 0
        assert np.array_equal(ad.cpu().numpy(), want)


def test_resample_degenerate(pf):
    gd = dev(np.zeros(300))
    ad = torch.zeros(300, dtype=torch.int32, device="cuda")
    assert pf.lib().pf_test_resample(300, gd.data_ptr(), 5, ad.data_ptr(), None) == pf.PF_EDEGENERATE


@pytest.mark.parametrize("N", [1, 7, 256, 257, 1000, 4097, 65549])
def test_resample_multinomial_bitexact(pf, oracle, N):
    rng = np.random.default_rng(1000 + N)
    for trial in range(3):
        g = rng.exponential(size=N) ** (1 + 2 * trial)
        g[rng.random(N) < 0.2] = 0.0
        if g.sum() == 0:
            g[0] = 1.0
        g /= g.sum()
        seed, step = int(rng.integers(0, 2**63)), 1 + trial * 17
        gd = dev(g)
        ad = torch.zeros(N, dtype=torch.int32, device="cuda")
        pf.check(pf.lib().pf_test_resample_multinomial(N, gd.data_ptr(), seed, step, ad.data_ptr(), None),
                 "multinomial")
        st, want = oracle.resample_multinomial(g, seed, step)
        assert st == 0
        assert np.array_equal(ad.cpu().numpy(), want)


def test_resample_multinomial_limits(pf):
    ad = torch.zeros(300, dtype=torch.int32, device="cuda")
    gd = dev(np.zeros(300))
    L = pf.lib()
    assert L.pf_test_resample_multinomial(300, gd.data_ptr(), 1, 1, ad.data_ptr(), None) == pf.PF_EDEGENERATE
    assert L.pf_test_resample_multinomial(300, gd.data_ptr(), 1, 0, ad.data_ptr(), None) == pf.PF_EINVAL
    assert L.pf_test_resample_multinomial((1 << 20) + 1, gd.data_ptr(), 1, 1, ad.data_ptr(), None) == pf.PF_EINVAL


# ---------------------------------------------------------------- init and one step
def _get(pf, f):
    x = torch.zeros((f.d, f.N), dtype=torch.float64, device="cuda")
    th = torch.zeros((f.p, f.N), dtype=torch.float64, device="cuda")
    lw = torch.zeros(f.N, dtype=torch.float64, device="cuda")
    pf.check(pf.lib().pf_test_get_ensemble(f.h, x.data_ptr(), th.data_ptr(), lw.data_ptr()), "get")
    return x.cpu().numpy().T, th.cpu().numpy().T, lw.cpu().numpy()


def _set(pf, f, ora):
    x, th, lw = dev(ora.x.T), dev(ora.theta.T), dev(ora.logw)
    mean, _ = ora.moments()
    L = np.ascontiguousarray(ora.chol())
    pf.check(pf.lib().pf_test_set_ensemble(f.h, x.data_ptr(), th.data_ptr(), lw.data_ptr(),
                                           pf._dp(np.ascontiguousarray(mean)), pf._dp(L), ora.j, ora.t),
             "set")


@pytest.mark.parametrize("prec", [0, 1])
def test_init_matches_oracle(pf, ctx, oracle, prec):
    prob = inputs.robertson(1000, 5, seed=4)
    f = pf.Filter(ctx, pf.Config(prob, prec))
    ora = oracle.Filter(prob)
    x, th, lw = _get(pf, f)
    assert np.allclose(th, ora.theta, rtol=1e-13, atol=1e-13)
    assert np.array_equal(x, ora.x)
    assert np.allclose(lw, ora.logw, rtol=1e-14)
    post = f.posterior()
    mean, cov = ora.moments()
    assert np.allclose(post["mean"], mean, rtol=1e-12, atol=1e-13)
    assert np.allclose(post["cov"], cov, rtol=1e-10, atol=1e-14)
    assert post["ess"] == pytest.approx(1000, rel=1e-12)
    f.close()


def _innovation_scale(oracle, prob, x_in, t_in, anc, theta_new, step):
    """Per slot and component, the scale of the terms of x_{j+1} = Psi(x_j) + v:
    max(|Psi|, sqrt(Gamma) max(|z|, 1)).  A state formed by cancellation of the
    two is judged against the terms that formed it, and the innovation against
    its own standard deviation (an FP32 normal is accurate to ~1e-6 absolute)."""
    h = (prob.times[step - 1] - t_in) / prob.substeps
    out = np.zeros((len(anc), prob.d))
    for n, k in enumerate(anc):
        xt, gam, _ = oracle.psi(prob.model, x_in[k], theta_new[n], h, prob.substeps, prob.order,
                                lte=True, rtol=prob.newton_rtol_fp64, kmax=prob.newton_max_iter,
                                floor=prob.state_floor, mc=prob.model_consts,
                                rates_fixed=prob.rates_fixed, lmm=prob.lmm)
        z = oracle.normals(prob.seed, step, n, oracle.PUR_INNOV, prob.d)
        out[n] = np.maximum(np.abs(xt), np.sqrt(gam) * np.maximum(np.abs(z), 1.0))
    return out


def _step_case(pf, ctx, oracle, prob, prec, j0):
    ora = oracle.Filter(prob)
    for j in range(j0):
        assert ora.step(prob.times[j], prob.y[j], prob.sigma[j])["status"] == 0
    x_in, t_in = ora.x.copy(), ora.t
    f = pf.Filter(ctx, pf.Config(prob, prec))
    _set(pf, f, ora)
    rc, g, anc_o = ora.stage1(prob.times[j0], prob.y[j0], prob.sigma[j0])
    assert rc == 0
    st = f.assimilate(prob.times[j0], prob.y[j0], prob.sigma[j0])
    assert st == pf.PF_OK
    out = ora.step(prob.times[j0], prob.y[j0], prob.sigma[j0])
    assert out["status"] == 0
    anc = torch.zeros(f.N, dtype=torch.int32, device="cuda")
    pf.check(pf.lib().pf_test_last_ancestors(f.h, anc.data_ptr()), "anc")
    anc_g = anc.cpu().numpy()
    x, th, lw = _get(pf, f)
    post = f.posterior()
    f.close()
    scale = np.maximum(_innovation_scale(oracle, prob, x_in, t_in, anc_o, ora.theta, j0 + 1),
                       prob.state_floor)
    return ora, out, anc_o, anc_g, x, th, lw, post, scale


def _fp32_all_slots(oracle, prob, j0, anc_g, x, th):
    """The FP32 step against the oracle's step taken with the GPU's own
    ancestors (FP32 predictions can move a borderline integer weight, so the
    two index draws may differ in a few slots): every slot's state within
    the FP32 bound, every slot's parameters within the FP32 jitter bound."""
    orb = oracle.Filter(prob)
    for j in range(j0):
        assert orb.step(prob.times[j], prob.y[j], prob.sigma[j])["status"] == 0
    x_in, t_in, L = orb.x.copy(), orb.t, orb.chol()
    assert orb.step_given(prob.times[j0], prob.y[j0], prob.sigma[j0], anc_g) == 0
    scale = np.maximum(_innovation_scale(oracle, prob, x_in, t_in, anc_g, orb.theta, j0 + 1),
                       prob.state_floor)
    err = np.abs(x - orb.x) / scale
    bound = JB.fp32_jitter_bound(oracle, prob, L, j0 + 1, len(th))
    dth = np.abs(th - orb.theta)
    print("FP32 step, all slots with the GPU's ancestors: state error %.2e, worst |d theta| / bound %.3f"
          % (err.max(), (dth / bound).max()))
    assert err.max() < TOL[1], err.max()
    assert np.all(dth <= bound)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("j0", [0, 7, 30])
def test_step_parity_robertson(pf, ctx, oracle, prec, j0):
    prob = inputs.robertson(1000, 50, seed=2)
    ora, out, anc_o, anc_g, x, th, lw, post, scale = _step_case(pf, ctx, oracle, prob, prec, j0)
    same = anc_o == anc_g
    if prec == 0:
        assert same.all()
    else:
        assert same.mean() > 0.98
        _fp32_all_slots(oracle, prob, j0, anc_g, x, th)
    err = np.abs(x[same] - ora.x[same]) / scale[same]
    assert err.max() < TOL[prec], err.max()
    if prec == 0:
        assert np.allclose(th[same], ora.theta[same], rtol=1e-12, atol=1e-12)
    else:
        # FP32 propagation draws the proliferation normals in FP32: the bound
        # of their Box-Muller rounding carried through s L z
        pre = oracle.Filter(prob)
        for j in range(j0):
            pre.step(prob.times[j], prob.y[j], prob.sigma[j])
        bound = JB.fp32_jitter_bound(oracle, prob, pre.chol(), j0 + 1, len(th))
        dev_ = np.abs(th - ora.theta)
        print("FP32 jitter: worst |d theta| / bound %.3f, max |d theta| %.2e"
              % ((dev_[same] / bound[same]).max(), dev_[same].max()))
        assert np.all(dev_[same] <= bound[same])
    if prec == 0:
        fin = np.isfinite(ora.logw)
        assert np.allclose(lw[fin], ora.logw[fin], rtol=0, atol=1e-8)
        mean, cov = ora.moments()
        assert np.allclose(post["mean"], mean, rtol=1e-10, atol=1e-12)
        # the covariance against its largest entry (entries near zero are formed
        # by cancellation in both sums): measured at most 1.7e-14
        cerr = np.abs(post["cov"] - cov).max() / np.abs(cov).max()
        print("FP64 step: covariance error %.2e of its largest entry" % cerr)
        assert cerr < 1e-12, cerr
        assert post["ess"] == pytest.approx(out["ess"], rel=1e-8)
        assert np.allclose(post["state_mean"], out["state_mean"], rtol=1e-9, atol=1e-15)


@pytest.mark.parametrize("N", [1 << 17, (1 << 17) + 300])
def test_step_parity_robertson_large_n(pf, ctx, oracle, N):
    """One FP64 step from the prior draw at the largest tile counts: at 2^17
    particles (512 tiles) the filter-wide combines (first-stage log-sum-exp,
    moments) take two tiles per lane; above that they loop over the tiles.
    Ancestors bit-exact, states and posterior summaries to rounding."""
    prob = inputs.robertson(N, 5, seed=3)
    ora = oracle.Filter(prob)
    f = pf.Filter(ctx, pf.Config(prob, pf.PF_PREC_FP64))
    rc, _, anc_o = ora.stage1(prob.times[0], prob.y[0], prob.sigma[0])
    assert rc == 0
    assert f.assimilate(prob.times[0], prob.y[0], prob.sigma[0]) == pf.PF_OK
    out = ora.step(prob.times[0], prob.y[0], prob.sigma[0])
    assert out["status"] == 0
    anc = torch.zeros(f.N, dtype=torch.int32, device="cuda")
    pf.check(pf.lib().pf_test_last_ancestors(f.h, anc.data_ptr()), "anc")
    assert (anc.cpu().numpy() == anc_o).all()
    x, th, lw = _get(pf, f)
    post = f.posterior()
    f.close()
    err = np.abs(x - ora.x) / np.maximum(np.abs(ora.x), prob.state_floor)
    assert err.max() < 1e-10, err.max()
    assert np.allclose(th, ora.theta, rtol=1e-12, atol=1e-12)
    mean, cov = ora.moments()
    assert np.allclose(post["mean"], mean, rtol=1e-10, atol=1e-12)
    # the covariance against its largest entry (entries near zero are formed
    # by cancellation in both sums): measured at most 1.7e-14
    cerr = np.abs(post["cov"] - cov).max() / np.abs(cov).max()
    print("FP64 step: covariance error %.2e of its largest entry" % cerr)
    assert cerr < 1e-12, cerr
    assert post["ess"] == pytest.approx(out["ess"], rel=1e-8)


@pytest.mark.parametrize("prec", [0, 1])
def test_step_parity_robertson_multinomial(pf, ctx, oracle, prec):
    prob = inputs.robertson(1000, 50, seed=2)
    prob.resampling = 1
    ora, out, anc_o, anc_g, x, th, lw, post, scale = _step_case(pf, ctx, oracle, prob, prec, 7)
    same = anc_o == anc_g
    if prec == 0:
        assert same.all()
    else:
        assert same.mean() > 0.98
        _fp32_all_slots(oracle, prob, 7, anc_g, x, th)
    assert not np.all(np.diff(anc_o) >= 0)     # multinomial ancestors are not sorted
    err = np.abs(x[same] - ora.x[same]) / scale[same]
    assert err.max() < TOL[prec], err.max()
    if prec == 0:
        mean, cov = ora.moments()
        assert np.allclose(post["mean"], mean, rtol=1e-10, atol=1e-12)
        # the covariance against its largest entry (entries near zero are formed
        # by cancellation in both sums): measured at most 1.7e-14
        cerr = np.abs(post["cov"] - cov).max() / np.abs(cov).max()
        print("FP64 step: covariance error %.2e of its largest entry" % cerr)
        assert cerr < 1e-12, cerr


@pytest.mark.parametrize("prec", [0, 1])
def test_step_parity_robertson_am1(pf, ctx, oracle, prec):
    prob = inputs.robertson(1000, 50, seed=2)
    prob.lmm, prob.order = 1, 1
    ora, out, anc_o, anc_g, x, th, lw, post, scale = _step_case(pf, ctx, oracle, prob, prec, 7)
    same = anc_o == anc_g
    if prec == 0:
        assert same.all()
    else:
        assert same.mean() > 0.98
        _fp32_all_slots(oracle, prob, 7, anc_g, x, th)
    err = np.abs(x[same] - ora.x[same]) / scale[same]
    assert err.max() < TOL[prec], err.max()
    if prec == 0:
        mean, cov = ora.moments()
        assert np.allclose(post["mean"], mean, rtol=1e-10, atol=1e-12)
        # the covariance against its largest entry (entries near zero are formed
        # by cancellation in both sums): measured at most 1.7e-14
        cerr = np.abs(post["cov"] - cov).max() / np.abs(cov).max()
        print("FP64 step: covariance error %.2e of its largest entry" % cerr)
        assert cerr < 1e-12, cerr


@pytest.mark.parametrize("prec", [0, 1])
def test_propagate_chain_sdirk(pf, oracle, prec):
    prob, sets = _chain_inputs()
    prob.lmm = pf.PF_LMM_BDF_SDIRK        # order 3: two SDIRK3 start-up steps
    rtol = prob.newton_rtol_fp64 if prec == 0 else prob.newton_rtol_fp32
    for x, th, h in sets:
        xg, gg, _ = _propagate_gpu(pf, prob, prec, x, th, h, True)
        xo, go, _ = _propagate_oracle(oracle, prob, x, th, h, True, rtol)
        err = relerr(xg, xo, prob.state_floor)
        assert err.max() < TOL[prec], (h, err.max())


@pytest.mark.parametrize("prec", [0, 1])
def test_step_parity_robertson_sdirk(pf, ctx, oracle, prec):
    prob = inputs.robertson(1000, 50, seed=2)
    prob.lmm, prob.order = pf.PF_LMM_BDF_SDIRK, 3
    ora, out, anc_o, anc_g, x, th, lw, post, scale = _step_case(pf, ctx, oracle, prob, prec, 7)
    same = anc_o == anc_g
    if prec == 0:
        assert same.all()
    else:
        assert same.mean() > 0.98
        _fp32_all_slots(oracle, prob, 7, anc_g, x, th)
    err = np.abs(x[same] - ora.x[same]) / scale[same]
    assert err.max() < TOL[prec], err.max()
    if prec == 0:
        fin = np.isfinite(ora.logw)
        assert np.allclose(lw[fin], ora.logw[fin], rtol=0, atol=1e-8)
        mean, cov = ora.moments()
        assert np.allclose(post["mean"], mean, rtol=1e-10, atol=1e-12)
        # the covariance against its largest entry (entries near zero are formed
        # by cancellation in both sums): measured at most 1.7e-14
        cerr = np.abs(post["cov"] - cov).max() / np.abs(cov).max()
        print("FP64 step: covariance error %.2e of its largest entry" % cerr)
        assert cerr < 1e-12, cerr


@pytest.mark.parametrize("prec", [0, 1])
def test_step_parity_chain(pf, ctx, oracle, prec):
    """One step of the chain from the oracle's ensemble after three steps.
    FP64: the bidiagonal forward substitution and the oracle's pivoted dense
    LU agree to rounding (a CPU replay of the device integrator gives states
    within 5e-15 and identical ancestors), so ancestors are bit-exact and
    weights, moments and ESS agree to rounding."""
    prob = inputs.chain16(2000, 10, seed=1)
    ora, out, anc_o, anc_g, x, th, lw, post, scale = _step_case(pf, ctx, oracle, prob, prec, 3)
    same = anc_o == anc_g
    if prec == 0:
        assert same.all(), (~same).sum()
    else:
        assert same.mean() > 0.95
        _fp32_all_slots(oracle, prob, 3, anc_g, x, th)
    err = np.abs(x[same] - ora.x[same]) / scale[same]
    assert err.max() < TOL[prec], err.max()
    if prec == 0:
        assert np.allclose(th, ora.theta, rtol=1e-12, atol=1e-12)
        fin = np.isfinite(ora.logw)
        assert np.array_equal(np.isfinite(lw), fin)
        print("chain FP64 step: logw max abs err", np.abs(lw[fin] - ora.logw[fin]).max())
        assert np.allclose(lw[fin], ora.logw[fin], rtol=0, atol=1e-8)
        mean, cov = ora.moments()
        print("chain FP64 step: mean rel err", np.abs(post["mean"] - mean).max() / np.abs(mean).max(),
              "cov rel err", np.abs(post["cov"] - cov).max() / np.abs(cov).max())
        assert np.allclose(post["mean"], mean, rtol=1e-10, atol=1e-12)
        assert np.abs(post["cov"] - cov).max() < 1e-9 * np.abs(cov).max()
        assert post["ess"] == pytest.approx(out["ess"], rel=1e-8)


# ---------------------------------------------------------------- negative states (reading R4)
def _negative_inputs(oracle, prob):
    """Robertson states with x2 < 0 (as an innovation could leave them) at
    several intervals of the small schedule, prior parameter draws, and the
    oracle's pivoted-LU result; kept where the oracle's Newton converges at
    every step (for x2 below about -1e-5 the kinetics x2' = -k2 x2^2 run away
    within the interval and neither side converges)."""
    rng = np.random.default_rng(21)
    xs, ths, hs, ref = [], [], [], []
    for j in (1, 5, 20):
        t0, t1 = prob.times[j - 1], prob.times[j]
        h = (t1 - t0) / prob.substeps
        for neg in (-1e-9, -1e-7, -1e-6, -1e-5):
            for _ in range(8):
                x = prob.x_true[j - 1].copy()
                x[1] = neg * (1.0 + rng.random())
                th = prob.theta_true + 0.5 * rng.standard_normal(3)
                xo, go, st = oracle.psi(prob.model, x, th, h, prob.substeps, prob.order, lte=True,
                                        rtol=prob.newton_rtol_fp64, kmax=prob.newton_max_iter,
                                        floor=prob.state_floor)
                if st["newton_fails"] == 0:
                    xs.append(x)
                    ths.append(th)
                    hs.append(h)
                    ref.append((xo, go))
    return xs, ths, hs, ref


def test_propagate_robertson_negative_states(pf, oracle):
    """The unpivoted elimination of I - c J (reading R4) on states with a
    negative x2, where its pivots are no longer bounded below by 1, against
    the oracle's partial pivoting in FP64: the same results to 1e-10."""
    prob = inputs.robertson(1000, 50)
    xs, ths, hs, ref = _negative_inputs(oracle, prob)
    assert len(xs) >= 60, len(xs)
    worst = 0.0
    for x, th, h, (xo, go) in zip(xs, ths, hs, ref):
        xg, gg, _ = _propagate_gpu(pf, prob, 0, x[None, :], th[None, :], h, True)
        err = relerr(xg[0], xo, prob.state_floor)
        worst = max(worst, err.max())
        assert err.max() < TOL[0], (x, th, h, err.max())
        # the estimate of a component whose local error is below its own
        # rounding (x1 ~ 1, sqrt(Gamma) ~ 1e-14) is rounding noise; bound
        # the rest relatively
        dev_ = np.abs(np.sqrt(gg[0]) - np.sqrt(go))
        assert np.all(dev_ <= 1e-7 * np.sqrt(go) + 64 * 2.0**-52 * np.abs(xo)), (x, th, h)
    print("negative x2 inputs:", len(xs), "worst rel err %.2e" % worst)


def test_negative_state_counter(pf, ctx, oracle):
    """pf_stats counts new states with a negative component: none on the
    small configuration; every particle when the ensemble sits at
    x = (0, -1e-9, 0), where x2' = -k2 x2^2 keeps x2 negative over the
    interval.  That step still equals the oracle's in FP64."""
    prob = inputs.robertson(1000, 50, seed=2)
    f = pf.Filter(ctx, pf.Config(prob, pf.PF_PREC_FP64))
    for j in range(10):
        assert f.assimilate(prob.times[j], prob.y[j], prob.sigma[j]) == pf.PF_OK
    assert f.stats()["negative_states"] == 0
    f.close()
    ora = oracle.Filter(prob)
    ora.step(prob.times[0], prob.y[0], prob.sigma[0])
    x = np.tile([0.0, -1e-9, 0.0], (prob.n_particles, 1))
    mean, cov = ora.moments()
    ora.set_ensemble(x, ora.theta, ora.logw, mean, cov, ora.chol(), ora.j, ora.t)
    f = pf.Filter(ctx, pf.Config(prob, pf.PF_PREC_FP64))
    _set(pf, f, ora)
    sig = np.full(1, 1e3)     # uninformative: every slot keeps a particle
    assert f.assimilate(prob.times[1], prob.y[1], sig) == pf.PF_OK
    out = ora.step(prob.times[1], prob.y[1], sig)
    assert out["status"] == 0
    assert np.all(ora.x[:, 1] < 0)
    assert f.stats()["negative_states"] == prob.n_particles
    xg, thg, _ = _get(pf, f)
    err = relerr(xg, ora.x, prob.state_floor)
    assert err.max() < TOL[0], err.max()
    f.close()
