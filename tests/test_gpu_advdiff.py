"""GPU parity of the advection-diffusion model (Sec. 4) against the FP64
oracle, through the C ABI.

The GPU solves each implicit step mode by mode in Fourier space; the oracle
runs Newton with a dense pivoted LU on the assembled operator.  The results
agree to rounding: FP64 states within 1e-10 of the field's largest value,
FP32 within a few 1e-6 (a transform mixes every grid value, so its rounding
error is uniform over the field and is measured against the field's scale,
not point by point).  Grids: odd and even sides on the one-wavefront shape
(nt = 7, 8, 19) and the four-wavefront shape (nt = 39, d = 1521)."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from paper_1411_1702_amd import inputs
import jitter_bound as JB

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

XTOL = {0: 1e-10, 1: 5e-6}     # state, relative to the particle's largest value
GTOL = {0: 1e-8, 1: 3e-3}      # sqrt(Gamma), relative to its largest value


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


def _inputs(n, count, seed):
    prob = inputs.advdiff(64, 3, seed=seed, n=n)
    rng = np.random.default_rng(seed)
    x = np.tile(prob.x0, (count, 1)) * (1 + 0.05 * rng.standard_normal((count, prob.d)))
    th = prob.prior_mean + 0.5 * rng.standard_normal((count, prob.p))
    return prob, x, th


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


def _propagate_oracle(oracle, prob, x, theta, h, lte):
    def one(i):
        xo, go, _ = oracle.psi(prob.model, x[i], theta[i], h, prob.substeps, prob.order, lte=lte,
                               rtol=prob.newton_rtol_fp64, kmax=prob.newton_max_iter, floor=prob.state_floor,
                               mc=prob.model_consts, lmm=prob.lmm)
        return xo, go
    with ThreadPoolExecutor(8) as ex:
        res = list(ex.map(one, range(x.shape[0])))
    return np.array([r[0] for r in res]), np.array([r[1] for r in res])


def _check_prop(xg, gg, xo, go, prec, lte, what):
    ex = (np.abs(xg - xo).max(axis=1) / np.abs(xo).max(axis=1)).max()
    print(what, "state err", ex)
    assert ex < XTOL[prec], (what, ex)
    if lte:
        sg, so = np.sqrt(gg), np.sqrt(go)
        eg = (np.abs(sg - so).max(axis=1) / so.max(axis=1)).max()
        print(what, "sqrt gamma err", eg)
        assert eg < GTOL[prec], (what, eg)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("lte", [False, True])
@pytest.mark.parametrize("n,lmm,order", [(8, 0, 2), (9, 0, 2), (8, 0, 1), (8, 2, 3), (9, 2, 2), (20, 0, 2)])
def test_propagate_matches_oracle(pf, oracle, prec, lte, n, lmm, order):
    prob, x, th = _inputs(n, 24 if n < 20 else 8, seed=n + order)
    prob.lmm, prob.order = lmm, order
    h = 0.1
    xg, gg, it = _propagate_gpu(pf, prob, prec, x, th, h, lte)
    xo, go = _propagate_oracle(oracle, prob, x, th, h, lte)
    _check_prop(xg, gg, xo, go, prec, lte, (n, lmm, order))
    assert it == x.shape[0] * prob.substeps      # one linear solve per step


@pytest.mark.parametrize("prec", [0, 1])
def test_propagate_largest_grid(pf, oracle, prec):
    # nt = 39 (d = 1521, four wavefronts per particle); short interval so the
    # oracle's dense LU (2.3 GFLOP per factorisation) stays affordable
    prob, x, th = _inputs(40, 2, seed=5)
    prob.substeps = 3
    xg, gg, _ = _propagate_gpu(pf, prob, prec, x, th, 0.1, True)
    xo, go = _propagate_oracle(oracle, prob, x, th, 0.1, True)
    _check_prop(xg, gg, xo, go, prec, True, "nt=39")


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
    prob = inputs.advdiff(1000, 3, seed=4, n=8)
    f = pf.Filter(ctx, pf.Config(prob, prec))
    ora = oracle.Filter(prob)
    x, th, lw = _get(pf, f)
    assert np.allclose(th, ora.theta, rtol=1e-13, atol=1e-13)
    assert np.allclose(x, ora.x, rtol=0 if prec == 0 else 1e-7, atol=0)
    post = f.posterior()
    mean, cov = ora.moments()
    assert np.allclose(post["mean"], mean, rtol=1e-12, atol=1e-13)
    assert np.allclose(post["cov"], cov, rtol=1e-10, atol=1e-13)
    assert np.array_equal(post["state_mean"], prob.x0)
    f.close()


def _step_case(pf, ctx, oracle, prob, prec, j0):
    ora = oracle.Filter(prob)
    for j in range(j0):
        assert ora.step(prob.times[j], prob.y[j], prob.sigma[j])["status"] == 0
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
    return ora, out, anc_o, anc_g, x, th, lw, post


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n,N,j0", [(8, 1000, 0), (8, 1000, 2), (20, 128, 0)])
def test_step_matches_oracle(pf, ctx, oracle, prec, n, N, j0):
    prob = inputs.advdiff(N, 4, seed=2, n=n)
    ora, out, anc_o, anc_g, x, th, lw, post = _step_case(pf, ctx, oracle, prob, prec, j0)
    same = anc_o == anc_g
    if prec == 0:
        assert same.all()
    else:
        assert same.mean() > 0.95, same.mean()
    # states after the innovation, against each particle's largest value
    ex = (np.abs(x[same] - ora.x[same]).max(axis=1) / np.abs(ora.x[same]).max(axis=1)).max()
    print("step state err", ex)
    assert ex < (1e-10 if prec == 0 else 2e-4), ex
    if prec == 0:
        assert np.allclose(th[same], ora.theta[same], rtol=1e-12, atol=1e-12)
    else:
        # FP32 proliferation normals: their Box-Muller rounding through s L z
        pre = oracle.Filter(prob)
        for j in range(j0):
            pre.step(prob.times[j], prob.y[j], prob.sigma[j])
        bound = JB.fp32_jitter_bound(oracle, prob, pre.chol(), j0 + 1, len(th))
        dev_ = np.abs(th - ora.theta)
        print("FP32 jitter: worst |d theta| / bound %.3f" % (dev_[same] / bound[same]).max())
        assert np.all(dev_[same] <= bound[same])
        # every slot, against the oracle's step taken with the GPU's ancestors
        orb = oracle.Filter(prob)
        for j in range(j0):
            orb.step(prob.times[j], prob.y[j], prob.sigma[j])
        assert orb.step_given(prob.times[j0], prob.y[j0], prob.sigma[j0], anc_g) == 0
        ea = (np.abs(x - orb.x).max(axis=1) / np.abs(orb.x).max(axis=1)).max()
        print("FP32 step, all slots with the GPU's ancestors: state err", ea)
        assert ea < 2e-4, ea
        assert np.all(np.abs(th - orb.theta) <= bound)
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
        assert np.allclose(post["state_mean"], out["state_mean"], rtol=1e-9, atol=1e-12)
    else:
        assert np.allclose(post["state_mean"], out["state_mean"], rtol=1e-3)


def test_configuration_limits(pf, ctx):
    prob = inputs.advdiff(300, 2, seed=1, n=8)
    L = pf.lib()
    cfg = pf.Config(prob)
    assert L.pf_filter_bytes(cfg.ptr()) > 0
    for mutate in (lambda c: setattr(c.c, "lmm", pf.PF_LMM_AM), lambda c: setattr(c.c, "p", 4),
                   lambda c: setattr(c.c, "d", 50), lambda c: setattr(c.c, "m", 33)):
        cfg = pf.Config(prob)
        mutate(cfg)
        assert L.pf_filter_bytes(cfg.ptr()) == 0
    # a batch row holds 4 observations: an advdiff filter with 20 sites is refused
    f = pf.Filter(ctx, pf.Config(prob))
    with pytest.raises(pf.PfError):
        ctx.assimilate_batch([f], [prob.times[0]], [prob.y[0]], [prob.sigma[0]])
    f.close()


def test_batched_equals_alone(pf, ctx):
    # an advdiff filter with 4 sites next to a Robertson filter in one batch
    # gives the same result, bit for bit, as each filter alone
    ad = inputs.advdiff(700, 3, seed=3, n=8, sites=4)
    rb = inputs.robertson(900, 3, seed=3)
    alone = []
    for prob in (ad, rb):
        f = pf.Filter(ctx, pf.Config(prob))
        for j in range(3):
            assert f.assimilate(prob.times[j], prob.y[j], prob.sigma[j]) == pf.PF_OK
        alone.append(f.posterior())
        f.close()
    fs = [pf.Filter(ctx, pf.Config(p)) for p in (ad, rb)]
    for j in range(3):
        tk = ctx.assimilate_batch(fs, [ad.times[j], rb.times[j]], [ad.y[j], rb.y[j]], [ad.sigma[j], rb.sigma[j]])
        assert all(f.wait(t) == pf.PF_OK for f, t in zip(fs, tk))
    for f, a in zip(fs, alone):
        b = f.posterior()
        assert np.array_equal(a["mean"], b["mean"]) and np.array_equal(a["cov"], b["cov"])
        assert np.array_equal(a["state_mean"], b["state_mean"])
        f.close()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n", [4, 23, 24, 26])
def test_propagate_generic_grid_sides(pf, oracle, prec, n):
    # the generic instances (grid side not a compile-time constant): the
    # smallest grid (3 x 3), the one-wavefront shape at its limit (22 x 22),
    # and the four-wavefront shape below 39 (23 x 23, 25 x 25)
    prob, x, th = _inputs(n, 8 if n < 24 else 4, seed=n)
    xg, gg, _ = _propagate_gpu(pf, prob, prec, x, th, 0.1, True)
    xo, go = _propagate_oracle(oracle, prob, x, th, 0.1, True)
    _check_prop(xg, gg, xo, go, prec, True, ("generic", n))


@pytest.mark.parametrize("N,sites,lmm,order", [(257, 20, 0, 2), (1013, 32, 0, 2), (700, 20, 2, 3)])
def test_step_ragged_max_sites_startup(pf, ctx, oracle, N, sites, lmm, order):
    # a ragged last tile, the largest number of observed sites, and BDF3 with
    # the SDIRK start-up, through a whole FP64 step
    prob = inputs.advdiff(N, 3, seed=5, n=8, sites=sites)
    prob.lmm, prob.order = lmm, order
    ora, out, anc_o, anc_g, x, th, lw, post = _step_case(pf, ctx, oracle, prob, 0, 1)
    assert np.array_equal(anc_o, anc_g)
    ex = (np.abs(x - ora.x).max(axis=1) / np.abs(ora.x).max(axis=1)).max()
    assert ex < 1e-10, ex
    fin = np.isfinite(ora.logw)
    assert np.allclose(lw[fin], ora.logw[fin], rtol=0, atol=1e-8)
    mean, cov = ora.moments()
    assert np.allclose(post["mean"], mean, rtol=1e-10, atol=1e-12)
    # the covariance against its largest entry (entries near zero are formed
    # by cancellation in both sums): measured at most 1.7e-14
    cerr = np.abs(post["cov"] - cov).max() / np.abs(cov).max()
    print("FP64 step: covariance error %.2e of its largest entry" % cerr)
    assert cerr < 1e-12, cerr
    assert np.allclose(post["state_mean"], out["state_mean"], rtol=1e-9, atol=1e-12)
