"""The single-filter step's systematic draw, done inside the update kernel
(each output slot finds its own ancestor), against the oracle's resampling on
weights that drive each of its search paths: even weights and one heavy
particle far from the slots (a workgroup's ancestors in at most four tiles,
whose prefixes it stages in LDS), and light particles one per tile (a
workgroup's slots drawing from more tiles than it stages: the search in
global memory).  A flat likelihood (sigma = 1e150) makes the first-stage
weights the committed ones, so the ancestors follow from the chosen
log-weights alone; they must equal the oracle's bit for bit, in both
propagation precisions."""
import numpy as np
import pytest

from paper_1411_1702_amd import inputs
import test_gpu_parity as TP

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N = 8192          # 32 tiles


def _logw(kind):
    w = np.zeros(N)
    if kind == "even":
        w[:] = 1.0
    elif kind == "far_heavy":
        w[:] = 1e-5
        w[N - 1] = 1.0
    elif kind == "light_per_tile":
        # tiles 0..9: one particle each with about 50 copies; the rest to the last particle
        for t in range(10):
            w[256 * t] = 50.0 / N
        w[N - 1] = 1.0 - w.sum()
    with np.errstate(divide="ignore"):
        return np.log(w)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kind", ["even", "far_heavy", "light_per_tile"])
def test_folded_draw_matches_oracle(pf, oracle, prec, kind):
    prob = inputs.robertson(N, 50, seed=7)
    j0 = 4
    ora = oracle.Filter(prob)
    rng = np.random.default_rng(31)
    x = np.tile(prob.x_true[j0 - 1], (N, 1))
    th = prob.theta_true + 0.1 * rng.standard_normal((N, prob.p))
    lw = _logw(kind)
    tb = prob.theta_true.copy()
    ora.set_ensemble(x, th, lw, tb, np.zeros((3, 3)), np.zeros((3, 3)), j0, prob.times[j0 - 1])
    sigma = np.full(prob.m, 1e150)
    rc, g, anc_o = ora.stage1(prob.times[j0], prob.y[j0], sigma)
    assert rc == 0
    with pf.Context(0, 1 << 30) as ctx:
        f = pf.Filter(ctx, pf.Config(prob, prec))
        TP._set(pf, f, ora)
        assert f.assimilate(prob.times[j0], prob.y[j0], sigma) == pf.PF_OK
        anc = torch.zeros(N, dtype=torch.int32, device="cuda")
        pf.check(pf.lib().pf_test_last_ancestors(f.h, anc.data_ptr()), "anc")
        anc_g = anc.cpu().numpy()
        f.close()
    print(kind, "precision", prec, "distinct ancestors", len(np.unique(anc_o)),
          "mismatches", int((anc_g != anc_o).sum()))
    assert np.array_equal(anc_g, anc_o)


@pytest.fixture(scope="module")
def pf():
    from paper_1411_1702_amd import pf as _pf
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _pf.lib()
    return _pf


def test_filter_above_the_fold_limit_uses_the_scatter_pass(pf, oracle):
    """A single filter of more than 2^19 particles keeps the separate scatter
    pass (its tile offsets would not fit the update kernel's LDS): its first
    step's ancestors must equal the oracle's, bit for bit (FP64, so that both
    sides resample on the same integer weights)."""
    n = (1 << 19) + 777
    prob = inputs.robertson(n, 50, seed=11)
    ora = oracle.Filter(prob)
    rc, g, anc_o = ora.stage1(prob.times[0], prob.y[0], prob.sigma[0])
    assert rc == 0
    with pf.Context(0, 1 << 30) as ctx:
        f = pf.Filter(ctx, pf.Config(prob, pf.PF_PREC_FP64))
        assert f.assimilate(prob.times[0], prob.y[0], prob.sigma[0]) == pf.PF_OK
        anc = torch.zeros(n, dtype=torch.int32, device="cuda")
        pf.check(pf.lib().pf_test_last_ancestors(f.h, anc.data_ptr()), "anc")
        anc_g = anc.cpu().numpy()
        f.close()
    print("N", n, "distinct ancestors", len(np.unique(anc_o)), "mismatches", int((anc_g != anc_o).sum()))
    assert np.array_equal(anc_g, anc_o)
