"""Whole-run parity in FP64: the GPU filter and the oracle, given the same
seed, follow the same trajectory over every observation of a run.

Both draw every random number from the same counter-based streams and take
the resampling decisions on the same integer weights, so with FP64
propagation the only differences are rounding-order ones (tree reductions,
the kinetic models' unpivoted solves, the advection-diffusion transforms).
Those stay far below the spacing of the integer weights' resampling
thresholds, so no ancestor changes and the posterior summaries agree to
rounding at every step.  This is a deterministic check of the whole of
Algorithm 1 over long runs; the statistical tests then cover the FP32
propagation, whose trajectories decorrelate."""
import numpy as np
import pytest

from paper_1411_1702_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pf():
    from paper_1411_1702_amd import pf as _pf
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _pf.lib()
    return _pf


def _cases():
    small = inputs.config_small()
    am1 = inputs.config_small()
    am1.lmm, am1.order = 1, 1
    sd3 = inputs.config_small()
    sd3.lmm, sd3.order = 2, 3
    mult = inputs.config_small()
    mult.resampling = 1
    return [
        ("robertson_bdf2_50", small, 50, 3, 1e-9),
        ("robertson_bdf2_200_n8192", inputs.robertson(8192, 200, seed=0), 200, 2, 1e-9),
        ("robertson_am1_50", am1, 50, 2, 1e-9),
        ("robertson_bdf3_sdirk_50", sd3, 50, 2, 1e-9),
        ("robertson_multinomial_50", mult, 50, 2, 1e-9),
        ("advdiff_7x7_n512", inputs.advdiff(512, 5, seed=0, n=8), 5, 2, 1e-9),
        ("advdiff_19x19_n64", inputs.advdiff(64, 2, seed=0, n=20), 2, 1, 1e-9),
        ("chain16_bdf3_n1024_30", inputs.chain16(1024, 100, seed=0), 30, 2, 1e-9),
    ]


@pytest.mark.parametrize("name,prob,T,R,tol", _cases(), ids=[c[0] for c in _cases()])
def test_fp64_run_follows_the_oracle(pf, oracle, name, prob, T, R, tol):
    with pf.Context(0, 2 << 30) as ctx:
        for seed in range(R):
            om, osd, oess = oracle.Filter(prob, seed=seed).run(T)
            gm, gsd, gess = pf.run_filter(ctx, prob, pf.PF_PREC_FP64, T=T, seed=seed)
            scale = np.maximum(np.abs(om), osd)
            err_m = np.abs(gm - om) / scale
            err_s = np.abs(gsd - osd) / osd
            print(name, seed, "mean err", err_m.max(), "sd err", err_s.max())
            assert err_m.max() < tol, (seed, err_m.max())
            assert err_s.max() < tol, (seed, err_s.max())
            fin = np.isfinite(oess)
            assert np.allclose(gess[fin], oess[fin], rtol=tol, atol=0)
