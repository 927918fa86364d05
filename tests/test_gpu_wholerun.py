"""Whole-run parity in FP64: the GPU filter and the oracle, given the same
seed, follow the same trajectory over every observation of a run.

Both draw every random number from the same counter-based streams and take
the resampling decisions on the same integer weights, so with FP64
propagation the only differences are rounding-order ones (tree reductions,
the kinetic models' unpivoted solves, the advection-diffusion transforms).
Those stay far below the spacing of the integer weights' resampling
thresholds, so no ancestor changes and the posterior summaries agree to
rounding at every step: within the flat floor `tol`, or a fixed multiple of
the oracle's own spread under fused multiply-adds where the run amplifies
rounding (tests/rounding_yardstick.py).

The 16-state chain is not among the whole runs: its first observation leaves
1-5 particles with weight, the parameter covariance is then rank-deficient
with a rounding-noise null space, and the jittered Cholesky factor differs
between evaluation orders by far more than rounding (shown on the CPU in
test_rounding_yardstick.py).  It is compared step by step from a shared
ensemble (test_gpu_parity.py, test_gpu_batch_oracle.py) and statistically
over all 100 observations (test_gpu_statistical.py).  This is a deterministic check of the whole of
Algorithm 1 over long runs; the statistical tests then cover the FP32
propagation, whose trajectories decorrelate."""
import numpy as np
import pytest

from paper_1411_1702_amd import inputs
import rounding_yardstick as Y

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
    ]


@pytest.mark.parametrize("name,prob,T,R,tol", _cases(), ids=[c[0] for c in _cases()])
def test_fp64_run_follows_the_oracle(pf, oracle, name, prob, T, R, tol):
    with pf.Context(0, 2 << 30) as ctx:
        for seed in range(R):
            (om, osd, oess), sp = Y.spread(oracle, prob, T, seed=seed)
            tm, ts, te = (np.maximum(tol, t) for t in Y.tolerances(sp))
            gm, gsd, gess = pf.run_filter(ctx, prob, pf.PF_PREC_FP64, T=T, seed=seed)
            err_m, err_s = Y.summary_errors(gm, gsd, om, osd)
            print(name, seed, "mean err %.2e sd err %.2e; oracle spread %.2e %.2e; worst/tol %.2f %.2f"
                  % (err_m.max(), err_s.max(), sp[0].max(), sp[1].max(), (err_m / tm).max(), (err_s / ts).max()))
            assert (err_m < tm).all(), (seed, int(np.argmax(err_m / tm)), err_m.max())
            assert (err_s < ts).all(), (seed, int(np.argmax(err_s / ts)), err_s.max())
            fin = np.isfinite(oess)
            assert (np.abs(gess[fin] - oess[fin]) <= te[fin] * oess[fin]).all()
