"""The whole-run FP64 tolerances' yardstick (tests/rounding_yardstick.py) on
the CPU: the fused-multiply-add build of the oracle is a different rounding
of the same computation (it moves the chain's posterior), its spread on
Robertson stays far below the flat floor the Robertson runs are held to, and
on the chain it follows the chain's own amplification of rounding."""
import numpy as np

from paper_1411_1702_amd import inputs
import rounding_yardstick as Y


def test_robertson_spread_far_below_the_floor(oracle):
    _, (em, es, ee) = Y.spread(oracle, inputs.robertson(1000, 50, seed=0), 20)
    print("Robertson spread: mean %.1e sd %.1e ess %.1e" % (em.max(), es.max(), ee.max()))
    assert em.max() < Y.FLOOR / 100 and es.max() < Y.FLOOR / 100 and ee.max() < Y.FLOOR / 100


def test_chain_spread_is_a_real_rounding_change(oracle):
    prob = inputs.chain16(1024, 100, seed=4, model_seed=inputs.CHAIN_INSTANCES[0])
    (om, osd, _), (em, es, _) = Y.spread(oracle, prob, 10)
    print("chain spread by step: sd", " ".join("%.0e" % v for v in es))
    # the two builds differ (the yardstick measures something) ...
    assert es.max() > 0.0
    # ... by rounding, not by a different computation: far below the
    # posterior's own scale
    assert em.max() < 1e-6 and es.max() < 1e-6
    # and the tolerances never drop below the floor
    tm, ts, te = Y.tolerances((em, es, es))
    assert (tm >= Y.FLOOR).all() and (ts >= Y.FLOOR).all()
    assert np.isfinite(om).all() and (osd > 0).all()


def test_chain_first_observation_collapses(oracle):
    """Why the chain has no whole-run FP64 comparison: after its first
    observation only a handful of particles keep weight, so the 12 x 12
    parameter covariance has rank at most 5 and its other eigenvalues are
    rounding noise; the Cholesky factor needs the jitter, and its null-space
    columns (from which step 4(a) draws) are set by that noise."""
    prob = inputs.chain16(1024, 100, seed=0)
    F = oracle.Filter(prob, seed=0)
    out = F.step(prob.times[0], prob.y[0], prob.sigma[0])
    w = np.exp(F.logw - F.logw.max())
    w /= w.sum()
    _, C = F.moments()
    ev = np.sort(np.abs(np.linalg.eigvalsh(C)))
    print("chain step 1: ess %.3f, weights > 1e-12: %d, |eigenvalues| of C:" % (out["ess"], (w > 1e-12).sum()),
          " ".join("%.0e" % v for v in ev))
    assert out["ess"] < 5.0
    assert (w > 1e-12).sum() <= 6
    assert out["jitters"] >= 1
    # seven of the twelve eigenvalues are below 1e-10 of the largest
    assert (ev < 1e-10 * ev[-1]).sum() >= 7
