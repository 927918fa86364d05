"""Calibration of the statistical parity rule (tests/stat_rule.py) on the
oracle alone: two independent oracle seed sets are two samples of the same
distribution, so the rule must accept them.  Each case compares disjoint
pairs of R = 16 seed sets on the configurations the GPU statistical tests
use, and prints the observed fraction of z-scores beyond 3 and the largest
|z|: the evidence behind the 10% / |z| < 5 allowance."""
import numpy as np
import pytest

import stat_rule as S
from paper_1411_1702_amd import inputs


def _small(lmm=0, order=2, resampling=0):
    p = inputs.config_small()
    p.lmm, p.order, p.resampling = lmm, order, resampling
    return p


CASES = [
    ("small_bdf2", _small(), 50, 16, 4),
    ("small_am1", _small(lmm=1, order=1), 50, 16, 4),
    ("small_multinomial", _small(resampling=1), 50, 16, 4),
    ("small_bdf3_sdirk", _small(lmm=2, order=3), 50, 16, 2),
]


@pytest.mark.slow
@pytest.mark.parametrize("name,prob,T,R,pairs", CASES, ids=[c[0] for c in CASES])
def test_independent_oracle_sets_pass_the_rule(oracle, name, prob, T, R, pairs):
    worst = {"mean": (0.0, 0.0), "sd": (0.0, 0.0)}
    for k in range(pairs):
        # seed sets 1000 k + [0, R) and 1000 k + 500 + [0, R): disjoint
        a = S.replicates(lambda sd: oracle.Filter(prob, seed=sd).run(T), R, 1000 * k)
        b = S.replicates(lambda sd: oracle.Filter(prob, seed=sd).run(T), R, 1000 * k + 500)
        m = S.margins(a[0], a[1], b[0], b[1])
        print(name, "pair", k, {q: (round(f, 3), round(z, 2)) for q, (f, z) in m.items()})
        for q in worst:
            worst[q] = (max(worst[q][0], m[q][0]), max(worst[q][1], m[q][1]))
        assert S.passes(m), (name, k, m)
    print(name, "worst over pairs", worst)
