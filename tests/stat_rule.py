"""The two-sample rule of the statistical parity tests, shared by the GPU
comparison (test_gpu_statistical.py) and its calibration on the oracle
alone (test_stat_rule_calibration.py).

Each side runs R replicate filters with independent seeds.  At every
observation step, for every parameter's posterior mean and sd, z =
(mean_a - mean_b) / sqrt(var_a / R + var_b / R) over the replicates.  The
rule: at most 10% of the (step, parameter) z-scores beyond 3, none beyond 5.
The z-scores of one comparison are strongly correlated over steps (the
posterior at step j carries into step j + 1), so one replicate set's
excursion spans many steps; the 10% allowance is what two independent
oracle seed sets need (calibration test)."""
import numpy as np

FRAC_BEYOND_3 = 0.10
MAX_Z = 5.0


def replicates(run, R, seed0):
    ms, ss = [], []
    for r in range(R):
        m, s, _ = run(seed0 + r)
        ms.append(m)
        ss.append(s)
    return np.array(ms), np.array(ss)


def zscores(a, b):
    R = a.shape[0]
    se = np.sqrt(a.var(axis=0, ddof=1) / R + b.var(axis=0, ddof=1) / R)
    return (a.mean(axis=0) - b.mean(axis=0)) / np.maximum(se, 1e-300)


def margins(a_m, a_s, b_m, b_s):
    """{'mean': (fraction beyond 3, max |z|), 'sd': (...)} of one comparison."""
    out = {}
    for name, z in (("mean", zscores(a_m, b_m)), ("sd", zscores(a_s, b_s))):
        z = z[np.isfinite(z)]
        out[name] = (float(np.mean(np.abs(z) > 3.0)), float(np.abs(z).max()))
    return out


def passes(m):
    return all(f <= FRAC_BEYOND_3 and zmax < MAX_Z for f, zmax in m.values())
