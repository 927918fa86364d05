"""How far the oracle moves from itself under another valid rounding.

A whole FP64 run of the filter (Algorithm 1 over T observations) maps
rounding-level differences in the states to differences in the posterior
summaries.  The map is mild for Robertson and can be steep for the 16-state
chain: the Newton stopping rule (relative step 1e-12) turns a rounding change
into a 1e-12 change of a state when a lane's test flips, and the likelihood
weights with 2% noise scale state changes by (x / sigma)^2 before the moments
see them, more so when few particles carry the weight.

The yardstick is the same oracle source compiled with fused multiply-adds
(gcc -mfma -ffp-contract=fast): every a*b+c in it rounds once instead of
twice, an equally valid FP64 evaluation.  The spread between the two builds at
each step measures the rounding sensitivity of that run; the GPU, whose
rounding differs from the oracle's in a comparable way (fused multiply-adds,
other reduction trees, device exp/log), is held to a fixed multiple of it,
and never looser than the flat floor of the insensitive runs.
TEST INFRASTRUCTURE ONLY (it loads the oracle)."""
from __future__ import annotations

import importlib.util
import os
import tempfile

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WRAPPER = os.path.join(ROOT, "oracle", "oracle.py")
FMA_FLAGS = ["-std=gnu11", "-mfma", "-ffp-contract=fast"]
# flat floor of the whole-run tolerances, and the multiple of the oracle's
# own spread a GPU run may reach
FLOOR = 1e-9
FACTOR = 30.0

_fma = None


def fma_oracle():
    """A second, independent load of the oracle built with fused multiply-adds."""
    global _fma
    if _fma is None:
        d = tempfile.mkdtemp(prefix="oracle_fma_")
        spec = importlib.util.spec_from_file_location("oracle_fma", WRAPPER)
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        mod.LIB = os.path.join(d, "liboracle_fma.so")
        mod.LIB_OVERRIDE = None
        mod.compile_to(mod.SRC, mod.LIB, FMA_FLAGS)
        mod._lib = None
        _fma = mod
    return _fma


def summary_errors(gm, gs, om, osd):
    """Per-step errors of a run's posterior summaries against the oracle's:
    the mean relative to max(|mean|, sd), the sd relative to the sd (max over
    parameters; a zero oracle sd compares absolutely)."""
    gm, gs, om, osd = (np.atleast_2d(np.asarray(v, dtype=float)) for v in (gm, gs, om, osd))
    em = (np.abs(gm - om) / np.maximum(np.abs(om), osd)).max(axis=1)
    es = (np.abs(gs - osd) / np.where(osd > 0, osd, 1.0)).max(axis=1)
    return em, es


def spread(oracle, prob, T, seed=None):
    """Oracle run (means, sds, ess) and the per-step spread (mean, sd, ess)
    of the fused-multiply-add build from it."""
    om, osd, oess = oracle.Filter(prob, seed=seed).run(T)
    fm, fsd, fess = fma_oracle().Filter(prob, seed=seed).run(T)
    em, es = summary_errors(fm, fsd, om, osd)
    fin = np.isfinite(oess) & np.isfinite(fess)
    ee = np.zeros(len(oess))
    ee[fin] = np.abs(fess[fin] - oess[fin]) / oess[fin]
    return (om, osd, oess), (em, es, ee)


def tolerances(sp):
    """Per-step tolerances (mean, sd, ess) from the spread."""
    return tuple(np.maximum(FLOOR, FACTOR * s) for s in sp)
