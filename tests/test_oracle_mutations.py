"""Mutation check of the composition pins (tests/oracle_pins.py): plausible
one-line slips in the oracle's Algorithm 1 step are planted in a copy of
the oracle source, compiled on the CPU, and every slip must make at least one
pin fail.  The untouched oracle passes every pin (test_oracle_composition)."""
import importlib.util
import os

import pytest

import oracle_pins as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "pf_oracle.c")
WRAPPER = os.path.join(ROOT, "oracle", "oracle.py")

# (name, text in or_filter_step, slipped text)
SLIPS = [
    # step 3(a): fitness weight without the committed weight w_j
    ("drop_wj_in_fitness", "lg[n] = s->logw[n] + lbar[n];", "lg[n] = lbar[n];"),
    # steps 4(c)-(d): no innovation, or Gamma used as a standard deviation
    ("drop_innovation", "xn[n * d + i] = xt[i] + sqrt(gam[i]) * zz[i];", "xn[n * d + i] = xt[i];"),
    ("gamma_as_sd", "xn[n * d + i] = xt[i] + sqrt(gam[i]) * zz[i];", "xn[n * d + i] = xt[i] + gam[i] * zz[i];"),
    # step 5: no predictive-likelihood denominator, or the slot's own one
    ("drop_step5_denominator", "xn + n * d) - lbar_anc;", "xn + n * d);"),
    ("own_denominator", "double lbar_anc = lbar[k];", "double lbar_anc = lbar[n];"),
    # step 3(c): the slot's own state or shrunk parameters instead of the ancestor's
    ("own_state", "const double* xj = s->x + k * d;", "const double* xj = s->x + n * d;"),
    ("own_shrunk_theta", "const double* mj = mshr + k * p;", "const double* mj = mshr + n * p;"),
    # steps 2 and 4(a): kernel width s^2 for s, shrink weights swapped
    ("s_squared", "sh = sqrt(1.0 - a * a);", "sh = 1.0 - a * a;"),
    ("swapped_shrink",
     "mshr[n * p + i] = a * s->theta[n * p + i] + (1.0 - a) * s->theta_bar[i];",
     "mshr[n * p + i] = (1.0 - a) * s->theta[n * p + i] + a * s->theta_bar[i];"),
]


def _mutant(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"slip site of {name} not found once in the oracle"
    c = tmp_path / f"mut_{name}.c"
    c.write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location(f"oracle_mut_{name}", WRAPPER)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod.SRC = str(c)
    mod.LIB = str(tmp_path / f"mut_{name}.so")
    mod.compile_to(mod.SRC, mod.LIB)
    mod._lib = None
    return mod


@pytest.mark.slow
@pytest.mark.parametrize("name,old,new", SLIPS, ids=[s[0] for s in SLIPS])
def test_slip_fails_a_pin(tmp_path, name, old, new):
    O = _mutant(tmp_path, name, old, new)
    failed = []
    for pin in P.PINS:
        try:
            pin(O)
        except AssertionError as e:
            failed.append((pin.__name__, str(e)[:120]))
    print(name, "caught by", [f[0] for f in failed])
    assert failed, f"slip {name} passes every composition pin"
