"""CPU checks of the C ABI library: it loads, exports every symbol the
headers declare, and its pure-host entry points behave (no GPU calls)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1411_1702_amd import inputs, pf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in ("pf.h", "pf_test.h"):
        txt = open(os.path.join(ROOT, "include", h)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names |= set(re.findall(r"\b(pf_[a-z_0-9]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    L = pf.lib()
    declared = _declared()
    assert declared, "no declarations found"
    assert declared == set(pf.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


def test_config_struct_layout():
    # pf_config is 8-byte aligned with the fields in header order
    names = [f[0] for f in pf.pf_config._fields_]
    txt = open(os.path.join(ROOT, "include", "pf.h")).read()
    body = txt[txt.index("typedef struct {\n    uint32_t struct_size"):txt.index("} pf_config;")]
    decl = re.findall(r"\b(\w+)(?:\s*,\s*(\w+))?(?:\s*,\s*(\w+))?\s*;", re.sub(r"/\*.*?\*/", "", body, flags=re.S))
    hdr = [n for tup in decl for n in tup if n]
    assert hdr == names


def test_allocator_struct_layout():
    txt = open(os.path.join(ROOT, "include", "pf.h")).read()
    body = txt[txt.index("typedef struct {\n    void* (*alloc)"):txt.index("} pf_allocator;")]
    hdr = re.findall(r"\(\*(\w+)\)|void\* (\w+);", body)
    names = [a or b for a, b in hdr]
    assert names == [f[0] for f in pf.pf_allocator._fields_] == ["alloc", "free", "user"]


def test_status_strings():
    L = pf.lib()
    for s in range(9):
        assert L.pf_status_str(s)
    assert b"unknown" in L.pf_status_str(99)


def test_filter_bytes_host_only():
    L = pf.lib()
    cfg = pf.Config(inputs.robertson(1000, 5), pf.PF_PREC_FP32_PROP)
    b32 = L.pf_filter_bytes(cfg.ptr())
    cfg64 = pf.Config(inputs.robertson(1000, 5), pf.PF_PREC_FP64)
    b64 = L.pf_filter_bytes(cfg64.ptr())
    assert 0 < b32 < b64
    # 1024 padded particles: states, params, weights, scratch, ~= 120 B/particle + tiles
    assert 100 * 1024 < b32 < 400 * 1024
    big = pf.Config(inputs.robertson(1000, 5), pf.PF_PREC_FP32_PROP, n_particles=1 << 17)
    assert L.pf_filter_bytes(big.ptr()) > 100 * (1 << 17)


def test_bad_configs_rejected_on_host():
    L = pf.lib()
    prob = inputs.robertson(100, 5)
    for mutate in (lambda c: setattr(c.c, "order", 4), lambda c: setattr(c.c, "shrink_a", 1.0),
                   lambda c: setattr(c.c, "n_particles", 0), lambda c: setattr(c.c, "d", 4),
                   lambda c: setattr(c.c, "struct_size", 8), lambda c: setattr(c.c, "m", 0),
                   lambda c: setattr(c.c, "substeps", 65537), lambda c: setattr(c.c, "newton_max_iter", 65),
                   lambda c: setattr(c.c, "lmm", 3), lambda c: setattr(c.c, "resampling", 2)):
        cfg = pf.Config(prob)
        mutate(cfg)
        assert L.pf_filter_bytes(cfg.ptr()) == 0
    # the largest accepted sizes (the packed Newton counters are sized for them)
    cfg = pf.Config(prob)
    cfg.c.substeps, cfg.c.newton_max_iter = 65536, 64
    assert L.pf_filter_bytes(cfg.ptr()) > 0
    for lmm in (pf.PF_LMM_BDF, pf.PF_LMM_AM, pf.PF_LMM_BDF_SDIRK):
        cfg = pf.Config(prob)
        cfg.c.lmm = lmm
        assert L.pf_filter_bytes(cfg.ptr()) > 0


def test_advdiff_configs_on_host():
    L = pf.lib()
    for n in (4, 8, 20, 40):
        prob = inputs.advdiff(1000, 2, n=n)
        cfg = pf.Config(prob, pf.PF_PREC_FP32_PROP)
        b = L.pf_filter_bytes(cfg.ptr())
        # two particle-major fields of d floats per particle, plus the rest
        assert b > 2 * 4 * prob.d * 1024
    prob = inputs.advdiff(1000, 2, n=8)
    for mutate in (lambda c: setattr(c.c, "lmm", pf.PF_LMM_AM), lambda c: setattr(c.c, "p", 3),
                   lambda c: setattr(c.c, "d", 48), lambda c: setattr(c.c, "m", 33),
                   lambda c: setattr(c.c, "n_model_consts", 0)):
        cfg = pf.Config(prob)
        mutate(cfg)
        assert L.pf_filter_bytes(cfg.ptr()) == 0
    # grid sides 3..39 only
    big = inputs.advdiff(100, 2, n=8)
    cfg = pf.Config(big)
    cfg.mc[0] = 40.0
    cfg.c.d = 1600
    assert L.pf_filter_bytes(cfg.ptr()) == 0
    # the kinetic models keep at most 4 observed components
    rb = pf.Config(inputs.robertson(100, 5))
    rb.c.m = 5
    assert L.pf_filter_bytes(rb.ptr()) == 0


def test_product_never_loads_the_oracle():
    # the binding and the HIP sources do not reference the oracle
    for path in ("paper_1411_1702_amd/pf.py", "paper_1411_1702_amd/inputs.py",
                 "paper_1411_1702_amd/csrc/pf_runtime.hip", "paper_1411_1702_amd/csrc/pf_kernels.hip",
                 "paper_1411_1702_amd/csrc/pf_device.hpp"):
        txt = open(os.path.join(ROOT, path)).read()
        for pat in ("from oracle", "import oracle", "liboracle", "pf_oracle"):
            assert pat not in txt, (path, pat)
