"""The batched and the served submission paths against the oracle, in FP64
(Algorithm 1 for many filters at once).

Several filters with different particle counts, integrators and resampling
draws run through one pf_assimilate_batch per observation step (step graphs
on), and through the continuous-batching server; every filter's posterior is
compared with an oracle filter of the same seed.  As in the single-filter
whole runs, both sides draw the same random numbers and resample on the same
integer weights, so the runs follow one trajectory and the posterior
summaries agree to rounding at every step."""
import os

import numpy as np
import pytest

from paper_1411_1702_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-9


@pytest.fixture(scope="module")
def pf():
    from paper_1411_1702_amd import pf as _pf
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _pf.lib()
    return _pf


def _filters():
    """(problem, observations assimilated): BDF2, BDF3 with the SDIRK
    start-up, AM1, multinomial draw, and the chain with BDF3."""
    bdf2 = inputs.robertson(1000, 50, seed=0)
    sd3 = inputs.robertson(1500, 50, seed=1)
    sd3.lmm, sd3.order = 2, 3
    am1 = inputs.robertson(700, 50, seed=2)
    am1.lmm, am1.order = 1, 1
    mult = inputs.robertson(1200, 50, seed=3)
    mult.resampling = 1
    chain = inputs.chain16(1024, 100, seed=4, model_seed=inputs.CHAIN_INSTANCES[0])
    return [(bdf2, 50), (sd3, 50), (am1, 50), (mult, 50), (chain, 24)]


def _oracle_runs(oracle, fs):
    out = []
    for prob, T in fs:
        m, s, e = oracle.Filter(prob).run(T)
        out.append((m, s, e))
    return out


def _err(gm, gs, om, osd):
    """Mean error relative to max(|mean|, sd); sd error relative to the sd."""
    scale = np.maximum(np.abs(om), osd)
    return (np.abs(gm - om) / scale).max(), (np.abs(gs - osd) / osd).max()


def _ctx(pf, pool=1 << 30):
    old = os.environ.get("PF_GRAPHS")
    os.environ["PF_GRAPHS"] = "1"
    try:
        return pf.Context(0, pool)
    finally:
        if old is None:
            del os.environ["PF_GRAPHS"]
        else:
            os.environ["PF_GRAPHS"] = old


def test_batched_fp64_follows_the_oracle(pf, oracle):
    fs = _filters()
    ref = _oracle_runs(oracle, fs)
    Tmax = max(T for _, T in fs)
    with _ctx(pf) as ctx:
        hs = [pf.Filter(ctx, pf.Config(prob, pf.PF_PREC_FP64)) for prob, _ in fs]
        worst = [0.0, 0.0]
        for j in range(Tmax):
            members = [i for i, (_, T) in enumerate(fs) if j < T]
            tk = ctx.assimilate_batch([hs[i] for i in members], [fs[i][0].times[j] for i in members],
                                      [fs[i][0].y[j] for i in members], [fs[i][0].sigma[j] for i in members])
            for i, t in zip(members, tk):
                st = hs[i].wait(t)
                assert st in (pf.PF_OK, pf.PF_EDEGENERATE), (i, j, st)
            for i in members:
                post = hs[i].posterior()
                om, osd, oess = ref[i][0][j], ref[i][1][j], ref[i][2][j]
                gs = np.sqrt(np.diag(post["cov"]))
                em, es = _err(post["mean"], gs, om, osd)
                worst = [max(worst[0], em), max(worst[1], es)]
                assert em < TOL and es < TOL, (fs[i][0].name, j, em, es)
                if np.isfinite(oess):
                    assert post["ess"] == pytest.approx(oess, rel=TOL), (i, j)
                # a degenerate step is skipped on both sides
                assert post["step"] == np.isfinite(ref[i][2][: j + 1]).sum(), (i, j, post["step"])
        print("batched FP64 vs oracle: worst mean err %.2e, sd err %.2e" % tuple(worst))
        for h in hs:
            h.close()


def test_served_fp64_follows_the_oracle(pf, oracle):
    """The same filters as served streams: opened one after another,
    observations submitted in a random interleaving, the posterior of every
    stream read at its midpoint (while the others keep running) and at the end."""
    fs = _filters()
    ref = _oracle_runs(oracle, fs)
    rng = np.random.default_rng(5)
    with pf.Context(0, 1 << 30) as ctx:
        srv = pf.Server(ctx, max_inflight=3)
        sids = [srv.open(pf.Config(prob, pf.PF_PREC_FP64)) for prob, _ in fs]
        nxt = [0] * len(fs)
        checked = []
        while any(nxt[i] < fs[i][1] for i in range(len(fs))):
            live = [i for i in range(len(fs)) if nxt[i] < fs[i][1]]
            i = int(rng.choice(live))
            prob, T = fs[i]
            j = nxt[i]
            srv.submit(sids[i], prob.times[j], prob.y[j], prob.sigma[j])
            nxt[i] += 1
            if nxt[i] in (T // 2, T):
                post = srv.posterior(sids[i], prob.p)
                checked.append((i, nxt[i] - 1, post))
                if nxt[i] == T:
                    srv.close(sids[i])
        srv.drain()
        report = srv.stats()
        srv.destroy()
        assert ctx.memory()[0] == 0
    assert report["mean_batch"] > 1.0
    assert len(checked) == 2 * len(fs)
    for i, j, post in checked:
        om, osd = ref[i][0][j], ref[i][1][j]
        em, es = _err(post["mean"], np.sqrt(np.diag(post["cov"])), om, osd)
        print("served", fs[i][0].name, "step", j + 1, "mean err %.2e sd err %.2e" % (em, es))
        assert em < TOL and es < TOL, (fs[i][0].name, j, em, es)
