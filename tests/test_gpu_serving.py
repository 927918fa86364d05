"""GPU tests of the continuous-batching server: streams served in a mix give
the same results, bit for bit, as the same filters run alone; admission by
pool memory; latency accounting."""
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


def _streams():
    out = []
    for k in range(8):
        if k % 3 == 2:
            prob = inputs.chain16(1500 + 300 * k, 100, seed=40 + k, model_seed=inputs.CHAIN_INSTANCES[k % 4])
        else:
            prob = inputs.robertson(1000 + 700 * k, 50, seed=40 + k)
        out.append((prob, 1 if k % 4 else 0))
    return out


def _alone(pf, streams, T):
    res = []
    with pf.Context(0, 1 << 30) as ctx:
        for prob, prec in streams:
            f = pf.Filter(ctx, pf.Config(prob, prec))
            for j in range(T):
                f.assimilate(prob.times[j], prob.y[j], prob.sigma[j])
            res.append(f.posterior())
            f.close()
    return res


def _serve(pf, streams, T, pool, rng_seed=0):
    rng = np.random.default_rng(rng_seed)
    with pf.Context(0, pool) as ctx:
        srv = pf.Server(ctx, max_inflight=3)
        sids = [None] * len(streams)
        nxt = [0] * len(streams)
        # stream k arrives after 2k submissions; afterwards submissions come
        # in a random interleaving of the open streams
        pending = []
        order = []
        for k in range(len(streams)):
            order += [("open", k)]
            order += [("obs", None)] * 2
        order += [("obs", None)] * (T * len(streams))
        for kind, k in order:
            if kind == "open":
                sids[k] = srv.open(pf.Config(*streams[k]))
                continue
            live = [i for i in range(len(streams)) if sids[i] is not None and nxt[i] < T]
            if not live:
                continue
            i = int(rng.choice(live))
            prob = streams[i][0]
            tk = srv.submit(sids[i], prob.times[nxt[i]], prob.y[nxt[i]], prob.sigma[nxt[i]])
            pending.append((i, tk))
            nxt[i] += 1
            if nxt[i] == T:
                srv.close(sids[i])      # memory returns to the pool once its steps are done
        for i in range(len(streams)):
            prob = streams[i][0]
            while nxt[i] < T:
                pending.append((i, srv.submit(sids[i], prob.times[nxt[i]], prob.y[nxt[i]], prob.sigma[nxt[i]])))
                nxt[i] += 1
                if nxt[i] == T:
                    srv.close(sids[i])
        srv.drain()
        stat = []
        for i, tk in pending:
            st, lat = srv.poll(sids[i], tk)
            stat.append(st)
            assert st != pf.PF_EBUSY
            assert lat >= 0.0
        posts = [srv.posterior(sids[i], streams[i][0].p) for i in range(len(streams))]
        report = srv.stats()
        closed = report["streams_closed"]
        srv.destroy()
        assert ctx.memory()[0] == 0
    return posts, stat, report, closed


def _same(a, b):
    return np.array_equal(a["mean"], b["mean"]) and np.array_equal(a["cov"], b["cov"]) and a["ess"] == b["ess"]


def test_served_mix_bit_identical_to_alone(pf):
    streams = _streams()
    T = 10
    ref = _alone(pf, streams, T)
    posts, stat, report, closed = _serve(pf, streams, T, pool=1 << 30)
    assert all(s in (pf.PF_OK, pf.PF_EDEGENERATE) for s in stat)
    for i, (a, b) in enumerate(zip(posts, ref)):
        assert _same(a, b), i
        assert a["step"] == b["step"]
    assert report["steps_completed"] + report["steps_skipped"] == T * len(streams)
    assert report["ticks"] < T * len(streams)          # steps of different streams were batched
    assert report["mean_batch"] > 1.0
    assert 0.0 <= report["latency_p50_ms"] <= report["latency_p99_ms"] <= report["latency_max_ms"]
    assert closed == len(streams)


def test_admission_by_memory(pf):
    streams = _streams()[:6]
    T = 6
    ref = _alone(pf, streams, T)
    cfgs = [pf.Config(p, prec) for p, prec in streams]
    need = max(pf.lib().pf_filter_bytes(c.ptr()) for c in cfgs)
    # room for about two ensembles at a time
    posts, stat, report, closed = _serve(pf, streams, T, pool=int(2.2 * need), rng_seed=1)
    for i, (a, b) in enumerate(zip(posts, ref)):
        assert _same(a, b), i
    assert report["streams_admitted"] == len(streams)
    assert report["admit_wait_p99_ms"] > 0.0


def test_posterior_of_a_fresh_stream_returns(pf):
    """pf_server_posterior on a stream with no submissions waits only for its
    admission and returns the prior's summary (the same as pf_create's)."""
    import threading
    prob = inputs.robertson(2000, 5, seed=7)
    with pf.Context(0, 1 << 30) as ctx:
        f = pf.Filter(ctx, pf.Config(prob, pf.PF_PREC_FP64))
        ref = f.posterior()
        f.close()
        srv = pf.Server(ctx)
        sid = srv.open(pf.Config(prob, pf.PF_PREC_FP64))
        box = {}
        th = threading.Thread(target=lambda: box.update(post=srv.posterior(sid, prob.p)), daemon=True)
        th.start()
        th.join(timeout=30)
        assert not th.is_alive(), "pf_server_posterior did not return"
        post = box["post"]
        assert post["step"] == 0
        assert np.array_equal(post["mean"], ref["mean"]) and np.array_equal(post["cov"], ref["cov"])
        # the stream still serves afterwards
        tk = srv.submit(sid, prob.times[0], prob.y[0], prob.sigma[0])
        srv.drain()
        assert srv.poll(sid, tk)[0] == pf.PF_OK
        assert srv.posterior(sid, prob.p)["step"] == 1
        srv.close(sid)
        srv.destroy()
