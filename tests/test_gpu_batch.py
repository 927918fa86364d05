"""GPU tests of the submission paths: graph replay vs eager launch, batched
vs alone (bit-identical), tickets, and the error paths of the C ABI."""
import os

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


def _ctx(pf, graphs, pool=1 << 30):
    old = os.environ.get("PF_GRAPHS")
    os.environ["PF_GRAPHS"] = "1" if graphs else "0"
    try:
        return pf.Context(0, pool)
    finally:
        if old is None:
            del os.environ["PF_GRAPHS"]
        else:
            os.environ["PF_GRAPHS"] = old


def _ensemble(pf, f):
    x = torch.zeros((f.d, f.N), dtype=torch.float64, device="cuda")
    th = torch.zeros((f.p, f.N), dtype=torch.float64, device="cuda")
    lw = torch.zeros(f.N, dtype=torch.float64, device="cuda")
    pf.check(pf.lib().pf_test_get_ensemble(f.h, x.data_ptr(), th.data_ptr(), lw.data_ptr()), "get")
    return x.cpu().numpy(), th.cpu().numpy(), lw.cpu().numpy()


def test_graph_replay_matches_eager(pf):
    prob = inputs.robertson(4096, 20, seed=3)
    eager = _ctx(pf, False)
    graph = _ctx(pf, True)
    fe = pf.Filter(eager, pf.Config(prob, pf.PF_PREC_FP32_PROP))
    fg = pf.Filter(graph, pf.Config(prob, pf.PF_PREC_FP32_PROP))
    for j in range(12):
        assert fe.assimilate(prob.times[j], prob.y[j], prob.sigma[j]) == pf.PF_OK
        assert fg.assimilate(prob.times[j], prob.y[j], prob.sigma[j]) == pf.PF_OK
        a, b = fe.posterior(), fg.posterior()
        # eager work and a synchronisation between replays: read the ensembles
        xa, ta, la = _ensemble(pf, fe)
        xb, tb, lb = _ensemble(pf, fg)
        assert np.array_equal(a["mean"], b["mean"]) and np.array_equal(a["cov"], b["cov"]), j
        assert a["ess"] == b["ess"] and a["step"] == b["step"] == j + 1
        assert np.array_equal(xa, xb) and np.array_equal(ta, tb) and np.array_equal(la, lb), j
    # async replays back to back, then the same comparison
    tk_e = [fe.assimilate_async(prob.times[j], prob.y[j], prob.sigma[j]) for j in range(12, 20)]
    tk_g = [fg.assimilate_async(prob.times[j], prob.y[j], prob.sigma[j]) for j in range(12, 20)]
    assert all(fe.wait(t) == pf.PF_OK for t in tk_e) and all(fg.wait(t) == pf.PF_OK for t in tk_g)
    a, b = fe.posterior(), fg.posterior()
    assert np.array_equal(a["mean"], b["mean"]) and np.array_equal(a["cov"], b["cov"])
    fe.close()
    fg.close()
    eager.close()
    graph.close()


def _mixed_problems():
    return [
        (inputs.robertson(3000, 20, seed=11), 1),
        (inputs.robertson(1000, 20, seed=12), 0),
        (inputs.chain16(2000, 20, seed=13, model_seed=0), 1),
        (inputs.robertson(700, 20, seed=14, order=3), 1),
    ]


@pytest.mark.parametrize("graphs", [False, True])
def test_batched_bit_identical_to_alone(pf, graphs):
    probs = _mixed_problems()
    steps = 6
    alone = []
    with _ctx(pf, graphs) as ctx:
        for prob, prec in probs:
            f = pf.Filter(ctx, pf.Config(prob, prec))
            for j in range(steps):
                assert f.assimilate(prob.times[j], prob.y[j], prob.sigma[j]) == pf.PF_OK
            alone.append((f.posterior(), _ensemble(pf, f)))
            f.close()
    with _ctx(pf, graphs) as ctx:
        fs = [pf.Filter(ctx, pf.Config(prob, prec)) for prob, prec in probs]
        for j in range(steps):
            tk = ctx.assimilate_batch(fs, [p.times[j] for p, _ in probs], [p.y[j] for p, _ in probs],
                                      [p.sigma[j] for p, _ in probs])
            for f, t in zip(fs, tk):
                assert f.wait(t) == pf.PF_OK
        for i, f in enumerate(fs):
            post, ens = f.posterior(), _ensemble(pf, f)
            ref_post, ref_ens = alone[i]
            assert np.array_equal(post["mean"], ref_post["mean"]), i
            assert np.array_equal(post["cov"], ref_post["cov"]), i
            assert post["ess"] == ref_post["ess"]
            for u, v in zip(ens, ref_ens):
                assert np.array_equal(u, v), i
            f.close()


def test_autotuned_launch_shapes(pf):
    """The launch-shape tuner tries every candidate grid on the first
    submissions of a batch, keeps one per launch group, and changes no
    result: a tuned context and one with the tuner off give the same
    ensembles bit for bit, and each tuned grid is a candidate."""
    probs = [(inputs.robertson(65536 - 300 * i, 40, seed=20 + i), 1) for i in range(6)]
    probs.append((inputs.chain16(16384, 40, seed=30, model_seed=0), 1))
    tiles = sum((p.n_particles + 255) // 256 for p, _ in probs)
    cu = torch.cuda.get_device_properties(0).multi_processor_count
    steps = 24
    runs = []
    for tuned in (True, False):
        with _ctx(pf, True) as ctx:
            ctx.autotune(tuned)
            fs = [pf.Filter(ctx, pf.Config(prob, prec)) for prob, prec in probs]
            for j in range(steps):
                tk = ctx.assimilate_batch(fs, [p.times[j] for p, _ in probs], [p.y[j] for p, _ in probs],
                                          [p.sigma[j] for p, _ in probs])
                for f, t in zip(fs, tk):
                    assert f.wait(t) == pf.PF_OK
            for group in (0, 1, 2):
                grid, ok = ctx.launch_grid(group, tiles)
                assert ok == tuned, group
                if tuned:
                    assert grid in {min(tiles, c) for c in (tiles, 16 * cu, 8 * cu, 4 * cu, 2 * cu)}, grid
                else:
                    assert grid == min(tiles, 8 * cu)
            assert pf.lib().pf_context_launch_grid(ctx.h, 3, tiles, None, None) == pf.PF_EINVAL
            assert pf.lib().pf_context_launch_grid(ctx.h, 0, 0, None, None) == pf.PF_EINVAL
            runs.append([(f.posterior(), _ensemble(pf, f)) for f in fs])
            for f in fs:
                f.close()
    for i, ((pa, ea), (pb, eb)) in enumerate(zip(*runs)):
        assert np.array_equal(pa["mean"], pb["mean"]) and np.array_equal(pa["cov"], pb["cov"]), i
        for u, v in zip(ea, eb):
            assert np.array_equal(u, v), i


def test_batch_with_uneven_schedules(pf):
    # filters join and leave the batch: each one's trajectory still matches
    # running it alone
    probs = _mixed_problems()[:3]
    with _ctx(pf, True) as ctx:
        ref = []
        for prob, prec in probs:
            f = pf.Filter(ctx, pf.Config(prob, prec))
            for j in range(5):
                f.assimilate(prob.times[j], prob.y[j], prob.sigma[j])
            ref.append(f.posterior()["mean"])
            f.close()
        fs = [pf.Filter(ctx, pf.Config(prob, prec)) for prob, prec in probs]
        done = [0, 0, 0]
        schedule = [[0, 1, 2], [0, 2], [1], [0, 1, 2], [2, 0], [1, 0, 2], [1, 2], [1]]
        for members in schedule:
            members = [m for m in members if done[m] < 5]
            if not members:
                continue
            tk = ctx.assimilate_batch([fs[m] for m in members], [probs[m][0].times[done[m]] for m in members],
                                      [probs[m][0].y[done[m]] for m in members],
                                      [probs[m][0].sigma[done[m]] for m in members])
            for m, t in zip(members, tk):
                assert fs[m].wait(t) == pf.PF_OK
                done[m] += 1
        assert done == [5, 5, 5]
        for i, f in enumerate(fs):
            assert np.array_equal(f.posterior()["mean"], ref[i])
            f.close()


def test_error_paths(pf):
    prob = inputs.robertson(2000, 10, seed=5)
    with _ctx(pf, True) as ctx:
        f = pf.Filter(ctx, pf.Config(prob, pf.PF_PREC_FP32_PROP))
        assert f.assimilate(prob.times[0], prob.y[0], prob.sigma[0]) == pf.PF_OK
        snap = _ensemble(pf, f)
        post = f.posterior()
        # time not increasing
        st = pf.lib().pf_assimilate(f.h, float(prob.times[0]), pf._dp(np.array(prob.y[0])),
                                    pf._dp(np.array(prob.sigma[0])))
        assert st == pf.PF_EORDER
        # NaN observation, zero sigma
        st = pf.lib().pf_assimilate(f.h, float(prob.times[1]), pf._dp(np.array([np.nan])), pf._dp(np.array([1.0])))
        assert st == pf.PF_EINVAL
        st = pf.lib().pf_assimilate(f.h, float(prob.times[1]), pf._dp(np.array([1e-5])), pf._dp(np.array([0.0])))
        assert st == pf.PF_EINVAL
        # an impossible observation: every weight underflows -> skipped, unchanged
        st = f.assimilate(prob.times[1], [1e200], [1e-200])
        assert st == pf.PF_EDEGENERATE
        after = _ensemble(pf, f)
        for u, v in zip(snap, after):
            assert np.array_equal(u, v)
        assert f.posterior()["step"] == post["step"] == 1
        # and the filter carries on with the next real observation
        assert f.assimilate(prob.times[2], prob.y[2], prob.sigma[2]) == pf.PF_OK
        assert f.posterior()["step"] == 2
        # too many steps in flight
        tk = [f.assimilate_async(prob.times[3] + 1e-9 * i, prob.y[3], prob.sigma[3]) for i in range(64)]
        with pytest.raises(pf.PfError) as e:
            f.assimilate_async(prob.times[3] + 1.0, prob.y[3], prob.sigma[3])
        assert e.value.status == pf.PF_EBUSY
        for t in tk:
            assert f.wait(t) in (pf.PF_OK, pf.PF_EDEGENERATE)
        assert f.wait(tk[0]) == pf.PF_EINVAL   # already waited on
        f.close()
    # pool exhaustion
    with _ctx(pf, True, pool=4 << 20) as ctx:
        with pytest.raises(pf.PfError) as e:
            pf.Filter(ctx, pf.Config(inputs.robertson(1 << 17, 5), pf.PF_PREC_FP64))
        assert e.value.status == pf.PF_ENOMEM
        small = pf.Filter(ctx, pf.Config(inputs.robertson(1000, 5), pf.PF_PREC_FP64))
        used, cap = ctx.memory()
        assert 0 < used <= cap
        small.close()
        assert ctx.memory()[0] == 0


def test_pool_full_now_is_admit_not_enomem(pf):
    # a pool that holds one filter: the second is refused with PF_EADMIT
    # (retry later) and admitted once the first is destroyed
    cfg = pf.Config(inputs.robertson(5000, 4, seed=1))
    need = pf.lib().pf_filter_bytes(cfg.ptr())
    with _ctx(pf, True, pool=need + 4096) as ctx:
        f1 = pf.Filter(ctx, cfg)
        with pytest.raises(pf.PfError) as e:
            pf.Filter(ctx, pf.Config(inputs.robertson(5000, 4, seed=2)))
        assert e.value.status == pf.PF_EADMIT
        f1.close()
        f2 = pf.Filter(ctx, pf.Config(inputs.robertson(5000, 4, seed=2)))
        f2.close()


def test_caller_allocator_provides_the_pool(pf):
    # the pool from the caller's allocator (device memory from torch here):
    # one alloc at creation, one free at destruction, and the filter's
    # results are those of a hipMalloc'ed pool, bit for bit
    prob = inputs.robertson(3000, 4, seed=3)
    held, calls = {}, []

    def alloc(n, stream):
        t = torch.empty(n, dtype=torch.uint8, device="cuda")
        held[t.data_ptr()] = t
        calls.append(("alloc", n))
        return t.data_ptr()

    def free(p, stream):
        calls.append(("free", p))
        held.pop(p)

    posts = []
    for a in (None, (alloc, free)):
        with pf.Context(0, 64 << 20, allocator=a) as ctx:
            f = pf.Filter(ctx, pf.Config(prob))
            for j in range(prob.T):
                assert f.assimilate(prob.times[j], prob.y[j], prob.sigma[j]) == pf.PF_OK
            posts.append(f.posterior())
            f.close()
            if a is not None:
                assert calls == [("alloc", 64 << 20)]
    assert [c[0] for c in calls] == ["alloc", "free"] and not held
    for k in ("mean", "cov", "state_mean"):
        assert np.array_equal(posts[0][k], posts[1][k])
