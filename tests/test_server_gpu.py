"""The continuous-batching server: results identical alone and in the mix,
requests joining while others run, the memory budget, cancellation."""
import math

import numpy as np
import pytest

import oracle
from paper_1505_02100_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kp():
    from paper_1505_02100_amd import kdeplugin
    return kdeplugin


@pytest.fixture(scope="module")
def ctx(kp):
    c = kp.Context(kp.KDE_FP32_COMP)
    yield c
    c.close()


def _mix(count, seed, lo=200, hi=40000):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        out.append(synth.draw(synth.DISTS[k % 3], n, 1000 * seed + k))
    return out


def test_alone_equals_mix_bitwise(kp, ctx):
    from paper_1505_02100_amd.server import Server
    xs = _mix(40, 1)
    alone = [ctx.plugin_bandwidth(x) for x in xs]
    with Server(ctx, max_active=16, step_pairs=1 << 28) as srv:
        ids = [srv.submit(x) for x in xs]
        res = {c.id: c for c in srv.drain()}
    assert sorted(res) == sorted(ids)
    for rid, x, a in zip(ids, xs, alone):
        c = res[rid]
        assert c.status == 0
        assert (c.h, c.psi6, c.psi4) == (a.h, a.psi6, a.psi4), (x.size,)
    for rid, x in zip(ids[:10], xs[:10]):
        ref = oracle.plugin(x)
        assert abs(res[rid].h - ref.h) / ref.h < 1e-6


def test_requests_join_while_others_run(kp, ctx):
    from paper_1505_02100_amd.server import Server
    big = synth.bimodal(150000, 5)
    small = _mix(12, 2, 300, 5000)
    with Server(ctx, max_active=8, step_pairs=1 << 27) as srv:
        rid_big = srv.submit(big)
        srv.step()
        srv.step()
        ids = []
        for x in small:                      # arrive while the big one is on the device
            ids.append(srv.submit(x))
            srv.step()
        got = {c.id: c for c in srv.drain()}
    # small requests admitted later finish before the big one
    assert all(got[i].t_done_ms <= got[rid_big].t_done_ms for i in ids[:4])
    assert got[rid_big].h == ctx.plugin_bandwidth(big).h
    for rid, x in zip(ids, small):
        assert got[rid].h == ctx.plugin_bandwidth(x).h


def test_memory_budget_admission_and_rejection(kp, ctx):
    from paper_1505_02100_amd.server import Server
    xs = [synth.normal(100000, k) for k in range(4)]     # 0.8 MB samples
    with Server(ctx, mem_budget=2 << 20, max_active=8) as srv:  # room for two at a time
        with pytest.raises(kp.KdeError) as e:
            srv.submit(synth.normal(400000, 9))          # 3.2 MB can never fit
        assert e.value.code == kp.KDE_ENOMEM
        ids = [srv.submit(x) for x in xs]
        st = srv.step()
        assert st.active <= 2 and st.active + st.queued == 4
        res = {c.id: c for c in srv.drain()}
    for rid, x in zip(ids, xs):
        assert res[rid].h == ctx.plugin_bandwidth(x).h


def test_cancel_queued_and_device_samples(kp, ctx):
    import torch
    from paper_1505_02100_amd.server import Server
    xs = [synth.t3(5000, k) if hasattr(synth, "t3") else synth.student_t3(5000, k) for k in range(3)]
    with Server(ctx, max_active=1) as srv:
        ids = [srv.submit(torch.from_numpy(x).cuda()) for x in xs]
        srv.cancel(ids[2])                   # still queued behind the first
        res = {c.id: c for c in srv.drain()}
        with pytest.raises(kp.KdeError):
            srv.cancel(ids[0])               # already finished
    assert sorted(res) == ids[:2]
    for rid, x in zip(ids[:2], xs[:2]):
        assert res[rid].h == ctx.plugin_bandwidth(x).h


def test_serve_trace_small(kp, ctx):
    from paper_1505_02100_amd.server import serve_trace
    trace = synth.serving_trace(rate=40.0, duration=2.0, master=11, n_lo=300, n_hi=20000)
    rep = serve_trace(ctx, trace, duration_s=2.0, drain=True, keep_samples=True)
    assert len(rep["completions"]) == len(trace)
    assert rep["latency_ms"]["p50"] > 0 and rep["latency_ms"]["p99"] >= rep["latency_ms"]["p50"]
    for c in rep["completions"][:12]:
        x = rep["samples"][c.id].cpu().numpy()
        ref = oracle.plugin(x)
        assert c.status == 0 and abs(c.h - ref.h) / ref.h < 1e-6
