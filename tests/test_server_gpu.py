"""The continuous-batching server: results identical alone and in the mix,
requests joining while others run, the memory budget, cancellation, a step
that fails (forced from the host) erroring only its requests, smallest-first
admission with aging, and the serving loop's reporting."""
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


@pytest.mark.parametrize("policy,fill", [("fcfs", "share"), ("sjf", "priority")])
def test_alone_equals_mix_bitwise(kp, ctx, policy, fill):
    from paper_1505_02100_amd.server import Server
    xs = _mix(40, 1)
    alone = [ctx.plugin_bandwidth(x) for x in xs]
    with Server(ctx, max_active=16, step_pairs=1 << 28, policy=policy, fill=fill, aging_ms=50) as srv:
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
    assert len(rep["completions"]) == len(trace) == rep["arrived"]
    assert rep["unfinished"] == 0 and rep["failed"] == 0
    assert rep["latency_ms"]["p50"] > 0 and rep["latency_ms"]["p99"] >= rep["latency_ms"]["p50"]
    # drained: the all-arrivals figures are the completed ones, uncensored,
    # and nothing is owed
    assert rep["latency_ms_all_arrivals"]["p99"] == rep["latency_ms"]["p99"]
    assert not rep["latency_ms_all_arrivals"]["p99_is_lower_bound"]
    assert rep["backlog"]["remaining_pair_evals"] == 0
    for c in rep["completions"][:12]:
        x = rep["samples"][c.id].cpu().numpy()
        ref = oracle.plugin(x)
        assert c.status == 0 and abs(c.h - ref.h) / ref.h < 1e-6


def test_serve_trace_backlog_when_overloaded(kp, ctx):
    # about 30 requests of 1e12-4e12 pair evaluations each arrive within 1 s,
    # far more than one GPU serves in that time: the window ends with work
    # owed, which is reported with the time the device would need to drain it
    from paper_1505_02100_amd.server import serve_trace
    trace = synth.serving_trace(rate=30.0, duration=1.0, master=12, n_lo=1e6, n_hi=2e6)
    rep = serve_trace(ctx, trace, duration_s=1.0)
    b = rep["backlog"]
    offered = sum(n * (n - 1) for _, n, _, _ in trace)
    assert rep["unfinished"] > 0
    assert 0 < b["remaining_pair_evals"] <= offered
    assert b["drain_s_at_device_rate"] > 0 and math.isfinite(b["drain_s_at_device_rate"])
    assert rep["device_pair_evals_per_s"] > 0


def test_failed_step_errors_only_its_requests(kp, ctx):
    # a step that cannot run (forced from the host, nothing is launched) fails
    # the requests it lists; requests admitted after it complete, bitwise as alone
    from paper_1505_02100_amd.server import Server
    first = [synth.draw(synth.DISTS[k], 20000 + 1000 * k, 500 + k) for k in range(3)]
    later = _mix(4, 7, 500, 8000)
    with Server(ctx, max_active=3, step_pairs=1 << 26) as srv:
        ids_first = [srv.submit(x) for x in first]
        srv.step()                      # admits the three, launches a step listing them
        srv.fail_next_step(kp.KDE_EDEVICE)
        st = srv.step()                 # the next step lists them again and fails
        assert st.failed_steps == 1
        ids_later = [srv.submit(x) for x in later]
        res = {c.id: c for c in srv.drain()}
    assert sorted(res) == sorted(ids_first + ids_later)
    for rid in ids_first:               # each spans many steps, so each was in the failed one
        assert res[rid].status == kp.KDE_EDEVICE and math.isnan(res[rid].h)
    for rid, x in zip(ids_later, later):
        a = ctx.plugin_bandwidth(x)
        assert res[rid].status == 0 and (res[rid].h, res[rid].psi6, res[rid].psi4) == (a.h, a.psi6, a.psi4)
    with pytest.raises(kp.KdeError):
        kp.kde_server_fail_next_step(None, kp.KDE_EDEVICE)


def test_smallest_first_with_aging(kp, ctx):
    # admission happens only inside a step, so the order is decided by the
    # keys at that moment: a large request that has waited 150 ms is admitted
    # before newer small ones when every ms of waiting halves its key's pair
    # count; without aging the small ones go first
    import time
    from paper_1505_02100_amd.server import Server
    order = {}
    for aging in (0, 1):
        with Server(ctx, max_active=1, policy="sjf", aging_ms=aging) as srv:
            a = srv.submit(synth.normal(2000, 1))
            srv.step()                          # a takes the only slot
            big = srv.submit(synth.normal(30000, 2))
            time.sleep(0.15)
            small = [srv.submit(synth.normal(600 + 10 * k, 3 + k)) for k in range(3)]
            res = {c.id: c for c in srv.drain()}
        assert all(c.status == 0 for c in res.values())
        order[aging] = sorted(res, key=lambda r: res[r].t_admit_ms)
        assert order[aging][0] == a
    assert order[0][-1] == big                  # pure smallest first: the large one last
    assert order[1][1] == big                   # with aging: the large one next


def test_priority_fill_finishes_in_key_order(kp, ctx):
    # FCFS with the priority fill: the oldest request takes the step budget
    # first, so equal-sized requests finish in submission order; with the
    # round-robin fill they share the device and finish together at the end
    from paper_1505_02100_amd.server import Server
    xs = [synth.draw(synth.DISTS[k % 3], 20000, 700 + k) for k in range(5)]
    done = {}
    for fill in ("priority", "share"):
        with Server(ctx, max_active=8, step_pairs=1 << 27, policy="fcfs", fill=fill) as srv:
            ids = [srv.submit(x) for x in xs]
            res = {c.id: c for c in srv.drain()}
        assert all(res[i].h == ctx.plugin_bandwidth(x).h for i, x in zip(ids, xs))
        done[fill] = [res[i].t_done_ms for i in ids]
    assert done["priority"] == sorted(done["priority"])
    assert done["priority"][0] < done["priority"][-1]
    span = lambda t: max(t) - min(t)
    assert span(done["share"]) < span(done["priority"])


def test_device_sample_written_on_another_stream(kp, ctx):
    # the sample is still being written on a side stream (behind a ~20 ms spin)
    # when it is submitted; the server's stream waits for that stream's work
    import torch
    from paper_1505_02100_amd.server import Server
    x = synth.draw("t3", 30000, 77)
    src = torch.from_numpy(x).cuda()
    dst = torch.full_like(src, float("nan"))
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    with Server(ctx, max_active=4, step_pairs=1 << 26) as srv:
        with torch.cuda.stream(side):
            torch.cuda._sleep(50_000_000)
            dst.copy_(src)
            rid = srv.submit(dst)            # producer: the side stream
        res = {c.id: c for c in srv.drain()}
    torch.cuda.synchronize()
    alone = ctx.plugin_bandwidth(src)
    assert res[rid].status == 0 and (res[rid].h, res[rid].psi6, res[rid].psi4) == (alone.h, alone.psi6, alone.psi4)
