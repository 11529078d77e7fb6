"""The host runtime around the kernels, through the C ABI: the context's
device-memory budget and its plan cache (eviction and reuse), contexts used
from several host threads at once (one context per thread, and the literal
calls' shared default context), thread-local error state, and the bound on
in-kernel waits.  Results must be bitwise those of the same calls made one at
a time."""
import ctypes
import math
import threading

import numpy as np
import pytest

import oracle
from paper_1505_02100_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kp():
    from paper_1505_02100_amd import kdeplugin
    return kdeplugin


def test_memory_budget_refuses_and_evicts(kp):
    import torch
    # device samples: the budget then covers the plans alone (work lists,
    # slots, states: about 10, 61 and 181 KB for these sizes)
    xs = [torch.from_numpy(synth.normal(n, 60 + n)).cuda() for n in (3000, 20000, 70000)]
    with kp.Context(kp.KDE_FP32_COMP) as free:
        want = [free.plugin_bandwidth(x) for x in xs]
    # a budget below one plan refuses the call
    with kp.Context(kp.KDE_FP32_COMP, mem_budget=4096) as tiny:
        with pytest.raises(kp.KdeError) as e:
            tiny.plugin_bandwidth(xs[2])
        assert e.value.code == kp.KDE_ENOMEM
    # a budget that holds the largest plan but not two of the larger ones:
    # a new size evicts the least recently used plans, and revisiting a size
    # rebuilds its plan with equal results
    with kp.Context(kp.KDE_FP32_COMP, mem_budget=200 << 10) as small:
        for _ in range(2):
            for x, w in zip(xs, want):
                r = small.plugin_bandwidth(x)
                assert (r.h, r.psi6, r.psi4) == (w.h, w.psi6, w.psi4)


def test_plan_cache_beyond_its_capacity(kp):
    # more distinct sizes than the cache keeps (16): results stay bitwise equal
    sizes = [300 + 97 * k for k in range(24)]
    xs = [synth.bimodal(n, n) for n in sizes]
    with kp.Context(kp.KDE_FP64_PLAIN) as c:
        first = [c.plugin_bandwidth(x).h for x in xs]
        again = [c.plugin_bandwidth(x).h for x in reversed(xs)][::-1]
    assert first == again
    for k in (0, 23):
        assert abs(first[k] - oracle.plugin(xs[k]).h) <= 1e-12 * first[k]


@pytest.mark.parametrize("rep", range(3))
def test_contexts_on_several_threads(kp, rep):
    # one context per thread, all launching at once (ctypes releases the GIL);
    # new contexts build their plans (and graphs) while the others launch
    xs = [synth.draw(synth.DISTS[k % 3], 5000 + 1111 * k + rep, 70 + k) for k in range(6)]
    with kp.Context(kp.KDE_FP32_COMP) as c:
        want = [c.plugin_bandwidth(x).h for x in xs]
    got = {}
    errors = []

    def work(t):
        try:
            with kp.Context(kp.KDE_FP32_COMP) as ctx:
                got[t] = [[ctx.plugin_bandwidth(x).h for x in xs] for _ in range(3)]
        except Exception as exc:  # reported below
            errors.append(exc)

    threads = [threading.Thread(target=work, args=(t,)) for t in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(120)
    assert not errors, errors
    for t in range(4):
        for rep in got[t]:
            assert rep == want


def test_literal_calls_share_the_default_context_safely(kp):
    xs = [synth.normal(2000 + 500 * k, 80 + k) for k in range(4)]
    want = [kp.kde_plugin_bandwidth(x) for x in xs]
    got = {}

    def work(t):
        got[t] = [kp.kde_plugin_bandwidth(xs[(t + k) % 4]) for k in range(8)]

    threads = [threading.Thread(target=work, args=(t,)) for t in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(120)
    for t in range(4):
        assert got[t] == [want[(t + k) % 4] for k in range(8)]


def test_errors_are_per_thread(kp):
    seen = {}
    barrier = threading.Barrier(2)

    def bad():
        kp._lib.kde_psi_num_items(None, 10)       # sets KDE_EINVAL on this thread
        barrier.wait()
        barrier.wait()
        seen["bad"] = kp.kde_last_error()

    def good():
        barrier.wait()
        res = kp.kde_result()
        x = np.ascontiguousarray(synth.normal(100, 1))
        with kp.Context(kp.KDE_FP64_PLAIN) as c:
            code = kp._lib.kde_plugin_bandwidth_ex(c.handle, x.ctypes.data, 100, kp.KDE_MEM_HOST, kp.KDE_F64,
                                                   None, ctypes.byref(res))
        seen["good"] = (code, kp.kde_last_error())
        barrier.wait()

    ta, tb = threading.Thread(target=bad), threading.Thread(target=good)
    ta.start()
    tb.start()
    ta.join(60)
    tb.join(60)
    assert seen["bad"] == kp.KDE_EINVAL
    assert seen["good"] == (kp.KDE_OK, kp.KDE_OK)


def test_wait_limit_fails_the_sample_and_the_launch_ends(kp):
    # a 1 us limit on the in-kernel waits for an earlier stage, forced from the
    # host: at n = 2^18 the first blocks to run out of Step IV items wait tens
    # of microseconds for the stage's last items, so the selection fails with
    # KDE_ETIMEOUT (h NaN) while every block still leaves the kernel; a limit
    # of 10 s, and the default limit, give the normal result bitwise
    import torch
    x = torch.from_numpy(synth.bimodal(1 << 18, 21)).cuda()
    with kp.Context(kp.KDE_FP32_COMP, wait_limit_us=1) as c:
        for _ in range(2):
            r = c.plugin_bandwidth(x, check=False)
            assert r.status == kp.KDE_ETIMEOUT and math.isnan(r.h)
        with pytest.raises(kp.KdeError) as e:
            c.plugin_bandwidth(x)
        assert e.value.code == kp.KDE_ETIMEOUT
        out = c.plugin_bandwidth_batch([x, x[:5000].contiguous()])
        assert out[0].status == kp.KDE_ETIMEOUT
    with kp.Context(kp.KDE_FP32_COMP) as c:
        want = c.plugin_bandwidth(x)
    with kp.Context(kp.KDE_FP32_COMP, wait_limit_us=10_000_000) as c:
        got = c.plugin_bandwidth(x)
    assert want.status == 0 and (got.h, got.psi6, got.psi4) == (want.h, want.psi6, want.psi4)


def test_four_wave_kernel_for_large_samples(kp):
    # with its own tile configuration a context runs launches whose pair stage
    # holds 2^34 pairs or more (n = 2^18 alone, or a batch of smaller samples)
    # on the kernel held to four waves per SIMD, smaller ones on the three-wave
    # kernel; the arithmetic is the same, so results are bitwise those of a
    # context pinned to three blocks per CU (three-wave kernel)
    import torch
    big = torch.from_numpy(synth.bimodal((1 << 18) + 5, 31)).cuda()
    small = torch.from_numpy(synth.bimodal((1 << 17) + 3, 32)).cuda()
    with kp.Context(kp.KDE_FP32_COMP) as a, kp.Context(kp.KDE_FP32_COMP, blocks_per_cu=3) as b:
        for x, waves in ((big, 4), (small, 3)):
            ra = a.plugin_bandwidth(x)
            la = a.last_launch()
            rb = b.plugin_bandwidth(x)
            lb = b.last_launch()
            assert la["waves_per_simd"] == waves and lb["waves_per_simd"] == 3
            cus = torch.cuda.get_device_properties(0).multi_processor_count
            assert 0 < la["blocks"] <= waves * cus and 0 < lb["blocks"] <= 3 * cus
            assert (ra.h, ra.psi6, ra.psi4, ra.g2) == (rb.h, rb.psi6, rb.psi4, rb.g2)
        # the no-allocation entry point stays on the three-wave kernel (no
        # scratch memory), bitwise again
        out = torch.zeros(ctypes.sizeof(kp.kde_result), dtype=torch.uint8, device="cuda")
        a.plugin_bandwidth_noalloc(big, out)
        torch.cuda.synchronize()
        got = kp.batch_results(out, 1)[0]
        assert a.last_launch()["waves_per_simd"] == 3
        want = b.plugin_bandwidth(big)
        assert (got.h, got.psi6, got.psi4) == (want.h, want.psi6, want.psi4)
        # a batch of samples too small alone, but with 2^34 pairs per stage in all
        xs = [torch.from_numpy(synth.bimodal(70000, 40 + k)).cuda() for k in range(8)]
        ga = a.plugin_bandwidth_batch(xs)
        assert a.last_launch()["waves_per_simd"] == 4
        gb = b.plugin_bandwidth_batch(xs)
        assert b.last_launch()["waves_per_simd"] == 3
        assert [(r.h, r.psi6, r.psi4) for r in ga] == [(r.h, r.psi6, r.psi4) for r in gb]
    with kp.Context(kp.KDE_FP64_PLAIN) as c:
        c.plugin_bandwidth(big)
        assert c.last_launch()["waves_per_simd"] == 3


def test_tune_tables_and_the_four_wave_kernel(kp, tmp_path):
    # a tune table whose blocks per CU is 0 leaves the choice to the context
    # (four-wave kernel for large samples); a table that names a count pins
    # the three-wave kernel; results are bitwise equal either way
    import json
    import torch
    x = torch.from_numpy(synth.bimodal((1 << 18) + 5, 33)).cuda()
    res = {}
    for bpc in (0, 3):
        p = tmp_path / f"t{bpc}.json"
        p.write_text(json.dumps({"precision": kp.KDE_FP32_COMP, "rows_per_lane": 1, "blocks_per_cu": bpc,
                                 "targets": [[18, 8192]]}))
        with kp.Context(kp.KDE_FP32_COMP, tune_table=str(p)) as c:
            r = c.plugin_bandwidth(x)
            res[bpc] = (r.h, r.psi6, r.psi4, c.last_launch()["waves_per_simd"])
    assert res[0][3] == 4 and res[3][3] == 3
    assert res[0][:3] == res[3][:3]
