"""kde_plugin_bandwidth_noalloc (static device scratch, no allocation) against
kde_plugin_bandwidth_ex on the same context: bitwise-equal results on two
calls in a row, the second with a smaller sample, for FP64 and FP32, with
the result in device memory and in pinned host memory; the FP64 result also
against the oracle; error paths that the host rejects before enqueuing.
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1505_02100_amd import synth

pytestmark = pytest.mark.gpu

FIELDS = ("h", "mean", "sigma", "psi8", "g1", "psi6", "g2", "psi4", "status")


@pytest.fixture(scope="module")
def kp():
    from paper_1505_02100_amd import kdeplugin
    return kdeplugin


def _out(kp, pinned):
    import torch
    nbytes = ctypes.sizeof(kp.kde_result)
    if pinned:
        return torch.zeros(nbytes, dtype=torch.uint8, pin_memory=True)
    return torch.zeros(nbytes, dtype=torch.uint8, device="cuda")


def _noalloc(kp, ctx, xd, pinned):
    import torch
    out = _out(kp, pinned)
    ctx.plugin_bandwidth_noalloc(xd, out)
    torch.cuda.synchronize()
    return kp.batch_results(out, 1)[0]


@pytest.mark.parametrize("prec", ["KDE_FP64_PLAIN", "KDE_FP32_COMP"])
@pytest.mark.parametrize("pinned", [False, True])
def test_noalloc_equals_the_allocating_call(kp, prec, pinned):
    import torch
    with kp.Context(getattr(kp, prec)) as ctx:
        # two calls in a row, the second with a smaller sample (the scratch
        # keeps the first call's contents)
        for n, dist, seed in ((70001, "bimodal", 5), (3001, "t3", 6), (2, "normal", 7)):
            x = synth.draw(dist, n, seed)
            xd = torch.from_numpy(x).cuda()
            got = _noalloc(kp, ctx, xd, pinned)
            want = ctx.plugin_bandwidth(xd)
            for k in FIELDS:
                assert getattr(got, k) == getattr(want, k), (n, k, getattr(got, k), getattr(want, k))
            if prec == "KDE_FP64_PLAIN":
                ref = oracle.plugin(x)
                assert abs(got.h - ref.h) <= 1e-12 * ref.h, (n, got.h, ref.h)


@pytest.mark.parametrize("R", [2, 4])
def test_noalloc_with_other_tile_shapes(kp, R):
    # contexts with 2 or 4 rows per lane: the device-built work list follows
    # the context's geometry like the host-built one
    import torch
    with kp.Context(kp.KDE_FP32_COMP, rows_per_lane=R, target_items=300) as ctx:
        for n, seed in ((50001, 11), (777, 12)):
            xd = torch.from_numpy(synth.draw("bimodal", n, seed)).cuda()
            got = _noalloc(kp, ctx, xd, False)
            want = ctx.plugin_bandwidth(xd)
            for k in FIELDS:
                assert getattr(got, k) == getattr(want, k), (R, n, k)


def test_noalloc_float32_input_and_device_status(kp):
    import torch
    with kp.Context(kp.KDE_FP32_COMP) as ctx:
        x = synth.draw("normal", 4097, 8).astype(np.float32)
        xd = torch.from_numpy(x).cuda()
        got = _noalloc(kp, ctx, xd, False)
        want = ctx.plugin_bandwidth(xd)
        assert (got.h, got.psi6, got.psi4) == (want.h, want.psi6, want.psi4)
        # a NaN sample: the device reports it in the result, h is NaN
        bad = torch.from_numpy(synth.draw("normal", 1000, 9)).cuda()
        bad[500] = float("nan")
        r = _noalloc(kp, ctx, bad, True)
        assert r.status == kp.KDE_ENONFINITE and np.isnan(r.h)
        # the next call after a failed one is clean again
        got2 = _noalloc(kp, ctx, xd, True)
        assert (got2.h, got2.psi6, got2.psi4) == (want.h, want.psi6, want.psi4)


def test_noalloc_rejects_before_enqueuing(kp):
    import torch
    with kp.Context(kp.KDE_FP64_PLAIN) as ctx:
        x = synth.draw("normal", 1000, 10)
        xd = torch.from_numpy(x).cuda()
        out = _out(kp, False)
        res_ptr = ctypes.cast(out.data_ptr(), ctypes.POINTER(kp.kde_result))
        lib = kp._lib
        # host sample pointer
        assert lib.kde_plugin_bandwidth_noalloc(ctx.handle, x.ctypes.data, x.size, kp.KDE_F64, None,
                                                res_ptr) == kp.KDE_EINVAL
        # result in pageable host memory
        host_res = kp.kde_result()
        assert lib.kde_plugin_bandwidth_noalloc(ctx.handle, xd.data_ptr(), x.size, kp.KDE_F64, None,
                                                ctypes.byref(host_res)) == kp.KDE_EINVAL
        # n < 2, bad dtype, null pointers
        assert lib.kde_plugin_bandwidth_noalloc(ctx.handle, xd.data_ptr(), 1, kp.KDE_F64, None,
                                                res_ptr) == kp.KDE_EINVAL
        assert lib.kde_plugin_bandwidth_noalloc(ctx.handle, xd.data_ptr(), x.size, 7, None,
                                                res_ptr) == kp.KDE_EINVAL
        assert lib.kde_plugin_bandwidth_noalloc(None, xd.data_ptr(), x.size, kp.KDE_F64, None,
                                                res_ptr) == kp.KDE_EINVAL
    # a work list over the scratch's item limit
    with kp.Context(kp.KDE_FP64_PLAIN, target_items=300000) as big:
        n = 65536
        assert 2 * big.psi_num_items(n) > kp.KDE_NOALLOC_MAX_ITEMS
        xd = torch.from_numpy(synth.draw("normal", n, 11)).cuda()
        with pytest.raises(kp.KdeError) as e:
            big.plugin_bandwidth_noalloc(xd, _out(kp, False))
        assert e.value.code == kp.KDE_EINVAL and "exceeds" in str(e.value)


@pytest.mark.parametrize("prec", ["KDE_FP64_PLAIN", "KDE_FP32_COMP"])
def test_noalloc_row_major_list_equals_the_banded_one(kp, prec):
    # n = 2^19 + 12345: the allocating call lists the pair items band-wise
    # (chunk-major in bands of 512 row blocks, a ragged last band), the
    # no-allocation call row-block major; the sums are exact, so any item
    # missing from or repeated in either list would change the bits
    import torch
    n = (1 << 19) + 12345
    xd = torch.from_numpy(synth.draw("t3", n, 13)).cuda()
    with kp.Context(getattr(kp, prec)) as ctx:
        got = _noalloc(kp, ctx, xd, False)
        want = ctx.plugin_bandwidth(xd)
    for k in FIELDS:
        assert getattr(got, k) == getattr(want, k), (prec, k)
