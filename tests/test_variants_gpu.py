"""Parity of every selectable configuration with the FP64 CPU oracle.

* rows_per_lane R = 2 and 4 (tile heights 512 and 1024 rows) for every
  precision: ragged sizes, a many-tile size and the full bimodal n = 65536
  sample.  R > 1 runs the generic pair loops (R = 1 takes the asm loops,
  tested in test_parity_gpu.py).
* the clamped FP32 variant, taken when the largest scaled deviation
  max|x - mean| / g exceeds 1e6: its pairs far apart must give exactly 0
  (without the clamp their Hermite factor would overflow FP32 and the sum
  would turn NaN).
* Psi_r(g) of equations (6)-(7) on samples without spread: n = 1 gives
  K^(r)(0) / g^(r+1) exactly (no pair, only the analytic diagonal), and ties
  are ordinary K^(r)(0) terms.
* asynchronous batches on two streams, results in device and pinned host
  memory, bitwise equal to the synchronous call.

Tolerances are those of test_parity_gpu.py: FP64 1e-12 relative, FP32 h 1e-6
and Psi 2e-5; the Q32.32 emulation within the bound its own arithmetic gives
(test_parity_gpu._q32_psi_bound).
"""
import math

import numpy as np
import pytest

import oracle
from paper_1505_02100_amd import synth

from test_parity_gpu import TOL32_H, TOL32_PSI, TOL64, _check, _q32_psi_bound, _rel

pytestmark = pytest.mark.gpu

SQ2PI = math.sqrt(2.0 * math.pi)
K0 = {4: 3.0 / SQ2PI, 6: -15.0 / SQ2PI}


@pytest.fixture(scope="module")
def kp():
    from paper_1505_02100_amd import kdeplugin
    return kdeplugin


PRECS = ("FP64_PLAIN", "FP32_COMP", "FP32_COMP_EXACT", "FP32_POLYEXP", "Q32_32")


@pytest.fixture(scope="module")
def ctxs(kp):
    made = {}
    for R in (1, 2, 4):
        for name in PRECS:
            made[(name, R)] = kp.Context(getattr(kp, "KDE_" + name), rows_per_lane=R)
    yield made
    for c in made.values():
        c.close()


def _tol(name):
    return (TOL64, TOL64) if name == "FP64_PLAIN" else (TOL32_H, TOL32_PSI)


@pytest.mark.parametrize("R", [2, 4])
@pytest.mark.parametrize("n", [2, 65, 513, 1025, 4097])
@pytest.mark.parametrize("name", PRECS)
def test_rows_per_lane_ragged(ctxs, name, R, n):
    ctx = ctxs[(name, R)]
    assert ctx.config()["rows_per_lane"] == R
    x = synth.draw(["normal", "bimodal", "t3"][n % 3], n, 300 + n)
    ref = oracle.plugin(x)
    res = ctx.plugin_bandwidth(x)
    if name == "Q32_32":
        assert res.status == 0
        b6 = _q32_psi_bound(x, 6, ref.g1) + 1e-12 * abs(ref.psi6)
        assert abs(res.psi6 - ref.psi6) <= b6
        rel4 = (_q32_psi_bound(x, 4, ref.g2) + 1e-12 * ref.psi4) / ref.psi4 + 10 * _rel(res.g2, ref.g2)
        assert _rel(res.psi4, ref.psi4) <= rel4
        assert _rel(res.h, ref.h) <= 0.2 * rel4 + 1e-12
        # the same integer sums as the R = 1 tiling: bitwise equal
        r1 = ctxs[(name, 1)].plugin_bandwidth(x)
        assert (r1.h, r1.psi6, r1.psi4) == (res.h, res.psi6, res.psi4)
    else:
        _check(res, ref, *_tol(name))
    # fixed-g Psi through the same loops
    for r, g in ((4, 0.4), (6, 0.05)):
        want = oracle.psi(x, r, g)
        got = ctx.psi(x, r, g)
        if name == "Q32_32":
            assert abs(got - want) <= _q32_psi_bound(x, r, g) + 1e-12 * abs(want)
        else:
            assert _rel(got, want) < _tol(name)[1], (r, g, got, want)


@pytest.mark.parametrize("R", [2, 4])
@pytest.mark.parametrize("name", PRECS[:4])
def test_rows_per_lane_many_tiles(ctxs, name, R):
    x = synth.bimodal(33333, 8)
    _check(ctxs[(name, R)].plugin_bandwidth(x), oracle.plugin(x), *_tol(name))


@pytest.mark.parametrize("R", [2, 4])
def test_rows_per_lane_full_bimodal_65536(ctxs, R):
    import torch
    x = synth.workload_single_bimodal(65536, 1)
    ref = oracle.plugin(x)
    xd = torch.from_numpy(x).cuda()
    for name in PRECS[:4]:
        res = ctxs[(name, R)].plugin_bandwidth(xd)
        tol_h, tol_psi = _tol(name)
        _check(res, ref, tol_h, tol_psi if name == "FP64_PLAIN" else 1e-5)


def _outlier_sample(n, seed):
    # N(0, 1) bulk with two outliers at +-1e10: the mean stays near 0 and the
    # bulk keeps its FP32 resolution, while max|x - mean| / g is about 1e10 / g
    x = synth.normal(n, seed)
    x[n // 3] = 1.0e10
    x[(2 * n) // 3] = -1.0e10
    return x


@pytest.mark.parametrize("R", [1, 2, 4])
@pytest.mark.parametrize("name", PRECS[:4])
def test_clamped_variant_far_outliers(ctxs, name, R):
    x = _outlier_sample(4099, 5)
    ctx = ctxs[(name, R)]
    for r, g in ((4, 0.5), (6, 0.3)):
        want = oracle.psi(x, r, g)
        got = ctx.psi(x, r, g)
        assert math.isfinite(got)
        assert _rel(got, want) < _tol(name)[1], (name, R, r, got, want)
    # the full selection on the same sample: g1 is large there, so this runs
    # the unclamped loops on extreme data
    _check(ctx.plugin_bandwidth(x), oracle.plugin(x), *_tol(name))


@pytest.mark.parametrize("r", [4, 6])
@pytest.mark.parametrize("name", PRECS)
def test_psi_without_spread(ctxs, name, r):
    ctx = ctxs[(name, 1)]
    g = 0.7
    # n = 1: only the diagonal, K(0) / g^(r+1), exactly as the host-side FP64
    # formula (2 * 0 + 1 * K(0)) / (1 * g^(r+1)) rounds it
    one = ctx.psi(np.array([2.5]), r, g)
    assert _rel(one, oracle.psi([2.5], r, g)) < 1e-15
    assert _rel(one, K0[r] / g ** (r + 1)) < 1e-15
    tol = 1e-12 if name == "FP64_PLAIN" else 1e-6
    for x in (np.array([-1.25, -1.25]), np.full(300, 4.0), np.full(1000, -3.0e4)):
        want = oracle.psi(x, r, g)
        # every pair is a tie: Psi = K(0) / g^(r+1) whatever n is
        assert _rel(want, K0[r] / g ** (r + 1)) < 1e-13
        assert _rel(ctx.psi(x, r, g), want) < tol, (name, x.size)
    # ties mixed with distinct values
    x = np.concatenate([np.full(40, 0.5), synth.normal(200, 9), np.full(7, -1.0)])
    want = oracle.psi(x, r, g)
    got = ctx.psi(x, r, g)
    if name == "Q32_32":
        assert abs(got - want) <= _q32_psi_bound(x, r, g) + 1e-12 * abs(want)
    else:
        assert _rel(got, want) < (TOL64 if name == "FP64_PLAIN" else TOL32_PSI)


def test_psi_without_spread_literal_and_range(kp, ctxs):
    x = np.full(513, 1.5)
    for r in (4, 6):
        assert _rel(kp.kde_psi(x, r, 0.25), oracle.psi(x, r, 0.25)) < 1e-12
        assert _rel(kp.kde_psi(np.array([1.0]), r, 0.25), oracle.psi([1.0], r, 0.25)) < 1e-15
    ctx = ctxs[("FP32_COMP", 1)]
    m = ctx.psi_num_items(513)
    tot = sum(ctx.psi_range(x, 4, 0.25, k, k + 1) for k in range(m))
    assert _rel(tot, 513 * 512 / 2 * K0[4]) < 1e-7
    # the full selection still rejects a sample without spread (Step II)
    r = ctx.plugin_bandwidth(x, check=False)
    assert r.status == kp.KDE_EDEGENERATE and math.isnan(r.h)


def _records(kp, out, m):
    return kp.batch_results(out, m)


def test_async_batch_two_streams(kp, ctxs):
    import torch
    ctx = ctxs[("FP32_COMP", 1)]
    xa, _ = synth.workload_batch(count=40, master=71, n_lo=256, n_hi=20000)
    xb, _ = synth.workload_batch(count=17, master=72, n_lo=300, n_hi=9000)
    da = [torch.from_numpy(x).cuda() for x in xa]
    db = [torch.from_numpy(x).cuda() for x in xb]
    ref_a = ctx.plugin_bandwidth_batch(da)
    ref_b = ctx.plugin_bandwidth_batch(db)
    rec = 72  # sizeof(kde_result)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    for rep in range(3):
        o1 = torch.empty(len(da) * rec, dtype=torch.uint8, device="cuda")
        o2 = torch.empty(len(db) * rec, dtype=torch.uint8, pin_memory=True)
        o3 = torch.empty(len(da) * rec, dtype=torch.uint8, pin_memory=True)
        with torch.cuda.stream(s1):
            ctx.plugin_bandwidth_batch_async(da, o1)
        with torch.cuda.stream(s2):
            ctx.plugin_bandwidth_batch_async(db, o2)
            # the same batch as on s1, in flight at the same time: ordered
            # behind s1's use of the shared work list by the library
            ctx.plugin_bandwidth_batch_async(da, o3)
        outs.append((o1, o2, o3))
    torch.cuda.synchronize()
    for o1, o2, o3 in outs:
        for got, ref in ((_records(kp, o1, len(da)), ref_a), (_records(kp, o2, len(db)), ref_b),
                         (_records(kp, o3, len(da)), ref_a)):
            for g, r in zip(got, ref):
                assert g.status == 0
                assert (g.h, g.sigma, g.psi8, g.g1, g.psi6, g.g2, g.psi4) == \
                       (r.h, r.sigma, r.psi8, r.g1, r.psi6, r.g2, r.psi4)


def test_async_batch_statuses(kp, ctxs):
    import torch
    ctx = ctxs[("FP64_PLAIN", 1)]
    good = synth.normal(3000, 3)
    xs = [torch.from_numpy(good).cuda(), torch.tensor([1.0], dtype=torch.float64, device="cuda"),
          torch.tensor([1.0, float("nan"), 2.0], dtype=torch.float64, device="cuda"),
          torch.full((64,), 2.0, dtype=torch.float64, device="cuda")]
    out = torch.empty(len(xs) * 72, dtype=torch.uint8, pin_memory=True)
    torch.cuda.synchronize()
    ctx.plugin_bandwidth_batch_async(xs, out)
    torch.cuda.synchronize()
    got = kp.batch_results(out, len(xs))
    assert got[0].status == 0 and _rel(got[0].h, oracle.plugin(good).h) < TOL64
    assert got[1].status == kp.KDE_EINVAL and math.isnan(got[1].h)
    assert got[2].status == kp.KDE_ENONFINITE and math.isnan(got[2].h)
    assert got[3].status == kp.KDE_EDEGENERATE and math.isnan(got[3].h)
    sync = ctx.plugin_bandwidth_batch([x for x in xs])
    assert [r.status for r in sync] == [r.status for r in got]
