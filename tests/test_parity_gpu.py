"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances (relative):
  * FP64 plain: h, Psi6, Psi4 within 1e-12.  Both sides evaluate the same
    sums in FP64 in different orders, with different (faithfully rounded) exp
    implementations and a reciprocal instead of a division for 1/g; the
    rounding error of a sum of n^2 terms with cancellation factor
    k = sum|terms| / |sum| stays below ~1e-14 k for the sizes tested.
  * FP32 (compensated sums): h within 1e-6 (the bound the FP32 path is built to);
    Psi6 and Psi4 within 2e-5 (their FP32 rounding is amplified by the
    cancellation inside the Hermite factor and the sum).
"""
import math

import numpy as np
import pytest

import oracle
from paper_1505_02100_amd import synth

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32_H = 1e-6
TOL32_PSI = 2e-5


@pytest.fixture(scope="module")
def kp():
    from paper_1505_02100_amd import kdeplugin
    return kdeplugin


@pytest.fixture(scope="module")
def ctx64(kp):
    c = kp.Context(kp.KDE_FP64_PLAIN)
    yield c
    c.close()


@pytest.fixture(scope="module")
def ctx32(kp):
    c = kp.Context(kp.KDE_FP32_COMP)
    yield c
    c.close()


@pytest.fixture(scope="module")
def ctx32x(kp):
    c = kp.Context(kp.KDE_FP32_COMP_EXACT)
    yield c
    c.close()


@pytest.fixture(scope="module")
def ctx32p(kp):
    c = kp.Context(kp.KDE_FP32_POLYEXP)
    yield c
    c.close()


@pytest.fixture(scope="module")
def ctxq(kp):
    c = kp.Context(kp.KDE_Q32_32)
    yield c
    c.close()


def _rel(a, b):
    return abs(a - b) / abs(b)


def _check(res, ref, tol_h, tol_psi):
    assert res.status == 0
    assert _rel(res.sigma, ref.sigma) < 1e-13
    # Step II in FP64 on both sides from the same sigma (sigma^9 amplifies
    # sigma's rounding ninefold)
    assert _rel(res.psi8, ref.psi8) < 1e-11, (res.psi8, ref.psi8)
    assert _rel(res.g1, ref.g1) < 1e-13
    assert _rel(res.psi6, ref.psi6) < tol_psi, (res.psi6, ref.psi6)
    assert _rel(res.g2, ref.g2) < tol_psi
    assert _rel(res.psi4, ref.psi4) < tol_psi, (res.psi4, ref.psi4)
    assert _rel(res.h, ref.h) < tol_h, (res.h, ref.h, _rel(res.h, ref.h))


RAGGED = [2, 3, 5, 63, 64, 65, 255, 256, 257, 511, 512, 513, 1000, 1023, 1024, 1025, 2047, 4097]


@pytest.mark.parametrize("n", RAGGED)
def test_plugin_fp64_ragged(ctx64, n):
    x = synth.draw(["normal", "bimodal", "t3"][n % 3], n, 50 + n)
    _check(ctx64.plugin_bandwidth(x), oracle.plugin(x), TOL64, TOL64)


@pytest.mark.parametrize("n", RAGGED)
def test_plugin_fp32_ragged(ctx32, ctx32x, n):
    x = synth.draw(["normal", "bimodal", "t3"][n % 3], n, 50 + n)
    ref = oracle.plugin(x)
    _check(ctx32.plugin_bandwidth(x), ref, TOL32_H, TOL32_PSI)
    _check(ctx32x.plugin_bandwidth(x), ref, TOL32_H, TOL32_PSI)


def test_small_config_normal_1024(ctx64, ctx32):
    # n = 1024 draws of N(0, 1), seed 0, checked in both precisions
    x = synth.workload_single_normal(1024, 0)
    ref = oracle.plugin(x)
    _check(ctx64.plugin_bandwidth(x), ref, TOL64, TOL64)
    _check(ctx32.plugin_bandwidth(x), ref, TOL32_H, TOL32_PSI)


@pytest.mark.parametrize("n", [20000, 33333])
def test_plugin_many_tiles(ctx64, ctx32, n):
    x = synth.bimodal(n, 7)
    ref = oracle.plugin(x)
    _check(ctx64.plugin_bandwidth(x), ref, TOL64, TOL64)
    _check(ctx32.plugin_bandwidth(x), ref, TOL32_H, TOL32_PSI)


@pytest.mark.parametrize("n", [2, 65, 1000, 4097, 33333])
def test_plugin_fp32_polynomial_exp2(ctx32p, n):
    # the Gaussian factor from the Remez polynomial instead of v_exp_f32:
    # the same FP32 tolerances against the oracle, deterministic
    x = synth.draw(["normal", "bimodal", "t3"][n % 3], n, 70 + n)
    ref = oracle.plugin(x)
    a = ctx32p.plugin_bandwidth(x)
    _check(a, ref, TOL32_H, TOL32_PSI)
    b = ctx32p.plugin_bandwidth(x)
    assert (a.h, a.psi6, a.psi4) == (b.h, b.psi6, b.psi4)
    for r, g in ((4, 0.4), (6, 0.05)):
        assert _rel(ctx32p.psi(x, r, g), oracle.psi(x, r, g)) < TOL32_PSI


def _q32_psi_bound(x, r, g):
    """Bound on the Psi_r(g) error of the Q32.32 mode, from its arithmetic.

    In units of one Q32.32 step (2^-32), per pair with |u| < 16: the
    z-scores truncate (|dd| <= 2), u = d (sigma/g) truncates (|du| <=
    2 ginv + 1 + |d|), t = u^2 (|dt| <= 2|u| du + 1), the exponent
    a = (t/2) log2(e) (|da| <= 0.73 dt + 2 + a/2).  The Gaussian factor is a
    Horner polynomial (at most 12 steps of error) shifted right by
    n = round(a) with a truncation: |de| <= min(1, e 2^32) + 12 2^-n, plus
    e ln2 da from its argument.  The Hermite factor carries |p'(t)| dt and
    its own truncations (1 + t), the product one more step:
        |dterm| <= |p| (min(1, e 2^32) + 12 2^-n + e ln2 da) + e (|p'| dt + 1 + t) + 1.
    The pair sum S enters Psi as 2 S / (sqrt(2 pi) n^2 g^(r+1)).  The first
    part dominates at small g: the Gaussian factor has an absolute, not a
    relative, resolution, so tail terms (t of 30 to 50, where e is a few
    steps) lose their accuracy, multiplied by |p| ~ t^3.  This is the
    fixed-point design's accuracy limit, which the mode is there to show.
    """
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    sig = x.std(ddof=1)
    z = (x - x.mean()) / sig
    ginv = sig / g
    q = 2.0 ** 32
    tot = 0.0
    for i in range(n - 1):
        u = (z[i] - z[i + 1:]) * ginv
        u = u[np.abs(u) < 16]
        d = u / ginv
        t = u * u
        e = np.exp(-t / 2)
        a = 0.7213475204444817 * t
        if r == 6:
            pv = ((t - 15) * t + 45) * t - 15
            dp = (3 * t - 30) * t + 45
        else:
            pv = (t - 6) * t + 3
            dp = 2 * t - 6
        du = 2 * ginv + 1 + np.abs(d)
        dt = 2 * np.abs(u) * du + 1
        da = 0.73 * dt + 2 + a / 2
        de = np.minimum(1.0, e * q) + 12.0 * np.exp2(-np.round(a)) + e * math.log(2) * da
        tot += np.sum(np.abs(pv) * de + e * (np.abs(dp) * dt + 1 + t) + 1)
    return 2 * tot / q / math.sqrt(2 * math.pi) / (n * n * g ** (r + 1))


@pytest.mark.parametrize("n", [2, 65, 1000, 4097])
def test_plugin_q32_fixed_point(ctxq, n):
    # the FPGA design's Q32.32 arithmetic against the oracle, within the
    # bounds its arithmetic gives (_q32_psi_bound): Psi6 at g1, Psi4 at g2 (plus
    # the effect of g2's own small error), h = (R(K)/(n Psi4))^(1/5) through
    # Psi4 alone; Psi at fixed g likewise.  The sums are integers added
    # exactly, so the result repeats bitwise.
    x = synth.draw(["normal", "bimodal", "t3"][n % 3], n, 90 + n)
    ref = oracle.plugin(x)
    a = ctxq.plugin_bandwidth(x)
    assert a.status == 0
    b6 = _q32_psi_bound(x, 6, ref.g1) + 1e-12 * abs(ref.psi6)
    assert abs(a.psi6 - ref.psi6) <= b6
    dg2 = _rel(a.g2, ref.g2)
    rel4 = (_q32_psi_bound(x, 4, ref.g2) + 1e-12 * ref.psi4) / ref.psi4 + 10 * dg2
    assert _rel(a.psi4, ref.psi4) <= rel4
    assert _rel(a.h, ref.h) <= 0.2 * rel4 + 1e-12
    b = ctxq.plugin_bandwidth(x)
    assert (a.h, a.psi6, a.psi4) == (b.h, b.psi6, b.psi4)
    for r, g in ((4, 0.4), (6, 0.05)):
        want = oracle.psi(x, r, g)
        bound = _q32_psi_bound(x, r, g) + 1e-12 * abs(want)
        assert abs(ctxq.psi(x, r, g) - want) <= bound, (r, g, bound / abs(want))


def test_q32_sums_do_not_depend_on_the_decomposition(kp, ctxq):
    # integer sums: any split of the work into items gives the same Psi bitwise
    x = synth.bimodal(9000, 4)
    a = ctxq.psi(x, 6, 0.3)
    with kp.Context(kp.KDE_Q32_32, target_items=97) as other:
        assert other.psi(x, 6, 0.3) == a


@pytest.mark.parametrize("r", [4, 6])
@pytest.mark.parametrize("g", [0.05, 0.4, 3.0])
def test_psi_fixed_g(ctx64, ctx32, r, g):
    x = synth.student_t3(3001, 9)
    ref = oracle.psi(x, r, g)
    assert _rel(ctx64.psi(x, r, g), ref) < TOL64
    assert _rel(ctx32.psi(x, r, g), ref) < TOL32_PSI


def test_psi_literal_calls(kp):
    x = synth.normal(777, 4)
    assert _rel(kp.kde_psi(x, 6, 0.5), oracle.psi(x, 6, 0.5)) < TOL64
    assert _rel(kp.kde_plugin_bandwidth(x), oracle.plugin(x).h) < TOL64
    assert math.isnan(kp.kde_plugin_bandwidth([1.0]))
    assert math.isnan(kp.kde_psi(x, 5, 0.5))


def _abs_block_sum(x, r, g, r0, r1, c0, c1):
    """sum |K^(r)((x_i - x_j)/g)| over the block's pairs j > i: the scale of
    the rounding error bound (not a reference value)."""
    from scipy import special
    tot = 0.0
    for i in range(r0, r1):
        j0 = max(c0, i + 1)
        if j0 >= c1:
            continue
        y = (x[i] - x[j0:c1]) / g
        tot += np.sum(np.abs(special.eval_hermitenorm(r, y)) * np.exp(-0.5 * y * y)) / math.sqrt(2 * math.pi)
    return tot


def test_psi_range_items_match_oracle_blocks(ctx64, ctx32):
    n = 9000
    x = synth.student_t3(n, 3)
    g = 0.3
    for ctx, eps in ((ctx64, 1e-13), (ctx32, 2e-6)):
        m = ctx.psi_num_items(n)
        assert m > 4
        for k in sorted({0, 1, m // 2, m - 2, m - 1}):
            r0, r1, c0, c1 = ctx.psi_item_geometry(n, k)
            got = ctx.psi_range(x, 6, g, k, k + 1)
            ref = oracle.block_sum(x, 6, g, r0, r1, c0, c1)
            bound = eps * _abs_block_sum(x, 6, g, r0, r1, c0, c1) + 1e-300
            assert abs(got - ref) <= bound, (k, got, ref, bound)
        # shards of a partition add up to the whole strict upper triangle
        cuts = [0, m // 3, (2 * m) // 3, m]
        total = sum(ctx.psi_range(x, 6, g, a, b) for a, b in zip(cuts[:-1], cuts[1:]))
        ref = oracle.pair_sum(x, 6, g)
        assert abs(total - ref) <= eps * _abs_block_sum(x, 6, g, 0, n, 0, n)


def test_batch_equals_single_bitwise(ctx64, ctx32):
    xs = [synth.draw(d, n, 100 + i) for i, (d, n) in
          enumerate([("normal", 300), ("bimodal", 2048), ("t3", 77), ("normal", 5000), ("t3", 2)])]
    for ctx in (ctx64, ctx32):
        batch = ctx.plugin_bandwidth_batch(xs)
        for x, b in zip(xs, batch):
            s = ctx.plugin_bandwidth(x)
            assert b.status == 0
            assert (b.h, b.psi6, b.psi4, b.g2) == (s.h, s.psi6, s.psi4, s.g2)


def test_batch_matches_oracle(ctx64, ctx32):
    xs, _ = synth.workload_batch(count=24, master=31, n_lo=256, n_hi=4096)
    r64 = ctx64.plugin_bandwidth_batch(xs)
    r32 = ctx32.plugin_bandwidth_batch(xs)
    for x, a, b in zip(xs, r64, r32):
        ref = oracle.plugin(x)
        _check(a, ref, TOL64, TOL64)
        _check(b, ref, TOL32_H, TOL32_PSI)


@pytest.mark.parametrize("n,offset", [(300_001, 1e6), (1_000_003, -3e4)])
def test_step1_many_chunks_far_from_origin(ctx64, ctx32, n, offset):
    # Step I merges many chunks (the last one ragged) of a sample whose mean
    # is far from 0 in units of its spread; every precision runs the same
    # FP64 Step I, so mean and sigma agree bitwise across precisions
    x = offset + 3.0 * synth.normal(n, 77)
    m, s = oracle.moments(x)
    r64 = ctx64.plugin_bandwidth(x)
    r32 = ctx32.plugin_bandwidth(x)
    assert r64.status == 0 and r32.status == 0
    assert _rel(r64.mean, m) < 1e-14 and _rel(r64.sigma, s) < 1e-12, (r64.mean, m, r64.sigma, s)
    assert (r32.mean, r32.sigma, r32.g1) == (r64.mean, r64.sigma, r64.g1)


def test_stage_timeline(ctx32):
    # Step I publishes its two stages at once; the pair stages follow in order,
    # all inside the launch's device time
    ctx32.plugin_bandwidth(synth.bimodal(20000, 3))
    tl = ctx32.last_timeline(0)
    assert len(tl) == 4 and tl[0] == tl[1]
    assert 0.0 <= tl[1] <= tl[2] <= tl[3] <= ctx32.last_device_ms(), tl


def test_deterministic_repeat(ctx32):
    x = synth.bimodal(12345, 5)
    a = ctx32.plugin_bandwidth(x)
    b = ctx32.plugin_bandwidth(x)
    assert (a.h, a.psi6, a.psi4) == (b.h, b.psi6, b.psi4)


@pytest.mark.parametrize("a,b", [(1e3, -5e2), (-2.5, 7.0)])
def test_scale_shift_equivariance(ctx64, ctx32, a, b):
    x = synth.lognormal(5000, 12)
    for ctx, tol in ((ctx64, 1e-12), (ctx32, 2e-6)):
        h0 = ctx.plugin_bandwidth(x).h
        h1 = ctx.plugin_bandwidth(a * x + b).h
        assert _rel(h1, abs(a) * h0) < tol


def test_error_cases(ctx64, ctx32, kp):
    for ctx in (ctx64, ctx32):
        r = ctx.plugin_bandwidth(np.array([1.0, np.nan, 2.0]), check=False)
        assert r.status == kp.KDE_ENONFINITE and math.isnan(r.h)
        r = ctx.plugin_bandwidth(np.array([1.0, np.inf, 2.0]), check=False)
        assert r.status == kp.KDE_ENONFINITE
        r = ctx.plugin_bandwidth(np.full(100, 3.25), check=False)
        assert r.status == kp.KDE_EDEGENERATE
        r = ctx.plugin_bandwidth(np.array([1.0]), check=False)
        assert r.status == kp.KDE_EINVAL
        with pytest.raises(kp.KdeError):
            ctx.psi(np.ones(10), 4, -1.0)
        # the context stays usable after errors
        x = synth.normal(100, 1)
        assert _rel(ctx.plugin_bandwidth(x).h, oracle.plugin(x).h) < TOL32_H


def test_f32_input_and_device_tensors(ctx64, ctx32):
    import torch
    x = synth.bimodal(3000, 19)
    ref = oracle.plugin(x)
    xd = torch.from_numpy(x).cuda()
    _check(ctx64.plugin_bandwidth(xd), ref, TOL64, TOL64)
    _check(ctx32.plugin_bandwidth(xd), ref, TOL32_H, TOL32_PSI)
    x32 = x.astype(np.float32)
    ref32 = oracle.plugin(x32.astype(np.float64))
    _check(ctx64.plugin_bandwidth(x32), ref32, TOL64, TOL64)
    _check(ctx64.plugin_bandwidth(torch.from_numpy(x32).cuda()), ref32, TOL64, TOL64)


def test_calls_on_alternating_streams(ctx32):
    # a plan's states are reset after each call on that call's stream; a call
    # on another stream waits for that reset
    import torch
    xd = torch.from_numpy(synth.bimodal(30000, 29)).cuda()
    ref = ctx32.plugin_bandwidth(xd)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for k in range(6):
        with torch.cuda.stream(s1 if k % 2 == 0 else s2):
            r = ctx32.plugin_bandwidth(xd)
        assert (r.status, r.h, r.psi6, r.psi4) == (0, ref.h, ref.psi6, ref.psi4)


def test_autotune_tables_roundtrip(kp, tmp_path):
    x = synth.bimodal(3000, 23)
    ref = oracle.plugin(x)
    p1 = str(tmp_path / "single.json")
    t1 = kp.kde_autotune(kp.KDE_FP32_COMP, [1024, 4096], p1, mode=kp.KDE_TUNE_SINGLE, reps=2)
    assert t1["rows_per_lane"] in (1, 2, 4) and len(t1["targets"]) == 2
    with kp.Context(kp.KDE_FP32_COMP, tune_table=p1) as c:
        cfg = c.config()
        assert cfg["rows_per_lane"] == t1["rows_per_lane"]
        # 0 leaves the blocks per CU to the context (its occupancy limit)
        assert cfg["blocks_per_cu"] == t1["blocks_per_cu"] or (t1["blocks_per_cu"] == 0 and cfg["blocks_per_cu"] >= 1)
        _check(c.plugin_bandwidth(x), ref, TOL32_H, TOL32_PSI)
    p2 = str(tmp_path / "batch.json")
    t2 = kp.kde_autotune(kp.KDE_FP32_COMP, [300, 1000, 2500], p2, mode=kp.KDE_TUNE_BATCH, reps=2)
    assert t2["pair_budget"] > 0
    with kp.Context(kp.KDE_FP32_COMP, tune_table=p2) as c:
        res = c.plugin_bandwidth_batch([x, x[:500]])
        _check(res[0], ref, TOL32_H, TOL32_PSI)
    with pytest.raises(kp.KdeError):
        kp.Context(kp.KDE_FP64_PLAIN, tune_table=p1)
    # the FP32 search also times the polynomial exponential and records its pick
    assert t1["exp_poly"] in (0, 1) and t2["exp_poly"] in (0, 1)


def test_tune_table_selects_the_polynomial_exponential(kp, tmp_path):
    # an FP32 table with exp_poly = 1 runs the polynomial-exponential kernels:
    # bitwise what a KDE_FP32_POLYEXP context computes, within the FP32 bounds
    # of the oracle; exp_poly = 0 keeps v_exp_f32; a table for another
    # precision may not select it
    x = synth.student_t3(5000, 31)
    ref = oracle.plugin(x)
    with kp.Context(kp.KDE_FP32_POLYEXP) as cp, kp.Context(kp.KDE_FP32_COMP) as ch:
        rp, rh = cp.plugin_bandwidth(x), ch.plugin_bandwidth(x)
    for flag, want in ((1, rp), (0, rh)):
        p = str(tmp_path / f"exp{flag}.json")
        with open(p, "w") as f:
            f.write('{"precision": %d, "rows_per_lane": 1, "blocks_per_cu": 0, "exp_poly": %d}' %
                    (kp.KDE_FP32_COMP, flag))
        with kp.Context(kp.KDE_FP32_COMP, tune_table=p) as c:
            r = c.plugin_bandwidth(x)
        assert (r.h, r.psi6, r.psi4) == (want.h, want.psi6, want.psi4), flag
        _check(r, ref, TOL32_H, TOL32_PSI)
    bad = str(tmp_path / "bad.json")
    with open(bad, "w") as f:
        f.write('{"precision": %d, "exp_poly": 1}' % kp.KDE_FP64_PLAIN)
    with pytest.raises(kp.KdeError):
        kp.Context(kp.KDE_FP64_PLAIN, tune_table=bad)
