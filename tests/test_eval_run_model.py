"""The density evaluation's FP32 terms (evenly spaced runs, and the
per-point path on narrow groups), replayed in FP32 on the CPU against the
exact Gaussian factor (no GPU).

The GPU kernel forms each column's terms for a run of 32 evenly spaced
points from four exp2 (two sub-runs of 16 sharing one ratio R) and FP32
multiplications; the error bound the GPU tests use (about 6.4e-6 per point)
is derived term by term in tests/test_eval_gpu.py.  This test replays that
arithmetic step by step with numpy's FP32 operations (its exp2 is more
accurate than the hardware's, whose one-ulp error the derivation adds) and
checks every term within its part of the bound: the exponents formed in FP64
and rounded to FP32 once, at most 8 chain steps from each reference, for
spacings up to the span limit (4/15 scaled units) and references far from
zero.  Terms below 2^-24 of a point's largest possible term (which is 1)
are left out, as in the derivation.
"""
import numpy as np
import pytest

U32 = 2.0 ** -24
K = 24.0
SUB, SUB_REF = 16, 8
ARG_MAX = np.float32(60.0)


def run_terms(vx, u0, ds):
    """Per column vx (FP64 array): the 32 point terms E_b R^j in FP32 as the
    kernel forms them (row p = point p of the run); each point's factor
    2^(-K - j^2 ds^2 - 2 j b SUB ds^2) is applied by the caller."""
    u1 = u0 + SUB * ds
    d0 = u0 - vx
    d1 = u1 - vx
    with np.errstate(over="ignore"):     # a far column's exponent rounds to -inf, as on the GPU
        ea0 = (K - d0 * d0).astype(np.float32)
        ea1 = (K - d1 * d1).astype(np.float32)
    ra = np.clip((d0 * (-2.0 * ds)).astype(np.float32), -ARG_MAX, ARG_MAX)
    e = [np.exp2(ea0), np.exp2(ea1)]
    r = np.exp2(ra)
    ri = np.exp2(-ra)
    terms = np.empty((32, vx.size), np.float32)
    for b in range(2):
        terms[b * SUB + SUB_REF] = e[b]
        t = e[b].copy()
        for j in range(1, SUB - SUB_REF):
            t = (t * r).astype(np.float32)
            terms[b * SUB + SUB_REF + j] = t
        t = e[b].copy()
        for j in range(1, SUB_REF + 1):
            t = (t * ri).astype(np.float32)
            terms[b * SUB + SUB_REF - j] = t
    return terms


@pytest.mark.parametrize("ds", [0.01, 0.13, 0.2123, 4.0 / 15.0])
@pytest.mark.parametrize("u0", [0.0, 0.37, -517.25, 1000.3])
def test_run_terms_within_the_derived_bound(ds, u0):
    # columns densely around the run (every term that matters, and beyond)
    rng = np.random.default_rng(7)
    span = 31 * ds
    vx = np.concatenate([np.linspace(u0 - SUB_REF * ds - 7.0, u0 + span + 7.0, 4001),
                         u0 - 8 * ds + rng.uniform(-6.0, span + 6.0, 2000)])
    terms = run_terms(vx, u0, ds).astype(np.float64)
    worst = 0.0
    for p in range(32):
        b, i = divmod(p, SUB)
        j = i - SUB_REF
        vp = u0 + (b * SUB + j) * ds                 # the point's scaled position
        exact = np.exp2(-(vp - vx) ** 2)
        got = terms[p] * np.exp2(-K - j * j * ds * ds - 2.0 * j * b * SUB * ds * ds)
        keep = exact >= U32
        rel = np.abs(got[keep] - exact[keep]) / exact[keep]
        # the derivation's per-term part: E's exponent (ln2 |K - d_b^2| u32)
        # plus |j| steps of (ln2 |2 ds d_0| + 2 + 1) u32, over |d_b| <= 7.2,
        # |d_0| <= 11.5; here for this point's own |j| and the columns kept
        d_b = (u0 + b * SUB * ds) - vx[keep]
        d_0 = u0 - vx[keep]
        bound = (np.log(2) * np.abs(K - d_b * d_b) + abs(j) * (np.log(2) * np.abs(2 * ds * d_0) + 3.0) + 2.0) * U32
        assert np.all(rel <= bound), (p, float(rel.max()), float(bound[np.argmax(rel - bound)]))
        worst = max(worst, float(rel.max()))
    # and the whole derivation's per-term figure (19 + 58 + 2 u32)
    assert worst <= 79 * U32, worst


def test_far_columns_contribute_nothing_or_their_value():
    # a column too far for E_b to stay in FP32's normal range gives 0 (its
    # exact terms are below 2^-100), never inf or NaN, also at zero spacing
    for ds in (0.0, 0.2):
        vx = np.array([-1e30, -80.0, -13.5, 13.5 + 31 * ds, 80.0, 1e30])
        terms = run_terms(vx, 0.0, ds)
        assert np.all(np.isfinite(terms))
        exact_max = np.exp2(-(np.minimum(np.abs(vx), np.abs(vx - 31 * ds)) - 0.0) ** 2)
        assert np.all((terms == 0) | (exact_max > 2.0 ** -130))


def fma32(a, b, c):
    """FP32 fused multiply-add: the product of two FP32 values is exact in
    FP64, the sum is rounded once more to FP32 (the FP64 rounding in between
    is far below FP32's)."""
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(np.float32)


@pytest.mark.parametrize("c", [0.0, 3.3, -1234.5, 1e6])
def test_point_terms_within_the_derived_bound(c):
    # the per-point path on a narrow group: centred scaled values rounded to
    # FP32 (|v_y| <= 4), columns stored as (v_x, -fl(v_x^2)), the term
    # 2^(fma(v_x, 2 v_y, -v_x^2)) scaled by 2^(-v_y^2) in FP64; each term that
    # matters (|d| <= 5) within ln2 |delta a| + 2 ln2 |d| |delta d| + u32, the
    # bound the GPU tests' tolerance is derived from
    rng = np.random.default_rng(11)
    s = 0.85
    y = c + rng.uniform(-4.0, 4.0, 64) / s
    x = c + rng.uniform(-9.5, 9.5, 6000) / s
    vy = ((y - c) * s).astype(np.float32)
    vx = ((x - c) * s).astype(np.float32)
    mvx2 = (-(vx * vx)).astype(np.float32)
    worst = 0.0
    for k in range(y.size):
        a = fma32(vx, np.float32(2.0) * vy[k], mvx2)
        got = np.exp2(a.astype(np.float32)).astype(np.float64) * np.exp2(-float(vy[k]) ** 2)
        d = (y[k] - x) * s
        exact = np.exp2(-d * d)
        keep = np.abs(d) <= 5.0
        rel = np.abs(got[keep] - exact[keep]) / exact[keep]
        va, vxa = np.abs(a[keep]).astype(np.float64), vx[keep].astype(np.float64)
        bound = (np.log(2) * (vxa * vxa + va) + 2 * np.log(2) * np.abs(d[keep]) * (abs(float(vy[k])) + np.abs(vxa))
                 + 1.0) * U32 + 2 * U32
        assert np.all(rel <= bound), (k, float(rel.max()))
        worst = max(worst, float(rel.max()))
    # the derivation's figure over the terms that matter: 4.4e-6 + 5.4e-6 + 1e-7
    assert worst <= 1e-5, worst
