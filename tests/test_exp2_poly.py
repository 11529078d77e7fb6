"""The minimax polynomial for 2^f behind the KDE_FP32_POLYEXP precision.

Pinned against the mathematics, not against its own code: the committed
coefficients are the generator's output; the exact minimax polynomial
equioscillates (degree + 2 extrema of equal size and alternating sign, the
characterisation of the best uniform approximation); the FP32-rounded
polynomial stays within its stated relative error of libm's exp2 on
[-1/2, 1/2]; and the full evaluation 2^n p(f) in emulated FP32 arithmetic
(each fma rounded once) stays within a few FP32 ulps of libm's exp2 over the
argument range the pair path uses.  The GPU parity of the mode is in
test_parity_gpu.py.
"""
import math
import os
import re

import numpy as np
import pytest

from paper_1505_02100_amd import remez_exp2 as rz

HERE = os.path.dirname(os.path.abspath(__file__))
HEADER = os.path.join(HERE, "..", "paper_1505_02100_amd", "csrc", "kde_exp2_poly.h")


@pytest.fixture(scope="module")
def generated():
    return rz.generate()


def _committed():
    text = open(HEADER).read()
    return [float(v) for v in re.findall(r"^\s+([0-9.eE+-]+)f,", text, re.M)], text


def test_committed_header_is_the_generator_output(generated):
    c32, E, err32 = generated
    cq, Eq = rz.generate_q32()
    vals, text = _committed()
    assert vals == c32
    assert text == rz.header_text(c32, E, err32, cq, Eq)


def test_q32_polynomial_within_a_q32_ulp():
    # the Q32.32 coefficients, evaluated exactly, stay within 2^-33 of 2^f
    cq, Eq = rz.generate_q32()
    assert float(Eq) < 2.0 ** -34
    f = np.linspace(-0.5, 0.5, 100001)
    p = np.zeros_like(f)
    for ck in reversed(cq):
        p = p * f + ck / 2.0 ** 32
    assert np.max(np.abs(p - np.exp2(f))) < 2.0 ** -31


def test_minimax_equioscillates():
    import mpmath as mp
    c, E = rz.remez()
    mp.mp.dps = 40
    xs = [rz.LO + (rz.HI - rz.LO) * i / 4000 for i in range(4001)]
    es = [rz.rel_err(c, x) for x in xs]
    # local extrema of the error, including the ends
    ext = [es[0]] + [es[i] for i in range(1, len(es) - 1)
                     if (es[i] - es[i - 1]) * (es[i + 1] - es[i]) <= 0] + [es[-1]]
    big = [e for e in ext if abs(e) > 0.99 * float(E)]
    assert len(big) == rz.DEGREE + 2
    assert all(big[i] * big[i + 1] < 0 for i in range(len(big) - 1))
    assert max(abs(float(e)) for e in es) <= float(E) * (1 + 1e-4)


def test_rounded_polynomial_against_libm(generated):
    c32, E, err32 = generated
    f = np.linspace(-0.5, 0.5, 200001)
    p = np.zeros_like(f)
    for ck in reversed(c32):
        p = p * f + ck
    rel = np.abs(p / np.exp2(f) - 1.0)
    assert rel.max() <= 1.6e-8
    assert abs(rel.max() - err32) <= 1e-9
    # the rounding error is odd in f (mostly c1's): its mean is tiny
    assert abs(np.mean(p / np.exp2(f) - 1.0)) <= 2e-9


def _fma32(a, b, c):
    # a*b is exact in float64 for float32 inputs; one rounding of the sum to float32
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(np.float32)


def test_full_evaluation_in_emulated_fp32(generated):
    c32, _, _ = generated
    c = [np.float32(v) for v in c32]
    t = np.concatenate([np.linspace(-149.0, 3.7, 400001), -np.logspace(-8, 2, 10001)]).astype(np.float32)
    tc = np.maximum(t, np.float32(-200.0))
    n = np.rint(tc).astype(np.float32)
    f = (tc - n).astype(np.float32)
    p = np.full_like(f, c[-1])
    for ck in reversed(c[:-1]):
        p = _fma32(p, f, np.full_like(f, ck))
    got = np.ldexp(p.astype(np.float64), n.astype(np.int64)).astype(np.float32).astype(np.float64)
    ref = np.exp2(t.astype(np.float64))
    normal = ref >= 2.0 ** -126
    rel = np.abs(got[normal] / ref[normal] - 1.0)
    assert rel.max() <= 4 * 2.0 ** -24
    # below FP32's range the value is tiny or zero, never large
    assert np.all(got[~normal] <= 2.0 ** -125)
    assert float(np.ldexp(np.float32(1.0), -250)) == 0.0
