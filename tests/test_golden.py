"""The oracle and the sample generator reproduce their committed records."""
import json
import os

import pytest

import oracle
from paper_1505_02100_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
with open(os.path.join(HERE, "golden", "oracle_records.json")) as f:
    RECORDS = json.load(f)


def _input(key, rec):
    if key == "toy8":
        return rec["x"]
    if key == "normal_n1024_seed0":
        return synth.workload_single_normal(1024, 0)
    dist, n, seed = key.split("_")
    return synth.draw(dist, int(n[1:]), int(seed[4:]))


@pytest.mark.parametrize("key", sorted(RECORDS))
def test_golden_record(key):
    rec = RECORDS[key]
    x = _input(key, rec)
    if "sha256" in rec:
        assert synth.sha256(x) == rec["sha256"]
    got = oracle.plugin(x)
    for k, hexval in rec["plugin"].items():
        assert getattr(got, k) == pytest.approx(float.fromhex(hexval), rel=1e-15, abs=0), k


with open(os.path.join(HERE, "golden", "full_size_records.json")) as f:
    FULL = json.load(f)


def test_full_size_records_match_their_samples():
    # the stored records were made from exactly these bytes
    assert synth.sha256(synth.workload_single_bimodal(65536, 1)) == FULL["bimodal65536"]["sha256"]
    assert synth.sha256(synth.workload_single_lognormal(1 << 20, 2)) == FULL["lognormal1m"]["sha256"]
    xs, names = synth.workload_batch(512, 3)
    recs = FULL["batch512"]["samples"]
    assert [r["sha256"] for r in recs] == [synth.sha256(x) for x in xs]
    assert [r["dist"] for r in recs] == names and [r["n"] for r in recs] == [x.size for x in xs]


@pytest.mark.parametrize("j", range(5))
def test_full_size_batch_records_reproduce(j):
    # the oracle reproduces its stored record of the j-th batch sample with
    # n <= 8192 (kept quick)
    xs, _ = synth.workload_batch(512, 3)
    k = [q for q, x in enumerate(xs) if x.size <= 8192][j]
    got = oracle.plugin(xs[k])
    for name, hexval in FULL["batch512"]["samples"][k]["plugin"].items():
        assert getattr(got, name) == pytest.approx(float.fromhex(hexval), rel=1e-15, abs=0), name
