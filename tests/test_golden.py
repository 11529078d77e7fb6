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
