"""Write the oracle's records for small fixed inputs into tests/golden/.

Calls only the FP64 oracle (and the seeded sample generator).  Run from the
repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1505_02100_amd import synth  # noqa: E402

FIELDS = ("mean", "sigma", "psi8", "g1", "psi6", "g2", "psi4", "h")


def record(x):
    r = oracle.plugin(x)
    return {k: float(getattr(r, k)).hex() for k in FIELDS}


def main():
    out = {}
    # The paper's toy dataset (Section 2, eight points shown with three KDEs).
    toy = [0.0, 1.0, 1.1, 1.5, 1.9, 2.8, 2.9, 3.5]
    out["toy8"] = {"source": "Section 2 toy dataset", "x": toy, "plugin": record(toy)}
    # One dataset of n = 1024 draws from N(0, 1), seed 0.
    x = synth.workload_single_normal(1024, 0)
    out["normal_n1024_seed0"] = {"source": "synth.workload_single_normal(1024, 0)",
                                 "sha256": synth.sha256(x), "plugin": record(x)}
    # Small mixed datasets covering ragged sizes.
    for n, dist, seed in ((2, "normal", 11), (3, "t3", 12), (63, "bimodal", 13),
                          (64, "normal", 14), (65, "t3", 15), (257, "bimodal", 16),
                          (1000, "t3", 17)):
        x = synth.draw(dist, n, seed)
        out[f"{dist}_n{n}_seed{seed}"] = {"source": f"synth.draw({dist!r}, {n}, {seed})",
                                          "sha256": synth.sha256(x), "plugin": record(x)}
    with open(os.path.join(HERE, "oracle_records.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
