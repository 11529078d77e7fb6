"""Write the FP64 oracle's Algorithm 1 records (Steps I-VII) for the full-size
workloads into tests/golden/full_size_records.json.

Calls only the oracle (oracle/) and the seeded sample generator (synth), never
the HIP library.  Each record keys the sample by the SHA-256 of its float64
bytes, so a test that regenerates the sample can check it has the same bytes
before it compares against the stored values.

Workloads:
  bimodal65536   n = 65536, 0.5 N(-1, (2/3)^2) + 0.5 N(1, (2/3)^2), seed 1
  lognormal1m    n = 2^20, 1e3 exp(Z) - 5e2, Z ~ N(0, 1), seed 2
                 (about 1.1e12 FP64 pair evaluations: minutes on a few cores)
  batch512/k     the 512 samples of the batch workload (master seed 3),
                 n log-uniform in [256, 65536], N(0,1) / bimodal / t3

Run from the repository root:  python tests/golden/make_full_size.py [names...]
With names, only those workloads are recomputed; the others keep their
stored records.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1505_02100_amd import synth  # noqa: E402

OUT = os.path.join(HERE, "full_size_records.json")
FIELDS = ("mean", "sigma", "psi8", "g1", "psi6", "g2", "psi4", "h")


def record(x):
    r = oracle.plugin(x)
    return {k: float(getattr(r, k)).hex() for k in FIELDS}


def single(name):
    if name == "bimodal65536":
        x = synth.workload_single_bimodal(65536, 1)
        src = "synth.workload_single_bimodal(65536, 1)"
    elif name == "lognormal1m":
        x = synth.workload_single_lognormal(1 << 20, 2)
        src = "synth.workload_single_lognormal(1 << 20, 2)"
    else:
        raise KeyError(name)
    t0 = time.perf_counter()
    rec = {"source": src, "n": int(x.size), "sha256": synth.sha256(x), "plugin": record(x)}
    rec["oracle_seconds"] = round(time.perf_counter() - t0, 1)
    rec["oracle_threads"] = oracle.num_threads()
    return rec


def batch():
    xs, names = synth.workload_batch(512, 3)
    t0 = time.perf_counter()
    recs = []
    for k, (x, nm) in enumerate(zip(xs, names)):
        recs.append({"k": k, "dist": nm, "n": int(x.size), "sha256": synth.sha256(x),
                     "plugin": record(x)})
    return {"source": "synth.workload_batch(512, 3)", "samples": recs,
            "oracle_seconds": round(time.perf_counter() - t0, 1),
            "oracle_threads": oracle.num_threads()}


def main(argv):
    names = argv or ["bimodal65536", "lognormal1m", "batch512"]
    out = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            out = json.load(f)
    for name in names:
        t0 = time.perf_counter()
        out[name] = batch() if name == "batch512" else single(name)
        print(f"{name}: {time.perf_counter() - t0:.1f} s", flush=True)
        with open(OUT, "w") as f:
            json.dump(out, f, indent=1, sort_keys=True)
            f.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:])
