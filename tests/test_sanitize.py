"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

* The FP64 oracle (oracle/oracle.c) with a C driver over ordinary, edge-case
  and invalid inputs, built here with gcc (CPU).
* The library's host runtime (contexts, work lists, plans, the server, the
  tune-table reader, the no-allocation entry point) built by build() with
  host-only sanitizers (device code unchanged) into a standalone driver,
  tests/sanitize/kde_san_driver, that exercises it on the GPU.
A sanitizer report aborts the process (-fno-sanitize-recover), so the tests
check the exit status and that no report was printed.
"""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = os.path.join(HERE, "sanitize")

REPORT_MARKERS = ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer")


def _run(cmd, env_extra, timeout):
    env = dict(os.environ)
    env.update(env_extra)
    return subprocess.run(cmd, capture_output=True, text=True, timeout=timeout, env=env)


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fno-fast-math", "-ffp-contract=off",
           "-fopenmp", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", exe,
           os.path.join(SAN, "oracle_driver.c"), os.path.join(ROOT, "oracle", "oracle.c"), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = _run([exe], {"ASAN_OPTIONS": "detect_leaks=1", "OMP_NUM_THREADS": "4"}, 120)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out
    assert not any(m in out for m in REPORT_MARKERS), out
    assert "ok" in r.stdout


@pytest.mark.gpu
def test_host_runtime_under_asan_ubsan():
    exe = os.path.join(SAN, "kde_san_driver")
    if not os.path.exists(exe):
        pytest.fail("tests/sanitize/kde_san_driver is not built: run __graft_entry__.build()")
    # the HIP runtime's own allocations are not ours to audit: no leak check
    r = _run([exe], {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0", "UBSAN_OPTIONS": "print_stacktrace=1"},
             240)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert not any(m in out for m in REPORT_MARKERS), out[-4000:]
    assert "host runtime under sanitizers: ok" in r.stdout
