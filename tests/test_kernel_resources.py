"""Register, scratch and occupancy figures of the built kernels (CPU test).

build() records what hipcc reports for every kernel of the device sources
(paper_1505_02100_amd/kernel_resources.txt).  The pair kernel's speed rests on
them: every persistent-kernel build held to three waves per SIMD must fit
(168 VGPRs at most) without spilling, the default precision's four-wave build
must reach four waves, and so must the density evaluation's FP32 kernel.  A
change that pushes one of them over (an edit of the hand-placed loops, a new
live value in the kernel) fails here, before any GPU run.
"""
import os
import re

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
RESOURCES = os.path.join(os.path.dirname(HERE), "paper_1505_02100_amd", "kernel_resources.txt")


@pytest.fixture(scope="module")
def kernels():
    if not os.path.exists(RESOURCES):
        pytest.skip("kernel_resources.txt not written: run __graft_entry__.build()")
    out = {}
    for line in open(RESOURCES):
        if line.startswith("#") or not line.strip():
            continue
        name, vgprs, scratch, occ = line.split()
        out[name] = (int(vgprs), int(scratch), int(occ))
    return out


def _persistent(kernels):
    found = {}
    for name, v in kernels.items():
        m = re.fullmatch(r"_ZN3kde12k_persistentILi(\d)ELi(\d)ELi256ELi(\d)EEEvNS_10LaunchArgsE", name)
        if m:
            found[tuple(int(g) for g in m.groups())] = v
    return found


def test_three_wave_builds_fit_without_spilling(kernels):
    pk = _persistent(kernels)
    three = {k: v for k, v in pk.items() if k[2] == 3}
    # five precisions x R in {1, 2, 4}
    assert len(three) == 15, sorted(pk)
    for (prec, r, _), (vgprs, scratch, occ) in three.items():
        assert occ == 3 and vgprs <= 168 and scratch == 0, (prec, r, vgprs, scratch, occ)


def test_four_wave_build_of_the_default_precision(kernels):
    pk = _persistent(kernels)
    four = {k: v for k, v in pk.items() if k[2] == 4}
    assert set(four) == {(1, 1, 4)}
    vgprs, scratch, occ = four[(1, 1, 4)]
    # its spills sit outside the pair loops (measured: 84 bytes per lane)
    assert occ == 4 and vgprs <= 128 and scratch <= 128, four


def test_density_evaluation_kernels(kernels):
    vgprs, scratch, occ = kernels["_ZN3kde4eval8k_eval32ENS0_8EvalArgsE"]
    # 32 points per thread in the run path: four waves, with a few values
    # spilled around the column loop (measured: 68 bytes per lane)
    assert occ >= 4 and vgprs <= 128 and scratch <= 128, (vgprs, scratch, occ)
    vgprs, scratch, occ = kernels["_ZN3kde4eval8k_eval64ENS0_8EvalArgsE"]
    assert scratch == 0
