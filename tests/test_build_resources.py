"""Register budget of the built kernels (compiler remarks recorded by the build).

A kernel that runs out of registers spills to scratch memory, and a spill in
a pass bound by memory costs it directly: one extra live value in the check
rule once made the FP32 degree-8 check kernel spill 20-28 bytes per lane and
run 15 % slower on the n=64800 workload, with every result unchanged.  These
checks read the per-kernel figures that `paper_1609_01567_amd.build` saves
beside the library and fail on any such regression.
"""
import json
import os
import re

import pytest

from paper_1609_01567_amd import build

# Kernels allowed to spill, with the most scratch bytes per lane they may use:
# the sum-product rows of 129..512 edges hold 32 edges per lane (u's and
# suffixes) in a 1024-thread workgroup, whose register budget is 128.
ALLOWED_SPILL = {r"check_wide_(level_)?kernel": 32}


@pytest.fixture(scope="module")
def resources():
    if not os.path.exists(build.RESOURCES):
        pytest.skip("no resource record: build the library with paper_1609_01567_amd.build first")
    if os.path.getmtime(build.RESOURCES) + 1 < os.path.getmtime(build.LIB):
        pytest.skip("resource record older than the library")
    with open(build.RESOURCES) as f:
        return json.load(f)


def test_record_covers_the_kernels(resources):
    names = " ".join(resources)
    for k in ("check_rows_kernel", "check_chunk_kernel", "check_wide_kernel", "check_hub_kernel", "bit_kernel",
              "check_rows_level_kernel", "bit_level_kernel", "level_decide_kernel", "level_move_kernel",
              "eng_check_rows", "eng_check_chunk", "eng_bit", "ingest_kernel", "egress_kernel"):
        assert k in names, k
    for name, r in resources.items():
        assert {"vgpr", "scratch", "occupancy"} <= set(r), name


def test_no_kernel_spills(resources):
    bad = []
    for name, r in resources.items():
        limit = next((b for pat, b in ALLOWED_SPILL.items() if re.search(pat, name)), 0)
        if r["scratch"] > limit:
            bad.append((name, r["scratch"]))
    assert not bad, f"kernels spilling to scratch (bytes per lane): {bad}"


def test_hot_check_kernels_keep_four_waves_per_simd(resources):
    # the register-row check kernels of the plain and engine paths: at most 128
    # registers, so that four wavefronts per SIMD hide the gathers' latency
    hot = {n: r for n, r in resources.items()
           if re.search(r"check_rows_(level_)?kernelILi\dELi4ELi8E|eng_check_rowsILi\dELi4ELi8E", n)}
    assert hot
    low = {n: (r["vgpr"], r["occupancy"]) for n, r in hot.items() if r["occupancy"] < 4}
    assert not low, low
