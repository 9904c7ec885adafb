"""Register and LDS budgets of the built kernels (no GPU needed).

The library's 1024-thread kernels are meant to run two workgroups per CU
(16 waves each, 8 per SIMD), which needs at most 64 VGPRs per lane, two LDS
tiles per CU and few enough scalar registers.  The compiler's occupancy
figure is not enough for the last: on the MI355X a persistent 1024-thread
sweep at 84, 88 or 95 scalar registers (occupancy 8 by the compiler's count)
got one workgroup per CU at a time (per-workgroup start clocks: the second
started when the first ended), while the same kernel capped at 62, 78 or 80
ran two at once.  So every 1024-thread kernel stays at or below 80.  The counts come from the compiler's kernel-resource-usage remarks,
which build() keeps in paper_1110_6745_amd/_build/kernel_resources.json.
"""
import json
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RESOURCES = os.path.join(ROOT, "paper_1110_6745_amd", "_build", "kernel_resources.json")
LDS_PER_CU = 160 * 1024


@pytest.fixture(scope="module")
def kernels():
    if not os.path.exists(RESOURCES):
        pytest.skip("no kernel resource record: run build() first")
    with open(RESOURCES) as f:
        return json.load(f)


def threads_of(name):
    m = re.search(r"(sweep_kernel|batch_kernel)ILi(\d+)E", name)
    return int(m.group(2)) if m else None


def test_every_library_kernel_is_recorded(kernels):
    names = list(kernels)
    assert any(re.search(r"sweep_kernelILi1024ELi0ELi256E", n) for n in names)
    assert any("batch_kernelILi1024E" in n for n in names)
    for n in names:
        assert {"sgpr", "vgpr", "agpr", "lds", "scratch", "occupancy"} <= set(kernels[n]), n


def test_1024_thread_kernels_fit_two_workgroups_per_cu(kernels):
    big = {n: r for n, r in kernels.items() if threads_of(n) == 1024}
    assert len(big) >= 36 + 4
    for n, r in big.items():
        assert r["sgpr"] <= 80, (n, r)
        assert r["vgpr"] + r["agpr"] <= 64, (n, r)
        assert 2 * r["lds"] <= LDS_PER_CU, (n, r)
        assert r["occupancy"] >= 8, (n, r)


def test_sweep_kernels_do_not_spill(kernels):
    sweeps = {n: r for n, r in kernels.items() if "sweep_kernel" in n}
    assert sweeps
    for n, r in sweeps.items():
        assert r["scratch"] == 0, (n, r)


def test_remark_parser():
    # the compiler's remark lines, as build() reads them
    from paper_1110_6745_amd.build import parse_resources

    text = "\n".join([
        "x.hip:20:1: remark: Function Name: _Z1kv [-Rpass-analysis=kernel-resource-usage]",
        "   20 | {",
        "      | ^",
        "x.hip:20:1: remark:     TotalSGPRs: 56 [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:20:1: remark:     VGPRs: 30 [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:20:1: remark:     AGPRs: 0 [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:20:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:20:1: remark:     Occupancy [waves/SIMD]: 8 [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:20:1: remark:     LDS Size [bytes/block]: 65920 [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:9:1: remark: Function Name: _Z2k2v [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:9:1: remark:     TotalSGPRs: 91 [-Rpass-analysis=kernel-resource-usage]",
    ])
    got = parse_resources(text)
    assert got == {"_Z1kv": {"sgpr": 56, "vgpr": 30, "agpr": 0, "scratch": 0, "occupancy": 8,
                             "lds": 65920},
                   "_Z2k2v": {"sgpr": 91}}
