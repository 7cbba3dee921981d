"""Register budgets of the FP32 scan kernels (and of the block form's two main kernels),
read from the compiler's resource report.

The balanced schedule places a whole number of workgroups (one wave per SIMD each) on
every compute unit, and its cut slices hand state between waves that must be resident
at the same time; the host clamps the plan to the occupancy the kernel allows, so a
kernel that grows past its register budget silently runs with fewer waves per SIMD.
These checks catch that at build time, without a GPU."""
import os
import re
import subprocess

import pytest

from paper_2011_06787_amd import build as hipbuild

SRC = os.path.join(hipbuild.CSRC, "scan_fp32.hip")


@pytest.fixture(scope="module")
def report(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("res") / "scan.o")
    cmd = [hipbuild.HIPCC, f"--offload-arch={hipbuild.ARCH}", "-O3", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(hipbuild.HERE, "..", "include"),
           "-c", SRC, "-o", out, "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True, check=True)
    kernels, name = {}, None
    for line in r.stderr.splitlines():
        if "Function Name:" in line:
            m = re.search(r"(scan_fp32_(?:[a-z]+_)?kernel)ILi(\d+)E", line)
            name = (m.group(1), int(m.group(2))) if m else None
            if name is not None:
                kernels[name] = {}
            continue
        m = re.search(r"remark:\s+(VGPRs|AGPRs|ScratchSize \[bytes/lane\]|Occupancy \[waves/SIMD\]): (\d+)",
                      line)
        if m and name is not None:
            kernels[name][m.group(1).split()[0]] = int(m.group(2))
    return kernels


def test_every_scan_kernel_is_reported(report):
    for kind in ("scan_fp32_kernel", "scan_fp32_balanced_kernel", "scan_fp32_persistent_kernel"):
        for maxm in (2, 4, 8):
            assert (kind, maxm) in report, (kind, maxm)


def test_scan_kernels_do_not_spill(report):
    for key, r in report.items():
        assert r.get("ScratchSize", 0) == 0, (key, r)


@pytest.mark.parametrize("maxm, waves", [(2, 4), (4, 4), (8, 3)])
def test_balanced_kernel_fits_its_waves_per_simd(report, maxm, waves):
    r = report[("scan_fp32_balanced_kernel", maxm)]
    assert r["Occupancy"] >= waves, r


@pytest.fixture(scope="module")
def block_report(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("res") / "block.o")
    cmd = [hipbuild.HIPCC, f"--offload-arch={hipbuild.ARCH}", "-O3", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(hipbuild.HERE, "..", "include"),
           "-c", os.path.join(hipbuild.CSRC, "block_bf16.hip"), "-o", out,
           "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True, check=True)
    kernels, name = {}, None
    for line in r.stderr.splitlines():
        if "Function Name:" in line:
            m = re.search(r"(block_state_kernel|block_output_kernel)", line)
            name = m.group(1) + (re.search(r"ILi(\d+)E", line).group(1) if "ILi" in line else "") \
                if m else None
            if name is not None:
                kernels[name] = {}
            continue
        m = re.search(r"remark:\s+(VGPRs|AGPRs|ScratchSize \[bytes/lane\]|Occupancy \[waves/SIMD\]): (\d+)",
                      line)
        if m and name is not None:
            kernels[name][m.group(1).split()[0]] = int(m.group(2))
    return kernels


def test_block_state_kernel_keeps_three_waves_per_simd(block_report):
    """The state kernel's W' register cache is sized for three waves per SIMD: a change
    that spills or drops it to two shows here."""
    r = block_report["block_state_kernel"]
    assert r.get("ScratchSize", 0) == 0 and r["Occupancy"] >= 3, r


@pytest.mark.parametrize("rw", [2, 4, 8])
def test_block_output_kernel_does_not_spill(block_report, rw):
    r = block_report[f"block_output_kernel{rw}"]
    assert r.get("ScratchSize", 0) == 0 and r["Occupancy"] >= 2, r
