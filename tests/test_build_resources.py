"""Build-time guard on the per-lane stack of every gfx950 kernel.

The HIP runtime gives each lane 1 KB of private segment by default.  A kernel
whose compiled stack exceeds that faults at launch (the fused stepper did,
when its tile variants were separate functions needing 1.4-1.9 KB per lane).
This test compiles each HIP source for the device only, with the compiler's
kernel resource-usage report, and fails if any kernel needs more than 1 KB
of scratch per lane or uses a dynamic stack.  CPU only: hipcc cross-compiles.
"""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1411_3487_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
LIMIT = 1024  # bytes per lane, the runtime's default private segment


def _flags():
    from paper_1411_3487_amd import build
    return [f for f in build.FLAGS if f not in ("-fPIC",)]


def resource_report(src):
    cmd = [HIPCC, *_flags(), "--cuda-device-only", "-Rpass-analysis=kernel-resource-usage",
           "-x", "hip", "-c", os.path.join(CSRC, src), "-o", os.devnull]
    out = subprocess.run(cmd, capture_output=True, text=True, check=True).stderr
    kernels, name = {}, None
    for line in out.splitlines():
        m = re.search(r"remark:\s+Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            kernels[name] = {}
            continue
        m = re.search(r"remark:\s+(ScratchSize \[bytes/lane\]|Dynamic Stack|Occupancy "
                      r"\[waves/SIMD\]): (\S+)", line)
        if m and name:
            kernels[name][m.group(1).split()[0]] = m.group(2)
    return kernels


@pytest.fixture(scope="module")
def reports():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    srcs = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    return {s: resource_report(s) for s in srcs}


def test_every_kernel_fits_the_default_private_segment(reports):
    seen = 0
    for src, kernels in reports.items():
        for name, r in kernels.items():
            if "ScratchSize" not in r:
                continue
            seen += 1
            assert int(r["ScratchSize"]) <= LIMIT, (src, name, r)
            assert r.get("Dynamic", "False") == "False", (src, name, r)
    assert seen >= 10


def test_fused_stepper_is_reported(reports):
    """Both precisions of the fused launch kernel are compiled and within the
    limit (the kernel that faulted when its stack exceeded it)."""
    fused = {n: r for n, r in reports["dm_fused.hip"].items() if "fused_kernel" in n}
    assert len(fused) >= 2, sorted(reports["dm_fused.hip"])
    for n, r in fused.items():
        assert int(r["ScratchSize"]) <= LIMIT, (n, r)
