"""Register budget of the HIP kernels (CPU: hipcc cross-compiles for gfx950).  Every kernel must
fit its vector registers without spilling to scratch memory: a spill turns register traffic into
memory traffic in kernels whose time is memory traffic.  (Scalar registers that the compiler
parks in vector-register lanes cost no memory traffic and are allowed.)"""
from __future__ import annotations

import os
import re
import shutil
import subprocess

import pytest

from paper_1503_06394_amd.build import CSRC, HIP_FLAGS, HIPCC


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="hipcc not available")
@pytest.mark.parametrize("src", ["ld_kernels.hip", "ld_prep.hip"])
def test_no_kernel_spills(tmp_path, src):
    cmd = [HIPCC, "-x", "hip", *HIP_FLAGS, "--cuda-device-only", "-Rpass-analysis=kernel-resource-usage", "-c",
           os.path.join(CSRC, src), "-o", str(tmp_path / "k.o")]
    out = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stderr[-2000:]
    kernels, cur = {}, None
    for line in out.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            kernels[cur] = {}
            continue
        m = re.search(r"remark:\s+(VGPRs Spill|ScratchSize \[bytes/lane\]): (\d+)", line)
        if m and cur:
            kernels[cur][m.group(1)] = int(m.group(2))
    assert kernels, "no resource remarks parsed"
    bad = {k: v for k, v in kernels.items() if any(v.values())}
    assert not bad, bad
