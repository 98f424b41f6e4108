"""Register budget of the device code: no kernel may spill to scratch memory. A spill turns
into per-lane private loads and stores on the hot path (one such spill in the row kernel cost
17 % of its time and wrote 160 MB per launch), so the compiler's resource report of every
kernel is checked at build time (hipcc cross-compiles gfx950 without a GPU)."""
import os
import re
import shutil
import subprocess

import pytest

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_2102_07167_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="hipcc not found")
@pytest.mark.parametrize("src", ["kur_kernels.hip", "ens_kernels.hip", "persist_kernels.hip"])
def test_no_kernel_uses_scratch(src, tmp_path):
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", str(tmp_path / "k.o"),
           "--offload-device-only", "-Rpass-analysis=kernel-resource-usage"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    found = re.findall(r"Function Name: (\S+).*?ScratchSize \[bytes/lane\]: (\d+)", res.stderr, re.S)
    assert found, "no resource report"
    spills = [(name, int(b)) for name, b in found if int(b) > 0]
    assert not spills, spills
