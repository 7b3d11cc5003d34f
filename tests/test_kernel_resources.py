"""Register budget of the compiled direct-sum kernels (no GPU needed).

Every variant of the persistent kernel must fit in 256 VGPRs per lane so that
two waves share each SIMD; above that the hardware runs one wave per SIMD and
the kernel slows by about half.  The check compiles the kernel source for
gfx950 to assembly with the same flags as the build and reads the register
counts from the code-object metadata.
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_2106_12655_amd import build

HIPCC = build._hipcc()


@pytest.mark.skipif(shutil.which(HIPCC) is None and not os.path.exists(HIPCC),
                    reason="hipcc not available")
def test_direct_sum_variants_fit_two_waves_per_simd(tmp_path):
    src = os.path.join(build.CSRC, "lk_ds.hip")
    out = str(tmp_path / "lk_ds.s")
    cmd = [HIPCC, *build.HIPFLAGS, "--cuda-device-only", "-S", src, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    text = open(out).read()
    found = re.findall(r"\.agpr_count:\s+(\d+).*?\.name:\s+(\S*ds_persistent\S*).*?"
                       r"\.vgpr_count:\s+(\d+).*?\.vgpr_spill_count:\s+(\d+)", text, re.S)
    assert len(found) >= 16, "kernel metadata not found"
    for agpr, name, vgpr, spill in found:
        assert int(vgpr) + int(agpr) <= 256, (name, vgpr, agpr)
        assert int(spill) == 0, (name, spill)
