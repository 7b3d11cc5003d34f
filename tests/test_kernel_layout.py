"""Placement of the FP32 direct-sum kernel's hot loops (no GPU needed).

On the MI355X the time of the packed FP32 kernel (R = 4, arctangent form 2)
depends on where its innermost walk loops start, with the same instructions:

* the loop of packed small pairs (chainmail): a loop header at 4 (mod 8)
  bytes into the kernel measured 0.457-0.469 ms on the chainmail workload and
  one at 0 (mod 8) bytes 0.486-0.505 ms (a sweep of 0-15 leading s_nop
  instructions on one box);
* the loop of big items (knit, long pairs): at 12 (mod 32) bytes it measured
  570 ms per knit call, at 4 (mod 32) 598 ms, at 16 (mod 32) 645 ms and
  620-627 ms elsewhere (a sweep of 0-16 s_nop instructions placed before
  it, which moves it alone).

The check compiles the kernel source for gfx950 with the build's flags,
disassembles the device code object and checks every innermost loop of the
walk (the loops with 20 square roots: four steps of R + 1 vertices).  In
address order the three are the packed small pairs, the whole-wave small
pairs and the big items.  An edit that moves them onto a slow placement
fails here instead of showing up as a slower bench.
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_2106_12655_amd import build

HIPCC = build._hipcc()
OBJDUMP = "/opt/rocm/llvm/bin/llvm-objdump"
KERNEL = "_ZN2lk12_GLOBAL__N_113ds_persistentIffLi2ELi4ELb1EEEvNS_6DsArgsE"


def _walk_loops(obj: str):
    d = subprocess.run([OBJDUMP, "-d", "--disassemble-symbols=" + KERNEL, obj],
                       capture_output=True, text=True).stdout.split("\n")
    ins = []
    for line in d:
        m = re.match(r"\s+(\S.*?)\s+//\s+([0-9A-F]+):", line)
        if m:
            ins.append((int(m.group(2), 16), m.group(1)))
    assert ins, "kernel not found in the device code"
    start = ins[0][0]
    index = {a: i for i, (a, _) in enumerate(ins)}
    heads = set()
    for k, (a, t) in enumerate(ins):
        m = re.search(r"s_c?branch\w* (\d+)$", t)
        if not m:
            continue
        off = int(m.group(1))
        off = off - 65536 if off >= 32768 else off
        tgt = a + 4 + 4 * off
        if tgt < a and tgt in index:
            body = ins[index[tgt]:k + 1]
            if sum(1 for _, x in body if x.startswith("v_sqrt_f32")) == 20:
                heads.add(tgt - start)
    return sorted(heads)


@pytest.mark.skipif((shutil.which(HIPCC) is None and not os.path.exists(HIPCC))
                    or not os.path.exists(OBJDUMP), reason="hipcc or llvm-objdump not available")
def test_walk_loop_placement(tmp_path):
    src = os.path.join(build.CSRC, "lk_ds.hip")
    obj = str(tmp_path / "lk_ds_device.o")
    cmd = [HIPCC, *build.HIPFLAGS, "--cuda-device-only", "--no-gpu-bundle-output", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    heads = _walk_loops(obj)
    assert len(heads) == 3, heads  # packed small pairs, whole-wave small pairs, big items
    assert all(h % 8 == 4 for h in heads), [hex(h) for h in heads]
    assert heads[2] % 32 == 12, [hex(h) for h in heads]
