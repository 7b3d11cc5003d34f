"""Build liblk.so (HIP, gfx950) in-tree with hipcc.

Usage: ``python -m paper_2106_12655_amd.build`` or :func:`build` from Python.
The library lands next to this file so that it travels with the source tree.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "liblk.so")
SOURCES = ["lk_ds.hip", "lk_aux.hip", "lk_bh.hip", "lk_dz.hip", "lk_runtime.hip", "lk_server.hip"]
ARCH = os.environ.get("LK_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are disabled for every HIP translation unit: the
# compiler must not fuse scalar float work into v_pk_* forms.
HIPFLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I" + INCLUDE, "-Wno-unused-command-line-argument"]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    return "hipcc"


# The direct-sum kernels' assembly is kept (-save-temps) and fingerprinted, so
# that measurements recorded for one build of a kernel can be matched to the
# exact machine code they were taken on.
ISA_SOURCE = "lk_ds.hip"
ISA_FILE = os.path.join(HERE, "liblk.kernels.json")
ISA_KERNELS = "ds_persistent"


def _compile(src: str, obj: str) -> None:
    cmd = [_hipcc(), *HIPFLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    if src == ISA_SOURCE:
        cmd.append("-save-temps=obj")
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed on %s" % src)


def kernel_isa_digests(asm_text: str, match: str = ISA_KERNELS) -> dict:
    """SHA-256 (16 hex digits) of each kernel's gfx950 assembly whose symbol
    contains ``match``: the function body from its label to its end marker
    plus its .amdhsa_kernel descriptor (registers, LDS, scratch), without
    comments.  Local labels are renumbered by first appearance, so code added
    elsewhere in the file does not change a kernel's digest."""
    import hashlib
    import re
    lines = asm_text.splitlines()
    out = {}
    label = re.compile(r"\.L[A-Za-z_]*\d+(?:_\d+)?")
    for i, line in enumerate(lines):
        m = re.match(r"^(_Z\w+):", line)
        if not m or match not in m.group(1):
            continue
        sym = m.group(1)
        body = []
        for ln in lines[i + 1:]:
            if re.match(r"^\.Lfunc_end\d+:", ln):
                break
            body.append(ln)
        desc, inside = [], False
        for ln in lines:
            t = ln.strip()
            if t == ".amdhsa_kernel " + sym:
                inside = True
            if inside:
                desc.append(t)
                if t == ".end_amdhsa_kernel":
                    break
        names = {}

        def ren(mm):
            return ".L%d" % names.setdefault(mm.group(0), len(names))
        code = [ln.split(";", 1)[0].strip() for ln in body + desc]  # comments vary by build mode
        text = "\n".join(label.sub(ren, ln) for ln in code if ln)
        out[sym] = hashlib.sha256(text.encode()).hexdigest()[:16]
    return out


def _write_isa_digests(objdir: str) -> None:
    import json
    asm = os.path.join(objdir, ISA_SOURCE.replace(".hip", "") + "-hip-amdgcn-amd-amdhsa-%s.s" % ARCH)
    with open(asm) as fh:
        dig = kernel_isa_digests(fh.read())
    tmp = ISA_FILE + ".tmp%d" % os.getpid()
    with open(tmp, "w") as fh:
        json.dump({"arch": ARCH, "kernels": dig}, fh, indent=1, sort_keys=True)
    os.replace(tmp, ISA_FILE)


def build(verbose: bool = False) -> str:
    """Compile every HIP source and link liblk.so; returns its path."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, s.replace(".hip", ".o")) for s in SOURCES]
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        list(ex.map(lambda a: _compile(*a), zip(SOURCES, objs)))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [_hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of liblk.so failed")
    os.replace(tmp, LIB)
    _write_isa_digests(objdir)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
