"""The build's fingerprint of kernel assembly (paper_2106_12655_amd.build):
comments and the numbering of local labels do not change it, a changed
instruction or kernel descriptor does.  bench.py relies on it to tell whether
recorded HBM counters belong to the kernel being measured."""
from paper_2106_12655_amd import build as B

ASM = """\
\t.text
\t.globl\t_ZN2lk12_GLOBAL__N_113ds_persistentIffLi2ELi4EEEvNS_6DsArgsE
_ZN2lk12_GLOBAL__N_113ds_persistentIffLi2ELi4EEEvNS_6DsArgsE: ; @k
; %bb.0:
\ts_load_dwordx2 s[0:1], s[4:5], 0x0
.LBB{n}_1:                               ; %loop
\tv_fmac_f32_e32 v1, v2, v3
\ts_cbranch_scc1 .LBB{n}_1
\ts_endpgm
.Lfunc_end{n}:
\t.amdhsa_kernel _ZN2lk12_GLOBAL__N_113ds_persistentIffLi2ELi4EEEvNS_6DsArgsE
\t\t.amdhsa_next_free_vgpr {v}
\t.end_amdhsa_kernel
"""


def _digest(n=7, v=124, extra=""):
    d = B.kernel_isa_digests(ASM.format(n=n, v=v).replace("\ts_endpgm", extra + "\ts_endpgm"))
    assert len(d) == 1
    return next(iter(d.values()))


def test_fingerprint_ignores_labels_and_comments():
    assert _digest(7) == _digest(42)
    assert _digest(7) == B.kernel_isa_digests(
        ASM.format(n=7, v=124).replace("; %loop", "; %Flow2881"))[
            "_ZN2lk12_GLOBAL__N_113ds_persistentIffLi2ELi4EEEvNS_6DsArgsE"]


def test_fingerprint_sees_code_and_descriptor():
    assert _digest(7) != _digest(7, extra="\tv_add_f32_e32 v1, v1, v1\n")
    assert _digest(7, v=124) != _digest(7, v=128)
