"""The C ABI library loads here (no GPU) and exports what include/lk.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lk.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lk_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("lk_build_pairs", "lk_direct_sum", "lk_verify", "lk_create", "lk_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2106_12655_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("liblk.so not built; run python -m paper_2106_12655_amd.build")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n
    assert sorted(_lib.EXPORTS) == _declared()


def test_header_constants_match_binding():
    from paper_2106_12655_amd import _lib
    src = open(HEADER).read()
    pairs = {
        "LK_FLAG_REFIT": _lib.FLAG_REFIT, "LK_FLAG_AMBIGUOUS": _lib.FLAG_AMBIGUOUS,
        "LK_FLAG_NONFINITE": _lib.FLAG_NONFINITE, "LK_FLAG_BADPAIR": _lib.FLAG_BADPAIR,
        "LK_FLAG_BADLOOP": _lib.FLAG_BADLOOP, "LK_EINVAL": _lib.EINVAL,
        "LK_ECAPACITY": _lib.ECAPACITY, "LK_MIXED": _lib.MIXED, "LK_PLAIN_F64": _lib.PLAIN_F64,
        "LK_OPT_TIMING": _lib.OPT_TIMING, "LK_OPT_ATAN": _lib.OPT_ATAN,
    }
    for name, val in pairs.items():
        m = re.search(r"\b%s\s*=\s*(-?\d+)" % name, src)
        assert m, name
        assert int(m.group(1)) == val, name


def test_no_device_means_clear_error():
    # without a GPU the binding refuses loudly instead of computing elsewhere
    import torch
    import paper_2106_12655_amd as lk
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError):
        lk.Context(0)


def test_status_codes_without_device():
    # lk_create on a machine without a HIP device fails with a status, no crash
    import torch
    from paper_2106_12655_amd import _lib
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.lk_create(ctypes.byref(h), 0) != _lib.OK
    assert lib.lk_set_option(None, 1, 5) == _lib.EINVAL
