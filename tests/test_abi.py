"""The C-ABI library loads and exports every entry point include/fslbm.h
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fslbm.h")
LIB = os.path.join(ROOT, "paper_2207_14496_amd", "libfslbm.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fslbm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("fslbm_init", "fslbm_step", "fslbm_refill_scheme", "fslbm_read_fields"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfslbm.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfslbm.so not built")
def test_binding_symbol_list_matches_header():
    from paper_2207_14496_amd import fslbm
    assert sorted(fslbm.SYMBOLS) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfslbm.so not built")
def test_workspace_bytes_and_validation_on_host():
    """Parameter validation runs on the host (no device needed)."""
    from paper_2207_14496_amd import fslbm
    p = fslbm.Params(64, 128, 1, periodic=(1, 0, 1), omega=1.8)
    n = fslbm.workspace_bytes(p)
    assert n >= 64 * 128 * 19 * 8
    p32 = fslbm.Params(64, 128, 1, periodic=(1, 0, 1), omega=1.8, storage=fslbm.F32)
    assert fslbm.workspace_bytes(p32) < n
    for bad in (dict(omega=2.0), dict(omega=0.0), dict(nx=0), dict(storage=7), dict(refill=9),
                dict(collision=3), dict(batch=0)):
        q = fslbm.Params(64, 128, 1, periodic=(1, 0, 1))
        for k, v in bad.items():
            setattr(q, k, v)
        with pytest.raises(fslbm.FslbmError) as e:
            fslbm.workspace_bytes(q)
        assert e.value.status == fslbm.EINVAL
