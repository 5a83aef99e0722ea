"""The C-ABI library loads and exports every entry point include/apx.h declares (CPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "apx.h")
LIB = os.path.join(ROOT, "paper_2308_01957_amd", "libapx.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(apx_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_hot_path():
    names = declared()
    for n in ["apx_render", "apx_chi2", "apx_jacobian", "apx_jtwj", "apx_lm_step", "apx_chi2_grad",
              "apx_render_vjp"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libapx.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    from paper_2308_01957_amd import apx
    assert sorted(apx.EXPORTS) == declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libapx.so not built")
def test_status_strings_and_struct_sizes():
    from paper_2308_01957_amd import apx
    lib = apx.load_library()
    assert lib.apx_status_string(apx.APX_OK) == b"ok"
    assert b"domain" in lib.apx_status_string(apx.APX_E_DOMAIN)
    assert lib.apx_version().startswith(b"apx")
    # C layouts (x86-64, checked against the header with gcc): image 80 B, comp 112 B, state 64 B
    assert ctypes.sizeof(apx.ImageDesc) == 80
    assert ctypes.sizeof(apx.CompDesc) == 112
    assert ctypes.sizeof(apx.LMState) == 64
