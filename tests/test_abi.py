"""The C-ABI library loads and exports every entry point the header
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "srp.h")
LIB = os.path.join(ROOT, "paper_2106_12060_amd", "libsrp.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "for", "return")))


def test_header_declares_entry_points():
    names = declared_functions()
    for expected in ["cca_solve", "lda_solve", "srp_countsketch", "srp_srht", "srp_sketch_factor",
                     "srp_gram_pass", "srp_default_options", "srp_last_error"]:
        assert expected in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsrp.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsrp.so not built")
def test_binding_signatures_cover_header():
    import paper_2106_12060_amd as srp
    assert set(declared_functions()) == set(srp.exported_symbols())


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsrp.so not built")
def test_default_options_host_only():
    import paper_2106_12060_amd as srp
    o = srp.srp_default_options()
    assert o.max_iter == 1000 and o.sketch == srp.SRP_COUNTSKETCH
    o2 = srp.srp_default_options(sketch="srht", max_iter=7)
    assert o2.sketch == srp.SRP_SRHT and o2.max_iter == 7


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsrp.so not built")
def test_struct_layouts_match_library():
    import paper_2106_12060_amd as srp
    from paper_2106_12060_amd import _lib
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    assert srp.lib().srp_abi_sizes(ctypes.byref(a), ctypes.byref(b)) == 0
    assert a.value == ctypes.sizeof(_lib.SrpOptions)
    assert b.value == ctypes.sizeof(_lib.SrpInfo)
