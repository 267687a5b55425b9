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
    a, b, c, d = (ctypes.c_size_t() for _ in range(4))
    assert srp.lib().srp_abi_sizes(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d)) == 0
    assert a.value == ctypes.sizeof(_lib.SrpOptions)
    assert b.value == ctypes.sizeof(_lib.SrpInfo)
    assert c.value == ctypes.sizeof(_lib.SrpRequest)
    assert d.value == ctypes.sizeof(_lib.SrpResult)


def test_request_footprint_host_only():
    """srp_request_footprint is host arithmetic: the solve workspace plus the
    staged copies, 0 for invalid sizes."""
    import paper_2106_12060_amd as srp
    from paper_2106_12060_amd import _lib
    L = srp.lib()
    req = _lib.SrpRequest()
    req.problem, req.n, req.dx, req.dy, req.k, req.sketch_size = srp.SRP_PROBLEM_CCA, 50000, 300, 200, 8, 1200
    req.lambda_x = req.lambda_y = 1e-3
    req.dtype = srp.SRP_F32
    srp.lib().srp_default_options(ctypes.byref(req.opt))
    ws = L.srp_cca_workspace_bytes(50000, 300, 200, 8, 1200, srp.SRP_F32, srp.SRP_COUNTSKETCH, srp.SRP_F32)
    assert ws > 0
    req.stage = srp.SRP_STAGE_NONE
    assert L.srp_request_footprint(ctypes.byref(req)) == ws
    req.stage = srp.SRP_STAGE_BF16
    f1 = L.srp_request_footprint(ctypes.byref(req))
    def al(b):   # the library places every buffer on a 256-byte boundary
        return (b + 255) // 256 * 256
    assert f1 - ws == al(2 * 50000 * 300) + al(2 * 50000 * 200)
    req.stage = srp.SRP_STAGE_BF16_FP8
    f2 = L.srp_request_footprint(ctypes.byref(req))
    ws8 = L.srp_cca_workspace_bytes(50000, 300, 200, 8, 1200, srp.SRP_F32, srp.SRP_COUNTSKETCH, srp.SRP_FP8E4M3)
    assert f2 == (al(2 * 50000 * 300) + al(2 * 50000 * 200) + al(50000 * 300) + al(50000 * 200)
                  + al(8 * 300) + al(8 * 200) + ws8)
    req.sketch_size = 100   # smaller than max(dx, dy): the Woodbury form, which needs lambda > 0
    lx, ly = req.lambda_x, req.lambda_y
    req.lambda_x = 0.0
    assert L.srp_request_footprint(ctypes.byref(req)) == 0
    req.lambda_x, req.lambda_y = lx, ly
    assert L.srp_request_footprint(ctypes.byref(req)) > 0
    assert L.srp_cca_workspace_bytes(50000, 300, 200, 8, 100, srp.SRP_F32, 0, srp.SRP_F32) > 0
    req.sketch_size = 0
    assert L.srp_request_footprint(ctypes.byref(req)) == 0
    assert L.srp_cca_workspace_bytes(50000, 300, 200, 8, 0, srp.SRP_F32, 0, srp.SRP_F32) == 0
    assert L.srp_lda_workspace_bytes(50000, 300, 10, 9, 1200, srp.SRP_F32, 0) > 0
    assert L.srp_lda_workspace_bytes(50000, 300, 10, 10, 1200, srp.SRP_F32, 0) == 0


def test_pass_kernel_choice_by_shape():
    """Host-side query of the pass kernel a shape takes (no device work):
    two FP32 views up to 1024 columns take the 4x4-block pass (k <= 10, or
    k <= 16 up to 512 columns), one FP32 view with k <= 20 the one-view
    4x4-block pass, other FP32 shapes within the LDS budget the streamed
    pass, the rest the register-staged one; out of limits: None."""
    srp = pytest.importorskip("paper_2106_12060_amd")
    q = srp.srp_gram_pass_kernel
    assert q("f32", "f32", 1000, 1000, 10) == "k_pass_quad"
    assert q("f32", "f32", 512, 500, 16) == "k_pass_quad"
    assert q("f32", "f32", 1000, 1000, 12) == "k_pass_dma"     # 4 slots: k <= 10
    assert q("f32", "f32", 2000, 0, 12) == "k_pass_quad1"      # one view
    assert q("f32", "f32", 2000, 0, 19) == "k_pass_quad1"
    assert q("f32", "f32", 2000, 0, 24) == "k_pass"            # one view, k > 20
    assert q("f32", "f32", 40, 30, 4) == "k_pass"              # views under 4 tiles
    assert q("f64", "f64", 300, 200, 8) == "k_pass"
    assert q("bf16", "bf16", 1000, 1000, 10) == "k_pass_bf"
    assert q("f32", "f32", 3000, 0, 4) is None                 # past the column limit
