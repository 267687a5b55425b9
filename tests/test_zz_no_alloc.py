"""The allocation-free CountSketch entry point (srp_countsketch_noalloc)
against srp_countsketch through the C ABI: the same bits on two calls in a
row, the second with a smaller input (the shared scratch keeps the first
call's contents), and its size limits."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda"


def _srp():
    import paper_2106_12060_amd as srp
    return srp


def _data(n, d, seed, dtype):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d)) * np.exp(rng.uniform(-3, 3, d))[None, :]
    return torch.from_numpy(X).to(DEV, dtype)


def test_noalloc_countsketch_matches_allocating_entry_point():
    srp = _srp()
    cases = [(200_003, 129, 5000, torch.float32, 101), (3001, 40, 300, torch.float64, 102)]
    outs = []
    # both calls enqueued back to back on one stream, then compared
    for n, d, s, dt, seed in cases:
        A = _data(n, d, seed, dt)
        out = torch.empty((s, d), dtype=torch.float64 if dt == torch.float64 else torch.float32, device=DEV)
        srp.srp_countsketch_noalloc(A, s, seed, out)
        outs.append((A, s, seed, out))
    torch.cuda.synchronize()
    for A, s, seed, out in outs:
        ref = srp.srp_countsketch(A, s, seed)
        assert torch.equal(out, ref), (A.shape, s)
    # and once more, largest first again after the small one
    A, s, seed, _ = outs[0]
    out = torch.empty((s, A.shape[1]), dtype=torch.float32, device=DEV)
    srp.srp_countsketch_noalloc(A, s, seed, out)
    torch.cuda.synchronize()
    assert torch.equal(out, srp.srp_countsketch(A, s, seed))


def test_noalloc_countsketch_rejects_sizes_past_its_scratch():
    srp = _srp()
    lib = srp.lib()
    A = torch.zeros((8, 4), dtype=torch.float32, device=DEV)
    out = torch.zeros((8, 4), dtype=torch.float32, device=DEV)
    p = ctypes.c_void_p
    rc = lib.srp_countsketch_noalloc(p(A.data_ptr()), srp.SRP_F32, (1 << 22) + 1, 4, 8, 1, p(out.data_ptr()), None)
    assert rc == srp.SRP_EINVAL
    assert b"scratch limit" in lib.srp_last_error()
    rc = lib.srp_countsketch_noalloc(p(A.data_ptr()), srp.SRP_F32, 8, 4, (1 << 20) + 1, 1, p(out.data_ptr()), None)
    assert rc == srp.SRP_EINVAL
    torch.cuda.synchronize()
