"""Parity at the benchmark shapes that can fail on a single wrong entry.
The inputs hold a few +-1 entries per row and the directions small
integers, so every FP32 (and BF16) sum the kernels form is an exact
integer, and the SRHT's 1/sqrt(s) is a power of two (s a power of 4): the
kernels must then reproduce the FP64 oracle bit for bit, at any n.  A
dropped row block, a sign error or a wrong index changes some output."""
import numpy as np
import pytest

import synth
from oracle import sketch as osk, stiefel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda"


def _srp():
    import paper_2106_12060_amd as srp
    return srp


def _int_dirs(d, k, seed):
    return np.random.default_rng(seed).integers(-2, 3, size=(d, k)).astype(np.float64)


@pytest.mark.parametrize("n,d0,d1,k,dt,comp,kernel", [
    (200_000, 1000, 1000, 10, "f32", "f32", "k_pass_quad"),       # the CCA benchmark pass
    (100_000, 2000, 0, 19, "f32", "f32", "k_pass_quad1"),         # the FDA benchmark pass
    (200_000, 1000, 1000, 10, "bf16", "bf16", "k_pass_bf"),       # the BF16 form's pass
    (100_000, 2000, 0, 24, "f32", "f32", "k_pass"),               # one view, k > 20
])
def test_pass_exact_at_benchmark_shape(n, d0, d1, k, dt, comp, kernel):
    srp = _srp()
    assert srp.srp_gram_pass_kernel(dt, comp, d0, d1, k) == kernel
    tdt = {"f32": torch.float32, "bf16": torch.bfloat16}[dt]
    A0 = synth.sparse_signs(n, d0, 3, seed=1 + d0)
    W0 = _int_dirs(d0, k, 2)
    if d1:
        A1 = synth.sparse_signs(n, d1, 3, seed=3 + d1)
        W1 = _int_dirs(d1, k, 4)
        J, _ = stiefel.data_products(A0, W0, A1, W1)
        G0, G1 = srp.srp_gram_pass(torch.from_numpy(A0).to(DEV, tdt), torch.from_numpy(W0).to(DEV),
                                   torch.from_numpy(A1).to(DEV, tdt), torch.from_numpy(W1).to(DEV), compute=comp)
        got = [G0.cpu().numpy(), G1.cpu().numpy()]
    else:
        J, _ = stiefel.data_products(A0, W0)
        G0, _ = srp.srp_gram_pass(torch.from_numpy(A0).to(DEV, tdt), torch.from_numpy(W0).to(DEV), compute=comp)
        got = [G0.cpu().numpy()]
    for g, ref in zip(got, J):
        assert np.abs(ref).max() < 2.0 ** 24           # exact in FP32 whatever the order
        np.testing.assert_array_equal(g, ref)


def test_srht_exact_at_benchmark_shape():
    """n = 200000 (n' = 2^18), d = 1000, s = 4096: 1/sqrt(s) = 2^-6.  Only
    every 16th column is nonzero (the oracle transforms those 64), so the
    other outputs must be exactly zero."""
    srp = _srp()
    n, d, s, seed = 200_000, 1000, 4096, 12061
    cols = np.arange(0, d, 16)
    X = synth.sparse_signs(n, d, 2, seed=5, cols=cols)
    out = srp.srp_srht(torch.from_numpy(X).to(DEV), s, seed).double().cpu().numpy()
    n_pad = osk.srht_padded_rows(n)
    ref = osk.srht_apply(X[:, cols].astype(np.float64), osk.srht_signs(n_pad, seed),
                         osk.srht_rows(n_pad, s, seed), s)
    np.testing.assert_array_equal(out[:, cols], ref)
    mask = np.ones(d, bool)
    mask[cols] = False
    assert not np.any(out[:, mask])


@pytest.mark.parametrize("n,d,s,per_row,col_step", [
    (200_000, 1000, 4000, 3, 7),   # the CCA benchmark sketch: B = 128, two row ranges per column slice
    (200_000, 1000, 1024, 3, 7),   # B = 64 and 1/sqrt(s) = 2^-5: bit for bit
    (50_000, 100, 3000, 4, 1),     # last column slice holds 4 of its 16 columns
    (140_000, 36, 2000, 4, 1),     # B = 64, three column slices: many row ranges
    (3_000, 12, 2500, 4, 1),       # n' = 4096, one column slice, one row range
    (700, 16, 1024, 2, 1),         # under four blocks per row range
])
def test_srht_one_read_exact(n, d, s, per_row, col_step):
    """The one-read SRHT (FP32 data, d a multiple of 4, B = 64 or 128, that
    is s from 1024 to 4095) on +-1 data: every partial sum is an exact
    integer, so the only rounding left is the final 1/sqrt(s) (none when s
    is a power of 4).  Columns outside the chosen set must stay zero."""
    srp = _srp()
    seed = 900 + s + n
    cols = np.arange(0, d, col_step)
    X = synth.sparse_signs(n, d, per_row, seed=seed, cols=cols)
    print("srht one-read exact", n, d, s, flush=True)
    out = srp.srp_srht(torch.from_numpy(X).to(DEV), s, seed).double().cpu().numpy()
    n_pad = osk.srht_padded_rows(n)
    ref = osk.srht_apply(X[:, cols].astype(np.float64), osk.srht_signs(n_pad, seed),
                         osk.srht_rows(n_pad, s, seed), s)
    got = out[:, cols]
    if (s & (s - 1)) == 0 and (s.bit_length() - 1) % 2 == 0:
        np.testing.assert_array_equal(got, ref)
    else:
        assert np.all(np.abs(got - ref) <= 2.0 ** -22 * np.abs(ref))
    mask = np.ones(d, bool)
    mask[cols] = False
    assert not np.any(out[:, mask])


def test_countsketch_exact_at_benchmark_shape():
    srp = _srp()
    n, d, s, seed = 200_000, 1000, 4000, 12062
    cols = np.arange(3, d, 16)
    X = synth.sparse_signs(n, d, 2, seed=6, cols=cols)
    out = srp.srp_countsketch(torch.from_numpy(X).to(DEV), s, seed).double().cpu().numpy()
    h, g = osk.countsketch_hash(n, s, seed)
    ref = osk.countsketch_apply(X[:, cols].astype(np.float64), h, g, s)
    np.testing.assert_array_equal(out[:, cols], ref)
    mask = np.ones(d, bool)
    mask[cols] = False
    assert not np.any(out[:, mask])
