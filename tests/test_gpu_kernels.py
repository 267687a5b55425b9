"""Kernel-level parity of the HIP library (through the C ABI) against the
FP64 oracle's definitions, on seeded inputs spanning several tiles and a
ragged tail.  Floating-point bounds come from the standard summation
bound |fl(sum a_i) - sum a_i| <= (m - 1) u sum |a_i| with the oracle
computing the magnitudes; integer work (hash buckets, sampled rows) is
bit-exact."""
import numpy as np
import pytest

import synth
from oracle import sketch as osk, stiefel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda"
U32, U64 = 2.0 ** -24, 2.0 ** -53
TORCH_DT = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}


def _srp():
    import paper_2106_12060_amd as srp
    return srp


def quantised(X, dt):
    """Device tensor of X in dtype dt and the exact FP64 values it holds."""
    t = torch.from_numpy(np.ascontiguousarray(X)).to(DEV, TORCH_DT[dt])
    return t, t.double().cpu().numpy()


def rand_data(n, d, seed, decades=2.0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, d)) * synth.column_scales(d, decades, True)[None, :]


# ------------------------------------------------------------ CountSketch
@pytest.mark.parametrize("n,d,s,dt", [(1000, 37, 50, "f64"), (5003, 300, 700, "f32"),
                                      (777, 5, 13, "f32"), (2048, 70, 100, "bf16"),
                                      (1, 3, 1, "f64"), (4096, 1, 4096, "f32")])
def test_countsketch_matches_definition(n, d, s, dt):
    srp = _srp()
    seed = 1000 + n + s
    X, Xq = quantised(rand_data(n, d, seed), dt)
    out = srp.srp_countsketch(X, s, seed).double().cpu().numpy()
    h, g = osk.countsketch_hash(n, s, seed)
    ref = osk.countsketch_apply(Xq, h, g, s)
    mag = osk.countsketch_apply(np.abs(Xq), h, np.abs(g), s)
    m = np.bincount(h, minlength=s).astype(float)[:, None]
    u = U64 if dt == "f64" else U32
    bound = np.maximum(m - 1, 0) * u * mag + 1e-300
    assert np.all(np.abs(out - ref) <= bound)


def test_countsketch_bitwise_reproducible():
    srp = _srp()
    X, _ = quantised(rand_data(20000, 130, 7), "f32")
    a = srp.srp_countsketch(X, 900, 99)
    b = srp.srp_countsketch(X, 900, 99)
    assert torch.equal(a, b)


# ------------------------------------------------------------------ SRHT
@pytest.mark.parametrize("n,s", [(2000, 240), (200_000, 4000), (13, 16), (1, 2), (1 << 12, 1 << 12),
                                 (70_000, 5)])
def test_srht_rows_bit_exact(n, s):
    srp = _srp()
    seed = 31 + n
    rows = srp.srp_srht_rows(n, s, seed).cpu().numpy()
    ref = osk.srht_rows(osk.srht_padded_rows(n), s, seed)
    np.testing.assert_array_equal(rows, ref)


@pytest.mark.parametrize("n,d,s,dt", [(3000, 40, 300, "f64"), (3001, 129, 257, "f32"),
                                      (700, 16, 1024, "f32"), (5000, 33, 64, "bf16"),
                                      (140000, 37, 512, "f32"), (600000, 3, 256, "f32"),
                                      (70000, 70, 400, "f64")])
def test_srht_matches_definition(n, d, s, dt):
    srp = _srp()
    seed = 77 + d
    X, Xq = quantised(rand_data(n, d, seed), dt)
    out = srp.srp_srht(X, s, seed).double().cpu().numpy()
    n_pad = osk.srht_padded_rows(n)
    D = osk.srht_signs(n_pad, seed)
    rows = osk.srht_rows(n_pad, s, seed)
    ref = osk.srht_apply(Xq, D, rows, s)
    mag = np.abs(Xq).sum(axis=0)[None, :] / np.sqrt(s)
    u = U64 if dt == "f64" else U32
    levels = int(np.log2(n_pad)) + (n_pad >> ((int(np.log2(n_pad)) + 1) // 2))
    assert np.all(np.abs(out - ref) <= levels * u * mag + 1e-300)


def test_srht_full_sample_is_isometry():
    srp = _srp()
    X, Xq = quantised(rand_data(1000, 12, 5), "f64")
    SX = srp.srp_srht(X, 1024, 5).cpu().numpy()
    np.testing.assert_allclose(SX.T @ SX, Xq.T @ Xq, rtol=1e-12, atol=1e-10)


# ------------------------------------------------------- metric factor R
@pytest.mark.parametrize("s,d,dt,lam", [(500, 120, "f64", 1e-3), (900, 200, "f32", 1e-2),
                                        (64, 64, "f64", 0.5), (300, 65, "f32", 1e-4),
                                        # 128 x 128 Gram tiles with ragged edges and a split contraction
                                        # (FP32 rows of 16-byte multiples: load-to-LDS stages; else
                                        # register-staged)
                                        (1300, 300, "f32", 1e-3), (2100, 520, "f64", 1e-2),
                                        (1100, 258, "f32", 1e-3)])
def test_sketch_factor_matches_cholesky(s, d, dt, lam):
    srp = _srp()
    SA, SAq = quantised(rand_data(s, d, 11 + d, decades=1.0), dt)
    R, Rinv = srp.srp_sketch_factor(SA, lam)
    R = R.cpu().numpy()
    Rinv = Rinv.cpu().numpy()
    ref = osk.sketch_factor(SAq, lam)
    assert np.allclose(np.tril(R, -1), 0.0) and np.all(np.diag(R) > 0)
    G = SAq.T @ SAq + lam * np.eye(d)
    kappa = np.linalg.cond(G)
    assert np.max(np.abs(R.T @ R - G)) <= 1e-13 * d * np.max(np.abs(G))
    assert np.max(np.abs(R - ref)) <= 1e-14 * kappa * np.max(np.abs(ref))
    np.testing.assert_allclose(Rinv @ R, np.eye(d), atol=1e-13 * np.sqrt(kappa) * d)


@pytest.mark.parametrize("s,d", [(4000, 1000), (8000, 2000)])
def test_sketch_factor_at_solver_sizes(s, d):
    """The factor at the sizes the solvers use (16 and 32 diagonal blocks of
    64 columns, 128 x 128 Gram tiles over a split contraction): R^T R equals
    the sketched Gram plus lambda I to FP64 rounding, and R^-1 R = I."""
    srp = _srp()
    SA, SAq = quantised(rand_data(s, d, 300 + d, decades=2.0), "f32")
    lam = 1e-4
    R, Rinv = srp.srp_sketch_factor(SA, lam)
    R = R.cpu().numpy()
    Rinv = Rinv.cpu().numpy()
    assert np.allclose(np.tril(R, -1), 0.0) and np.all(np.diag(R) > 0)
    assert np.allclose(np.tril(Rinv, -1), 0.0)
    G = SAq.T @ SAq + lam * np.eye(d)
    assert np.max(np.abs(R.T @ R - G)) <= 1e-13 * d * np.max(np.abs(G))
    ref = osk.sketch_factor(SAq, lam)
    w = np.linalg.eigvalsh(G)
    kappa = w[-1] / w[0]
    assert np.max(np.abs(R - ref)) <= 1e-14 * kappa * np.max(np.abs(ref))
    np.testing.assert_allclose(Rinv @ R, np.eye(d), atol=1e-13 * np.sqrt(kappa) * d)


def test_sketch_factor_reports_not_spd():
    srp = _srp()
    SA = torch.zeros((40, 8), dtype=torch.float64, device=DEV)
    with pytest.raises(srp.SrpError) as e:
        srp.srp_sketch_factor(SA, 0.0)
    assert e.value.code == srp.SRP_ENOTSPD


# ----------------------------------------------------------- data pass
@pytest.mark.parametrize("n,d0,d1,k,dt,comp", [(3000, 70, 45, 7, "f64", "f64"), (5001, 130, 200, 10, "f32", "f32"),
                                               (4097, 300, 0, 19, "f32", "f32"), (999, 17, 33, 16, "f32", "f64"),
                                               (2000, 1000, 1000, 10, "f32", "f32"), (64, 5, 3, 1, "f64", "f64"),
                                               (3333, 2000, 0, 19, "f32", "f32"), (1500, 90, 60, 5, "bf16", "f32"),
                                               (1003, 1000, 0, 10, "f32", "f32"), (777, 260, 516, 16, "f32", "f32"),
                                               (130, 66, 70, 3, "f32", "f32"), (5, 64, 0, 4, "f32", "f32"),
                                               (40001, 2000, 0, 12, "f32", "f32"),
                                               (3000, 120, 96, 8, "bf16", "bf16"), (999, 40, 0, 5, "bf16", "bf16")])
def test_gram_pass_matches_products(n, d0, d1, k, dt, comp):
    """Fused pass against the FP64 products of the same (quantised) data.
    compute="bf16" on views narrower than the matrix-core pass's row chunk
    runs the FP32-arithmetic pass on the BF16 data, hence the FP32 bound."""
    srp = _srp()
    rng = np.random.default_rng(n + d0)
    A0, A0q = quantised(rand_data(n, d0, n), dt)
    W0 = rng.standard_normal((d0, k))
    W0t = torch.from_numpy(W0).to(DEV)
    if d1:
        A1, A1q = quantised(rand_data(n, d1, n + 1), dt)
        W1 = rng.standard_normal((d1, k))
        W1t = torch.from_numpy(W1).to(DEV)
        J, Jabs = stiefel.data_products(A0q, W0, A1q, W1)
        G0, G1 = srp.srp_gram_pass(A0, W0t, A1, W1t, compute=comp)
        got = [G0.cpu().numpy(), G1.cpu().numpy()]
    else:
        J, Jabs = stiefel.data_products(A0q, W0)
        G0, _ = srp.srp_gram_pass(A0, W0t, compute=comp)
        got = [G0.cpu().numpy()]
    u = U64 if comp == "f64" else U32
    for g, ref, mag in zip(got, J, Jabs):
        bound = (d0 + d1 + n + 2) * u * mag + 1e-300
        assert np.all(np.abs(g - ref) <= bound), np.max(np.abs(g - ref) / bound)


# Two FP32 views of at most 1024 columns each take the 4x4-block pass: every
# tile-slot count (at most 32 / 64 tiles per view), every k class
# (ceil(k / 2) = 1 .. 8 with 2 slots, .. 6 with 4), 16-byte and 4-byte row
# loads (columns not a multiple of 4), views of unequal width (tiles without
# work), fewer rows than one block, ragged last blocks.
@pytest.mark.parametrize("n,d0,d1,k", [(3001, 512, 500, 1), (3001, 512, 500, 3), (3001, 512, 500, 5),
                                       (3001, 512, 500, 8), (3001, 512, 500, 9), (3001, 512, 500, 12),
                                       (3001, 512, 500, 13), (3001, 512, 500, 16),
                                       (2500, 1000, 1024, 2), (2500, 1000, 1024, 7), (2500, 1000, 1024, 10),
                                       (2500, 1000, 1024, 11), (1777, 1001, 333, 10), (7, 300, 200, 6),
                                       (4099, 64, 1000, 11), (513, 70, 90, 4)])
def test_gram_pass_4x4_blocks(n, d0, d1, k):
    srp = _srp()
    rng = np.random.default_rng(7 * n + k)
    A0, A0q = quantised(rand_data(n, d0, n + k), "f32")
    A1, A1q = quantised(rand_data(n, d1, n + k + 1), "f32")
    W0 = rng.standard_normal((d0, k))
    W1 = rng.standard_normal((d1, k))
    J, Jabs = stiefel.data_products(A0q, W0, A1q, W1)
    G0, G1 = srp.srp_gram_pass(A0, torch.from_numpy(W0).to(DEV), A1, torch.from_numpy(W1).to(DEV), compute="f32")
    for g, ref, mag in zip([G0.cpu().numpy(), G1.cpu().numpy()], J, Jabs):
        assert g.shape == ref.shape
        bound = (d0 + d1 + n + 2) * U32 * mag + 1e-300
        assert np.all(np.abs(g - ref) <= bound), np.max(np.abs(g - ref) / bound)


# One FP32 view of at most 2048 columns with k <= 20 takes the one-view
# 4x4-block pass: 4 and 8 tile slots, one to five direction-column groups
# (whole 16-column P tiles and 4-column remainders), 4-byte row loads,
# fewer rows than one block, the widest view.
@pytest.mark.parametrize("n,d,k", [(3001, 1000, 1), (3001, 1000, 4), (3001, 1000, 7), (3001, 1000, 12),
                                   (3001, 1000, 16), (3001, 1000, 19), (3001, 1000, 20), (2500, 2000, 3),
                                   (2500, 2000, 9), (2500, 2000, 13), (2500, 2000, 19), (2500, 2000, 20),
                                   (1777, 1001, 10), (7, 300, 6), (4099, 2048, 17), (513, 70, 5)])
def test_gram_pass_4x4_blocks_one_view(n, d, k):
    srp = _srp()
    rng = np.random.default_rng(11 * n + k)
    A, Aq = quantised(rand_data(n, d, n + 3 * k), "f32")
    W = rng.standard_normal((d, k))
    J, Jabs = stiefel.data_products(Aq, W)
    G, _ = srp.srp_gram_pass(A, torch.from_numpy(W).to(DEV), compute="f32")
    g, ref, mag = G.cpu().numpy(), J[0], Jabs[0]
    assert g.shape == ref.shape
    bound = (d + n + 2) * U32 * mag + 1e-300
    assert np.all(np.abs(g - ref) <= bound), np.max(np.abs(g - ref) / bound)


# ---------------------------------------------------------- staging
def test_stage_bf16_bit_exact():
    from oracle import quant
    srp = _srp()
    rng = np.random.default_rng(11)
    X = (rng.standard_normal((1037, 129)) * np.exp(rng.uniform(-20, 20, (1037, 129)))).astype(np.float32)
    X[0, :5] = [0.0, -0.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -3.0e38]
    # infinities, NaNs whose payload sits only in the low 16 bits (they must
    # stay NaN), FLT_MAX (overflows to inf), ties at the largest BF16 values
    # and subnormal ties
    special = np.array([0x7F800000, 0xFF800000, 0x7F800001, 0xFF80FFFF, 0x7FC00000, 0x7F7FFFFF,
                        0x7F7F7FFF, 0x7F7F8000, 0x7F7E8000, 0x00008000, 0x00018000, 0x80000001],
                       dtype=np.uint32).view(np.float32)
    X[1, :special.size] = special
    got = srp.srp_stage_bf16(torch.from_numpy(X).to(DEV)).float().cpu().numpy()
    np.testing.assert_array_equal(got.view(np.uint32), quant.bf16_round(X).view(np.uint32))


@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_stage_fp8_bit_exact(dt):
    from oracle import quant
    srp = _srp()
    rng = np.random.default_rng(12)
    n, d = 3001, 67
    X = (rng.standard_normal((n, d)) * np.exp(rng.uniform(-12, 12, d))[None, :]).astype(np.float32)
    X[:, 5] = 0.0                                   # empty column: scale 1
    X[7, 6] = 448.0 * 2.0 ** 3                      # column max exactly 448 2^3
    X[:, 8] = np.float32(2.0 ** -9) * rng.integers(-20, 20, n)   # subnormal grid and ties
    Xt = torch.from_numpy(X).to(DEV)
    if dt == "bf16":
        Xt = Xt.to(torch.bfloat16)
        X = Xt.float().cpu().numpy()
    codes, scales = srp.srp_stage_fp8(Xt)
    ref_codes, ref_scales = quant.fp8_stage(X.astype(np.float64))
    np.testing.assert_array_equal(scales.cpu().numpy(), ref_scales)
    np.testing.assert_array_equal(codes.cpu().numpy(), ref_codes)


@pytest.mark.parametrize("kind", ["countsketch", "srht"])
def test_sketch_of_fp8_codes(kind):
    """Sketch of the FP8-staged matrix = sketch of the decoded codes times the
    column scales (exact: powers of two), against the oracle's sketch of the
    unstaged-and-rescaled matrix."""
    from oracle import quant
    srp = _srp()
    rng = np.random.default_rng(13)
    n, d, s = 5000, 40, 256
    X = rng.standard_normal((n, d)).astype(np.float32) * 3.0
    codes, scales = srp.srp_stage_fp8(torch.from_numpy(X).to(DEV))
    fn = srp.srp_countsketch if kind == "countsketch" else srp.srp_srht
    out = fn(codes, s, 99).double().cpu().numpy() * scales.cpu().numpy()[None, :]
    Xq = quant.fp8_unstage(codes.cpu().numpy(), scales.cpu().numpy())
    ref = osk.sketch(Xq, kind, s, 99)
    mag = np.abs(osk.sketch(np.abs(Xq), kind, s, 99)) + np.abs(Xq).sum(axis=0)[None, :] / np.sqrt(s)
    assert np.all(np.abs(out - ref) <= 40 * U32 * mag)


@pytest.mark.parametrize("n,d0,d1,k", [(3000, 520, 600, 10), (2001, 130, 200, 10), (1500, 1000, 0, 16),
                                       (777, 264, 130, 3)])
def test_gram_pass_bf16_products(n, d0, d1, k):
    """BF16 matrix-core pass against the oracle on the same quantised
    operands: BF16 data, BF16 direction, P = A W rounded to BF16 before
    A^T P.  The bound allows P's rounding to land one BF16 ulp apart (the
    kernel rounds an FP32 sum) plus FP32 accumulation."""
    from oracle import quant
    srp = _srp()
    rng = np.random.default_rng(n + d0 + 7)
    A0 = torch.from_numpy(rand_data(n, d0, n)).to(DEV).to(torch.bfloat16)
    A0q = A0.float().cpu().numpy().astype(np.float64)
    W0 = rng.standard_normal((d0, k))
    W0q = quant.bf16_round(W0.astype(np.float32)).astype(np.float64)
    blocks = [(A0, A0q, W0, W0q)]
    if d1:
        A1 = torch.from_numpy(rand_data(n, d1, n + 1)).to(DEV).to(torch.bfloat16)
        A1q = A1.float().cpu().numpy().astype(np.float64)
        W1 = rng.standard_normal((d1, k))
        W1q = quant.bf16_round(W1.astype(np.float32)).astype(np.float64)
        blocks.append((A1, A1q, W1, W1q))
    P = np.concatenate([Aq @ Wq for _, Aq, _, Wq in blocks], axis=1)
    Pq = quant.bf16_round(P.astype(np.float32)).astype(np.float64)
    if d1:
        G0, G1 = srp.srp_gram_pass(A0, torch.from_numpy(W0).to(DEV), A1, torch.from_numpy(W1).to(DEV),
                                   compute="bf16")
        got = [G0.cpu().numpy(), G1.cpu().numpy()]
    else:
        G0, _ = srp.srp_gram_pass(A0, torch.from_numpy(W0).to(DEV), compute="bf16")
        got = [G0.cpu().numpy()]
    for g, (_, Aq, _, _) in zip(got, blocks):
        ref = Aq.T @ Pq
        bound = 2.0 ** -7 * (np.abs(Aq).T @ np.abs(P)) + (Aq.shape[1] + n) * U32 * (np.abs(Aq).T @ np.abs(Pq))
        assert np.all(np.abs(g - ref) <= bound + 1e-300), np.max(np.abs(g - ref) / (bound + 1e-300))
