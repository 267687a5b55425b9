"""End-to-end parity of cca_solve / lda_solve (through the C ABI) against
the FP64 oracle's closed forms: objective, constraint residual, correlations
and, where the spectrum pins them, the weight vectors themselves."""
import numpy as np
import pytest

import synth
from oracle import direct, metrics

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda"


def _srp():
    import paper_2106_12060_amd as srp
    return srp


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    return t if dtype is None else t.to(dtype)


def cca_errors(U, V, X, Y, lam, sig_true):
    Uh, Vh = U.cpu().numpy(), V.cpu().numpy()
    err = metrics.cca_rel_objective_error(Uh, Vh, X, Y, lam, lam, sig_true)
    cons = max(metrics.constraint_residual(Uh, X, lam), metrics.constraint_residual(Vh, Y, lam))
    return err, cons


def test_cca_f64_small_workload():
    """FP64 CCA, n=2000, dx=60, dy=40, k=5, lambda=1e-3, CountSketch s=240.
    The latent strengths span one decade, so the top correlations are 2-10 %
    apart and the FP64 iteration reaches the closed form to about 1e-12."""
    srp = _srp()
    wl = synth.workload("cca-f64-small")
    X, Y = wl.generate()
    lam = wl.lam_value
    sig_true, _, _ = direct.cca_direct(X, Y, lam, lam)
    U, V, sig, info = srp.cca_solve(dev(X), dev(Y), wl.k, lam, lam, wl.s, tol=1e-12,
                                    options=srp.srp_default_options(max_iter=2000))
    err, cons = cca_errors(U, V, X, Y, lam, sig_true)
    print("cca-f64-small", info, err, cons)
    assert cons < 1e-12
    assert err < 1e-10
    np.testing.assert_allclose(sig.cpu().numpy(), sig_true[:wl.k], rtol=0, atol=1e-8)
    assert np.all(np.diff(sig.cpu().numpy()) <= 0)


@pytest.mark.parametrize("dt,tol,bar", [("f32", 1e-6, 1e-6), ("f64", 1e-12, 1e-10)])
def test_cca_unequal_wide_views(dt, tol, bar):
    """dx = 300, dy = 264 (views wider than one 256-wide Gram tile pair, of
    different widths), n = 8000, k = 6, lambda = 1e-3, s = 1200: the sketch
    Grams and the cross Gram of the warm start take the 128 x 128-tile GEMM
    with ragged edges and a split contraction.  Latent strengths span one
    decade and the noise is twice the factor scale, so the top correlations
    run from 0.99 down to 0.82 with sigma_7 = 0.72 (with little noise they
    cluster near 1 and the k-th gap all but closes)."""
    srp = _srp()
    X, Y = synth.cca_latent(8000, 300, 264, r=8, noise=2.0, x_decades=1.0, factor_decades=1.0, seed=41,
                            dtype=np.float32 if dt == "f32" else np.float64)
    lam, k = 1e-3, 6
    sig_true, _, _ = direct.cca_direct(X, Y, lam, lam)
    U, V, sig, info = srp.cca_solve(dev(X), dev(Y), k, lam, lam, 1200, tol=tol, mu=[1.0] * k,
                                    options=srp.srp_default_options(max_iter=3000, warm_start_iters=12))
    err, cons = cca_errors(U, V, X, Y, lam, sig_true)
    print("unequal wide views", dt, info, err, cons)
    assert info["warm_iterations"] > 0
    assert err < bar and cons < bar
    np.testing.assert_allclose(sig.cpu().numpy(), sig_true[:k], rtol=0, atol=10 * bar)


def test_cca_f64_two_reads_every_iteration():
    """FP64 CCA with dx + dy = 960, past the fused FP64 pass: every data
    product takes the two-read FP64 route (X W by row blocks over the whole
    contraction, then X^T P split over the rows), n = 6000, k = 4,
    lambda = 1e-3, s = 2000; the iteration reaches the closed form."""
    srp = _srp()
    X, Y = synth.cca_latent(6000, 500, 460, r=6, noise=2.0, factor_decades=1.0, seed=23, dtype=np.float64)
    lam, k = 1e-3, 4
    sig_true, _, _ = direct.cca_direct(X, Y, lam, lam)
    U, V, sig, info = srp.cca_solve(dev(X), dev(Y), k, lam, lam, 2000, tol=1e-11, mu=[1.0] * k,
                                    options=srp.srp_default_options(max_iter=3000))
    err, cons = cca_errors(U, V, X, Y, lam, sig_true)
    print("f64 two reads", info, err, cons)
    assert err < 1e-10 and cons < 1e-10
    np.testing.assert_allclose(sig.cpu().numpy(), sig_true[:k], rtol=0, atol=1e-8)


def test_poll_interval_does_not_change_the_result():
    """The host reads the convergence flag of the previous batch after it
    has queued the next one; iterations queued after convergence return at
    once on the device.  So the poll interval changes neither the
    iterations nor any output bit."""
    srp = _srp()
    wl = synth.workload("cca-f64-small")
    X, Y = wl.generate()
    lam = wl.lam_value
    outs = []
    for ce in (1, 3, 4):
        U, V, sig, info = srp.cca_solve(dev(X), dev(Y), wl.k, lam, lam, wl.s, tol=1e-10,
                                        options=srp.srp_default_options(max_iter=2000, check_every=ce))
        outs.append((U.cpu().numpy(), V.cpu().numpy(), sig.cpu().numpy(), info["iterations"]))
    for U, V, sig, it in outs[1:]:
        assert it == outs[0][3]
        assert np.array_equal(U, outs[0][0]) and np.array_equal(V, outs[0][1])
        assert np.array_equal(sig, outs[0][2])


def test_cca_planted_vectors_pinned():
    """lambda = 0, planted distinct correlations: the weights are pinned
    (A^-1, B^-1 columns) and sigma = rho.  The solve ends when the cost
    stops decreasing in FP64, so the subspace error e obeys
    e^2 * gap ~ u |f|: with gaps >= 0.1 the weights are pinned to about
    3e-7 of their scale (sigma, second order in e, to 1e-9)."""
    srp = _srp()
    rho = np.array([0.95, 0.85, 0.7, 0.5, 0.3, 0.1])
    X, Y, A, B = synth.planted_cca(4000, 6, rho, seed=5)
    k = 4
    U, V, sig, info = srp.cca_solve(dev(X), dev(Y), k, 0.0, 0.0, 60, tol=1e-13,
                                    options=srp.srp_default_options(max_iter=3000))
    print("planted", info)
    np.testing.assert_allclose(sig.cpu().numpy(), rho[:k], atol=1e-9)
    Ai, Bi = np.linalg.inv(A), np.linalg.inv(B)
    Uh, Vh = U.cpu().numpy(), V.cpu().numpy()
    for i in range(k):
        j = int(np.argmax(np.abs(Ai[:, i])))
        sgn = np.sign(Ai[j, i])
        np.testing.assert_allclose(Uh[:, i], sgn * Ai[:, i], atol=3e-7 * np.abs(Ai).max())
        np.testing.assert_allclose(Vh[:, i], sgn * Bi[:, i], atol=3e-7 * np.abs(Bi).max())


@pytest.mark.parametrize("sketch", ["srht", "countsketch"])
def test_cca_f32_scaled_workload(sketch):
    """FP32 CCA with the column-scaled latent recipe (10^(-4j/d)) at a size
    the oracle solves in seconds, latent rank = k so that the top-k block is
    separated from the rest: relative objective error <= 1e-6."""
    import dataclasses
    srp = _srp()
    wl = dataclasses.replace(synth.workload("cca-f32-srht").scaled(n=30_000, dx=200, dy=160, s=800), r=10,
                             noise=0.1, factor_decades=0.0)
    X, Y = wl.generate()
    lam = wl.lam_value
    sig_true, _, _ = direct.cca_direct(X, Y, lam, lam)
    opt = srp.srp_default_options(sketch=sketch, max_iter=300)
    U, V, sig, info = srp.cca_solve(dev(X), dev(Y), wl.k, lam, lam, wl.s, tol=1e-5, options=opt)
    err, cons = cca_errors(U, V, X.astype(np.float64), Y.astype(np.float64), lam, sig_true)
    print(sketch, info, err, cons)
    assert err < 1e-6
    assert cons < 1e-6


def test_cca_f32_clustered_workload():
    """Same recipe with latent rank 32 > k = 10, equal strengths and little
    noise: the k-cut splits a cluster of correlations a few 1e-6 apart, so
    convergence in the objective is slow (the CPU prototype of the same
    iteration needs > 300 iterations for 1e-6); checked at a looser 1e-5
    after 300 iterations."""
    import dataclasses
    srp = _srp()
    wl = dataclasses.replace(synth.workload("cca-f32-srht").scaled(n=30_000, dx=200, dy=160, s=800),
                             noise=0.1, factor_decades=0.0)
    X, Y = wl.generate()
    lam = wl.lam_value
    sig_true, _, _ = direct.cca_direct(X, Y, lam, lam)
    opt = srp.srp_default_options(sketch="srht", max_iter=300)
    U, V, sig, info = srp.cca_solve(dev(X), dev(Y), wl.k, lam, lam, wl.s, tol=1e-6, options=opt)
    err, cons = cca_errors(U, V, X.astype(np.float64), Y.astype(np.float64), lam, sig_true)
    print("clustered", info, err, cons)
    assert err < 1e-5
    assert cons < 1e-6


def test_lda_scaled_workload():
    """FP32 FDA, n=20000, d=200, 20 classes, k=19, CountSketch s=800.  The
    between-class spectrum spans 1.5 decades with relative gaps down to
    5e-3, so the weighted cost needs several hundred iterations (about 1000
    reach 4e-11).  The within-class covariance spans 6 decades, which puts
    the constraint residual of a retraction built from FP32 products at
    about 1e-6; the finishing pass runs in FP64 (final_f64 = -1)."""
    srp = _srp()
    wl = synth.workload("lda-f32")
    n, d = 20_000, 200
    X, y = synth.lda_classes(n, d, wl.c, seed=wl.seed, dtype=np.float32)
    lam = synth.lda_population_lambda(n, d)
    k = wl.c - 1
    rho_true, _ = direct.lda_direct(X, y, wl.c, lam, k=k)
    W, rho, info = srp.lda_solve(dev(X), dev(y), wl.c, k, lam, 800, tol=1e-7,
                                 options=srp.srp_default_options(max_iter=1500, final_f64=-1))
    _, _, _, Xh, Yh = direct.lda_scatter(X, y, wl.c)
    err = metrics.lda_rel_objective_error(W.cpu().numpy(), Xh, Yh, lam, rho_true)
    cons = metrics.constraint_residual(W.cpu().numpy(), Xh, lam)
    print("lda", info, err, cons)
    assert err < 1e-6
    assert cons < 1e-6
    # k = 19 is odd: the closing Rayleigh-Ritz eigensolve pads one row; the
    # returned rho are the Ritz values, ordered
    np.testing.assert_allclose(rho.cpu().numpy(), rho_true[:k], rtol=1e-5)


@pytest.mark.parametrize("d", [1000, 1003])
def test_lda_fp64_finish_two_reads(d):
    """FP32 FDA with d past the fused FP64 pass (d = 1000, and 1003, whose
    rows are not 16-byte multiples), n = 12000, 12 classes, k = 8,
    CountSketch s = 4000: the finishing pass takes the two-read FP64 route
    (P = X W, then X^T P split over the rows).  With the within-class
    covariance over 6 decades its constraint residual is about 2e-7; wrong
    products break the final retraction or leave residuals of order one."""
    srp = _srp()
    n, c, k = 12_000, 12, 8
    X, y = synth.lda_classes(n, d, c, seed=17, dtype=np.float32)
    lam = synth.lda_population_lambda(n, d)
    rho_true, _ = direct.lda_direct(X, y, c, lam, k=k)
    W, rho, info = srp.lda_solve(dev(X), dev(y), c, k, lam, 4000, tol=1e-5,
                                 options=srp.srp_default_options(max_iter=1500, final_f64=-1))
    _, _, _, Xh, Yh = direct.lda_scatter(X, y, c)
    err = metrics.lda_rel_objective_error(W.cpu().numpy(), Xh, Yh, lam, rho_true)
    cons = metrics.constraint_residual(W.cpu().numpy(), Xh, lam)
    print("lda two-read FP64 finish", d, info, err, cons)
    assert err < 1e-6
    assert cons < 1e-6


def test_lda_f64_two_classes_closed_form():
    srp = _srp()
    rng = np.random.default_rng(3)
    n1, n2, d = 600, 1000, 24
    X = rng.standard_normal((n1 + n2, d))
    X[:n1] += 0.7
    y = np.array([0] * n1 + [1] * n2, dtype=np.int32)
    lam = 0.1
    rho_true, W_true = direct.lda_direct(X, y, 2, lam, k=1)
    W, rho, info = srp.lda_solve(dev(X), dev(y), 2, 1, lam, 96, tol=1e-12)
    assert abs(rho.item() - rho_true[0]) < 1e-9 * rho_true[0]
    np.testing.assert_allclose(W.cpu().numpy()[:, 0], W_true[:, 0], rtol=1e-7, atol=1e-9)


def test_cca_rejects_bad_arguments():
    srp = _srp()
    X = torch.zeros((100, 6), dtype=torch.float64, device=DEV)
    Y = torch.zeros((100, 4), dtype=torch.float64, device=DEV)
    with pytest.raises(srp.SrpError) as e:
        srp.cca_solve(X, Y, 5, 0.1, 0.1, 20)          # k > min(dx, dy)
    assert e.value.code == srp.SRP_EINVAL
    with pytest.raises(srp.SrpError) as e:
        srp.cca_solve(X, Y, 2, 0.0, 0.1, 5)           # s < dx needs lambda_x > 0 (Woodbury form)
    assert e.value.code == srp.SRP_EINVAL
    with pytest.raises(srp.SrpError) as e:
        srp.cca_solve(X, Y, 2, -1.0, 0.1, 20)         # lambda < 0
    assert e.value.code == srp.SRP_EINVAL


def test_cca_rank_deficient_without_regularisation():
    srp = _srp()
    rng = np.random.default_rng(4)
    X = rng.standard_normal((500, 3)) @ rng.standard_normal((3, 8))   # rank 3 < 8
    Y = rng.standard_normal((500, 5))
    with pytest.raises(srp.SrpError) as e:
        srp.cca_solve(dev(X), dev(Y), 2, 0.0, 0.0, 40)
    assert e.value.code == srp.SRP_ENOTSPD


def _cca_case(n=30_000, dx=200, dy=160, s=800, r=10):
    import dataclasses
    # latent rank = k, equal strengths, little noise: the top-k block stands
    # clear of the noise-level correlations
    wl = dataclasses.replace(synth.workload("cca-f32-srht").scaled(n=n, dx=dx, dy=dy, s=s), r=r,
                             noise=0.1, factor_decades=0.0)
    X, Y = wl.generate()
    return wl, X, Y


def test_cca_equal_weights_objective_and_order():
    """N = I (unweighted trace): the top-k subspace, ordered by the closing
    Rayleigh-Ritz step; sigma against the oracle's."""
    srp = _srp()
    wl, X, Y = _cca_case()
    lam = wl.lam_value
    sig_true, _, _ = direct.cca_direct(X, Y, lam, lam)
    U, V, sig, info = srp.cca_solve(dev(X), dev(Y), wl.k, lam, lam, wl.s, tol=1e-6, mu=[1.0] * wl.k,
                                    options=srp.srp_default_options(sketch="srht", max_iter=300))
    err, cons = cca_errors(U, V, X.astype(np.float64), Y.astype(np.float64), lam, sig_true)
    print("N=I", info, err, cons)
    assert err < 1e-6 and cons < 1e-6
    s = sig.cpu().numpy()
    assert np.all(np.diff(s) <= 0)
    np.testing.assert_allclose(s, sig_true[:wl.k], rtol=0, atol=1e-5)


def test_cca_bf16_phase_then_fp32_refinement():
    """BF16 copies (srp_stage_bf16) drive the iteration on BF16 matrix
    cores; the same call then refines on the FP32 data.  The BF16-only
    answer is within 1e-3 of the FP64 objective; the refined one within
    1e-6 (tolerances of the low-precision and FP32 forms)."""
    srp = _srp()
    wl, X, Y = _cca_case()
    lam = wl.lam_value
    sig_true, _, _ = direct.cca_direct(X, Y, lam, lam)
    Xd, Yd = dev(X), dev(Y)
    Xb, Yb = srp.srp_stage_bf16(Xd), srp.srp_stage_bf16(Yd)
    X64, Y64 = X.astype(np.float64), Y.astype(np.float64)
    # BF16 phase only: the FP32 refinement gets no iterations to work with
    opt = srp.srp_default_options(sketch="srht", max_iter=1)
    opt.lowp_tol = 1e-4
    U, V, sig, info = srp.cca_solve(Xd, Yd, wl.k, lam, lam, wl.s, tol=1e-30, options=opt, mu=[1.0] * wl.k,
                                    lowp=(Xb, Yb))
    err_lp, _ = cca_errors(U, V, X64, Y64, lam, sig_true)
    print("bf16 only", info, err_lp)
    assert info["lowp_iterations"] >= 1
    assert err_lp < 1e-3
    opt = srp.srp_default_options(sketch="srht", max_iter=300)
    U, V, sig, info = srp.cca_solve(Xd, Yd, wl.k, lam, lam, wl.s, tol=1e-6, options=opt, mu=[1.0] * wl.k,
                                    lowp=(Xb, Yb))
    err, cons = cca_errors(U, V, X64, Y64, lam, sig_true)
    print("bf16 + fp32", info, err, cons)
    assert err < 1e-6 and cons < 1e-6


@pytest.mark.parametrize("fmt", ["fp8", "bf16"])
def test_cca_staged_sketch_inputs(fmt):
    """Sketch from an FP8 (with column scales) or BF16 staged copy: the
    preconditioner changes, the fixed point does not (the critical points
    do not depend on the metric), so the answer still meets 1e-6."""
    srp = _srp()
    wl, X, Y = _cca_case()
    lam = wl.lam_value
    sig_true, _, _ = direct.cca_direct(X, Y, lam, lam)
    Xd, Yd = dev(X), dev(Y)
    if fmt == "fp8":
        (cx, sx), (cy, sy) = srp.srp_stage_fp8(Xd), srp.srp_stage_fp8(Yd)
        staged = (cx, cy, sx, sy)
    else:
        staged = (srp.srp_stage_bf16(Xd), srp.srp_stage_bf16(Yd), None, None)
    U, V, sig, info = srp.cca_solve(Xd, Yd, wl.k, lam, lam, wl.s, tol=1e-6, mu=[1.0] * wl.k,
                                    options=srp.srp_default_options(sketch="srht", max_iter=300),
                                    sketch_input=staged)
    err, cons = cca_errors(U, V, X.astype(np.float64), Y.astype(np.float64), lam, sig_true)
    print(fmt, info, err, cons)
    assert err < 1e-6 and cons < 1e-6


def test_cca_views_whose_factor_splits_differ():
    """dx = 383 (6 tiles of 64) and dy = 399 (7 tiles): the narrower view's
    Gram takes the deeper split-K and the larger factor scratch, so each
    view's scratch must cover the larger need of the two."""
    srp = _srp()
    X, Y = synth.cca_latent(3000, 383, 399, r=8, noise=0.1, x_decades=3.0, seed=97)
    lam = 1e-3
    sig_true, _, _ = direct.cca_direct(X, Y, lam, lam)
    U, V, sig, info = srp.cca_solve(dev(X, torch.float32), dev(Y, torch.float32), 2, lam, lam, 1596, tol=1e-6,
                                    options=srp.srp_default_options(max_iter=1000), mu=[1.0, 1.0])
    err, cons = cca_errors(U, V, X, Y, lam, sig_true)
    print("split views", info["iterations"], err, cons)
    assert err < 1e-6 and cons < 1e-6


def test_cca_sign_convention_with_largest_entries_past_row_256():
    """The sign convention flips a column pair when the largest |entry| of
    the U column is negative.  Here every U column has its largest entry at
    a row past 256 (the columns of X are scaled over three decades, so the
    weights peak at the small-scale columns): the workgroup thread that owns
    that row negates it while the others decide whether to flip, so the
    decision must be taken once and shared before any write.  Two seeds give
    different signs before the fix; every column must end with a positive
    largest entry and the constraints intact."""
    srp = _srp()
    X, Y = synth.cca_latent(20000, 600, 520, r=8, noise=1.0, x_decades=3.0, factor_decades=1.0, seed=61,
                            dtype=np.float32)
    lam, k = 1e-3, 6
    sig_true, U_true, _ = direct.cca_direct(X, Y, lam, lam, k=k)
    assert np.all(np.argmax(np.abs(U_true), axis=0) >= 256)
    for seed in (3, 4):
        U, V, sig, info = srp.cca_solve(dev(X), dev(Y), k, lam, lam, 2400, tol=1e-6,
                                        options=srp.srp_default_options(max_iter=500, seed=seed))
        err, cons = cca_errors(U, V, X.astype(np.float64), Y.astype(np.float64), lam, sig_true)
        Uh = U.cpu().numpy()
        print("sign fix", seed, info, err, cons)
        j = np.argmax(np.abs(Uh), axis=0)
        assert np.all(Uh[j, np.arange(k)] > 0)
        assert cons < 1e-6 and err < 1e-6
        # same phase: u_i^T Sxy v_i >= 0 for every pair
        XU = X.astype(np.float64) @ Uh
        YV = Y.astype(np.float64) @ V.cpu().numpy()
        assert np.all(np.sum(XU * YV, axis=0) > 0)


@pytest.mark.parametrize("c,k", [(22, 21), (33, 32)])
def test_lda_more_than_twenty_directions(c, k):
    """FDA with k = 21 and k = 32 (the ABI's limit): the one-view pass past
    the 4x4-block instance (register-staged rows) and the controllers'
    largest k x k instances.  k = c - 1 takes every between-class
    direction, a subspace separated from the null space of S_B, so equal
    weights converge quickly; the closing Rayleigh-Ritz step orders it."""
    srp = _srp()
    n, d = c * 600, 200
    X, y = synth.lda_classes(n, d, c, decades=2.0, seed=70 + c, dtype=np.float32)
    lam = synth.lda_population_lambda(n, d)
    rho_true, _ = direct.lda_direct(X, y, c, lam, k=k)
    W, rho, info = srp.lda_solve(dev(X), dev(y), c, k, lam, 800, tol=1e-7, mu=[1.0] * k,
                                 options=srp.srp_default_options(max_iter=1000, final_f64=-1))
    _, _, _, Xh, Yh = direct.lda_scatter(X, y, c)
    err = metrics.lda_rel_objective_error(W.cpu().numpy(), Xh, Yh, lam, rho_true)
    cons = metrics.constraint_residual(W.cpu().numpy(), Xh, lam)
    print("lda k", k, info, err, cons)
    assert err < 1e-6 and cons < 1e-6
    np.testing.assert_allclose(rho.cpu().numpy(), rho_true[:k], rtol=1e-5)


def test_lda_rejects_too_many_classes():
    srp = _srp()
    X = torch.zeros((650, 8), dtype=torch.float32, device=DEV)
    y = torch.arange(650, dtype=torch.int32, device=DEV) % 65
    with pytest.raises(srp.SrpError) as e:
        srp.lda_solve(X, y, 65, 2, 0.1, 16)
    assert e.value.code == srp.SRP_EINVAL


def _sin_max_angle(A, B):
    """Sine of the largest principal angle between span(A) and span(B):
    the norm of the part of B's orthonormal basis outside span(A) (accurate
    for small angles, unlike sqrt(1 - cos^2))."""
    Qa, _ = np.linalg.qr(A)
    Qb, _ = np.linalg.qr(B)
    return float(np.linalg.norm(Qb - Qa @ (Qa.T @ Qb), 2))


@pytest.mark.parametrize("n,dx,dy,k,s,dt,sketch,iters,bar", [
    # block = min(dx, dy) columns: one product spans C^T C's range, exact
    (3000, 50, 40, 5, 200, "f64", "countsketch", 12, 1e-9),
    # 64-column block inside dmin = 200; the sketched correlations past the
    # block sit near 0.75 against 0.95 for the sixth, so the error falls
    # about 0.6x per iteration: 40 iterations reach the floor set by the
    # FP32 sketch (its rounding moves the sketched subspace by ~1e-6)
    (20000, 300, 200, 6, 1200, "f32", "srht", 40, 1e-5)])
def test_cca_warm_start_is_the_exact_sketched_solution(n, dx, dy, k, s, dt, sketch, iters, bar):
    """Algorithm CCAopt starts from exact-cca(SX, SY).  With max_iter = 0
    the solver returns that start point (after qf in the full metric and the
    closing Rayleigh-Ritz rotation, which keep its span): its span must be
    the span of the oracle's CCA of the sketched data, sketched with the
    same seed."""
    from oracle import sketch as osk
    srp = _srp()
    X, Y = synth.cca_latent(n, dx, dy, r=k, noise=0.5, factor_decades=0.5, seed=80 + dx,
                            dtype=np.float64 if dt == "f64" else np.float32)
    lam, seed = 1e-3, 17
    opt = srp.srp_default_options(sketch=sketch, seed=seed, max_iter=0, warm_start_iters=iters)
    U, V, sig, info = srp.cca_solve(dev(X), dev(Y), k, lam, lam, s, tol=1e-9, options=opt)
    assert info["warm_iterations"] >= 1
    X64, Y64 = X.astype(np.float64), Y.astype(np.float64)
    SX = osk.sketch(X64, sketch, s, seed)
    SY = osk.sketch(Y64, sketch, s, seed)
    sig_s, Us, Vs = direct.cca_direct(SX, SY, lam, lam, k=k)
    assert sig_s[k - 1] - sig_s[k] > 0.05          # the sketched top-k block is separated
    su = _sin_max_angle(U.cpu().numpy(), Us)
    sv = _sin_max_angle(V.cpu().numpy(), Vs)
    print("warm start", info, su, sv)
    assert su < bar and sv < bar


def test_lda_warm_start_is_the_exact_sketched_solution():
    """Algorithm LDAopt starts from exact-fda(SX): the leading generalized
    eigenvectors of (S_B, M) with M the sketched within-class Gram plus
    lambda I; k < c - 1 so the span is pinned by the eigengap, not by the
    range of S_B alone."""
    from oracle import sketch as osk
    srp = _srp()
    c, k, d, n, s = 10, 4, 120, 6000, 480
    X, y = synth.lda_classes(n, d, c, decades=2.0, seed=90, dtype=np.float64)
    lam, seed = 0.1, 5
    opt = srp.srp_default_options(seed=seed, max_iter=0, warm_start_iters=1)
    W, rho, info = srp.lda_solve(dev(X), dev(y), c, k, lam, s, tol=1e-9, options=opt)
    _, _, _, Xh, Yh = direct.lda_scatter(X, y, c)
    SXh = osk.sketch(Xh, "countsketch", s, seed)
    M = SXh.T @ SXh + lam * np.eye(d)
    import scipy.linalg as sla
    ev, Vg = sla.eigh(Yh.T @ Yh, M)
    ev, Vg = ev[::-1], Vg[:, ::-1]
    assert (ev[k - 1] - ev[k]) > 0.02 * ev[0]
    sw = _sin_max_angle(W.cpu().numpy(), Vg[:, :k])
    print("lda warm start", info, sw)
    assert sw < 1e-9
