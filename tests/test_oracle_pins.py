"""Pins for the FP64 oracle: each check ties it to something other than
itself (closed forms, an independent eigen-solver, brute force,
invariants, finite differences), chosen so that a dropped term, a wrong
sign or index, or a transposed operand fails at least one of them."""
import numpy as np
import pytest
import scipy.linalg as sla
from scipy.optimize import minimize

import synth
from oracle import direct, sketch, stiefel, metrics


def _rand_cca(n=80, dx=6, dy=4, seed=0):
    X, Y = synth.cca_latent(n, dx, dy, r=3, noise=0.3, x_decades=1.0, seed=seed)
    return X, Y


# ------------------------------------------------------------------ CCA --
@pytest.mark.parametrize("lam", [0.0, 1e-2, 3.0])
def test_cca_matches_generalized_eigensolve(lam):
    """Generalized eigenvalues of ([[0,Sxy],[Sxy^T,0]], blkdiag(Sxx,Syy)) are
    +-sigma_i plus |dx-dy| zeros (the pencil behind Definition CCA)."""
    X, Y = _rand_cca(seed=1)
    dx, dy = X.shape[1], Y.shape[1]
    Sxx, Syy, Sxy = stiefel.cca_blocks(X, Y, lam, lam)
    A = np.block([[np.zeros((dx, dx)), Sxy], [Sxy.T, np.zeros((dy, dy))]])
    Bm = sla.block_diag(Sxx, Syy)
    theta = sla.eigh(A, Bm, eigvals_only=True)
    top = np.sort(theta)[::-1][:min(dx, dy)]
    sig, U, V = direct.cca_direct(X, Y, lam, lam)
    np.testing.assert_allclose(sig, top, rtol=1e-10, atol=1e-12)


def test_cca_y_equals_x_closed_form():
    """Y = X, lam_x = lam_y = lam: sigma_i = s_i^2 / (s_i^2 + lam) with s_i the
    singular values of X, and U = V."""
    X, _ = _rand_cca(n=60, dx=5, seed=2)
    lam = 0.7
    s = np.linalg.svd(X, compute_uv=False)
    sig, U, V = direct.cca_direct(X, X, lam, lam, k=5)
    np.testing.assert_allclose(sig, s ** 2 / (s ** 2 + lam), rtol=1e-12)
    np.testing.assert_allclose(U, V, rtol=1e-8, atol=1e-10)


def test_cca_planted_correlations():
    """Planted pair: canonical correlations are exactly rho; weights are the
    columns of A^-1 and B^-1 up to sign."""
    rho = np.array([0.95, 0.8, 0.5, 0.2])
    X, Y, A, B = synth.planted_cca(200, 4, rho, seed=3)
    sig, U, V = direct.cca_direct(X, Y, 0.0, 0.0)
    np.testing.assert_allclose(sig, rho, atol=1e-12)
    Ai = np.linalg.inv(A)
    Bi = np.linalg.inv(B)
    for i in range(4):
        su = np.sign(U[:, i] @ Ai[:, i])
        np.testing.assert_allclose(U[:, i], su * Ai[:, i], atol=1e-9)
        np.testing.assert_allclose(V[:, i], su * Bi[:, i], atol=1e-9)


def test_cca_invariant_under_column_transforms():
    """lam = 0: sigma unchanged for X -> X A, Y -> Y B (A, B invertible)."""
    X, Y = _rand_cca(seed=4)
    rng = np.random.default_rng(5)
    A = rng.standard_normal((6, 6)) + 2 * np.eye(6)
    B = rng.standard_normal((4, 4)) + 2 * np.eye(4)
    s1, _, _ = direct.cca_direct(X, Y, 0.0, 0.0)
    s2, _, _ = direct.cca_direct(X @ A, Y @ B, 0.0, 0.0)
    np.testing.assert_allclose(s1, s2, rtol=1e-9)


def test_cca_constraints_and_diagonal():
    """U^T Sxx U = I, V^T Syy V = I, U^T Sxy V = diag(sigma_1..k)."""
    X, Y = _rand_cca(seed=6)
    lam = 0.05
    sig, U, V = direct.cca_direct(X, Y, lam, lam, k=3)
    Sxx, Syy, Sxy = stiefel.cca_blocks(X, Y, lam, lam)
    np.testing.assert_allclose(U.T @ Sxx @ U, np.eye(3), atol=1e-11)
    np.testing.assert_allclose(V.T @ Syy @ V, np.eye(3), atol=1e-11)
    np.testing.assert_allclose(U.T @ Sxy @ V, np.diag(sig[:3]), atol=1e-11)
    assert np.all(np.diff(sig) <= 0)
    assert metrics.constraint_residual(U, X, lam) < 1e-11
    assert metrics.cca_rel_objective_error(U, V, X, Y, lam, lam, sig) < 1e-12


def test_cca_gram_and_qr_routes_agree():
    X, Y = synth.cca_latent(300, 8, 7, r=4, noise=0.1, x_decades=3.0, seed=7)
    s1, U1, V1 = direct.cca_direct(X, Y, 1e-3, 1e-3, k=3)
    s2, U2, V2 = direct.cca_direct_qr(X, Y, 1e-3, 1e-3, k=3)
    np.testing.assert_allclose(s1, s2, rtol=1e-10)
    np.testing.assert_allclose(U1, U2, rtol=1e-6, atol=1e-8)


def test_cca_brute_force_top_correlation():
    """dx = dy = 2: maximise the correlation ratio
    u^T Sxy v / sqrt(u^T Sxx u * v^T Syy v) over angles (no factorisation
    involved) and compare with sigma_1."""
    X, Y = _rand_cca(n=40, dx=2, dy=2, seed=8)
    lam = 0.3
    Sxx, Syy, Sxy = stiefel.cca_blocks(X, Y, lam, lam)

    def neg_ratio(a):
        u = np.array([np.cos(a[0]), np.sin(a[0])])
        v = np.array([np.cos(a[1]), np.sin(a[1])])
        return -(u @ Sxy @ v) / np.sqrt((u @ Sxx @ u) * (v @ Syy @ v))

    th = np.linspace(0, np.pi, 181)
    grid = np.array([[neg_ratio((a, b)) for b in th] for a in th])
    i, j = np.unravel_index(np.argmin(grid), grid.shape)
    res = minimize(neg_ratio, [th[i], th[j]], method="Nelder-Mead",
                   options={"xatol": 1e-12, "fatol": 1e-15, "maxiter": 4000})
    sig, _, _ = direct.cca_direct(X, Y, lam, lam)
    assert abs(-res.fun - sig[0]) < 1e-9


# ------------------------------------------------------------------ FDA --
def test_lda_matches_generalized_eigensolve():
    X, y = synth.lda_classes(120, 7, 4, decades=2.0, seed=9)
    lam = 0.1
    rho, W = direct.lda_direct(X, y, 4, lam, k=3)
    _, _, _, Xh, Yh = direct.lda_scatter(X, y, 4)
    ev = sla.eigh(Yh.T @ Yh, Xh.T @ Xh + lam * np.eye(7), eigvals_only=True)
    np.testing.assert_allclose(rho[:3], np.sort(ev)[::-1][:3], rtol=1e-10)
    B = Xh.T @ Xh + lam * np.eye(7)
    np.testing.assert_allclose(W.T @ B @ W, np.eye(3), atol=1e-10)
    np.testing.assert_allclose(W.T @ (Yh.T @ Yh) @ W, np.diag(rho[:3]),
                               atol=1e-8 * rho[0])


def test_lda_two_class_closed_form():
    """l = 2: S_B = (n1 n2 / n) D D^T with D = m1 - m2, so the only nonzero
    generalized eigenvalue is (n1 n2 / n) D^T B^-1 D with vector B^-1 D."""
    rng = np.random.default_rng(10)
    n1, n2, d = 30, 50, 5
    X = rng.standard_normal((n1 + n2, d))
    X[:n1] += 1.5
    y = np.array([0] * n1 + [1] * n2)
    lam = 0.2
    m1, m2 = X[:n1].mean(0), X[n1:].mean(0)
    Dm = m1 - m2
    Xh = X - np.where(y[:, None] == 0, m1, m2)
    B = Xh.T @ Xh + lam * np.eye(d)
    w = np.linalg.solve(B, Dm)
    rho1 = n1 * n2 / (n1 + n2) * Dm @ w
    rho, W = direct.lda_direct(X, y, 2, lam, k=1)
    assert abs(rho[0] - rho1) < 1e-10 * rho1
    assert abs(rho[1]) < 1e-10 * rho1
    cos = abs(W[:, 0] @ w) / (np.linalg.norm(W[:, 0]) * np.linalg.norm(w))
    assert abs(cos - 1) < 1e-12


# -------------------------------------------------------------- sketches --
def test_splitmix64_vectorised_matches_integer_definition():
    rng = np.random.default_rng(11)
    for seed in [0, 1, 12060, int(rng.integers(0, 2**63))]:
        idx = np.array([0, 1, 2, 1000, 2**31, 2**40 + 7], dtype=np.uint64)
        v = sketch.splitmix64(seed, idx)
        ref = [sketch.splitmix64_reference(seed, int(i)) for i in idx]
        assert [int(x) for x in v] == ref


def test_splitmix64_stream_is_the_sequential_generator():
    """The i-th output equals stepping a sequential SplitMix64 state i+1
    times (the counter form is the published generator, not a variant)."""
    seed = 987654321
    state = seed
    outs = []
    for _ in range(5):
        state = (state + sketch.GOLDEN_GAMMA) & sketch.MASK64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & sketch.MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & sketch.MASK64
        outs.append(z ^ (z >> 31))
    assert outs == [int(x) for x in sketch.splitmix64(seed, np.arange(5, dtype=np.uint64))]


def test_countsketch_bucket_sum_equals_matrix_definition():
    X, _ = _rand_cca(n=50, dx=3, seed=12)
    h, g = sketch.countsketch_hash(50, 7, seed=13)
    assert h.min() >= 0 and h.max() < 7
    S = sketch.countsketch_matrix(h, g, 7)
    assert np.all(np.count_nonzero(S, axis=0) == 1)
    np.testing.assert_allclose(sketch.countsketch_apply(X, h, g, 7), S @ X,
                               atol=1e-13)


def test_countsketch_injective_hash_is_isometry():
    rng = np.random.default_rng(14)
    n, s = 20, 25
    h = rng.permutation(s)[:n]
    g = rng.choice([-1.0, 1.0], size=n)
    X = rng.standard_normal((n, 4))
    SX = sketch.countsketch_apply(X, h, g, s)
    np.testing.assert_allclose(SX.T @ SX, X.T @ X, atol=1e-12)


def test_countsketch_hash_statistics():
    n, s = 200_000, 64
    h, g = sketch.countsketch_hash(n, s, seed=15)
    counts = np.bincount(h, minlength=s)
    chi2 = np.sum((counts - n / s) ** 2 / (n / s))
    assert chi2 < 130            # 63 dof: p ~ 1e-6 tail
    assert abs(g.mean()) < 5 / np.sqrt(n)


def test_countsketch_unbiased_over_seeds():
    """E[S^T S] = I: average over many seeds is close to the identity."""
    n, s, reps = 12, 5, 4000
    acc = np.zeros((n, n))
    for seed in range(reps):
        h, g = sketch.countsketch_hash(n, s, seed)
        S = sketch.countsketch_matrix(h, g, s)
        acc += S.T @ S
    acc /= reps
    assert np.max(np.abs(acc - np.eye(n))) < 0.06


def test_hadamard_is_orthogonal_and_fwht_matches():
    for m in [1, 2, 5, 8]:
        H = sketch.hadamard(2 ** m)
        np.testing.assert_allclose(H @ H.T, 2 ** m * np.eye(2 ** m))
        r = np.random.default_rng(m).integers(0, 2 ** m, size=20)
        i = np.random.default_rng(m + 1).integers(0, 2 ** m, size=20)
        expect = np.array([(-1) ** bin(int(a) & int(b)).count("1") for a, b in zip(r, i)])
        np.testing.assert_array_equal(H[r, i], expect)
        A = np.random.default_rng(m).standard_normal((2 ** m, 3))
        np.testing.assert_allclose(sketch.fwht_rows(A), H @ A, atol=1e-10)


def test_srht_full_sample_preserves_gram():
    """s = n': S = n'^-1/2 H D is orthogonal, so (SX)^T (SX) = X^T X."""
    rng = np.random.default_rng(16)
    X = rng.standard_normal((13, 4))
    n_pad = sketch.srht_padded_rows(13)
    assert n_pad == 16
    D = sketch.srht_signs(n_pad, 17)
    rows = sketch.srht_rows(n_pad, n_pad, 17)
    np.testing.assert_array_equal(rows, np.arange(16))
    SX = sketch.srht_apply(X, D, rows, n_pad)
    np.testing.assert_allclose(SX.T @ SX, X.T @ X, atol=1e-12)
    SX2 = sketch.srht_apply(X, D, rows, n_pad, dense_limit=0)  # FWHT route
    np.testing.assert_allclose(SX2, SX, atol=1e-12)


def test_srht_rows_are_a_uniform_sample():
    n_pad, s = 64, 16
    rows = sketch.srht_rows(n_pad, s, 18)
    assert len(set(rows.tolist())) == s and np.all(np.diff(rows) > 0)
    counts = np.zeros(n_pad)
    for seed in range(3000):
        counts[sketch.srht_rows(n_pad, s, seed)] += 1
    p = counts / 3000
    assert np.max(np.abs(p - s / n_pad)) < 0.04


def test_srht_unbiased_over_seeds():
    n, s, reps = 8, 4, 3000
    acc = np.zeros((n, n))
    I = np.eye(n)
    for seed in range(reps):
        D = sketch.srht_signs(n, seed)
        rows = sketch.srht_rows(n, s, seed)
        S = sketch.srht_apply(I, D, rows, s)
        acc += S.T @ S
    acc /= reps
    assert np.max(np.abs(acc - np.eye(n))) < 0.08


def test_sketch_factor_is_cholesky_of_sketched_gram():
    X, _ = _rand_cca(n=100, dx=5, seed=19)
    SX = sketch.sketch(X, "countsketch", 30, 20)
    R = sketch.sketch_factor(SX, 0.1)
    assert np.allclose(R, np.triu(R)) and np.all(np.diag(R) > 0)
    Rq = np.linalg.qr(np.vstack([SX, np.sqrt(0.1) * np.eye(5)]), mode="r")
    Rq *= np.sign(np.diag(Rq))[:, None]
    np.testing.assert_allclose(R, Rq, rtol=1e-10, atol=1e-12)


def test_countsketch_lemma_statistically():
    """Lemma sketching: s >= 20 s_lam^2 / delta gives generalized eigenvalues
    of (Z^T Z + lam I, Z^T S^T S Z + lam I) in [1/2, 3/2] with probability
    at least 1 - delta."""
    rng = np.random.default_rng(21)
    Z = rng.standard_normal((4000, 6)) * np.array([3, 2, 1, .3, .1, .03])
    lam = 300.0
    sl = direct.statistical_dimension(Z, lam)
    delta = 0.25
    s = int(np.ceil(20 * sl ** 2 / delta))
    assert s < 4000
    ok = 0
    trials = 60
    B = Z.T @ Z + lam * np.eye(6)
    for seed in range(trials):
        SZ = sketch.sketch(Z, "countsketch", s, 1000 + seed)
        M = SZ.T @ SZ + lam * np.eye(6)
        ev = sla.eigh(B, M, eigvals_only=True)
        ok += int(ev.min() >= 0.5 and ev.max() <= 1.5)
    assert ok / trials >= 1 - delta


# --------------------------------------------------------- Table 1 parts --
def _spd(d, rng, cond=10.0):
    Q = stiefel_q(d, rng)
    return (Q * np.geomspace(1, cond, d)) @ Q.T


def stiefel_q(d, rng):
    Q, _ = np.linalg.qr(rng.standard_normal((d, d)))
    return Q


def _point(d, p, B, rng):
    return stiefel.qf_B(rng.standard_normal((d, p)), B)


def test_projection_properties():
    rng = np.random.default_rng(22)
    d, p = 7, 3
    B, M = _spd(d, rng, 50), _spd(d, rng, 20)
    X = _point(d, p, B, rng)
    np.testing.assert_allclose(X.T @ B @ X, np.eye(p), atol=1e-12)
    a, b = rng.standard_normal((d, p)), rng.standard_normal((d, p))
    Pa, Pb = stiefel.project(X, B, M, a), stiefel.project(X, B, M, b)
    T = X.T @ B @ Pa
    np.testing.assert_allclose(T + T.T, 0, atol=1e-11)                # tangent
    np.testing.assert_allclose(stiefel.project(X, B, M, Pa), Pa, atol=1e-11)
    assert abs(stiefel.inner(Pa, b, M) - stiefel.inner(a, Pb, M)) < 1e-10
    assert abs(stiefel.inner(a - Pa, Pb, M)) < 1e-10                # M-orthogonal
    # normal part has the Table 1 form M^-1 B X S with S symmetric
    S = stiefel.normal_coeff(X, B, M, a)
    np.testing.assert_allclose(S, S.T, atol=1e-11)


def test_projection_with_exact_metric_reduces_to_sym():
    """M = B: the Sylvester solution is S = sym(X^T B xi) (Appendix B)."""
    rng = np.random.default_rng(23)
    d, p = 6, 2
    B = _spd(d, rng, 30)
    X = _point(d, p, B, rng)
    xi = rng.standard_normal((d, p))
    S = stiefel.normal_coeff(X, B, B, xi)
    np.testing.assert_allclose(S, stiefel.sym(X.T @ B @ xi), atol=1e-11)
    np.testing.assert_allclose(stiefel.project(X, B, B, xi),
                               xi - X @ stiefel.sym(X.T @ B @ xi), atol=1e-11)


def test_qr_retraction_literal_and_on_manifold():
    rng = np.random.default_rng(24)
    d, p = 6, 3
    B = _spd(d, rng, 40)
    X = _point(d, p, B, rng)
    xi = 0.3 * rng.standard_normal((d, p))
    R1 = stiefel.retract_qr(X, xi, B)
    R2 = stiefel.retract_qr_literal(X, xi, B)
    np.testing.assert_allclose(R1, R2, atol=1e-10)
    np.testing.assert_allclose(R1.T @ B @ R1, np.eye(p), atol=1e-11)
    np.testing.assert_allclose(stiefel.retract_qr(X, 0 * xi, B), X, atol=1e-11)


def test_cca_gradient_matches_finite_differences():
    """<grad f, eta>_M = d/dt f(R(Z + t eta)) at t = 0 for tangent eta, on the
    product manifold with metric blkdiag(Mxx, Myy) (Eq. gradCCA)."""
    X, Y = _rand_cca(n=90, dx=5, dy=4, seed=25)
    lam = 0.1
    Sxx, Syy, Sxy = stiefel.cca_blocks(X, Y, lam, lam)
    rng = np.random.default_rng(26)
    Mxx, Myy = _spd(5, rng, 5) * 40, _spd(4, rng, 5) * 40
    mu = np.array([3.0, 2.0])
    U = _point(5, 2, Sxx, rng)
    V = _point(4, 2, Syy, rng)
    gu, gv = stiefel.cca_rgrad(U, V, Sxx, Syy, Sxy, Mxx, Myy, mu)
    eu = stiefel.project(U, Sxx, Mxx, rng.standard_normal((5, 2)))
    ev = stiefel.project(V, Syy, Myy, rng.standard_normal((4, 2)))
    h = 1e-5

    def f(t):
        return stiefel.cca_cost(stiefel.retract_qr(U, t * eu, Sxx),
                                stiefel.retract_qr(V, t * ev, Syy), Sxy, mu)

    fd = (f(h) - f(-h)) / (2 * h)
    ip = stiefel.inner(gu, eu, Mxx) + stiefel.inner(gv, ev, Myy)
    assert abs(fd - ip) < 1e-7 * max(1.0, abs(ip))
    # gradient is tangent
    T = U.T @ Sxx @ gu
    np.testing.assert_allclose(T + T.T, 0, atol=1e-10)


def test_lda_gradient_matches_finite_differences():
    X, y = synth.lda_classes(100, 6, 4, decades=1.0, seed=27)
    _, _, _, Xh, Yh = direct.lda_scatter(X, y, 4)
    lam = 0.5
    B = Xh.T @ Xh + lam * np.eye(6)
    SB = Yh.T @ Yh
    rng = np.random.default_rng(28)
    M = _spd(6, rng, 8) * 30
    mu = np.array([3.0, 2.0, 1.0])
    W = _point(6, 3, B, rng)
    g = stiefel.lda_rgrad(W, B, SB, M, mu)
    eta = stiefel.project(W, B, M, rng.standard_normal((6, 3)))
    h = 1e-5

    def f(t):
        return stiefel.lda_cost(stiefel.retract_qr(W, t * eta, B), SB, mu)

    fd = (f(h) - f(-h)) / (2 * h)
    ip = stiefel.inner(g, eta, M)
    assert abs(fd - ip) < 1e-7 * max(1.0, abs(ip))


def test_gradient_vanishes_at_direct_solution():
    """Theorem criticalpointofCCA / criticalpointsofLDA: the direct solution
    is critical for any metric."""
    X, Y = _rand_cca(n=120, dx=6, dy=5, seed=29)
    lam = 0.05
    sig, U, V = direct.cca_direct(X, Y, lam, lam, k=3)
    Sxx, Syy, Sxy = stiefel.cca_blocks(X, Y, lam, lam)
    rng = np.random.default_rng(30)
    Mxx, Myy = _spd(6, rng, 7) * 50, _spd(5, rng, 7) * 50
    mu = np.array([3.0, 2.0, 1.0])
    gu, gv = stiefel.cca_rgrad(U, V, Sxx, Syy, Sxy, Mxx, Myy, mu)
    U0 = _point(6, 3, Sxx, rng)
    V0 = _point(5, 3, Syy, rng)
    g0u, g0v = stiefel.cca_rgrad(U0, V0, Sxx, Syy, Sxy, Mxx, Myy, mu)
    assert np.linalg.norm(gu) + np.linalg.norm(gv) < 1e-10 * (
        np.linalg.norm(g0u) + np.linalg.norm(g0v))
    np.testing.assert_allclose(Sxy @ V, Sxx @ U @ np.diag(sig[:3]), atol=1e-10)
    assert metrics.weighted_suboptimality(sig, stiefel.cca_cost(U, V, Sxy, mu), mu) < 1e-13

    Xl, yl = synth.lda_classes(92, 6, 4, decades=1.0, seed=31)
    rho, W = direct.lda_direct(Xl, yl, 4, 0.2, k=3)
    _, _, _, Xh, Yh = direct.lda_scatter(Xl, yl, 4)
    B = Xh.T @ Xh + 0.2 * np.eye(6)
    gl = stiefel.lda_rgrad(W, B, Yh.T @ Yh, _spd(6, rng, 5), mu)
    assert np.linalg.norm(gl) < 1e-9 * rho[0]


def test_cca_solution_independent_of_column_order():
    """Permuting columns permutes the weights and leaves sigma unchanged."""
    X, Y = _rand_cca(seed=32)
    perm = np.array([3, 0, 5, 1, 4, 2])
    s1, U1, V1 = direct.cca_direct(X, Y, 0.1, 0.1, k=2)
    s2, U2, V2 = direct.cca_direct(X[:, perm], Y, 0.1, 0.1, k=2)
    np.testing.assert_allclose(s1, s2, rtol=1e-12)
    np.testing.assert_allclose(U1[perm], U2, atol=1e-10)


# ------------------------------------------------------------ staging
def test_bf16_round_definition():
    from oracle import quant
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -9, -2.5, 0.0], dtype=np.float32)
    r = quant.bf16_round(x)
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: tie to even -> 1
    # 1 + 3 2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: tie to even -> 1 + 2^-6
    np.testing.assert_array_equal(r, np.array([1.0, 1.0, 1.0 + 2.0 ** -6, 1.0, -2.5, 0.0], dtype=np.float32))
    # every BF16 value has 8 significant bits: the low 16 bits are zero
    assert np.all(r.view(np.uint32) & 0xFFFF == 0)
    rng = np.random.default_rng(0)
    y = rng.standard_normal(10000).astype(np.float32)
    ry = quant.bf16_round(y)
    assert np.all(np.abs(ry - y) <= 2.0 ** -8 * np.abs(y))   # unit roundoff of an 8-bit significand


def test_fp8_table_matches_format():
    from oracle import quant
    vals, codes = quant.fp8_e4m3_table()
    assert len(vals) == 127 and vals[0] == 0.0 and vals[-1] == 448.0
    assert vals[1] == 2.0 ** -9                       # smallest subnormal
    assert 2.0 ** -6 in vals and 2.0 ** -6 - 2.0 ** -9 in vals   # smallest normal, largest subnormal
    assert np.all(np.diff(vals) > 0)
    np.testing.assert_array_equal(quant.fp8_e4m3_decode(codes), vals)


def test_fp8_encode_rounding_and_saturation():
    from oracle import quant
    dec = lambda x: quant.fp8_e4m3_decode(quant.fp8_e4m3_encode(np.array(x, dtype=np.float64)))
    np.testing.assert_array_equal(dec([448.0, 500.0, 1e9, -1e9]), [448.0, 448.0, 448.0, -448.0])
    # ties: 1 + 1/16 between 1 (m=0) and 1.125 (m=1) -> 1; 1 + 3/16 between 1.125 and 1.25 (m=2) -> 1.25
    np.testing.assert_array_equal(dec([1.0625, 1.1875, -1.0625]), [1.0, 1.25, -1.0])
    # subnormal grid 2^-9 and its ties
    np.testing.assert_array_equal(dec([2.0 ** -9, 1.5 * 2.0 ** -9, 2.5 * 2.0 ** -9, 0.4 * 2.0 ** -9]),
                                  [2.0 ** -9, 2.0 * 2.0 ** -9, 2.0 * 2.0 ** -9, 0.0])
    # 464 = halfway between 448 and the (missing) 480: saturates to 448
    np.testing.assert_array_equal(dec([464.0]), [448.0])
    rng = np.random.default_rng(1)
    x = rng.uniform(-400, 400, 20000)
    q = dec(x)
    # relative error at most half an ulp of a 4-bit significand in the normal range
    nrm = np.abs(x) >= 2.0 ** -6
    assert np.all(np.abs(q[nrm] - x[nrm]) <= 2.0 ** -4 * np.abs(x[nrm]))


def test_fp8_column_scales_are_powers_of_two_and_exact():
    from oracle import quant
    rng = np.random.default_rng(2)
    X = rng.standard_normal((300, 7)) * np.array([1e-3, 1.0, 10.0, 448.0, 449.0, 1e5, 0.0])
    sc = quant.fp8_column_scales(X)
    assert np.all(np.log2(sc) == np.round(np.log2(sc)))
    assert np.all(np.max(np.abs(X), axis=0) / sc <= 448.0)
    assert sc[-1] == 1.0
    codes, sc2 = quant.fp8_stage(X)
    back = quant.fp8_unstage(codes, sc2)
    ok = np.abs(X) >= 2.0 ** -6 * sc2[None, :]
    assert np.all(np.abs(back - X)[ok] <= 2.0 ** -4 * np.abs(X)[ok])


def test_bf16_round_special_values():
    """Infinities, signed zeros, NaN (quiet, sign kept), the largest finite
    BF16 value, and overflow: FLT_MAX lies past the midpoint between the
    largest BF16 value and 2^128, so round-to-nearest overflows to inf."""
    from oracle import quant
    bits = np.array([0x7F800000, 0xFF800000, 0x00000000, 0x80000000, 0x7F800001, 0xFF800001,
                     0x7FC00000, 0xFFFFFFFF, 0x7F7F0000, 0x7F7FFFFF, 0x7F7F7FFF, 0x7F7F8000,
                     0x7F7E8000, 0x00000001, 0x00008000, 0x00018000], dtype=np.uint32)
    expect = np.array([0x7F80, 0xFF80, 0x0000, 0x8000, 0x7FC0, 0xFFC0,
                       0x7FC0, 0xFFFF, 0x7F7F, 0x7F80, 0x7F7F, 0x7F80,
                       0x7F7E, 0x0000, 0x0000, 0x0002], dtype=np.uint32)
    got = quant.bf16_round(bits.view(np.float32)).view(np.uint32)
    np.testing.assert_array_equal(got >> 16, expect)
    np.testing.assert_array_equal(got & 0xFFFF, 0)


def test_bf16_round_matches_search_over_all_values():
    """Nearest BF16 value found by searching the ordered list of every finite
    non-negative BF16 value (2^128 standing in for the overflow to inf),
    ties to the even code: an independent route to the same rounding."""
    from oracle import quant
    codes = np.arange(0x0000, 0x7F80, dtype=np.uint32)          # every finite magnitude
    vals = (codes << 16).view(np.float32).astype(np.float64)
    vals = np.append(vals, 2.0 ** 128)
    codes = np.append(codes, 0x7F80)
    rng = np.random.default_rng(3)
    # random patterns over the whole finite range plus dense sweeps at ties
    u = rng.integers(0, 0x7F800000, size=200_000, dtype=np.uint32)
    ties = (rng.integers(0, 0x7F7F, size=20_000, dtype=np.uint32) << 16) | 0x8000
    u = np.concatenate([u, ties, ties + 1, ties - 1])
    x = u.view(np.float32).astype(np.float64)
    hi = np.searchsorted(vals, x, side="left")
    lo = np.maximum(hi - 1, 0)
    dlo, dhi = x - vals[lo], vals[hi] - x
    pick = np.where((dhi < dlo) | ((dhi == dlo) & (codes[hi] % 2 == 0)), hi, lo)
    pick = np.where(vals[hi] == x, hi, pick)
    ref = codes[pick]
    sgn = rng.integers(0, 2, size=u.size).astype(np.uint32)
    got = quant.bf16_round((u | (sgn << 31)).view(np.float32)).view(np.uint32)
    np.testing.assert_array_equal(got >> 16, ref | (sgn << 15))


def test_splitmix64_published_reference_outputs():
    """The first outputs of the published splitmix64.c generator seeded with
    0 (the reference sequence of the generator's public test vectors)."""
    ref = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F,
           0xF88BB8A8724C81EC, 0x1B39896A51A8749B]
    assert [int(v) for v in sketch.splitmix64(0, np.arange(5, dtype=np.uint64))] == ref


# ------------------------------------------------------ statistical dimension
def test_statistical_dimension_definition_and_limits():
    """s_lambda(Z) = tr((Z^T Z + lambda I)^-1 Z^T Z) (Lemma sketching): equal
    to a linear solve, to rank(Z) as lambda -> 0, to d / (1 + lambda) for
    orthonormal columns, and decreasing in lambda."""
    rng = np.random.default_rng(40)
    Z = rng.standard_normal((50, 6)) * np.array([5, 2, 1, .5, .1, .01])
    G = Z.T @ Z
    for lam in [1e-3, 0.3, 7.0, 400.0]:
        ref = np.trace(np.linalg.solve(G + lam * np.eye(6), G))
        assert abs(direct.statistical_dimension(Z, lam) - ref) < 1e-12 * 6
    Q, _ = np.linalg.qr(rng.standard_normal((30, 5)))
    assert abs(direct.statistical_dimension(Q, 0.25) - 5 / 1.25) < 1e-12
    Zr = rng.standard_normal((40, 3)) @ rng.standard_normal((3, 7))      # rank 3
    assert abs(direct.statistical_dimension(Zr, 1e-6) - 3.0) < 1e-5
    vals = [direct.statistical_dimension(Z, lam) for lam in [0.01, 0.1, 1, 10]]
    assert np.all(np.diff(vals) < 0)


# ------------------------------------------------------------ Hessians
def _dense_cca_hessian(U, V, Sxx, Syy, Sxy, Mxx, Myy, mu):
    bu = stiefel.tangent_basis(U, Sxx, Mxx)
    bv = stiefel.tangent_basis(V, Syy, Myy)
    basis = [(b, np.zeros_like(V)) for b in bu] + [(np.zeros_like(U), b) for b in bv]
    m = len(basis)
    H = np.zeros((m, m))
    for a in range(m):
        hu, hv = stiefel.cca_rhess(U, V, Sxx, Syy, Sxy, Mxx, Myy, mu, *basis[a])
        for b in range(m):
            H[b, a] = stiefel.inner(basis[b][0], hu, Mxx) + stiefel.inner(basis[b][1], hv, Myy)
    return H


@pytest.mark.parametrize("dx,dy,p", [(5, 4, 2), (4, 6, 3), (5, 5, 1)])
def test_cca_hessian_spectrum_at_optimum(dx, dy, p):
    """With M = Sigma the Riemannian Hessian (Eq. HessCCA) at the optimum has
    exactly the spectrum of the proof of Theorem CCAHessiantheorem, and its
    condition number is kappa*_CCA."""
    X, Y = synth.cca_latent(90, dx, dy, r=3, noise=0.3, x_decades=1.0, seed=41 + dx + dy)
    lam = 0.05
    Sxx, Syy, Sxy = stiefel.cca_blocks(X, Y, lam, lam)
    mu = np.arange(p, 0, -1, dtype=float) * 1.5
    sig, U, V = direct.cca_direct(X, Y, lam, lam, k=p)
    H = _dense_cca_hessian(U, V, Sxx, Syy, Sxy, Sxx, Syy, mu)
    assert H.shape[0] == p * (dx + dy) - p * (p + 1)
    np.testing.assert_allclose(H, H.T, atol=1e-12 * np.abs(H).max())
    ev = np.sort(np.linalg.eigvalsh(0.5 * (H + H.T)))
    cf = direct.cca_hessian_spectrum(sig, mu, dx, dy)
    np.testing.assert_allclose(ev, cf, rtol=1e-9, atol=1e-12)
    assert ev[0] > 0
    assert abs(ev[-1] / ev[0] - direct.kappa_star_cca(sig, mu)) < 1e-8 * ev[-1] / ev[0]


def test_cca_hessian_condition_bound_with_sketched_metric():
    """Theorem CCAHessiantheorem: kappa(Hess) <= kappa*_CCA kappa(Sigma, M)
    for another SPD metric M (here the sketched one)."""
    X, Y = synth.cca_latent(400, 5, 4, r=3, noise=0.3, x_decades=2.0, seed=44)
    lam = 0.05
    Sxx, Syy, Sxy = stiefel.cca_blocks(X, Y, lam, lam)
    mu = np.array([2.0, 1.0])
    sig, U, V = direct.cca_direct(X, Y, lam, lam, k=2)
    SX = sketch.sketch(X, "countsketch", 60, 45)
    SY = sketch.sketch(Y, "countsketch", 60, 45)
    Mxx = SX.T @ SX + lam * np.eye(5)
    Myy = SY.T @ SY + lam * np.eye(4)
    H = _dense_cca_hessian(U, V, Sxx, Syy, Sxy, Mxx, Myy, mu)
    ev = np.linalg.eigvalsh(0.5 * (H + H.T))
    gx = sla.eigh(Sxx, Mxx, eigvals_only=True)
    gy = sla.eigh(Syy, Myy, eigvals_only=True)
    kap_m = max(gx.max(), gy.max()) / min(gx.min(), gy.min())
    assert ev.min() > 0
    assert ev.max() / ev.min() <= direct.kappa_star_cca(sig, mu) * kap_m * (1 + 1e-9)


def test_lda_hessian_spectrum_at_optimum():
    """With M = S_w + lam I the Riemannian Hessian (Eq. LDAhess) at the
    optimum has the spectrum of the proof of Theorem LDAHessiantheorem and
    condition number kappa*_FDA."""
    X, y = synth.lda_classes(152, 6, 4, decades=1.0, seed=46)
    lam = 0.2
    mu = np.array([3.0, 2.0, 1.0])
    rho, W = direct.lda_direct(X, y, 4, lam, k=3)
    _, _, _, Xh, Yh = direct.lda_scatter(X, y, 4)
    B = Xh.T @ Xh + lam * np.eye(6)
    SB = Yh.T @ Yh
    bas = stiefel.tangent_basis(W, B, B)
    m = len(bas)
    assert m == 3 * 6 - 6
    H = np.zeros((m, m))
    for a in range(m):
        h = stiefel.lda_rhess(W, B, SB, B, mu, bas[a])
        for b in range(m):
            H[b, a] = stiefel.inner(bas[b], h, B)
    np.testing.assert_allclose(H, H.T, atol=1e-12 * np.abs(H).max())
    ev = np.sort(np.linalg.eigvalsh(0.5 * (H + H.T)))
    rho_all = np.concatenate([rho, np.zeros(6 - len(rho))])    # rank S_B <= c - 1
    np.testing.assert_allclose(ev, direct.lda_hessian_spectrum(rho_all, mu), rtol=1e-9,
                               atol=1e-12 * rho[0])
    assert abs(ev[-1] / ev[0] - direct.kappa_star_fda(rho_all, mu)) < 1e-8 * ev[-1] / ev[0]


def _fd_hessian(grad_field, X, xi, h=1e-5):
    """Central difference of the extended gradient field Y -> grad(Y) along xi
    (projected on T_X by the caller): the Levi-Civita derivative on a
    Riemannian submanifold of the constant-metric ambient space."""
    return (grad_field(X + h * xi) - grad_field(X - h * xi)) / (2 * h)


def test_cca_hessian_matches_differentiated_gradient_field():
    """Away from critical points, with a non-trivial metric: Hess f[xi] =
    Pi_Z(D grad f[xi]) for the extension of the gradient formula off the
    manifold, and the Hessian is self-adjoint in the metric."""
    X, Y = synth.cca_latent(90, 5, 4, r=3, noise=0.3, x_decades=1.0, seed=47)
    lam = 0.1
    Sxx, Syy, Sxy = stiefel.cca_blocks(X, Y, lam, lam)
    rng = np.random.default_rng(48)
    Mxx, Myy = _spd(5, rng, 5) * 40, _spd(4, rng, 5) * 40
    mu = np.array([3.0, 2.0])
    U = _point(5, 2, Sxx, rng)
    V = _point(4, 2, Syy, rng)
    xu = stiefel.project(U, Sxx, Mxx, rng.standard_normal((5, 2)))
    xv = stiefel.project(V, Syy, Myy, rng.standard_normal((4, 2)))
    hu, hv = stiefel.cca_rhess(U, V, Sxx, Syy, Sxy, Mxx, Myy, mu, xu, xv)
    h = 1e-5
    gp = stiefel.cca_rgrad(U + h * xu, V + h * xv, Sxx, Syy, Sxy, Mxx, Myy, mu)
    gm = stiefel.cca_rgrad(U - h * xu, V - h * xv, Sxx, Syy, Sxy, Mxx, Myy, mu)
    fu = stiefel.project(U, Sxx, Mxx, (gp[0] - gm[0]) / (2 * h))
    fv = stiefel.project(V, Syy, Myy, (gp[1] - gm[1]) / (2 * h))
    scale = np.linalg.norm(hu) + np.linalg.norm(hv)
    assert np.linalg.norm(fu - hu) + np.linalg.norm(fv - hv) < 1e-7 * scale
    eu = stiefel.project(U, Sxx, Mxx, rng.standard_normal((5, 2)))
    ev = stiefel.project(V, Syy, Myy, rng.standard_normal((4, 2)))
    ku, kv = stiefel.cca_rhess(U, V, Sxx, Syy, Sxy, Mxx, Myy, mu, eu, ev)
    a = stiefel.inner(eu, hu, Mxx) + stiefel.inner(ev, hv, Myy)
    b = stiefel.inner(xu, ku, Mxx) + stiefel.inner(xv, kv, Myy)
    assert abs(a - b) < 1e-10 * max(1.0, abs(a))


def test_lda_hessian_matches_differentiated_gradient_field():
    X, y = synth.lda_classes(100, 6, 4, decades=1.0, seed=49)
    _, _, _, Xh, Yh = direct.lda_scatter(X, y, 4)
    lam = 0.5
    B = Xh.T @ Xh + lam * np.eye(6)
    SB = Yh.T @ Yh
    rng = np.random.default_rng(50)
    M = _spd(6, rng, 8) * 30
    mu = np.array([3.0, 2.0, 1.0])
    W = _point(6, 3, B, rng)
    xi = stiefel.project(W, B, M, rng.standard_normal((6, 3)))
    hx = stiefel.lda_rhess(W, B, SB, M, mu, xi)
    fd = stiefel.project(W, B, M, _fd_hessian(lambda Z: stiefel.lda_rgrad(Z, B, SB, M, mu), W, xi))
    assert np.linalg.norm(fd - hx) < 1e-7 * np.linalg.norm(hx)
    eta = stiefel.project(W, B, M, rng.standard_normal((6, 3)))
    he = stiefel.lda_rhess(W, B, SB, M, mu, eta)
    assert abs(stiefel.inner(eta, hx, M) - stiefel.inner(xi, he, M)) < 1e-10 * np.linalg.norm(hx) ** 2


# ------------------------------------------------------- metrics: negatives
def test_constraint_residual_flags_a_scaled_point():
    """U scaled by (1 + eps) has U^T Sxx U = (1 + eps)^2 I: residual 2 eps + eps^2."""
    X, Y = _rand_cca(seed=51)
    lam = 0.05
    _, U, V = direct.cca_direct(X, Y, lam, lam, k=3)
    for eps in [1e-7, 1e-4, 0.1]:
        r = metrics.constraint_residual((1 + eps) * U, X, lam)
        assert abs(r - (2 * eps + eps * eps)) < 1e-12 + 1e-9 * eps


def test_objective_error_of_a_rotated_point_is_closed_form():
    """Rotating the last column of the optimum towards the next canonical
    pair by theta (u_k -> cos u_k + sin u_{k+1}, same for v) keeps the
    constraints and, since u_i^T Sxy v_j = sigma_i delta_ij, lowers the
    objective by sin^2 theta (sigma_k - sigma_{k+1}): the metric must report
    exactly that."""
    X, Y = _rand_cca(n=120, dx=6, dy=5, seed=52)
    lam = 0.05
    sig, U, V = direct.cca_direct(X, Y, lam, lam, k=3)
    for th in [1e-3, 0.1, 0.7]:
        U2, V2 = U[:, :2].copy(), V[:, :2].copy()
        U2[:, 1] = np.cos(th) * U[:, 1] + np.sin(th) * U[:, 2]
        V2[:, 1] = np.cos(th) * V[:, 1] + np.sin(th) * V[:, 2]
        err = metrics.cca_rel_objective_error(U2, V2, X, Y, lam, lam, sig)
        # tr(U2^T Sxy V2) = sigma_1 + cos^2 sigma_2 + sin^2 sigma_3
        expect = (sig[1] - (np.cos(th) ** 2 * sig[1] + np.sin(th) ** 2 * sig[2])) / (sig[0] + sig[1])
        assert abs(err - expect) < 1e-12 + 1e-9 * expect
        assert metrics.constraint_residual(U2, X, lam) < 1e-10


def test_objective_error_of_random_feasible_points_is_positive():
    """Any feasible point scores at most sum sigma_i (von Neumann / Ky Fan):
    random qf points score strictly below it, and their weighted
    sub-optimality is positive."""
    X, Y = _rand_cca(n=100, dx=6, dy=5, seed=53)
    lam = 0.05
    sig, _, _ = direct.cca_direct(X, Y, lam, lam, k=2)
    Sxx, Syy, Sxy = stiefel.cca_blocks(X, Y, lam, lam)
    rng = np.random.default_rng(54)
    mu = np.array([2.0, 1.0])
    for _ in range(20):
        U = stiefel.qf_B(rng.standard_normal((6, 2)), Sxx)
        V = stiefel.qf_B(rng.standard_normal((5, 2)), Syy)
        assert metrics.cca_objective(U, V, X, Y, lam, lam) < sig[0] + sig[1]
        assert metrics.cca_rel_objective_error(U, V, X, Y, lam, lam, sig) > 1e-6
        assert metrics.weighted_suboptimality(sig, stiefel.cca_cost(U, V, Sxy, mu), mu) > 1e-6


def test_lda_objective_error_of_a_rotated_point_is_closed_form():
    X, y = synth.lda_classes(150, 6, 5, decades=1.0, seed=55)
    lam = 0.2
    rho, W = direct.lda_direct(X, y, 5, lam, k=3)
    _, _, _, Xh, Yh = direct.lda_scatter(X, y, 5)
    th = 0.3
    W2 = W[:, :2].copy()
    W2[:, 1] = np.cos(th) * W[:, 1] + np.sin(th) * W[:, 2]
    err = metrics.lda_rel_objective_error(W2, Xh, Yh, lam, rho)
    expect = (rho[1] - (np.cos(th) ** 2 * rho[1] + np.sin(th) ** 2 * rho[2])) / (rho[0] + rho[1])
    assert abs(err - expect) < 1e-12 + 1e-9 * expect


def test_principal_angles_of_a_plane_rotation():
    th = 0.37
    A = np.array([[1.0], [0.0], [0.0]])
    B = np.array([[np.cos(th)], [np.sin(th)], [0.0]])
    assert abs(metrics.principal_angles(A, B)[0] - th) < 1e-14
    S = np.diag([4.0, 1.0, 1.0])     # S-inner product of e_1 and (1, 2, 0)
    a = metrics.principal_angles(A, np.array([[1.0], [2.0], [0.0]]), S)[0]
    assert abs(np.cos(a) - 4.0 / (2.0 * np.sqrt(8.0))) < 1e-14   # <A,B>_S / (|A|_S |B|_S)


# ----------------------------------------------------------- CSR oracle
def _csr_case(n, d, per_row, seed):
    X, _ = synth.cca_sparse(n, d, 3, per_row=per_row, seed=seed, dtype=np.float64)
    return X


def test_csr_to_dense_matches_loop_and_scipy():
    import scipy.sparse as sp
    from oracle import sparse as osp
    X = _csr_case(300, 40, 6, 3)
    A = osp.csr_to_dense(X.row_ptr, X.col_idx, X.values, X.n_cols)
    L = np.zeros_like(A)
    for i in range(X.shape[0]):
        for e in range(X.row_ptr[i], X.row_ptr[i + 1]):
            L[i, X.col_idx[e]] += X.values[e]
    assert np.array_equal(A, L)
    S = sp.csr_matrix((X.values, X.col_idx, X.row_ptr), shape=X.shape).toarray()
    assert np.array_equal(A, S)
    assert np.any(np.diff(X.row_ptr) == 0)   # the pattern holds empty rows


@pytest.mark.parametrize("n,d,s", [(500, 30, 64), (1, 5, 3), (200, 1, 16)])
def test_csr_countsketch_matches_dense_definition(n, d, s):
    from oracle import sparse as osp
    X = _csr_case(n, d, 4, 11)
    A = osp.csr_to_dense(X.row_ptr, X.col_idx, X.values, X.n_cols)
    h, g = sketch.countsketch_hash(n, s, 7)
    got = osp.countsketch_csr(X.row_ptr, X.col_idx, X.values, X.n_cols, h, g, s)
    np.testing.assert_allclose(got, sketch.countsketch_apply(A, h, g, s), rtol=1e-14, atol=1e-13)
    np.testing.assert_allclose(got, sketch.countsketch_matrix(h, g, s) @ A, rtol=1e-14, atol=1e-13)


def test_csr_pass_matches_dense_products():
    from oracle import sparse as osp
    X, Y = synth.cca_sparse(400, 30, 20, per_row=5, seed=4, dtype=np.float64)
    rng = np.random.default_rng(0)
    W0, W1 = rng.standard_normal((30, 3)), rng.standard_normal((20, 3))
    A0 = osp.csr_to_dense(X.row_ptr, X.col_idx, X.values, X.n_cols)
    A1 = osp.csr_to_dense(Y.row_ptr, Y.col_idx, Y.values, Y.n_cols)
    blocks = [(X.row_ptr, X.col_idx, X.values, X.n_cols), (Y.row_ptr, Y.col_idx, Y.values, Y.n_cols)]
    J0, J1 = osp.pass_csr(blocks, [W0, W1])
    P = np.hstack([A0 @ W0, A1 @ W1])
    np.testing.assert_allclose(J0, A0.T @ P, rtol=1e-12, atol=1e-11)
    np.testing.assert_allclose(J1, A1.T @ P, rtol=1e-12, atol=1e-11)
    (J,) = osp.pass_csr(blocks[:1], [W0])
    np.testing.assert_allclose(J, A0.T @ (A0 @ W0), rtol=1e-12, atol=1e-11)


def test_closed_form_and_metrics_take_sparse_matrices():
    """The CCA closed form and the metrics on scipy sparse input equal
    those on the same matrices made dense."""
    import scipy.sparse as sps
    from oracle import sparse as osp
    X, Y = synth.cca_sparse(600, 25, 18, per_row=6, seed=9, dtype=np.float64)
    Xs = sps.csr_matrix((X.values, X.col_idx, X.row_ptr), shape=X.shape)
    Ys = sps.csr_matrix((Y.values, Y.col_idx, Y.row_ptr), shape=Y.shape)
    Xd, Yd = Xs.toarray(), Ys.toarray()
    s1, U1, V1 = direct.cca_direct(Xs, Ys, 1e-2, 1e-2, k=4)
    s2, U2, V2 = direct.cca_direct(Xd, Yd, 1e-2, 1e-2, k=4)
    np.testing.assert_allclose(s1, s2, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(U1, U2, rtol=1e-9, atol=1e-12)
    assert metrics.constraint_residual(U1, Xs, 1e-2) == pytest.approx(metrics.constraint_residual(U1, Xd, 1e-2),
                                                                       abs=1e-14)
    assert metrics.cca_rel_objective_error(U1, V1, Xs, Ys, 1e-2, 1e-2, s2) < 1e-13
