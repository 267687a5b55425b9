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
