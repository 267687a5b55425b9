"""Direct (closed-form) regularised CCA and FDA in FP64.

Parity status: pinned.  ``tests/test_oracle_pins.py`` checks these against
a dense generalized symmetric eigensolve, the Y = X closed form, planted
correlations, invariance under invertible column transforms (lambda = 0),
the two-class FDA closed form, and the constraint / diagonality conditions
of the definitions.  The Hessian spectra and kappa* are pinned to the
eigenvalues of the dense Riemannian Hessian operator (``stiefel``) at the
optimum; the statistical dimension to a linear solve and its closed forms
(rank at lambda -> 0, d / (1 + lambda) for orthonormal columns).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.linalg import solve_triangular


def _f64(a):
    """FP64 view of a matrix; a scipy sparse matrix stays sparse (its
    products below are sparse products, made dense)."""
    if sp.issparse(a):
        return sp.csr_matrix(a, dtype=np.float64)
    return np.asarray(a, dtype=np.float64)


def _gram(A, B):
    """A^T B as a dense FP64 array (A, B dense or scipy sparse)."""
    G = A.T @ B
    return G.toarray() if sp.issparse(G) else np.asarray(G)


def sign_normalize(U: np.ndarray, V: np.ndarray | None = None):
    """Column sign convention: flip column i (of U and, jointly, of V) so the
    entry of largest magnitude in U[:, i] is positive; ties go to the lowest
    index.  The optimum is unique only up to such joint flips (Theorem
    criticalpointofCCA, Theorem criticalpointsofLDA)."""
    U = U.copy()
    V = None if V is None else V.copy()
    for i in range(U.shape[1]):
        j = int(np.argmax(np.abs(U[:, i])))
        if U[j, i] < 0:
            U[:, i] = -U[:, i]
            if V is not None:
                V[:, i] = -V[:, i]
    return (U, V) if V is not None else U


def cca_direct(X, Y, lam_x: float, lam_y: float, k: int | None = None):
    """lambda-canonical correlations and weights (Definition of regularised
    CCA, Section 4): maximise tr(U^T X^T Y V) subject to
    U^T (X^T X + lam_x I) U = I, V^T (Y^T Y + lam_y I) V = I, with
    U^T X^T Y V diagonal and non-increasing.

    Closed form: with Sxx = Lx Lx^T and Syy = Ly Ly^T (Cholesky), the
    correlations are the singular values of C = Lx^-1 Sxy Ly^-T, and the
    weights are U = Lx^-T Uc, V = Ly^-T Vc (any square root of Sxx, Syy gives
    the same singular values; Appendix B, proof of Theorem
    criticalpointofCCA, uses the symmetric one).

    Returns ``(sigma_all, U, V)`` with ``sigma_all`` all min(dx, dy)
    correlations in descending order and ``U``, ``V`` the first ``k``
    weight columns, sign-normalised.
    """
    X = _f64(X)
    Y = _f64(Y)
    dx, dy = X.shape[1], Y.shape[1]
    if k is None:
        k = min(dx, dy)
    Sxx = _gram(X, X) + lam_x * np.eye(dx)
    Syy = _gram(Y, Y) + lam_y * np.eye(dy)
    Sxy = _gram(X, Y)
    Lx = np.linalg.cholesky(Sxx)
    Ly = np.linalg.cholesky(Syy)
    C = solve_triangular(Lx, Sxy, lower=True)               # Lx^-1 Sxy
    C = solve_triangular(Ly, C.T, lower=True).T             # ... Ly^-T
    Uc, sig, Vct = np.linalg.svd(C)
    U = solve_triangular(Lx.T, Uc[:, :k], lower=False)      # Lx^-T Uc
    V = solve_triangular(Ly.T, Vct[:k, :].T, lower=False)   # Ly^-T Vc
    U, V = sign_normalize(U, V)
    return sig, U, V


def cca_direct_qr(X, Y, lam_x: float, lam_y: float, k: int | None = None):
    """Same solution through the lambda-QR factorisation (the factorisation
    named in the proof of Lemma sketching): R from the QR of
    [X; sqrt(lam) I] satisfies R^T R = X^T X + lam I without forming the
    Gram.  Then C = (X Rx^-1)^T (Y Ry^-1).  Slower; more accurate when the
    data are badly conditioned."""
    X = _f64(X)
    Y = _f64(Y)
    dx, dy = X.shape[1], Y.shape[1]
    if k is None:
        k = min(dx, dy)
    Rx = np.linalg.qr(np.vstack([X, np.sqrt(lam_x) * np.eye(dx)]), mode="r")
    Ry = np.linalg.qr(np.vstack([Y, np.sqrt(lam_y) * np.eye(dy)]), mode="r")
    Rx *= np.sign(np.diag(Rx))[:, None]
    Ry *= np.sign(np.diag(Ry))[:, None]
    Qx = solve_triangular(Rx, X.T, trans="T", lower=False).T   # X Rx^-1
    Qy = solve_triangular(Ry, Y.T, trans="T", lower=False).T
    Uc, sig, Vct = np.linalg.svd(Qx.T @ Qy)
    U = solve_triangular(Rx, Uc[:, :k], lower=False)
    V = solve_triangular(Ry, Vct[:k, :].T, lower=False)
    U, V = sign_normalize(U, V)
    return sig, U, V


def lda_scatter(X, labels, c: int):
    """Class counts, means and the factors of Section 5.1: Xhat has rows
    x_i - m_{y_i} (so S_w = Xhat^T Xhat), Yhat has rows sqrt(n_k)(m_k - m)
    (so S_B = Yhat^T Yhat)."""
    X = _f64(X)
    labels = np.asarray(labels)
    nk = np.bincount(labels, minlength=c).astype(np.float64)
    if np.any(nk == 0):
        raise ValueError("empty class")
    sums = np.zeros((c, X.shape[1]))
    np.add.at(sums, labels, X)
    means = sums / nk[:, None]
    m = X.sum(axis=0) / X.shape[0]
    Xhat = X - means[labels]
    Yhat = np.sqrt(nk)[:, None] * (means - m[None, :])
    return nk, means, m, Xhat, Yhat


def lda_direct(X, labels, c: int, lam: float, k: int | None = None):
    """Regularised FDA (Definition of FDA, Section 5; problem Eq. LDAprob):
    the leading generalized eigenpairs of (S_B, S_w + lam I).

    Closed form: B = Xhat^T Xhat + lam I = L L^T; G = Yhat L^-T (c x d); the
    SVD G = P diag(gamma) Q^T gives rho = gamma^2 and W = L^-T Q[:, :k], so
    W^T B W = I and W^T S_B W = diag(rho).

    Returns ``(rho_all, W)`` with ``rho_all`` the min(c, d) largest
    generalized eigenvalues in descending order.
    """
    _, _, _, Xhat, Yhat = lda_scatter(X, labels, c)
    d = Xhat.shape[1]
    if k is None:
        k = min(c - 1, d)
    B = Xhat.T @ Xhat + lam * np.eye(d)
    L = np.linalg.cholesky(B)
    G = solve_triangular(L, Yhat.T, lower=True).T            # Yhat L^-T
    _, gam, Qt = np.linalg.svd(G, full_matrices=False)
    rho = gam ** 2
    W = solve_triangular(L.T, Qt[:k, :].T, lower=False)
    W = sign_normalize(W)
    return rho, W


def cca_hessian_spectrum(sigma, mu, dx: int, dy: int) -> np.ndarray:
    """Eigenvalues of the Riemannian Hessian at the CCA optimum with the
    metric M = Sigma (proof of Theorem CCAHessiantheorem, Appendix B), for
    sigma_1 > ... > sigma_p > sigma_{p+1} >= ... the min(dx, dy) canonical
    correlations and N = diag(mu):
    mu_j (sigma_j + sigma_i) and mu_j (sigma_j - sigma_i) for j <= p < i;
    mu_j sigma_j, |dx - dy| times each; and for j < i <= p the pair
    (mu_j + mu_i)(sigma_j + sigma_i) / 2, (mu_j - mu_i)(sigma_j - sigma_i) / 2.
    Sorted ascending; p d - p (p + 1) values in all (d = dx + dy)."""
    mu = np.asarray(mu, dtype=np.float64)
    s = np.asarray(sigma, dtype=np.float64)
    p = len(mu)
    q = min(dx, dy)
    ev = []
    for j in range(p):
        for i in range(p, q):
            ev += [mu[j] * (s[j] + s[i]), mu[j] * (s[j] - s[i])]
        ev += [mu[j] * s[j]] * abs(dx - dy)
        for i in range(j + 1, p):
            ev += [0.5 * (mu[j] + mu[i]) * (s[j] + s[i]), 0.5 * (mu[j] - mu[i]) * (s[j] - s[i])]
    return np.sort(np.array(ev))


def lda_hessian_spectrum(rho, mu) -> np.ndarray:
    """Eigenvalues of the Riemannian Hessian at the FDA optimum with the
    metric M = S_w + lam I (proof of Theorem LDAHessiantheorem, Appendix C),
    for rho the d generalized eigenvalues in descending order:
    mu_j (rho_j - rho_i) for j <= p < i <= d, and
    (mu_j - mu_i)(rho_j - rho_i) / 2 for j < i <= p.  Sorted ascending;
    p d - p (p + 1) / 2 values."""
    mu = np.asarray(mu, dtype=np.float64)
    r = np.asarray(rho, dtype=np.float64)
    p, d = len(mu), len(r)
    ev = []
    for j in range(p):
        ev += [mu[j] * (r[j] - r[i]) for i in range(p, d)]
        ev += [0.5 * (mu[j] - mu[i]) * (r[j] - r[i]) for i in range(j + 1, p)]
    return np.sort(np.array(ev))


def kappa_star_cca(sigma, mu) -> float:
    """kappa*_CCA of Theorem CCAHessiantheorem: the largest over the
    smallest value of the spectrum above (needs sigma_1..sigma_{p+1})."""
    p = len(mu)
    s = np.asarray(sigma, dtype=np.float64)
    num = mu[0] * (s[0] + s[p])
    if p > 1:
        num = max(num, 0.5 * (mu[0] + mu[1]) * (s[0] + s[1]))
    den = mu[p - 1] * (s[p - 1] - s[p])
    for j in range(p - 1):
        den = min(den, 0.5 * (mu[j] - mu[j + 1]) * (s[j] - s[j + 1]))
    return float(num / den)


def kappa_star_fda(rho, mu) -> float:
    """kappa*_FDA of Theorem LDAHessiantheorem (rho over all d values)."""
    p = len(mu)
    r = np.asarray(rho, dtype=np.float64)
    num = mu[0] * (r[0] - r[-1])
    den = mu[p - 1] * (r[p - 1] - r[p])
    for j in range(p - 1):
        den = min(den, 0.5 * (mu[j] - mu[j + 1]) * (r[j] - r[j + 1]))
    return float(num / den)


def statistical_dimension(Z, lam: float) -> float:
    """s_lambda(Z) = tr((Z^T Z + lam I)^-1 Z^T Z) (Lemma sketching)."""
    Z = _f64(Z)
    G = Z.T @ Z
    ev = np.linalg.eigvalsh(G)
    ev = np.clip(ev, 0.0, None)
    return float(np.sum(ev / (ev + lam)))
