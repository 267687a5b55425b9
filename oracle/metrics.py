"""Quality measures for a candidate solution, all in FP64 on the host.

* constraint residual max|U^T (X^T X + lam I) U - I| (Definition of
  regularised CCA, Section 4; FDA analogue Eq. LDAprob);
* relative objective error of tr(U'^T X^T Y V') against the sum of the
  top-k correlations, after an FP64 re-orthonormalisation U' = qf_Sxx(U)
  so that an infeasible point earns no credit;
* the paper's weighted sub-optimality |sum mu_i sigma_i + f(Z)| /
  sum mu_i sigma_i (Section 6.1);
* principal angles between subspaces.

Parity status: pinned.  Besides reading zero at the oracle's solution,
tests check that they flag wrong answers by the amounts the definitions
fix: a point scaled by (1 + eps) has constraint residual 2 eps + eps^2; a
column rotated by theta towards the next canonical pair loses exactly
sin^2 theta (sigma_k - sigma_{k+1}) of the objective (CCA and FDA); random
feasible points score below sum sigma_i (Ky Fan) with positive weighted
sub-optimality; principal angles of a plane rotation equal its angle.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _mat(Z):
    """FP64 data matrix; scipy sparse matrices stay sparse (Z @ U is then
    a sparse product with a dense result)."""
    return sp.csr_matrix(Z, dtype=np.float64) if sp.issparse(Z) else np.asarray(Z, dtype=np.float64)


def _qf(U, S):
    L = np.linalg.cholesky(U.T @ S @ U)
    return np.linalg.solve(L, U.T).T


def constraint_residual(U, Z, lam) -> float:
    U = np.asarray(U, dtype=np.float64)
    Z = _mat(Z)
    ZU = Z @ U
    G = ZU.T @ ZU + lam * (U.T @ U)
    return float(np.max(np.abs(G - np.eye(U.shape[1]))))


def cca_objective(U, V, X, Y, lam_x, lam_y, reorth: bool = True) -> float:
    """tr(U^T X^T Y V), optionally after FP64 qf re-orthonormalisation."""
    U = np.asarray(U, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    X = _mat(X)
    Y = _mat(Y)
    XU = X @ U
    YV = Y @ V
    if reorth:
        Lx = np.linalg.cholesky(XU.T @ XU + lam_x * U.T @ U)
        Ly = np.linalg.cholesky(YV.T @ YV + lam_y * V.T @ V)
        XU = np.linalg.solve(Lx, XU.T).T
        YV = np.linalg.solve(Ly, YV.T).T
    return float(np.trace(XU.T @ YV))


def cca_rel_objective_error(U, V, X, Y, lam_x, lam_y, sigma_true) -> float:
    k = np.asarray(U).shape[1]
    ref = float(np.sum(np.asarray(sigma_true)[:k]))
    return abs(ref - cca_objective(U, V, X, Y, lam_x, lam_y)) / ref


def lda_objective(W, Xhat, Yhat, lam, reorth: bool = True) -> float:
    """tr(W^T S_B W) after FP64 re-orthonormalisation in the
    (S_w + lam I)-inner product."""
    W = np.asarray(W, dtype=np.float64)
    XW = np.asarray(Xhat, dtype=np.float64) @ W
    YW = np.asarray(Yhat, dtype=np.float64) @ W
    if reorth:
        L = np.linalg.cholesky(XW.T @ XW + lam * W.T @ W)
        YW = np.linalg.solve(L, YW.T).T
    return float(np.sum(YW * YW))


def lda_rel_objective_error(W, Xhat, Yhat, lam, rho_true) -> float:
    k = np.asarray(W).shape[1]
    ref = float(np.sum(np.asarray(rho_true)[:k]))
    return abs(ref - lda_objective(W, Xhat, Yhat, lam)) / ref


def weighted_suboptimality(values_true, f_value, mu) -> float:
    """|sum mu_i v_i + f| / sum mu_i v_i (Section 6.1)."""
    mu = np.asarray(mu, dtype=np.float64)
    ref = float(np.sum(mu * np.asarray(values_true)[:len(mu)]))
    return abs(ref + f_value) / ref


def principal_angles(A, B, S=None):
    """Principal angles between span(A) and span(B) in the S-inner product
    (S = I when None)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    if S is None:
        S = np.eye(A.shape[0])
    Qa = _qf(A, S)
    Qb = _qf(B, S)
    c = np.linalg.svd(Qa.T @ S @ Qb, compute_uv=False)
    return np.arccos(np.clip(c, -1.0, 1.0))
