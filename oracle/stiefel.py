"""Preconditioned generalized-Stiefel components (Table 1) and the CCA /
FDA costs, in plain FP64 with explicitly formed d x d matrices.

St_B(p, d) = {X : X^T B X = I}, metric g(xi, eta) = tr(xi^T M eta) for a
fixed SPD preconditioner M (Section 3 uses the sketched
M = Z^T S^T S Z + lam I).  For CCA the manifold is the product
St_Sxx x St_Syy with metric blkdiag(Mxx, Myy) and every component acts
block by block (Section 4.2).

Parity status: pinned.  Tests check tangency, idempotence and
M-self-adjointness of the projection, that the Sylvester solve reduces to
S = sym(X^T B xi) when M = B (Appendix B), that the Cholesky form of the QR
retraction equals B^-1/2 qf(B^1/2 (X + xi)) literally, that the retraction
lands on the manifold, and that the Riemannian gradient reproduces finite
differences of the cost along retraction curves.  The Riemannian Hessians
are pinned to the closed-form spectra at the optimum with M = B (proofs of
Theorems CCAHessiantheorem and LDAHessiantheorem, Appendices B and C), to
central differences of the extended gradient field projected on the
tangent space (the Levi-Civita connection of a Riemannian submanifold of
the constant-metric ambient space), and to self-adjointness in the metric.
"""
from __future__ import annotations

import numpy as np


def sym(A):
    return 0.5 * (A + A.T)


def inner(xi, eta, M) -> float:
    """Riemannian metric tr(xi^T M eta) (Table 1)."""
    return float(np.trace(xi.T @ M @ eta))


def sylvester_kron(A, C):
    """Solve A S + S A = C (A SPD k x k) through the Kronecker form
    (I (x) A + A^T (x) I) vec(S) = vec(C)."""
    k = A.shape[0]
    K = np.kron(np.eye(k), A) + np.kron(A.T, np.eye(k))
    s = np.linalg.solve(K, C.reshape(-1, order="F"))
    return s.reshape((k, k), order="F")


def normal_coeff(X, B, M, xi):
    """S_xi of Table 1: (X^T B M^-1 B X) S + S (X^T B M^-1 B X) =
    X^T B xi + (X^T B xi)^T."""
    BX = B @ X
    A = BX.T @ np.linalg.solve(M, BX)
    C = BX.T @ xi
    return sylvester_kron(A, C + C.T)


def project(X, B, M, xi):
    """Orthogonal projection on T_X St_B in the M-metric (Table 1):
    xi - M^-1 B X S_xi."""
    S = normal_coeff(X, B, M, xi)
    return xi - np.linalg.solve(M, B @ X) @ S


def retract_qr(X, xi, B):
    """QR retraction (Table 1): B^-1/2 qf(B^1/2 (X + xi)), computed as
    (X + xi) L^-T with L L^T = (X + xi)^T B (X + xi), since qf(A) = A R^-1
    for the positive-diagonal R of A = QR and R^T R = A^T A."""
    Y = X + xi
    L = np.linalg.cholesky(Y.T @ B @ Y)
    return np.linalg.solve(L, Y.T).T


def retract_qr_literal(X, xi, B):
    """The same retraction written with B^1/2 and a Householder QR."""
    w, Q = np.linalg.eigh(B)
    Bh = (Q * np.sqrt(w)) @ Q.T
    Bmh = (Q / np.sqrt(w)) @ Q.T
    Qf, Rf = np.linalg.qr(Bh @ (X + xi))
    Qf = Qf * np.sign(np.diag(Rf))[None, :]
    return Bmh @ Qf


def transport(X_new, B, M, xi):
    """Vector transport by projection onto the new tangent space."""
    return project(X_new, B, M, xi)


def qf_B(X, B):
    """qf_B(X) = B^-1/2 qf(B^1/2 X): the start point map of Algorithms
    CCAopt and LDAopt."""
    return retract_qr(X, np.zeros_like(X), B)


def rhess(X, B, M, egrad, ehess_eta, rgrad, eta):
    """Riemannian Hessian applied to a tangent vector (Table 1):
    Pi_X(M^-1 (D^2 f[eta] - B eta (X^T grad_E f - X^T M grad f))), with the
    Euclidean gradient ``egrad``, the Euclidean Hessian applied to eta
    ``ehess_eta`` and the Riemannian gradient ``rgrad`` at X.  Valid for a
    constant metric M, the case of the sketched preconditioner."""
    inner_kk = X.T @ egrad - X.T @ M @ rgrad
    return project(X, B, M, np.linalg.solve(M, ehess_eta - B @ eta @ inner_kk))


def tangent_basis(X, B, M):
    """M-orthonormal basis (list of d x p matrices) of T_X St_B(p, d), of
    dimension p d - p (p + 1) / 2: the projections of the canonical basis,
    orthonormalised in the metric tr(xi^T M eta) (Table 1)."""
    d, p = X.shape
    cols = []
    for i in range(d):
        for j in range(p):
            E = np.zeros((d, p))
            E[i, j] = 1.0
            cols.append(project(X, B, M, E).reshape(-1))
    A = np.array(cols).T                      # (d p) x (d p) spanning set
    G = A.T @ np.kron(M, np.eye(p)) @ A       # metric Gram of the set
    w, Q = np.linalg.eigh(G)
    keep = w > 1e-10 * w.max()
    Bas = A @ (Q[:, keep] / np.sqrt(w[keep]))
    return [Bas[:, i].reshape(d, p) for i in range(Bas.shape[1])]


# --------------------------------------------------------------- CCA ---
def cca_blocks(X, Y, lam_x, lam_y):
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    Sxx = X.T @ X + lam_x * np.eye(X.shape[1])
    Syy = Y.T @ Y + lam_y * np.eye(Y.shape[1])
    Sxy = X.T @ Y
    return Sxx, Syy, Sxy


def cca_cost(U, V, Sxy, mu) -> float:
    """f_CCA(Z) = -1/2 tr(Z^T [[0, Sxy], [Sxy^T, 0]] Z N)
    = -tr(U^T Sxy V N) (Eq. costriemannianccaBrockett)."""
    return -float(np.sum(np.diag(U.T @ Sxy @ V) * np.asarray(mu)))


def cca_egrad(U, V, Sxy, mu):
    """Euclidean gradient of the extended cost: -[Sxy V N; Sxy^T U N]."""
    N = np.diag(mu)
    return -(Sxy @ V @ N), -(Sxy.T @ U @ N)


def cca_rgrad(U, V, Sxx, Syy, Sxy, Mxx, Myy, mu):
    """Riemannian gradient, Eq. gradCCA:
    -[Pi_U(Mxx^-1 Sxy V N); Pi_V(Myy^-1 Sxy^T U N)]."""
    gu, gv = cca_egrad(U, V, Sxy, mu)
    return (project(U, Sxx, Mxx, np.linalg.solve(Mxx, gu)),
            project(V, Syy, Myy, np.linalg.solve(Myy, gv)))


def cca_rhess(U, V, Sxx, Syy, Sxy, Mxx, Myy, mu, xu, xv):
    """Riemannian Hessian of the CCA cost applied to (xu, xv), Eq. HessCCA:
    Pi_Z(M^-1 [-Sigma_cca xi N + Sigma (xi_U U^T Sxy V N ; xi_V V^T Sxy^T U N)
    + Sigma (xi_U U^T ; xi_V V^T) M grad f]), block by block on the product
    manifold (the Table 1 formula with grad_E f = -[Sxy V N; Sxy^T U N] and
    D^2 f[xi] = -[Sxy xi_V N; Sxy^T xi_U N])."""
    N = np.diag(mu)
    gu, gv = cca_rgrad(U, V, Sxx, Syy, Sxy, Mxx, Myy, mu)
    eu, ev = cca_egrad(U, V, Sxy, mu)
    hu = rhess(U, Sxx, Mxx, eu, -(Sxy @ xv @ N), gu, xu)
    hv = rhess(V, Syy, Myy, ev, -(Sxy.T @ xu @ N), gv, xv)
    return hu, hv


# --------------------------------------------------------------- FDA ---
def lda_cost(W, SB, mu) -> float:
    """f_FDA(W) = -1/2 tr(W^T S_B W N) (Eq. lda_riemannian)."""
    return -0.5 * float(np.sum(np.diag(W.T @ SB @ W) * np.asarray(mu)))


def lda_egrad(W, SB, mu):
    """Euclidean gradient -S_B W N (the differential of the cost above)."""
    return -(SB @ W @ np.diag(mu))


def lda_rgrad(W, B, SB, M, mu):
    """Riemannian gradient Pi_W(M^-1 grad f) (Table 1 applied to the FDA
    cost; Eq. LDAgrad read as grad = Pi(M^-1 (-S_B W N)), its printed
    second term being the first written out)."""
    return project(W, B, M, np.linalg.solve(M, lda_egrad(W, SB, mu)))


def lda_rhess(W, B, SB, M, mu, xi):
    """Riemannian Hessian of the FDA cost applied to xi, Eq. LDAhess:
    Pi_W(M^-1 [-S_B xi N + B xi (W^T S_B W N + W^T M grad f)]).  The printed
    equation adds grad f (d x p) to a p x p matrix; it is read as W^T M grad f,
    the term of the Table 1 formula with grad_E f = -S_B W N."""
    N = np.diag(mu)
    g = lda_rgrad(W, B, SB, M, mu)
    return rhess(W, B, M, lda_egrad(W, SB, mu), -(SB @ xi @ N), g, xi)


# ----------------------------------------------------- data products ---
def data_products(A0, W0, A1=None, W1=None):
    """J_b = A_b^T [A_0 W_0 | A_1 W_1] in FP64: the products with the data
    matrices that the Riemannian components consume (Table costs).  Also
    returns the entrywise magnitudes |A_b|^T [|A_0||W_0| | |A_1||W_1|] that
    bound the rounding error of any summation order."""
    A0 = np.asarray(A0, dtype=np.float64)
    W0 = np.asarray(W0, dtype=np.float64)
    P = [A0 @ W0]
    Pa = [np.abs(A0) @ np.abs(W0)]
    As = [A0]
    if A1 is not None:
        A1 = np.asarray(A1, dtype=np.float64)
        W1 = np.asarray(W1, dtype=np.float64)
        P.append(A1 @ W1)
        Pa.append(np.abs(A1) @ np.abs(W1))
        As.append(A1)
    Pc = np.hstack(P)
    Pac = np.hstack(Pa)
    J = [A.T @ Pc for A in As]
    Jabs = [np.abs(A).T @ Pac for A in As]
    return J, Jabs
