"""Sketching transforms by definition (FP64), and the draw of their
randomness from a counter-based generator.

Parity status: pinned.  Tests check the bucket-sum form against the
explicit CountSketch matrix, that an injective hash gives S^T S = I, the
fast Walsh-Hadamard transform against the Sylvester-construction dense
Hadamard matrix, that the SRHT with s = n' preserves the Gram matrix
exactly, that E[S^T S] = I over seeds, and the SplitMix64 outputs against
an independent arbitrary-precision evaluation of its published definition.

Randomness (one stream per purpose, each the sequence of SplitMix64
outputs for a derived seed; the i-th output is ``splitmix64(seed, i)``):

* CountSketch row i: w = splitmix64(seed, i); bucket
  h(i) = ((w >> 32) * s) >> 32, sign g(i) = +1 if bit 0 of w is 0 else -1.
  (Section 3: h maps the n rows -- the paper prints the domain as
  {1..d}, read here as the row index set, since S is s x n.)
* SRHT signs: D_i = +1 if bit 0 of splitmix64(seed ^ SRHT_SIGN_SALT, i) is
  0 else -1, for i in [0, n').
* SRHT rows: the s indices r in [0, n') with the smallest keys
  splitmix64(seed ^ SRHT_ROW_SALT, r) (ties to the smaller index), in
  ascending order: a uniform sample without replacement (Definition SRHT).
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15
SRHT_SIGN_SALT = 0x5352485444494147   # arbitrary salts: distinct streams
SRHT_ROW_SALT = 0x535248545357524F


def splitmix64(seed: int, idx) -> np.ndarray:
    """i-th output (0-based) of SplitMix64 seeded with ``seed``.

    Published definition (Steele, Lea, Flood, "Fast splittable pseudorandom
    number generators", OOPSLA 2014; Vigna's splitmix64.c): the state
    advances by the golden gamma 0x9E3779B97F4A7C15 before each output, and
    the output is the state passed through the mix
    z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27;
    z *= 0x94D049BB133111EB; z ^= z >> 31 (all mod 2^64).
    """
    i = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & MASK64) + (i + np.uint64(1)) * np.uint64(GOLDEN_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def splitmix64_reference(seed: int, i: int) -> int:
    """The same definition evaluated with Python integers (a second,
    independent route used to pin the vectorised one)."""
    state = (seed + (i + 1) * GOLDEN_GAMMA) & MASK64
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def countsketch_hash(n: int, s: int, seed: int):
    """Bucket h (int64 in [0, s)) and sign g (+-1.0) for each of n rows."""
    w = splitmix64(seed, np.arange(n, dtype=np.uint64))
    h = ((w >> np.uint64(32)) * np.uint64(s)) >> np.uint64(32)
    g = np.where((w & np.uint64(1)) == 0, 1.0, -1.0)
    return h.astype(np.int64), g


def countsketch_matrix(h, g, s: int) -> np.ndarray:
    """Dense S (s x n): column j holds g(j) in row h(j) (Section 3)."""
    n = len(h)
    S = np.zeros((s, n))
    S[np.asarray(h), np.arange(n)] = g
    return S


def countsketch_apply(X, h, g, s: int) -> np.ndarray:
    """(S X)_b = sum over rows j with h(j) = b of g(j) X_j (Section 3)."""
    X = np.asarray(X, dtype=np.float64)
    out = np.zeros((s, X.shape[1]))
    np.add.at(out, np.asarray(h), np.asarray(g)[:, None] * X)
    return out


def srht_padded_rows(n: int) -> int:
    """n' = smallest power of two >= n (at least 2)."""
    p = 1
    while p < max(n, 2):
        p <<= 1
    return p


def srht_signs(n_pad: int, seed: int) -> np.ndarray:
    w = splitmix64(seed ^ SRHT_SIGN_SALT, np.arange(n_pad, dtype=np.uint64))
    return np.where((w & np.uint64(1)) == 0, 1.0, -1.0)


def srht_rows(n_pad: int, s: int, seed: int) -> np.ndarray:
    """s distinct rows of [0, n') chosen uniformly without replacement (the
    s smallest random keys), returned in ascending order."""
    keys = splitmix64(seed ^ SRHT_ROW_SALT, np.arange(n_pad, dtype=np.uint64))
    order = np.lexsort((np.arange(n_pad), keys))   # by key, then by index
    return np.sort(order[:s]).astype(np.int64)


def hadamard(n_pad: int) -> np.ndarray:
    """Unnormalised Sylvester Hadamard matrix, H[r, i] = (-1)^popcount(r&i)."""
    H = np.ones((1, 1))
    while H.shape[0] < n_pad:
        H = np.block([[H, H], [H, -H]])
    return H


def fwht_rows(A: np.ndarray) -> np.ndarray:
    """Unnormalised Walsh-Hadamard transform along axis 0 (H A), by the
    butterfly recursion H_{2m} = [[H_m, H_m], [H_m, -H_m]]."""
    A = np.array(A, dtype=np.float64, copy=True)
    n = A.shape[0]
    h = 1
    while h < n:
        A = A.reshape(n // (2 * h), 2, h, -1)
        a = A[:, 0].copy()
        b = A[:, 1].copy()
        A[:, 0] = a + b
        A[:, 1] = a - b
        A = A.reshape(n, -1)
        h *= 2
    return A


def srht_apply(X, D, rows, s: int, dense_limit: int = 4096) -> np.ndarray:
    """S X with S = sqrt(n'/s) R H D (Definition SRHT; the printed scale
    sqrt(s/n) is read as sqrt(n'/s) with H normalised, so that
    E[S^T S] = I), X zero-padded to n' rows.  Net factor 1/sqrt(s) on the
    unnormalised +-1 Hadamard matrix."""
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    n_pad = len(D)
    Xp = np.zeros((n_pad, d))
    Xp[:n] = X
    Xp *= np.asarray(D)[:, None]
    rows = np.asarray(rows)
    if n_pad <= dense_limit:
        HX = hadamard(n_pad)[rows] @ Xp
    else:
        HX = fwht_rows(Xp)[rows]
    return HX / np.sqrt(s)


def sketch(X, kind: str, s: int, seed: int) -> np.ndarray:
    """S X for the library's sketch kinds with its seeded randomness."""
    n = np.asarray(X).shape[0]
    if kind == "countsketch":
        h, g = countsketch_hash(n, s, seed)
        return countsketch_apply(X, h, g, s)
    if kind == "srht":
        n_pad = srht_padded_rows(n)
        return srht_apply(X, srht_signs(n_pad, seed), srht_rows(n_pad, s, seed), s)
    raise ValueError(kind)


def sketch_factor(SX, lam: float) -> np.ndarray:
    """Upper-triangular R with positive diagonal and R^T R =
    (S X)^T (S X) + lam I: the Cholesky factor of the preconditioner M
    (Section 3; equal to the R of the QR of [S X; sqrt(lam) I])."""
    SX = np.asarray(SX, dtype=np.float64)
    G = SX.T @ SX + lam * np.eye(SX.shape[1])
    return np.linalg.cholesky(G).T
