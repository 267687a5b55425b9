"""CSR data by definition (FP64): the dense matrix a CSR triple stands for,
its CountSketch (Section 3) and the data products of the iteration
(Table costs: their cost is in terms of nnz), written as sums over the
stored entries.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Parity status: pinned.  Tests check ``csr_to_dense`` against an entry-by-
entry loop and against scipy's CSR conversion, ``countsketch_csr`` against
the dense ``sketch.countsketch_apply`` (and the explicit S matrix) of the
same matrix, and ``pass_csr`` against dense products of the densified
matrices; zero rows, a single row and a single column are among the cases.
"""
from __future__ import annotations

import numpy as np


def _rows_of_entries(row_ptr) -> np.ndarray:
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    return np.repeat(np.arange(len(row_ptr) - 1, dtype=np.int64), np.diff(row_ptr))


def csr_to_dense(row_ptr, col_idx, values, n_cols: int) -> np.ndarray:
    """A (n x n_cols, FP64) with A[i, col_idx[e]] = values[e] for the
    entries e of row i, zeros elsewhere (column indices distinct in a row)."""
    n = len(row_ptr) - 1
    A = np.zeros((n, n_cols))
    A[_rows_of_entries(row_ptr), np.asarray(col_idx, dtype=np.int64)] = np.asarray(values, dtype=np.float64)
    return A


def countsketch_csr(row_ptr, col_idx, values, n_cols: int, h, g, s: int) -> np.ndarray:
    """(S A)[b, j] = sum over the stored entries (i, j) with h(i) = b of
    g(i) A[i, j]: the CountSketch of Section 3 restricted to the nonzeros."""
    rows = _rows_of_entries(row_ptr)
    out = np.zeros((s, n_cols))
    np.add.at(out, (np.asarray(h)[rows], np.asarray(col_idx, dtype=np.int64)),
              np.asarray(g)[rows] * np.asarray(values, dtype=np.float64))
    return out


def times_dense(row_ptr, col_idx, values, W) -> np.ndarray:
    """A W for the CSR matrix A: row i = sum over its entries of
    A[i, j] W[j, :]."""
    rows = _rows_of_entries(row_ptr)
    W = np.asarray(W, dtype=np.float64)
    out = np.zeros((len(row_ptr) - 1, W.shape[1]))
    np.add.at(out, rows, np.asarray(values, dtype=np.float64)[:, None] * W[np.asarray(col_idx, dtype=np.int64)])
    return out


def transpose_times_dense(row_ptr, col_idx, values, n_cols: int, P) -> np.ndarray:
    """A^T P for the CSR matrix A: row j = sum over the entries (i, j) of
    A[i, j] P[i, :]."""
    rows = _rows_of_entries(row_ptr)
    P = np.asarray(P, dtype=np.float64)
    out = np.zeros((n_cols, P.shape[1]))
    np.add.at(out, np.asarray(col_idx, dtype=np.int64), np.asarray(values, dtype=np.float64)[:, None] * P[rows])
    return out


def pass_csr(blocks, Ws):
    """J_b = A_b^T [A_0 W_0 | A_1 W_1] for CSR blocks A_b (given as
    (row_ptr, col_idx, values, n_cols)): the data products the Riemannian
    gradient, projection and retraction consume (Eq. gradCCA, Table 1)."""
    P = np.hstack([times_dense(b[0], b[1], b[2], W) for b, W in zip(blocks, Ws)])
    return [transpose_times_dense(b[0], b[1], b[2], b[3], P) for b in blocks]
