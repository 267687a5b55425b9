"""Seeded synthetic workloads for sketched Riemannian CCA / FDA.

This module only draws data.  It holds none of the method's arithmetic:
no sketch, no Gram, no factorisation, no solver step.  Both the FP64 CPU
oracle (``oracle/``) and the GPU library's tests and benchmark take their
inputs from here, so the two sides see bit-identical matrices.

Workload shapes follow the paper's setting of tall data with samples in
rows (Section 2, Section 4 problem statement, Section 5 problem statement):

* CCA: ``X`` (n x dx) and ``Y`` (n x dy) share a Gaussian latent factor
  ``Z`` (n x r) whose columns have strengths ``a_j = 10^(-fdec*j/r)``;
  ``X = (Z diag(a) Wx + noise*E) diag(cx)``, ``Y = (Z diag(a) Wy +
  noise*E') diag(cy)`` with geometric column scales
  ``c_j = 10^(-decades*j/(d-1))`` (or ``10^(-decades*j/d)``) that make
  ``X^T X`` ill conditioned the way the paper's synthetic experiment asks
  for (Section 6.2).  Spread strengths separate the canonical correlations;
  equal strengths with little noise cluster them near 1.
* FDA: ``c`` classes with exactly ``n/c`` samples each (shuffled), class
  means drawn from ``N(0, mean_std^2 I)``, and a shared within-class
  covariance ``Q diag(lam) Q^T`` with ``lam_j = 10^(-decades*j/d)`` and a
  Haar-random orthogonal ``Q``.
* Planted CCA: matrices whose canonical correlations are known exactly,
  used to pin the oracle.

All draws use ``numpy.random.default_rng(seed)`` (PCG64), except
``cca_latent_device``: the same latent recipe drawn directly in device
memory with torch's device generator (for the serving trace, whose 512
requests hold about 1e11 bytes of data; the host could not draw them in
reasonable time).
"""
from __future__ import annotations

import dataclasses

import numpy as np

__all__ = [
    "column_scales", "cca_latent", "cca_latent_device", "lda_classes", "planted_cca",
    "Workload", "workload", "serving_trace", "WORKLOADS", "sparse_signs",
    "CsrArrays", "sparse_pattern", "cca_sparse", "lda_sparse", "SparseWorkload", "SPARSE_WORKLOADS",
]


def column_scales(d: int, decades: float, inclusive_end: bool) -> np.ndarray:
    """Geometric column scales 1 -> 10^-decades.

    ``inclusive_end=True`` gives ``10^(-decades*j/(d-1))`` (last column is
    exactly ``10^-decades``); ``False`` gives ``10^(-decades*j/d)``.
    """
    if decades == 0 or d == 1:
        return np.ones(d)
    j = np.arange(d, dtype=np.float64)
    den = (d - 1) if inclusive_end else d
    return 10.0 ** (-decades * j / den)


def cca_latent(n: int, dx: int, dy: int, *, r: int, noise: float = 0.1,
               x_decades: float = 0.0, y_decades: float = 0.0,
               inclusive_end: bool = True, seed: int = 0,
               dtype=np.float64, factor_decades: float = 0.0):
    """Two views of one Gaussian latent factor (rows are samples)."""
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((n, r))
    if factor_decades:
        Z *= 10.0 ** (-factor_decades * np.arange(r) / r)[None, :]
    Wx = rng.standard_normal((r, dx))
    Wy = rng.standard_normal((r, dy))
    X = Z @ Wx
    X += noise * rng.standard_normal((n, dx))
    Y = Z @ Wy
    Y += noise * rng.standard_normal((n, dy))
    if x_decades:
        X *= column_scales(dx, x_decades, inclusive_end)[None, :]
    if y_decades:
        Y *= column_scales(dy, y_decades, inclusive_end)[None, :]
    return (np.ascontiguousarray(X, dtype=dtype),
            np.ascontiguousarray(Y, dtype=dtype))


def cca_latent_device(n: int, dx: int, dy: int, *, r: int, noise: float = 0.1,
                      x_decades: float = 0.0, y_decades: float = 0.0,
                      inclusive_end: bool = True, seed: int = 0, device="cuda",
                      factor_decades: float = 0.0):
    """``cca_latent``'s recipe drawn on the device in FP32 (torch's
    device generator seeded with ``seed``; a different stream from the
    host version, same distribution)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    f32 = torch.float32
    Z = torch.randn((n, r), generator=g, device=device, dtype=f32)
    if factor_decades:
        Z.mul_(torch.from_numpy(10.0 ** (-factor_decades * np.arange(r) / r)).to(device=device, dtype=f32)[None, :])
    out = []
    for d, dec in ((dx, x_decades), (dy, y_decades)):
        W = torch.randn((r, d), generator=g, device=device, dtype=f32)
        A = torch.randn((n, d), generator=g, device=device, dtype=f32)
        A.mul_(noise).addmm_(Z, W)
        if dec:
            A.mul_(torch.from_numpy(column_scales(d, dec, inclusive_end)).to(device=device, dtype=f32)[None, :])
        out.append(A.contiguous())
    return out[0], out[1]


def haar_orthogonal(d: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed orthogonal matrix (QR of a Gaussian, signs fixed)."""
    G = rng.standard_normal((d, d))
    Q, Rg = np.linalg.qr(G)
    Q *= np.sign(np.diag(Rg))[None, :]
    return Q


def lda_classes(n: int, d: int, c: int, *, mean_std: float = 2.0,
                decades: float = 6.0, haar: bool = True, seed: int = 0,
                dtype=np.float64):
    """Labelled samples with equal priors and a shared covariance.

    Returns ``(X, labels)`` with ``labels`` int32 in ``[0, c)``; every class
    has exactly ``n // c`` samples (``n`` must be a multiple of ``c``).
    """
    if n % c:
        raise ValueError("n must be a multiple of c for equal priors")
    rng = np.random.default_rng(seed)
    labels = np.repeat(np.arange(c, dtype=np.int32), n // c)
    rng.shuffle(labels)
    means = mean_std * rng.standard_normal((c, d))
    lam = 10.0 ** (-decades * np.arange(d, dtype=np.float64) / d)
    Q = haar_orthogonal(d, rng) if haar else np.eye(d)
    G = rng.standard_normal((n, d))
    G *= np.sqrt(lam)[None, :]
    X = G @ Q.T
    X += means[labels]
    return np.ascontiguousarray(X, dtype=dtype), labels


def sparse_signs(n: int, d: int, per_row: int, *, seed: int = 0, cols=None,
                 dtype=np.float32) -> np.ndarray:
    """n x d matrix with ``per_row`` entries of +-1 per row at random
    columns (drawn from ``cols`` when given; a repeated column adds up), the
    rest zero: small integers, so that every sum of products with small
    integers is exact in FP32."""
    rng = np.random.default_rng(seed)
    cols = np.arange(d) if cols is None else np.asarray(cols)
    idx = cols[rng.integers(0, len(cols), size=(n, per_row))]
    vals = rng.choice(np.array([-1.0, 1.0]), size=(n, per_row))
    X = np.zeros((n, d), dtype=np.float64)
    np.add.at(X, (np.repeat(np.arange(n), per_row), idx.reshape(-1)), vals.reshape(-1))
    return X.astype(dtype)


@dataclasses.dataclass
class CsrArrays:
    """A CSR matrix as host arrays: row_ptr (int64, n + 1), col_idx (int32,
    strictly increasing within a row), values, and the column count."""
    row_ptr: np.ndarray
    col_idx: np.ndarray
    values: np.ndarray
    n_cols: int

    @property
    def shape(self):
        return (len(self.row_ptr) - 1, self.n_cols)

    @property
    def nnz(self):
        return len(self.col_idx)


def sparse_pattern(n: int, d: int, per_row: float, rng: np.random.Generator, *, alpha: float = 0.7,
                   empty_frac: float = 0.02):
    """Sparsity pattern of a bag-of-words-like matrix: row i draws about
    ``per_row`` columns (Poisson count) from a Zipf-like popularity
    p_j ~ (j + 1)^-alpha, duplicates merged; a fraction ``empty_frac`` of the
    rows is left empty.  Returns (row_ptr int64, col_idx int32, row of each
    entry int64), entries in row order with ascending columns."""
    counts = rng.poisson(per_row, n)
    counts[rng.random(n) < empty_frac] = 0
    p = (np.arange(d) + 1.0) ** -alpha
    p /= p.sum()
    rows = np.repeat(np.arange(n, dtype=np.int64), counts)
    cols = rng.choice(d, size=rows.size, p=p)
    key = np.unique(rows * d + cols)
    rows, cols = key // d, key % d
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr[1:])
    return row_ptr, cols.astype(np.int32), rows


def cca_sparse(n: int, dx: int, dy: int, *, per_row: float = 16, r: int = 8, noise: float = 0.5,
               seed: int = 0, dtype=np.float32, integer: bool = False):
    """Two sparse views of one Gaussian latent factor: both views share the
    rows' latent z_i (r-dimensional); an entry (i, j) of view X, at a
    sparse position, holds z_i . a_j + noise * e with a_j ~ N(0, I_r) per
    column, so the views correlate through z on their supports.  With
    ``integer`` the values are instead drawn from {-2, -1, 1, 2} (exact in
    any summation order).  Returns (X, Y) as CsrArrays."""
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((n, r))
    out = []
    for d in (dx, dy):
        row_ptr, cols, rows = sparse_pattern(n, d, per_row, rng)
        if integer:
            vals = rng.choice(np.array([-2.0, -1.0, 1.0, 2.0]), size=cols.size)
        else:
            A = rng.standard_normal((d, r))
            vals = np.empty(cols.size)
            for b0 in range(0, cols.size, 1 << 22):
                b1 = min(cols.size, b0 + (1 << 22))
                vals[b0:b1] = np.einsum("ij,ij->i", Z[rows[b0:b1]], A[cols[b0:b1]])
            vals += noise * rng.standard_normal(cols.size)
        out.append(CsrArrays(row_ptr, cols, vals.astype(dtype), d))
    return out[0], out[1]


def lda_sparse(n: int, d: int, c: int, *, per_row: float = 24, mean_std: float = 1.0, noise: float = 0.5,
               seed: int = 0, dtype=np.float32):
    """Sparse labelled samples: labels uniform over c classes (every class
    present); an entry (i, j) at a sparse position holds mu[y_i, j] +
    noise * e, with class means mu ~ N(0, mean_std^2).  Returns
    (X as CsrArrays, labels int32)."""
    rng = np.random.default_rng(seed)
    labels = rng.integers(0, c, size=n).astype(np.int32)
    labels[:c] = np.arange(c, dtype=np.int32)
    means = mean_std * rng.standard_normal((c, d))
    row_ptr, cols, rows = sparse_pattern(n, d, per_row, rng)
    vals = means[labels[rows], cols] + noise * rng.standard_normal(cols.size)
    return CsrArrays(row_ptr, cols, vals.astype(dtype), d), labels


def planted_cca(n: int, r: int, rho, *, seed: int = 0, dtype=np.float64):
    """CCA pair with canonical correlations exactly ``rho`` (lambda = 0).

    ``X = E1 A`` and ``Y = (E1 diag(rho) + E2 diag(sqrt(1-rho^2))) B`` where
    ``[E1 E2]`` has orthonormal columns (n x 2r) and ``A``, ``B`` are
    invertible r x r.  Then the canonical correlations of (X, Y) are the
    entries of ``rho`` and the weights are ``A^-1`` / ``B^-1`` columns.
    Returns ``(X, Y, A, B)``.
    """
    rho = np.asarray(rho, dtype=np.float64)
    assert rho.shape == (r,)
    rng = np.random.default_rng(seed)
    E, _ = np.linalg.qr(rng.standard_normal((n, 2 * r)))
    E1, E2 = E[:, :r], E[:, r:]
    A = rng.standard_normal((r, r)) + 3.0 * np.eye(r)
    B = rng.standard_normal((r, r)) + 3.0 * np.eye(r)
    X = E1 @ A
    Y = (E1 * rho[None, :] + E2 * np.sqrt(1.0 - rho ** 2)[None, :]) @ B
    return (np.ascontiguousarray(X, dtype=dtype),
            np.ascontiguousarray(Y, dtype=dtype), A, B)


@dataclasses.dataclass(frozen=True)
class Workload:
    """One named synthetic workload (sizes and generator recipe)."""
    name: str
    problem: str          # "cca" or "lda"
    n: int
    dx: int
    dy: int               # 0 for LDA
    k: int
    lam: float            # lambda_x = lambda_y; LDA: NaN means the 1e-6 rule
    sketch: str           # "countsketch" or "srht"
    s: int
    dtype: str            # data dtype: "f64", "f32", "bf16"
    seed: int
    r: int = 8            # latent rank (CCA)
    x_decades: float = 0.0
    y_decades: float = 0.0
    inclusive_end: bool = True
    c: int = 0            # classes (LDA)
    noise: float = 0.1    # CCA noise level
    factor_decades: float = 0.0   # CCA latent strengths 10^(-fdec j / r)

    @property
    def lam_value(self) -> float:
        """lambda_x = lambda_y for CCA; the population 1e-6 rule for FDA."""
        if self.problem == "lda":
            return lda_population_lambda(self.n, self.dx)
        return self.lam

    def generate(self):
        np_dtype = np.float64 if self.dtype == "f64" else np.float32
        if self.problem == "cca":
            return cca_latent(self.n, self.dx, self.dy, r=self.r, noise=self.noise,
                              factor_decades=self.factor_decades,
                              x_decades=self.x_decades,
                              y_decades=self.y_decades,
                              inclusive_end=self.inclusive_end,
                              seed=self.seed, dtype=np_dtype)
        return lda_classes(self.n, self.dx, self.c, seed=self.seed,
                           dtype=np_dtype)

    def scaled(self, n: int | None = None, dx: int | None = None,
               dy: int | None = None, s: int | None = None,
               name: str | None = None) -> "Workload":
        """Same recipe at other sizes (for tests that the oracle finishes)."""
        return dataclasses.replace(
            self, n=n or self.n, dx=dx or self.dx,
            dy=(dy if dy is not None else self.dy), s=s or self.s,
            name=name or self.name + "-scaled")


WORKLOADS = {
    # FP64 CCA, CountSketch s = 4 dx, X columns scaled 1 -> 1e-3; latent
    # strengths over one decade (top correlations 2-10 % apart).
    "cca-f64-small": Workload("cca-f64-small", "cca", 2000, 60, 40, 5, 1e-3,
                              "countsketch", 240, "f64", 12060 + 0, r=8,
                              x_decades=3.0, inclusive_end=True,
                              noise=1.0, factor_decades=1.0),
    # FP32 CCA, SRHT s = 4000, both views scaled 10^(-4j/d); latent
    # strengths over two decades (top-10 correlations 3e-4 to 5e-3 apart).
    "cca-f32-srht": Workload("cca-f32-srht", "cca", 200_000, 1000, 1000, 10,
                             1e-4, "srht", 4000, "f32", 12060 + 1, r=32,
                             x_decades=4.0, y_decades=4.0,
                             inclusive_end=False, noise=1.0,
                             factor_decades=2.0),
    # The same shape with the recipe exactly as the FP32 CCA configuration
    # states it: latent Z ~ N(0, 1) of rank 32 with equal strengths, noise
    # 0.1 (the top 32 correlations then sit within ~1e-5 of 1).
    "cca-f32-srht-cfg1": Workload("cca-f32-srht-cfg1", "cca", 200_000, 1000, 1000, 10,
                                  1e-4, "srht", 4000, "f32", 12060 + 1, r=32,
                                  x_decades=4.0, y_decades=4.0,
                                  inclusive_end=False, noise=0.1,
                                  factor_decades=0.0),
    # FP32 FDA, CountSketch s = 8000 of the centred data, 20 classes.
    "lda-f32": Workload("lda-f32", "lda", 100_000, 2000, 0, 19, float("nan"),
                        "countsketch", 8000, "f32", 12060 + 2, c=20),
    # Precision variant of the FP32 CCA workload (BF16 data and GEMMs).
    "cca-bf16-srht": Workload("cca-bf16-srht", "cca", 200_000, 1000, 1000, 10,
                              1e-4, "srht", 4000, "bf16", 12060 + 1, r=32,
                              x_decades=4.0, y_decades=4.0,
                              inclusive_end=False, noise=1.0,
                              factor_decades=2.0),
}


@dataclasses.dataclass(frozen=True)
class SparseWorkload:
    """A CSR CCA workload (``cca_sparse`` recipe, CountSketch, FP32 values)."""
    name: str
    n: int
    dx: int
    dy: int
    k: int
    lam: float
    s: int
    per_row: float
    r: int = 8
    noise: float = 0.5
    seed: int = 0
    problem: str = "cca"
    sketch: str = "countsketch"
    dtype: str = "f32"

    def generate(self):
        return cca_sparse(self.n, self.dx, self.dy, per_row=self.per_row, r=self.r, noise=self.noise,
                          seed=self.seed, dtype=np.float32)


# Bag-of-words-like sparse views (the regime the paper states its costs
# for: nnz(X), nnz(Y) << n d): one million rows, 1000 columns per view,
# about 24 stored entries per row with Zipf-like column popularity; k = 8,
# the latent rank (the 9th correlation is in the noise bulk, 10x lower).
SPARSE_WORKLOADS = {
    "cca-csr": SparseWorkload("cca-csr", 1_000_000, 1000, 1000, 8, 1e-3, 4000, 24, seed=12065),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]


def lda_population_lambda(n: int, d: int, decades: float = 6.0) -> float:
    """Regularisation for the FDA workload: 1e-6 times the mean eigenvalue
    of the within-class scatter (the paper's synthetic rule, Section 6.2),
    taken at its population value ``n * mean_j 10^(-decades*j/d)`` so that
    it is fixed by the recipe rather than estimated from the draw."""
    lam = 10.0 ** (-decades * np.arange(d, dtype=np.float64) / d)
    return 1e-6 * n * float(lam.mean())


@dataclasses.dataclass(frozen=True)
class Request:
    rid: int
    arrival_s: float
    n: int
    dx: int
    dy: int
    k: int
    seed: int


def serving_trace(num: int = 512, rate_per_s: float = 200.0, *,
                  n_range=(5000, 100_000), d_range=(64, 1024),
                  k_range=(2, 16), seed: int = 12064):
    """Poisson arrivals with independent uniform sizes per request."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=num)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(num):
        out.append(Request(
            rid=i, arrival_s=float(t[i]),
            n=int(rng.integers(n_range[0], n_range[1] + 1)),
            dx=int(rng.integers(d_range[0], d_range[1] + 1)),
            dy=int(rng.integers(d_range[0], d_range[1] + 1)),
            k=int(rng.integers(k_range[0], k_range[1] + 1)),
            seed=1_000_000 + i))
    return out

