"""Sketches with fewer rows than columns (s < d): the metric kept in
Woodbury form (closing remark after Table costs).  The fixed point does not
depend on the metric, so every solve must reach the oracle's closed form."""
import numpy as np
import pytest

import synth
from oracle import direct, metrics
from oracle import sparse as osp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda"

# lambda large enough that the statistical dimension (65 here) sits well
# below the sketch size: with the noise eigenvalues of X^T X near 4e3-6e3
# the preconditioned Gram's condition number is about 6 at s = 150.  The
# latent strengths span one decade, so the top correlations are apart
# (0.994, 0.988, 0.976, 0.946, 0.890, 0.820).
LAM = 2e4


def _srp():
    import paper_2106_12060_amd as srp
    return srp


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.mark.parametrize("s,dt,method,sketch", [
    (150, np.float64, "rcg", "countsketch"),   # both views in Woodbury form
    (250, np.float64, "rcg", "srht"),          # X in Woodbury form, Y (200 columns) dense
    (150, np.float32, "rcg", "countsketch"),
    (150, np.float64, "rtr", "countsketch"),
])
def test_cca_woodbury_reaches_closed_form(s, dt, method, sketch):
    srp = _srp()
    X, Y = synth.cca_latent(20_000, 300, 200, r=6, noise=0.5, seed=3, dtype=dt, factor_decades=1.0)
    sig_true, _, _ = direct.cca_direct(X, Y, LAM, LAM)
    k = 5
    f64 = dt == np.float64
    opt = srp.srp_default_options(sketch=sketch, method=method, max_iter=1000, final_f64=0 if f64 else 3)
    U, V, sig, info = srp.cca_solve(dev(X), dev(Y), k, LAM, LAM, s, tol=1e-11 if f64 else 1e-6, options=opt)
    X64, Y64 = X.astype(np.float64), Y.astype(np.float64)
    Uh, Vh = U.cpu().numpy(), V.cpu().numpy()
    err = metrics.cca_rel_objective_error(Uh, Vh, X64, Y64, LAM, LAM, sig_true)
    cons = max(metrics.constraint_residual(Uh, X64, LAM), metrics.constraint_residual(Vh, Y64, LAM))
    print("woodbury cca", s, dt.__name__, method, sketch, info, err, cons)
    assert info["status"] == 0 and info["warm_iterations"] > 0
    bar = 1e-10 if f64 else 1e-6
    assert err < bar and cons < bar
    np.testing.assert_allclose(sig.cpu().numpy(), sig_true[:k], rtol=0, atol=1e-8 if f64 else 1e-5)


def test_lda_woodbury_reaches_closed_form():
    srp = _srp()
    n, d, c, k, s = 19_992, 300, 12, 4, 120
    X, y = synth.lda_classes(n, d, c, decades=2.0, seed=4)
    _, _, _, Xh, Yh = direct.lda_scatter(X, y, c)
    # about 5 times the mean within-class eigenvalue (4.3e3): the
    # preconditioned Gram's condition number is 3.3 at s = 120
    lam = 2e4
    rho_true, _ = direct.lda_direct(X, y, c, lam, k=k)
    W, rho, info = srp.lda_solve(dev(X), dev(y), c, k, lam, s, tol=1e-11,
                                 options=srp.srp_default_options(max_iter=1000))
    Wh = W.cpu().numpy()
    err = metrics.lda_rel_objective_error(Wh, Xh, Yh, lam, rho_true)
    cons = metrics.constraint_residual(Wh, Xh, lam)
    print("woodbury lda", info, err, cons)
    assert info["status"] == 0
    assert err < 1e-10 and cons < 1e-11
    np.testing.assert_allclose(rho.cpu().numpy(), rho_true[:k], rtol=1e-9)


def test_csr_cca_woodbury():
    srp = _srp()
    # column popularity spreads X^T X over 1e3 .. 4e5: lambda = 3e4 puts the
    # preconditioned Gram's condition number near 5 at s = 120
    n, dx, dy, k, s, lam = 30_000, 300, 200, 5, 120, 3e4
    Xs, Ys = synth.cca_sparse(n, dx, dy, per_row=14, r=8, seed=21, dtype=np.float32)
    Xd = osp.csr_to_dense(Xs.row_ptr, Xs.col_idx, Xs.values, dx)
    Yd = osp.csr_to_dense(Ys.row_ptr, Ys.col_idx, Ys.values, dy)
    sig_true, _, _ = direct.cca_direct(Xd, Yd, lam, lam)
    to = lambda M: srp.Csr(dev(M.row_ptr), dev(M.col_idx), dev(M.values), M.n_cols)
    U, V, sig, info = srp.cca_solve_csr(to(Xs), to(Ys), k, lam, lam, s, tol=1e-11,
                                        options=srp.srp_default_options(max_iter=1000))
    Uh, Vh = U.cpu().numpy(), V.cpu().numpy()
    err = metrics.cca_rel_objective_error(Uh, Vh, Xd, Yd, lam, lam, sig_true)
    cons = max(metrics.constraint_residual(Uh, Xd, lam), metrics.constraint_residual(Vh, Yd, lam))
    print("woodbury csr", info, err, cons)
    assert info["status"] == 0
    assert err < 1e-10 and cons < 1e-11


def test_woodbury_needs_positive_lambda():
    srp = _srp()
    X = torch.randn(500, 40, dtype=torch.float64, device=DEV)
    Y = torch.randn(500, 30, dtype=torch.float64, device=DEV)
    with pytest.raises(srp.SrpError) as e:
        srp.cca_solve(X, Y, 2, 0.0, 1.0, 35)
    assert e.value.code == srp.SRP_EINVAL
    y = (torch.arange(500, device=DEV) % 5).to(torch.int32)
    with pytest.raises(srp.SrpError) as e:
        srp.lda_solve(X, y, 5, 2, 0.0, 20)
    assert e.value.code == srp.SRP_EINVAL
