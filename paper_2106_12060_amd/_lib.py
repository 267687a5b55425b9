"""ctypes binding of ``libsrp.so`` (the C ABI in ``include/srp.h``).

Argument marshalling only: every step of the computation runs in the HIP
library.  Tensors are torch tensors on the current HIP device; outputs are
allocated here with torch (device memory) and filled by the library on
torch's current stream.  A missing library raises immediately: there is
no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsrp.so")

SRP_OK, SRP_EINVAL, SRP_ENOTSPD, SRP_ENOCONV, SRP_ENOMEM, SRP_EDEVICE = 0, 1, 2, 3, 4, 5
SRP_EBUSY, SRP_EREJECTED, SRP_PENDING = 6, 7, 8
SRP_F64, SRP_F32, SRP_BF16, SRP_FP8E4M3 = 0, 1, 2, 3
SRP_COUNTSKETCH, SRP_SRHT = 0, 1
SRP_RCG, SRP_RTR = 0, 1

STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOTSPD", 3: "ENOCONV", 4: "ENOMEM",
                5: "EDEVICE", 6: "EBUSY", 7: "EREJECTED", 8: "PENDING"}

# uint8 tensors hold FP8 E4M3 codes (sketch input only)
_DTYPES = {torch.float64: SRP_F64, torch.float32: SRP_F32, torch.bfloat16: SRP_BF16, torch.uint8: SRP_FP8E4M3}


class SrpOptions(ctypes.Structure):
    _fields_ = [("sketch", ctypes.c_int), ("seed", ctypes.c_uint64),
                ("max_iter", ctypes.c_int), ("warm_start_iters", ctypes.c_int),
                ("refresh_every", ctypes.c_int), ("check_every", ctypes.c_int),
                ("pass_compute", ctypes.c_int), ("final_f64", ctypes.c_int),
                ("mu", ctypes.POINTER(ctypes.c_double)), ("time_passes", ctypes.c_int),
                ("lowp_x", ctypes.c_void_p), ("lowp_y", ctypes.c_void_p), ("lowp_tol", ctypes.c_double),
                ("lowp_max_iter", ctypes.c_int), ("sketch_x", ctypes.c_void_p), ("sketch_y", ctypes.c_void_p),
                ("sketch_dtype", ctypes.c_int), ("sketch_scale_x", ctypes.c_void_p),
                ("sketch_scale_y", ctypes.c_void_p), ("method", ctypes.c_int), ("rtr_max_inner", ctypes.c_int)]


class SrpInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iterations", ctypes.c_int),
                ("warm_iterations", ctypes.c_int), ("passes", ctypes.c_int),
                ("f", ctypes.c_double), ("objective", ctypes.c_double),
                ("grad_norm", ctypes.c_double), ("ms_sketch", ctypes.c_double),
                ("ms_factor", ctypes.c_double), ("ms_warm", ctypes.c_double),
                ("ms_iterate", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("pass_ms", ctypes.c_double), ("pass_launches", ctypes.c_int),
                ("lowp_iterations", ctypes.c_int), ("ms_lowp", ctypes.c_double),
                ("lowp_pass_ms", ctypes.c_double), ("lowp_pass_launches", ctypes.c_int),
                ("lowp_status", ctypes.c_int), ("inner_iterations", ctypes.c_int)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class SrpRequest(ctypes.Structure):
    _fields_ = [("problem", ctypes.c_int), ("X", ctypes.c_void_p), ("Y", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("dx", ctypes.c_int), ("dy", ctypes.c_int), ("k", ctypes.c_int),
                ("lambda_x", ctypes.c_double), ("lambda_y", ctypes.c_double), ("sketch_size", ctypes.c_int),
                ("tol", ctypes.c_double), ("dtype", ctypes.c_int), ("stage", ctypes.c_int),
                ("opt", SrpOptions), ("U", ctypes.c_void_p), ("V", ctypes.c_void_p), ("sigma", ctypes.c_void_p)]


class SrpResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("slot", ctypes.c_int), ("t_submit_ms", ctypes.c_double),
                ("t_start_ms", ctypes.c_double), ("t_done_ms", ctypes.c_double),
                ("footprint_bytes", ctypes.c_size_t), ("info", SrpInfo), ("message", ctypes.c_char * 160)]

    def as_dict(self):
        d = {name: getattr(self, name) for name, _ in self._fields_ if name not in ("info", "message")}
        d["info"] = self.info.as_dict()
        d["message"] = self.message.decode(errors="replace")
        return d


class SrpCsr(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_cols", ctypes.c_int), ("dtype", ctypes.c_int),
                ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("values", ctypes.c_void_p)]


class SrpError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn} failed: {STATUS_NAMES.get(code, code)} ({msg})")
        self.code = code


_lib = None

# Exported C symbols and their signatures (names as in include/srp.h).
_P = ctypes.c_void_p
_SIGS = {
    "srp_default_options": (ctypes.c_int, [ctypes.POINTER(SrpOptions)]),
    "srp_last_error": (ctypes.c_char_p, []),
    "srp_abi_sizes": (ctypes.c_int, [ctypes.POINTER(ctypes.c_size_t)] * 4),
    "srp_cca_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                  ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "srp_lda_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                  ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "srp_engine_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(_P)]),
    "srp_engine_create2": (ctypes.c_int, [ctypes.c_int, ctypes.c_size_t, ctypes.c_int, ctypes.c_int,
                                          ctypes.POINTER(_P)]),
    "srp_engine_ticks": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_uint64)]),
    "srp_request_footprint": (ctypes.c_size_t, [ctypes.POINTER(SrpRequest)]),
    "srp_engine_submit": (ctypes.c_int, [_P, ctypes.POINTER(SrpRequest), ctypes.POINTER(ctypes.c_uint64)]),
    "srp_engine_poll": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(SrpResult)]),
    "srp_engine_wait": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(SrpResult)]),
    "srp_engine_stats": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_size_t),
                                        ctypes.POINTER(ctypes.c_size_t)]),
    "srp_engine_destroy": (ctypes.c_int, [_P]),
    "srp_countsketch": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_uint64, _P, _P]),
    "srp_countsketch_noalloc": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                               ctypes.c_uint64, _P, _P]),
    "srp_srht": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                ctypes.c_uint64, _P, _P]),
    "srp_srht_rows": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int, ctypes.c_uint64, _P, _P]),
    "srp_stage_bf16": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int, _P, _P]),
    "srp_stage_fp8": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int64, ctypes.c_int, _P, _P, _P]),
    "srp_sketch_factor": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                         _P, _P, _P]),
    "srp_gram_pass_kernel": (ctypes.c_char_p, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "srp_gram_pass": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_int, _P, _P, _P, _P, _P]),
    "srp_countsketch_csr": (ctypes.c_int, [ctypes.POINTER(SrpCsr), ctypes.c_int, ctypes.c_uint64, _P, _P]),
    "srp_gram_pass_csr": (ctypes.c_int, [ctypes.POINTER(SrpCsr), ctypes.POINTER(SrpCsr), ctypes.c_int, _P, _P,
                                         _P, _P, _P]),
    "cca_solve_csr": (ctypes.c_int, [ctypes.POINTER(SrpCsr), ctypes.POINTER(SrpCsr), ctypes.c_int,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                     ctypes.POINTER(SrpOptions), _P, _P, _P, _P, ctypes.POINTER(SrpInfo)]),
    "lda_solve_csr": (ctypes.c_int, [ctypes.POINTER(SrpCsr), _P, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_int, ctypes.c_double, ctypes.POINTER(SrpOptions), _P, _P, _P,
                                     ctypes.POINTER(SrpInfo)]),
    "cca_solve": (ctypes.c_int, [_P, _P, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                 ctypes.c_int, ctypes.POINTER(SrpOptions), _P, _P, _P, _P,
                                 ctypes.POINTER(SrpInfo)]),
    "lda_solve": (ctypes.c_int, [_P, _P, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                 ctypes.POINTER(SrpOptions), _P, _P, _P, ctypes.POINTER(SrpInfo)]),
}


def lib() -> ctypes.CDLL:
    """Load ``libsrp.so`` (fails loudly when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _check(fn, code):
    if code != SRP_OK:
        raise SrpError(fn, code, lib().srp_last_error().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _dtype(t):
    if t.dtype not in _DTYPES:
        raise TypeError(f"unsupported dtype {t.dtype}")
    return _DTYPES[t.dtype]


def _need_cuda(*ts):
    for t in ts:
        if t is not None and (not t.is_cuda or not t.is_contiguous()):
            raise ValueError("inputs must be contiguous tensors on the HIP device")


def srp_default_options(**overrides) -> SrpOptions:
    o = SrpOptions()
    _check("srp_default_options", lib().srp_default_options(ctypes.byref(o)))
    for key, val in overrides.items():
        if key == "mu":
            continue
        if key == "sketch" and isinstance(val, str):
            val = {"countsketch": SRP_COUNTSKETCH, "srht": SRP_SRHT}[val]
        if key == "pass_compute" and isinstance(val, str):
            val = {"f64": SRP_F64, "f32": SRP_F32}[val]
        if key == "method" and isinstance(val, str):
            val = {"rcg": SRP_RCG, "rtr": SRP_RTR}[val]
        setattr(o, key, val)
    return o


def _sketch_out(A, s):
    acc = torch.float64 if A.dtype == torch.float64 else torch.float32
    return torch.empty((s, A.shape[1]), dtype=acc, device=A.device)


def srp_countsketch(A: torch.Tensor, s: int, seed: int) -> torch.Tensor:
    _need_cuda(A)
    out = _sketch_out(A, s)
    _check("srp_countsketch", lib().srp_countsketch(_ptr(A), _dtype(A), A.shape[0], A.shape[1], s,
                                                    seed, _ptr(out), _stream()))
    return out


def srp_countsketch_noalloc(A: torch.Tensor, s: int, seed: int, out: torch.Tensor) -> torch.Tensor:
    """The allocation-free CountSketch: the caller passes the output (s x d,
    float64 for float64 input, float32 otherwise); the call is enqueued on
    torch's current stream and returns without synchronising."""
    _need_cuda(A, out)
    _check("srp_countsketch_noalloc", lib().srp_countsketch_noalloc(_ptr(A), _dtype(A), A.shape[0], A.shape[1], s,
                                                                    seed, _ptr(out), _stream()))
    return out


def srp_srht(A: torch.Tensor, s: int, seed: int) -> torch.Tensor:
    _need_cuda(A)
    out = _sketch_out(A, s)
    _check("srp_srht", lib().srp_srht(_ptr(A), _dtype(A), A.shape[0], A.shape[1], s, seed,
                                      _ptr(out), _stream()))
    return out


def srp_srht_rows(n: int, s: int, seed: int, device="cuda") -> torch.Tensor:
    rows = torch.empty(s, dtype=torch.int64, device=device)
    _check("srp_srht_rows", lib().srp_srht_rows(n, s, seed, _ptr(rows), _stream()))
    return rows


def srp_stage_bf16(X: torch.Tensor) -> torch.Tensor:
    """BF16 copy of an FP32 matrix (nearest, ties to even)."""
    _need_cuda(X)
    if X.dtype != torch.float32:
        raise TypeError("srp_stage_bf16 takes float32 data")
    out = torch.empty(X.shape, dtype=torch.bfloat16, device=X.device)
    _check("srp_stage_bf16", lib().srp_stage_bf16(_ptr(X), X.shape[0], X.shape[1], _ptr(out), _stream()))
    return out


def srp_stage_fp8(X: torch.Tensor):
    """(E4M3 codes as uint8, per-column power-of-two scales as float64)."""
    _need_cuda(X)
    out = torch.empty(X.shape, dtype=torch.uint8, device=X.device)
    scales = torch.empty(X.shape[1], dtype=torch.float64, device=X.device)
    _check("srp_stage_fp8", lib().srp_stage_fp8(_ptr(X), _dtype(X), X.shape[0], X.shape[1], _ptr(out),
                                                _ptr(scales), _stream()))
    return out, scales


def srp_sketch_factor(SA: torch.Tensor, lam: float, want_inverse: bool = True):
    _need_cuda(SA)
    s, d = SA.shape
    R = torch.empty((d, d), dtype=torch.float64, device=SA.device)
    Rinv = torch.empty((d, d), dtype=torch.float64, device=SA.device) if want_inverse else None
    _check("srp_sketch_factor", lib().srp_sketch_factor(_ptr(SA), _dtype(SA), s, d, lam, _ptr(R),
                                                        _ptr(Rinv), _stream()))
    return R, Rinv


def srp_gram_pass(A0, W0, A1=None, W1=None, compute: str = "f32"):
    _need_cuda(A0, A1, W0, W1)
    n, d0 = A0.shape
    k = W0.shape[1]
    d1 = A1.shape[1] if A1 is not None else 0
    nb = 2 if A1 is not None else 1
    J0 = torch.empty((d0, nb * k), dtype=torch.float64, device=A0.device)
    J1 = torch.empty((d1, nb * k), dtype=torch.float64, device=A0.device) if A1 is not None else None
    comp = {"f64": SRP_F64, "f32": SRP_F32, "bf16": SRP_BF16}[compute]
    _check("srp_gram_pass", lib().srp_gram_pass(_ptr(A0), _ptr(A1), _dtype(A0), comp, n, d0, d1, k,
                                                _ptr(W0), _ptr(W1), _ptr(J0), _ptr(J1), _stream()))
    return J0, J1


def srp_gram_pass_kernel(dtype: str, compute: str, d0: int, d1: int, k: int):
    """Name of the pass kernel the library runs for this shape (rows on
    16-byte boundaries), or None outside its limits."""
    dt = {"f64": SRP_F64, "f32": SRP_F32, "bf16": SRP_BF16}[dtype]
    comp = {"f64": SRP_F64, "f32": SRP_F32, "bf16": SRP_BF16}[compute]
    name = lib().srp_gram_pass_kernel(dt, comp, d0, d1, k)
    return name.decode() if name else None


def _attach_staged(opt, lowp, sketch_input):
    """Point the options at staged copies (kept alive by the caller)."""
    if lowp is not None:
        lx, ly = lowp
        _need_cuda(lx, ly)
        if lx.dtype != torch.bfloat16 or (ly is not None and ly.dtype != torch.bfloat16):
            raise TypeError("low-precision copies must be bfloat16 (srp_stage_bf16)")
        opt.lowp_x, opt.lowp_y = lx.data_ptr(), (ly.data_ptr() if ly is not None else None)
    if sketch_input is not None:
        sx, sy, scx, scy = sketch_input
        _need_cuda(sx, sy, scx, scy)
        opt.sketch_x, opt.sketch_y = sx.data_ptr(), (sy.data_ptr() if sy is not None else None)
        opt.sketch_dtype = _dtype(sx)
        opt.sketch_scale_x = scx.data_ptr() if scx is not None else None
        opt.sketch_scale_y = scy.data_ptr() if scy is not None else None


def cca_solve(X, Y, k, lambda_x, lambda_y, sketch_size, tol=1e-6, options: SrpOptions | None = None,
              mu=None, raise_on_noconv: bool = False, lowp=None, sketch_input=None):
    """Returns (U, V, sigma, info_dict).

    lowp = (Xb, Yb): BF16 copies for the low-precision phase (then refined on
    X, Y); sketch_input = (Sx, Sy, scale_x, scale_y): staged copies the sketch
    reads (FP8 codes with their column scales, or BF16 / F32 with None)."""
    _need_cuda(X, Y)
    if X.dtype != Y.dtype:
        raise TypeError("X and Y must share a dtype")
    n, dx = X.shape
    dy = Y.shape[1]
    opt = options if options is not None else srp_default_options()
    _attach_staged(opt, lowp, sketch_input)
    mu_buf = None
    if mu is not None:
        mu_buf = (ctypes.c_double * k)(*[float(m) for m in mu])
        opt.mu = ctypes.cast(mu_buf, ctypes.POINTER(ctypes.c_double))
    U = torch.empty((dx, k), dtype=torch.float64, device=X.device)
    V = torch.empty((dy, k), dtype=torch.float64, device=X.device)
    sigma = torch.empty(k, dtype=torch.float64, device=X.device)
    info = SrpInfo()
    rc = lib().cca_solve(_ptr(X), _ptr(Y), n, dx, dy, k, lambda_x, lambda_y, sketch_size, tol,
                         _dtype(X), ctypes.byref(opt), _stream(), _ptr(U), _ptr(V), _ptr(sigma),
                         ctypes.byref(info))
    if rc != SRP_OK and not (rc == SRP_ENOCONV and not raise_on_noconv):
        _check("cca_solve", rc)
    return U, V, sigma, info.as_dict()


def lda_solve(X, labels, n_classes, k, lam, sketch_size, tol=1e-6, options: SrpOptions | None = None,
              mu=None, raise_on_noconv: bool = False):
    """Returns (W, rho, info_dict)."""
    _need_cuda(X, labels)
    if labels.dtype != torch.int32:
        raise TypeError("labels must be int32")
    n, d = X.shape
    opt = options if options is not None else srp_default_options()
    mu_buf = None
    if mu is not None:
        mu_buf = (ctypes.c_double * k)(*[float(m) for m in mu])
        opt.mu = ctypes.cast(mu_buf, ctypes.POINTER(ctypes.c_double))
    W = torch.empty((d, k), dtype=torch.float64, device=X.device)
    rho = torch.empty(k, dtype=torch.float64, device=X.device)
    info = SrpInfo()
    rc = lib().lda_solve(_ptr(X), _ptr(labels), n, d, n_classes, k, lam, sketch_size, tol, _dtype(X),
                         ctypes.byref(opt), _stream(), _ptr(W), _ptr(rho), ctypes.byref(info))
    if rc != SRP_OK and not (rc == SRP_ENOCONV and not raise_on_noconv):
        _check("lda_solve", rc)
    return W, rho, info.as_dict()


# ------------------------------------------------------------ CSR data
class Csr:
    """A CSR matrix on the HIP device: row_ptr (int64, n + 1), col_idx
    (int32, strictly increasing within each row), values (float32 or
    float64) and the column count.  The tensors must stay alive while a
    call that takes the matrix runs."""

    def __init__(self, row_ptr, col_idx, values, n_cols):
        _need_cuda(row_ptr, col_idx, values)
        if row_ptr.dtype != torch.int64 or col_idx.dtype != torch.int32:
            raise TypeError("row_ptr must be int64 and col_idx int32")
        if values.dtype not in (torch.float32, torch.float64):
            raise TypeError("values must be float32 or float64")
        self.row_ptr, self.col_idx, self.values = row_ptr, col_idx, values
        self.shape = (row_ptr.numel() - 1, int(n_cols))

    @classmethod
    def from_torch(cls, A):
        """From a torch sparse CSR tensor (indices are converted)."""
        return cls(A.crow_indices().to(torch.int64).contiguous(), A.col_indices().to(torch.int32).contiguous(),
                   A.values().contiguous(), A.shape[1])

    def struct(self) -> SrpCsr:
        return SrpCsr(self.shape[0], self.shape[1], _dtype(self.values), self.values.numel(),
                      self.row_ptr.data_ptr(), self.col_idx.data_ptr(), self.values.data_ptr())


def srp_countsketch_csr(A: Csr, s: int, seed: int) -> torch.Tensor:
    out = torch.empty((s, A.shape[1]), dtype=torch.float64, device=A.values.device)
    a = A.struct()
    _check("srp_countsketch_csr", lib().srp_countsketch_csr(ctypes.byref(a), s, seed, _ptr(out), _stream()))
    return out


def srp_gram_pass_csr(A0: Csr, W0, A1: Csr | None = None, W1=None):
    _need_cuda(W0, W1)
    k = W0.shape[1]
    nb = 2 if A1 is not None else 1
    dev = A0.values.device
    J0 = torch.empty((A0.shape[1], nb * k), dtype=torch.float64, device=dev)
    J1 = torch.empty((A1.shape[1], nb * k), dtype=torch.float64, device=dev) if A1 is not None else None
    a0 = A0.struct()
    a1 = A1.struct() if A1 is not None else None
    _check("srp_gram_pass_csr", lib().srp_gram_pass_csr(ctypes.byref(a0), ctypes.byref(a1) if a1 else None, k,
                                                        _ptr(W0), _ptr(W1), _ptr(J0), _ptr(J1), _stream()))
    return J0, J1


def cca_solve_csr(X: Csr, Y: Csr, k, lambda_x, lambda_y, sketch_size, tol=1e-6,
                  options: SrpOptions | None = None, mu=None, raise_on_noconv: bool = False):
    """cca_solve for CSR data.  Returns (U, V, sigma, info_dict)."""
    opt = options if options is not None else srp_default_options()
    mu_buf = None
    if mu is not None:
        mu_buf = (ctypes.c_double * k)(*[float(m) for m in mu])
        opt.mu = ctypes.cast(mu_buf, ctypes.POINTER(ctypes.c_double))
    dev = X.values.device
    U = torch.empty((X.shape[1], k), dtype=torch.float64, device=dev)
    V = torch.empty((Y.shape[1], k), dtype=torch.float64, device=dev)
    sigma = torch.empty(k, dtype=torch.float64, device=dev)
    info = SrpInfo()
    x, y = X.struct(), Y.struct()
    rc = lib().cca_solve_csr(ctypes.byref(x), ctypes.byref(y), k, lambda_x, lambda_y, sketch_size, tol,
                             ctypes.byref(opt), _stream(), _ptr(U), _ptr(V), _ptr(sigma), ctypes.byref(info))
    if rc != SRP_OK and not (rc == SRP_ENOCONV and not raise_on_noconv):
        _check("cca_solve_csr", rc)
    return U, V, sigma, info.as_dict()


def lda_solve_csr(X: Csr, labels, n_classes, k, lam, sketch_size, tol=1e-6, options: SrpOptions | None = None,
                  mu=None, raise_on_noconv: bool = False):
    """lda_solve for CSR data.  Returns (W, rho, info_dict)."""
    _need_cuda(labels)
    if labels.dtype != torch.int32:
        raise TypeError("labels must be int32")
    opt = options if options is not None else srp_default_options()
    mu_buf = None
    if mu is not None:
        mu_buf = (ctypes.c_double * k)(*[float(m) for m in mu])
        opt.mu = ctypes.cast(mu_buf, ctypes.POINTER(ctypes.c_double))
    dev = X.values.device
    W = torch.empty((X.shape[1], k), dtype=torch.float64, device=dev)
    rho = torch.empty(k, dtype=torch.float64, device=dev)
    info = SrpInfo()
    x = X.struct()
    rc = lib().lda_solve_csr(ctypes.byref(x), _ptr(labels), n_classes, k, lam, sketch_size, tol,
                             ctypes.byref(opt), _stream(), _ptr(W), _ptr(rho), ctypes.byref(info))
    if rc != SRP_OK and not (rc == SRP_ENOCONV and not raise_on_noconv):
        _check("lda_solve_csr", rc)
    return W, rho, info.as_dict()


# ------------------------------------------------------------ serving engine
SRP_PROBLEM_CCA, SRP_PROBLEM_LDA = 0, 1
SRP_ENGINE_GROUPED = 1
SRP_STAGE_NONE, SRP_STAGE_BF16, SRP_STAGE_BF16_FP8 = 0, 1, 2


class Engine:
    """Continuous-batching engine (``srp_engine_*`` in include/srp.h).

    submit_* returns a ticket at once; poll / wait return the outputs and
    the engine's record for it.  Inputs are read on the engine's own
    streams, so submit first waits for torch's current stream (the inputs'
    producer); the tensors a request uses are held here until it ends."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 4, device: int | None = None,
                 grouped: bool = False):
        dev = torch.cuda.current_device() if device is None else int(device)
        h = ctypes.c_void_p()
        flags = SRP_ENGINE_GROUPED if grouped else 0
        _check("srp_engine_create2", lib().srp_engine_create2(dev, int(hbm_budget_bytes), int(max_slots), flags,
                                                               ctypes.byref(h)))
        self._h = h
        self.device = dev
        self._keep = {}

    def _submit(self, req, keep):
        torch.cuda.current_stream().synchronize()
        t = ctypes.c_uint64()
        _check("srp_engine_submit", lib().srp_engine_submit(self._h, ctypes.byref(req), ctypes.byref(t)))
        self._keep[t.value] = keep
        return t.value

    @staticmethod
    def _mu(opt, mu, k):
        if mu is None:
            return None
        buf = (ctypes.c_double * k)(*[float(m) for m in mu])
        opt.mu = ctypes.cast(buf, ctypes.POINTER(ctypes.c_double))
        return buf

    def cca_request(self, X, Y, k, lambda_x, lambda_y, sketch_size, tol=1e-6, options=None, mu=None,
                    stage=SRP_STAGE_NONE):
        """(SrpRequest, kept objects) for a CCA solve; outputs allocated here."""
        _need_cuda(X, Y)
        if X.dtype != Y.dtype:
            raise TypeError("X and Y must share a dtype")
        n, dx = X.shape
        dy = Y.shape[1]
        opt = options if options is not None else srp_default_options()
        req = SrpRequest()
        req.problem, req.X, req.Y, req.n, req.dx, req.dy, req.k = SRP_PROBLEM_CCA, X.data_ptr(), Y.data_ptr(), n, dx, dy, k
        req.lambda_x, req.lambda_y, req.sketch_size, req.tol = lambda_x, lambda_y, sketch_size, tol
        req.dtype, req.stage = _dtype(X), stage
        mu_buf = self._mu(opt, mu, k)
        req.opt = opt
        U = torch.empty((dx, k), dtype=torch.float64, device=X.device)
        V = torch.empty((dy, k), dtype=torch.float64, device=X.device)
        sigma = torch.empty(k, dtype=torch.float64, device=X.device)
        req.U, req.V, req.sigma = U.data_ptr(), V.data_ptr(), sigma.data_ptr()
        return req, {"kind": "cca", "in": (X, Y, mu_buf), "out": (U, V, sigma)}

    def lda_request(self, X, labels, n_classes, k, lam, sketch_size, tol=1e-6, options=None, mu=None):
        _need_cuda(X, labels)
        if labels.dtype != torch.int32:
            raise TypeError("labels must be int32")
        n, d = X.shape
        opt = options if options is not None else srp_default_options()
        req = SrpRequest()
        req.problem, req.X, req.Y, req.n, req.dx, req.dy, req.k = (SRP_PROBLEM_LDA, X.data_ptr(), labels.data_ptr(),
                                                                   n, d, n_classes, k)
        req.lambda_x, req.lambda_y, req.sketch_size, req.tol = lam, 0.0, sketch_size, tol
        req.dtype, req.stage = _dtype(X), SRP_STAGE_NONE
        mu_buf = self._mu(opt, mu, k)
        req.opt = opt
        W = torch.empty((d, k), dtype=torch.float64, device=X.device)
        rho = torch.empty(k, dtype=torch.float64, device=X.device)
        req.U, req.V, req.sigma = W.data_ptr(), None, rho.data_ptr()
        return req, {"kind": "lda", "in": (X, labels, mu_buf), "out": (W, rho)}

    @staticmethod
    def footprint(req) -> int:
        return int(lib().srp_request_footprint(ctypes.byref(req)))

    def submit_cca(self, *args, **kw) -> int:
        req, keep = self.cca_request(*args, **kw)
        return self._submit(req, keep)

    def submit_lda(self, *args, **kw) -> int:
        req, keep = self.lda_request(*args, **kw)
        return self._submit(req, keep)

    def _finish(self, ticket, rc, res, raise_on_error):
        keep = self._keep.pop(ticket)
        if raise_on_error and rc not in (SRP_OK, SRP_ENOCONV):
            raise SrpError("engine request", rc, res.message.decode(errors="replace"))
        return (*keep["out"], res.as_dict())

    def poll(self, ticket: int, raise_on_error: bool = True):
        """None while pending, else (outputs..., record).  A failed solve
        raises SrpError unless raise_on_error is False (then the record's
        status and message tell)."""
        res = SrpResult()
        rc = lib().srp_engine_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(res))
        if rc == SRP_PENDING:
            return None
        if ticket not in self._keep:
            _check("srp_engine_poll", rc)
        return self._finish(ticket, rc, res, raise_on_error)

    def wait(self, ticket: int, raise_on_error: bool = True):
        res = SrpResult()
        rc = lib().srp_engine_wait(self._h, ctypes.c_uint64(ticket), ctypes.byref(res))
        if ticket not in self._keep:
            _check("srp_engine_wait", rc)
        return self._finish(ticket, rc, res, raise_on_error)

    def stats(self):
        q, r, p = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        u, pk = ctypes.c_size_t(), ctypes.c_size_t()
        _check("srp_engine_stats", lib().srp_engine_stats(self._h, ctypes.byref(q), ctypes.byref(r), ctypes.byref(p),
                                                          ctypes.byref(u), ctypes.byref(pk)))
        t = ctypes.c_uint64()
        _check("srp_engine_ticks", lib().srp_engine_ticks(self._h, ctypes.byref(t)))
        return {"queued": q.value, "running": r.value, "peak_running": p.value, "pool_used": u.value,
                "pool_peak": pk.value, "grouped_ticks": t.value}

    def close(self):
        if self._h:
            lib().srp_engine_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
