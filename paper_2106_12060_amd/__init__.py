"""Sketch-preconditioned Riemannian CCA / FDA on one AMD MI355X (gfx950).

Python face of the C-ABI library ``libsrp.so`` (``include/srp.h``); see
``_lib`` for the functions.  Every computation runs in the HIP library.
"""
from ._lib import (  # noqa: F401
    SRP_OK, SRP_EINVAL, SRP_ENOTSPD, SRP_ENOCONV, SRP_ENOMEM, SRP_EDEVICE,
    SRP_F64, SRP_F32, SRP_BF16, SRP_FP8E4M3, SRP_COUNTSKETCH, SRP_SRHT, SRP_RCG, SRP_RTR,
    SrpError, SrpOptions, SrpInfo, LIB_PATH, lib, exported_symbols,
    srp_default_options, srp_countsketch, srp_countsketch_noalloc, srp_srht, srp_srht_rows,
    srp_sketch_factor, srp_gram_pass, srp_gram_pass_kernel, cca_solve, lda_solve, srp_stage_bf16, srp_stage_fp8,
    SRP_EBUSY, SRP_EREJECTED, SRP_PENDING, SRP_PROBLEM_CCA, SRP_PROBLEM_LDA,
    SRP_STAGE_NONE, SRP_STAGE_BF16, SRP_STAGE_BF16_FP8, SRP_ENGINE_GROUPED, SrpRequest, SrpResult, Engine,
    SrpCsr, Csr, srp_countsketch_csr, srp_gram_pass_csr, cca_solve_csr, lda_solve_csr,
)
