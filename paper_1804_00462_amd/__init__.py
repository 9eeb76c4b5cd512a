"""MI355X (gfx950) Subspace-Orbit Randomized SVD.

The computation lives in ``libsorsvd.so`` (HIP kernels behind the C ABI of
``include/sorsvd.h``); this package only marshals arguments. Importing it does
not load the library; the first call does, and fails loudly if it is missing.
"""
from . import _lib
from ._lib import SORSVD_BF16, SORSVD_DIAG, SORSVD_F16, SORSVD_F32, SORSVD_F64, SorsvdError, load
from .api import (MLP, Batch, Plan, auto, bounds, dtype_code, mlp_param_count, pack_f16, pass_timing,
                  pass_timing_read, philox_normal, predict_kq, probe_features, rpca, sorsvd, sorsvd_diag,
                  step_core_svd, step_orbit, step_project, step_qr, step_sketch, workspace_bytes)

__all__ = ["MLP", "Batch", "Plan", "SORSVD_BF16", "SORSVD_DIAG", "SORSVD_F16", "SORSVD_F32", "SORSVD_F64",
           "SorsvdError", "auto", "bounds", "dtype_code", "load", "mlp_param_count", "pack_f16", "pass_timing", "pass_timing_read", "philox_normal",
           "predict_kq", "probe_features", "rpca", "sorsvd", "sorsvd_diag", "step_core_svd", "step_orbit", "step_project",
           "step_qr", "step_sketch", "workspace_bytes"]
