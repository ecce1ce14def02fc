"""MI355X-native smallest eigenvalue of ill-conditioned Hankel moment matrices.

The compute path is libhk.so (HIP kernels for gfx950 behind the C-ABI in
include/hk.h); this package only binds it.  See hk.py.
"""
from .hk import (HK_INVERSE, HK_SECANT, HK_FLAG_NO_WORK_COUNT, HK_FLAG_TIME_UPDATES, HK_FLAG_CERTIFY, HK_FLAG_PANEL,
                 HK_FLAG_GROUP, HK_FLAG_LOOKAHEAD_ON, HK_FLAG_VECTOR_UPDATE, HK_UPDATE_MATRIX_CORES, HK_UPDATE_VECTOR,
                 HK_FLAG_LOOKAHEAD_OFF, HK_FLAG_LOOKAHEAD_FUSED, EXPORTS, HKError, Matrix, lib, smallest_eig,  # noqa: F401
                 workspace_bytes, batch_workspace_bytes, eig_batched, autotune,
                 mlp_nparams, mlp_cache_floats, mlp_forward, mlp_backward, mlp_mse, mlp_adam_step,
                 bracket_batched, mlp_meta, mlp_propose, eig_learned, moments_host, Batch, BatchMember, mpf_value,
                 mul_rate, smallest_eig_static, HK_RATE_MAD_I64_I32, HK_RATE_MAD_U64_U32, HK_RATE_MAD_U32_U24, HK_RATE_FMA_F64,
                 HK_RATE_MFMA_I8)
