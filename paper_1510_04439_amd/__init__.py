"""MI355X (gfx950) hot path of multi-dimensional FPCA (Chen & Jiang).

The compute lives in the HIP library `libfpca.so` (C ABI declared in
include/fpca.h). This package is its thin Python binding: `fpca_bin`,
`fpca_smooth_mean`, `fpca_smooth_cov`, `fpca_eig_randomized` and the handle
calls take torch tensors for device memory and marshal pointers and the
current HIP stream. Nothing here computes; if the library is missing, every
call raises.
"""
from ._binding import (  # noqa: F401
    FPCA_OK, FPCA_ERR_INVALID_ARG, FPCA_ERR_DOMAIN, FPCA_ERR_UNSUPPORTED, FPCA_ERR_WORKSPACE,
    FPCA_ERR_DEVICE, FPCA_STATUS_OK, FPCA_STATUS_FALLBACK, FPCA_STATUS_EMPTY, FPCA_BIN_MEAN,
    FPCA_BIN_COV, FPCA_IRREGULAR, FPCA_COMMON_GRID, FPCA_F64, FPCA_F32, FPCA_PREC_F64,
    FPCA_PREC_F32, FPCA_PREC_BF16X3, FPCA_K_EPANECHNIKOV, FPCA_CONV_DIRECT, FPCA_CONV_FFT, FPCA_CONV_AUTO, FPCA_COVOP_RECOMPUTE, FPCA_COVOP_STORE_BAND, FPCA_ENGINE_AUTO, FPCA_ENGINE_QUEUE, FPCA_ENGINE_PASSES, CovOp, FpcaError, Grid, Handle, LIB_PATH,
    EXPORTED_SYMBOLS, fpca_stream_create_cu_range, fpca_stream_destroy, fpca_bin, fpca_bin_common, fpca_cv_batched, fpca_cv_select, fpca_cv_loo, fpca_bw_search, fpca_set_conv, fpca_set_engine, fpca_eig_randomized, fpca_rng_normal, fpca_smooth_cov,
    fpca_smooth_mean, load_library, fpca_bw_features, fpca_bw_num_params, fpca_bw_mlp_forward,
    fpca_bw_mlp_backward, fpca_bw_adam_step, fpca_noise_variance,
    fpca_pace_scores, fpca_pace_scores_noalloc, fpca_reconstruct,
)
