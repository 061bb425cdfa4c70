"""MI355X-native semicoherent NUFFT resampling (gfx950 HIP kernels behind a C ABI).

The computation lives in ``libnufft_resample.so`` (built from ``csrc/``);
``nufft_resample`` is its ctypes binding.
"""
from .nufft_resample import (  # noqa: F401
    NrError, Plan, complex_view, load, nufft_resample_bin_offsets, nufft_resample_chirp_beta,
    nufft_resample_default_options, nufft_resample_destroy, nufft_resample_execute,
    nufft_resample_kernel_ft, nufft_resample_kernel_params, nufft_resample_last_error,
    nufft_resample_plan, nufft_resample_query, nufft_resample_query_class,
    nufft_resample_semicoherent_sum, nufft_resample_stage_times, nufft_resample_stat_offsets, nufft_resample_valid_mask,
    NR_OK, NR_ERR_INVALID_ARG, NR_ERR_TOL_UNATTAINABLE, NR_ERR_OUT_OF_MEMORY, NR_ERR_DEVICE,
    NR_ERR_NONFINITE_INPUT)
