"""MI355X (gfx950) batched homotopy-continuation path tracker.

The tracking itself lives in libhc.so (HIP kernels behind the C ABI of
include/hc.h); this package only builds it and binds it.
"""
from .hc import (HC_EVAL_MFMA, HC_EVAL_ROWS, HC_FP64, HC_LAYOUT_AUTO, HC_LAYOUT_DENSE, HC_LAYOUT_TERMS, HC_MAX_N, HC_MIXED,  # noqa: F401
                 HC_NOALLOC_SCRATCH_BYTES, HC_PARAMETER, HC_T_AT_INFINITY, HC_T_MAX_STEPS, HC_T_MIN_STEP,
                 HC_T_NONFINITE, HC_T_REFINE_FAILED, HC_T_SINGULAR, HC_T_SINGULAR_END, HC_T_SUCCESS,
                 HC_TOTAL_DEGREE, INFO_DTYPE, STATUS_NAMES, Context, HcError, Opts, System, Profile, Server,
                 default_opts, homogenize, lib)
