"""MI355X-native hot path of the Z-Model high-order step.

The computation lives in ``libzm.so`` (hand-written HIP kernels for gfx950
behind the C ABI in ``include/zm.h``); this package is its thin Python
binding.  Importing it loads the library and fails loudly if it has not been
built -- there is no CPU fallback.
"""
from ._zm import (  # noqa: F401
    EXPORTS, KERNELS, LIB_PATH, Batch, Context, Params, ZMError, batch_workspace_bytes,
    ZM_FLAG_GRAPH, autotune, batch_autotune, tuning_get, tuning_set, Pool, pool_request_bytes,
    ZM_REQ_UNKNOWN, ZM_REQ_QUEUED, ZM_REQ_LIVE, ZM_REQ_FINISHED, ZM_REQ_FAILED,
    ZM_ERR_CAPACITY, ZM_ERR_HIP, ZM_ERR_INVALID_ARG, ZM_ERR_NONFINITE,
    ZM_ERR_UNSUPPORTED, ZM_ERR_WORKSPACE, ZM_FLAG_CHECK_FINITE, ZM_FP32_PAIRS,
    ZM_FP64, ZM_OK, ZM_MODEL_HIGH, ZM_MODEL_LOW, ZM_MODEL_MEDIUM, ZM_BOUNDARY_PERIODIC,
    ZM_BOUNDARY_FREE, load, status_string, workspace_bytes, br_velocity_noalloc,
    NOALLOC_SCRATCH_BYTES, ZM_CUT_PATH_CELLS, ZM_CUT_PATH_WINDOW, ZM_CUT_PATH_STENCIL,
)

load()
