"""Exact grey-scale dilation / erosion on MI355X (gfx950) by the polynomial
(umbra) convolution method of arXiv 2305.03018.

This package is a thin binding over the C ABI of ``include/md.h`` (library
``libmd.so`` built by ``build.py``): it marshals torch device tensors and
numpy SE arrays into the C calls; every step of the computation runs in the
library's HIP kernels.  There is no CPU fallback: calling into the library
without a built ``libmd.so`` raises.
"""
from ._binding import (  # noqa: F401
    BLACKHAT,
    Batch,
    CLOSE,
    DILATE,
    ERODE,
    GRADIENT,
    MDError,
    OPEN,
    TOPHAT,
    OPT_AUTOTUNE,
    OPT_BAND,
    OPT_GRAPH,
    OPT_NR,
    OPT_PATH,
    OPT_PRECISION,
    OPT_PROFILE,
    OPT_STREAM_MB,
    OPT_STREAM_ROWS,
    OPT_SYNC,
    OPT_TILE,
    OPT_WORKSPACE_MB,
    debug_tile_values,
    dilate,
    dilate3,
    dilate3_host,
    dilate_batch,
    dilate_host,
    erode,
    erode3,
    erode3_host,
    erode_host,
    exported_symbols,
    get_option,
    get_stats,
    blackhat,
    closing,
    cost_model,
    gradient,
    morph,
    opening,
    tophat,
    library_path,
    load,
    options,
    profile_get,
    profile_reset,
    release,
    set_option,
)
