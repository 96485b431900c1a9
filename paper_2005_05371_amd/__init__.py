"""MI355X-native hybrid de-noiser: adaptive median filter + adaptive Wiener filter.

The compute lives in ``libhybrid_denoise.so`` (hand-written HIP for gfx950, C ABI in
``include/hybrid_denoise.h``); this package only marshals torch GPU tensors into it.
"""
from ._binding import (HD_AMF_UNRESOLVED_KEEP, HD_CONTRAST_STRETCH, HD_OPT_FAIL_ALLOC, HD_OPT_SURROGATE_FUSED, HD_OPT_TILE_ROWS,
                       HD_OPT_FUSE_MOMENTS, HD_OPT_GRAPHS, HD_OPT_RESIDENT, HD_OPT_SELECT,
                       HD_OPT_WAIT_LIMIT_US, HD_U8, HD_U16, HDError,
                       LIB_PATH, amf_filter, autotune_batched, autotune_hybrid, check_errors, contrast_stretch,
                       degrade_image,
                       hybrid_denoise,
                       hybrid_denoise_batched, hybrid_denoise_batched_timed, hybrid_denoise_noalloc, hybrid_paper, hybrid_partitioned, load,
                       release_plans, wiener_fft,
                       resident_capacity,
                       set_option, tiles_of, wiener_filter, Surrogate)

__all__ = ["HD_AMF_UNRESOLVED_KEEP", "HD_CONTRAST_STRETCH", "HD_OPT_FAIL_ALLOC", "HD_OPT_SURROGATE_FUSED", "HD_OPT_TILE_ROWS", "HD_OPT_FUSE_MOMENTS",
           "HD_OPT_GRAPHS", "HD_OPT_RESIDENT", "HD_OPT_SELECT", "HD_OPT_WAIT_LIMIT_US", "HD_U8",
           "HD_U16", "HDError", "LIB_PATH", "amf_filter", "autotune_batched", "autotune_hybrid", "check_errors",
           "contrast_stretch", "degrade_image", "hybrid_denoise",
           "hybrid_denoise_batched", "hybrid_denoise_batched_timed", "hybrid_denoise_noalloc", "hybrid_paper", "hybrid_partitioned", "load", "wiener_fft",
           "release_plans", "resident_capacity", "set_option", "tiles_of", "wiener_filter",
           "Surrogate"]
