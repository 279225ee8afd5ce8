"""cfsim: MI355X-native coupled similarity of CFG pairs (arXiv 1707.02423).

The compute path is libcfsim.so (HIP kernels for gfx950, C ABI in
include/cfsim.h); `cfsim.py` is the thin ctypes binding.
"""
from .cfsim import (  # noqa: F401
    F32, F64, CONVERGED, HIT_MAX_ITER, DEGENERATE, INVALID_INPUT, NEAR_TIE, FP64_FINAL, NUM_BUCKETS, RESULT_DTYPE,
    RESULT_BYTES, RESULT_STRIDE, TUNE_CLASSES, NOALLOC_SCRATCH_BYTES, Batch, CfsimError, CfsimScore, Context,
    GraphSet, NUM_DISTANCES, DISTANCE_NAMES, backward, distances, bucket_kernel, check_jumps, lib, options, pack,
    score, score_batch, score_damped, assign, ward, topk,
)
