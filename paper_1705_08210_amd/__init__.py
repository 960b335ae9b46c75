"""MI355X (gfx950) library for the 2-way and 3-way Proportional Similarity
metric (Joubert et al., arXiv 1705.08210).  The compute path is the C ABI of
include/ps.h (libps.so, hand-written HIP kernels); ``ps`` is its binding."""

from .ps import (BatchedPlan, PSError, ps2, ps2_batched, ps2_compute, ps2_compute_batched,
                 ps3, ps3_compute, ps3_stage_size, ps_vector_sums, stage_size, tile_configs,
                 tune_clear, tune_register, vector_sums)

from . import autotune as _autotune

_autotune.load()  # tuned tile choices, if a cache was written on this machine type

__all__ = ["BatchedPlan", "PSError", "ps2", "ps2_batched", "ps2_compute",
           "ps2_compute_batched", "ps3", "ps3_compute", "ps3_stage_size", "ps_vector_sums",
           "stage_size", "tile_configs", "tune_clear", "tune_register", "vector_sums"]
