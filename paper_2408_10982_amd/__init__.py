"""MI355X-native hot path of GreediRIS-style influence maximization.

RRR sampling under IC/LT and max-k-cover seed selection (standard greedy,
RandGreedi local greedy, streaming bucket cover with truncation, IMM driver),
as hand-written HIP kernels for gfx950 behind the C ABI in include/im.h.
This package is the thin Python face of that library.
"""
from .binding import (IC, LT, SEL_GREEDIRIS, SEL_GREEDY, SEL_RANDGREEDI, greedi_offline, Forward, prepare_forward, influence, opim, scratch_bytes, EXPORTS, Graph, ImError, RRR,
                      build_incidence, greedy_cover, greedy_cover_static, lib, prepare_graph, randgreedi, release,
                      sample_rrr, solve, solve_batch, stream_cover, version,
                      imm_plan, sample_into, tune_set, tune_get, TUNE_SAMPLE_BLOCKS,
                      TUNE_BIG_SHAPE, TUNE_APPLY_BLOCKS, TUNE_DENSE_RATIO, TUNE_LT_BLOCKS, TUNE_LT_GRAB, TUNE_GRAPH)

__all__ = ["IC", "LT", "SEL_GREEDY", "SEL_GREEDIRIS", "SEL_RANDGREEDI", "greedi_offline", "Forward",
           "prepare_forward", "influence", "opim", "scratch_bytes", "EXPORTS", "Graph", "ImError", "RRR",
           "build_incidence", "greedy_cover", "greedy_cover_static", "lib", "prepare_graph", "randgreedi", "release",
           "sample_rrr", "solve", "solve_batch", "stream_cover", "version", "imm_plan",
           "sample_into", "tune_set", "tune_get", "TUNE_SAMPLE_BLOCKS", "TUNE_BIG_SHAPE",
           "TUNE_APPLY_BLOCKS", "TUNE_DENSE_RATIO", "TUNE_LT_BLOCKS", "TUNE_LT_GRAB", "TUNE_GRAPH"]
