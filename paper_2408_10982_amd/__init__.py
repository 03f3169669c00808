"""MI355X-native hot path of GreediRIS-style influence maximization.

RRR sampling under IC/LT and max-k-cover seed selection (standard greedy,
RandGreedi local greedy, streaming bucket cover with truncation, IMM driver),
as hand-written HIP kernels for gfx950 behind the C ABI in include/im.h.
This package is the thin Python face of that library.
"""
from .binding import (IC, LT, SEL_GREEDIRIS, SEL_GREEDY, SEL_RANDGREEDI, EXPORTS, Forward, Graph,
                      ImError, RRR, TUNE_APPLY_BLOCKS, TUNE_BIG_SHAPE, TUNE_DENSE_RATIO,
                      TUNE_GRAPH, TUNE_LISTS, TUNE_LT_BLOCKS, TUNE_LT_GRAB, TUNE_SAMPLE_BLOCKS,
                      WS_BATCH, WS_FORWARD, WS_GREEDY, WS_INCIDENCE, WS_INFLUENCE, WS_OFFLINE,
                      WS_OPIM, WS_PREPARE_GRAPH, WS_RANDGREEDI, WS_SAMPLE, WS_SOLVE, WS_STREAM,
                      build_incidence, drop_workspaces, greedi_offline, greedy_cover,
                      greedy_cover_static, imm_plan, influence, lib, lt_index_size, opim, prepare_forward,
                      prepare_graph, randgreedi, release, sample_into, sample_rrr, solve,
                      solve_batch, stream_cover, tune_get, tune_set, version, workspace_bytes,
                      workspace_need, workspace_size)

__all__ = ["IC", "LT", "SEL_GREEDY", "SEL_GREEDIRIS", "SEL_RANDGREEDI", "EXPORTS", "Forward",
           "Graph", "ImError", "RRR", "TUNE_APPLY_BLOCKS", "TUNE_BIG_SHAPE", "TUNE_DENSE_RATIO",
           "TUNE_GRAPH", "TUNE_LISTS", "TUNE_LT_BLOCKS", "TUNE_LT_GRAB", "TUNE_SAMPLE_BLOCKS", "WS_BATCH",
           "WS_FORWARD", "WS_GREEDY", "WS_INCIDENCE", "WS_INFLUENCE", "WS_OFFLINE", "WS_OPIM",
           "WS_PREPARE_GRAPH", "WS_RANDGREEDI", "WS_SAMPLE", "WS_SOLVE", "WS_STREAM",
           "build_incidence", "drop_workspaces", "greedi_offline", "greedy_cover",
           "greedy_cover_static", "imm_plan", "influence", "lib", "lt_index_size", "opim", "prepare_forward",
           "prepare_graph", "randgreedi", "release", "sample_into", "sample_rrr", "solve",
           "solve_batch", "stream_cover", "tune_get", "tune_set", "version", "workspace_bytes",
           "workspace_need", "workspace_size"]
