"""MI355X-native parallel Gene-pool Optimal Mixing (GOM) with partial evaluations on weighted
Max-Cut, parallelised by Welsh-Powell colouring of the linkage-model interaction graph
(Bouter & Bosman, arXiv 2203.08680).

The compute path is libgom.so (HIP kernels for gfx950 behind the C ABI in include/gom.h);
paper_2203_08680_amd.gom is its thin ctypes binding.
"""
from .gom import (  # noqa: F401
    GOM_FOS_NEIGHBOURHOOD, GOM_FOS_UNIVARIATE, GOM_MAX_POP, GOM_NEUTRAL_ALWAYS,
    GOM_NEUTRAL_PAPER, GOM_ORDER_FIXED, GOM_ORDER_RANDOM, GOM_SCHED_AUTO, GOM_SCHED_BITSLICED,
    GOM_SCHED_CLASS_LAUNCH, GOM_SCHED_RESIDENT, GomBatch, GomError, GomServer, Instance,
    gom_batch_init, gom_batch_run, gom_batch_set_graph, gom_colour, gom_colour_get, gom_debug_stop_after_class,
    gom_fos_build, gom_fos_build_lt, gom_fos_from_sets, gom_generation, gom_ims_run,
    gom_iterated_local_search, gom_local_search,
    gom_run_to_target,
    gom_state_autotune, gom_state_bytes, gom_state_get_block, gom_state_get_fi, gom_state_get_schedule, gom_state_hash, gom_state_init,
    gom_state_read, gom_state_reseed, gom_state_set_block, gom_state_set_fi, gom_state_set_schedule, gom_state_write,
    gom_timing_enable, gom_timing_read, gom_version, lib, mc_graph_load,
)
