"""MI355X (gfx950) lower/upper-bound single-source shortest paths.

The method (V. K. Garg, "Removing Sequential Bottleneck of Dijkstra's
Algorithm for the Shortest Path Problem") keeps an upper bound D and a lower
bound C per vertex and fixes every vertex whose bounds meet, many per round.
The rounds run as hand-written HIP kernels in libsssp.so behind the C ABI of
include/sssp.h; this package is its Python binding.
"""
from ._abi import (  # noqa: F401
    EXPORTS, LIB_PATH, SSSP_ERR_ARG, SSSP_ERR_CAPACITY, SSSP_ERR_GRAPH, SSSP_ERR_HIP,
    SSSP_ERR_INTERNAL,
    SSSP_ERR_NOMEM, SSSP_ERR_OVERFLOW, SSSP_ERR_WEIGHT, SSSP_F32, SSSP_I32, SSSP_OK,
    SSSP_ORDER_AUTO, SSSP_ORDER_DEGREE, SSSP_ORDER_INPUT, SSSP_RELAX_AUTO,
    SSSP_RELAX_CORRECTING, SSSP_RELAX_SETTING, SSSP_SCOPE_ALL, SSSP_SCOPE_AUTO,
    SSSP_SCOPE_OPEN, SSSP_PLAN_BATCH, SSSP_PLAN_SEQUENCE, Csr, Launch,
    KERNELS, Policy, SSSPError, Stats, lib, sssp_backward, sssp_check, sssp_policy_of,
    sssp_set_round_limit, sssp_profile_enable, sssp_profile_read,
    sssp_build_csr, sssp_build_csr_bytes, sssp_release_workspace, sssp_set_weights, sssp_solve,
    sssp_solve_batch, sssp_solve_noalloc, sssp_solve_target, sssp_strerror, sssp_set_launch,
    sssp_permute_edges, sssp_plan_create,
    sssp_plan_run, sssp_plan_stats, sssp_plan_destroy, sssp_autotune)
from .graph import (  # noqa: F401
    I32_INF, Graph, Plan, SSSPFunction, autotune, backward, batch_layout, check,
    set_launch, set_round_limit, shortest_paths, solve, solve_batch, solve_target)
