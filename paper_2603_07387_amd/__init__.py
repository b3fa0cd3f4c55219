"""MI355X (gfx950) sketching estimators for full tensor network contraction.

Python binding of libtnsketch.so (C ABI in include/tn_sketch.h).  The binding
only marshals arguments: every step of the estimators runs in the library's
HIP kernels.  PyTorch supplies device memory and the current stream.

Importing this package requires the built library (see build.py); there is no
fallback path.
"""
from ._binding import (  # noqa: F401
    TN_OK, TN_ERR_ARG, TN_ERR_DIMS, TN_ERR_HYPEREDGE, TN_ERR_SELFLOOP, TN_ERR_CYCLIC,
    TN_ERR_PARTIAL, TN_ERR_OOM, TN_ERR_HIP, TN_ERR_UNSUPPORTED, TN_F64, TN_F32, TN_BF16,
    TN_CYCLIC, TN_ACYCLIC, TN_FLAG_GRAPH, TN_FLAG_PROFILE, TN_FLAG_AUTOTUNE, TN_FLAG_MFMA_BF16, TN_FLAG_PERSISTENT, TN_FLAG_PROFILE_SKETCH, TN_KERNEL_HASH, TN_KERNEL_SKETCH,
    TN_KERNEL_COMBINE, TN_KERNEL_STATS, TNError, NetworkSpec, Plan, lib_path, load,
    tn_sketch_plan, tn_sketch_estimate, tn_contract_exact, tn_plan_destroy, tn_last_error,
    tn_plan_query, tn_plan_stream, tn_plan_get_hashes, tn_plan_set_hashes, tn_plan_get_sketches,
    tn_plan_kernel_time, MLP, tn_mlp_create, tn_mlp_num_params, tn_mlp_get_params,
    tn_mlp_set_params, tn_mlp_predict, tn_mlp_grad, tn_mlp_step, tn_mlp_train, tn_mlp_destroy,
    tn_tensor_stats, tn_tensor_stats_noalloc, tn_median_of_means, median_of_means,
)
