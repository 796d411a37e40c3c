"""CS-RBF least-squares approximation of big scattered data on one MI355X.

Python entry points with the names of the C-ABI in include/rbf.h; they only
marshal arguments (torch tensors give device memory and the stream) and every
step of the computation runs in the HIP kernels of librbf.so:

    plan = rbf_fit_plan(points, centers, rho, lambda_rel=1e-4)
    rbf_assemble(plan, "w31", "fp32", values)
    coeffs, info = rbf_solve(plan, rtol=1e-10)
    f, rmse = rbf_eval(plan, queries, coeffs, values=heldout_values)

Points that need not (or cannot) sit in HBM together stream through in chunks:

    plan = rbf_stream_begin(centers, max_chunk, rho, phi="w31", prec="fp32")
    for x, h in chunks:                      # GPU tensors, or pinned host tensors
        rbf_stream_add(plan, x, h)
    rbf_stream_finish(plan)
    coeffs, info = rbf_solve(plan, rtol=1e-10)
"""
from .binding import (Plan, rbf_assemble, rbf_eval, rbf_eval_noalloc, rbf_fit_plan,  # noqa: F401
                      rbf_plan_info,
                      rbf_plan_pattern, rbf_solve, rbf_system_export, rbf_poly_export, rbf_set_values,
                      rbf_solve_batch, rbf_solve_lsqr, rbf_stream_begin, rbf_stream_add, rbf_stream_finish,
                      rbf_plan_destroy,
                      rbf_profile, rbf_profile_read, rbf_density_features, rbf_block_sq_err,
                      rbf_radius_broadcast, Mlp)
