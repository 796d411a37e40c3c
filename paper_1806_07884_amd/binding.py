"""Thin torch-facing binding of librbf (argument marshalling only).

Device buffers come from torch tensors (float64, CUDA/HIP, contiguous); the
stream is torch's current stream unless one is given; every buffer the plan
owns is taken from torch's caching allocator through the C allocator hooks.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib as L


def _need(t: torch.Tensor, name: str, shape=None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != torch.float64 or not t.is_cuda:
        raise ValueError(f"{name} must be a float64 GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


class Plan:
    """Owner of one rbf_plan handle (and of the allocator callbacks it uses)."""

    def __init__(self):
        self.handle = ctypes.c_void_p()
        self.dim = self.n = self.m = 0
        self.n_poly = 0       # dim + 1 with a linear polynomial
        self.device = None
        self.stream = None
        self._alloc = None
        self._keep = []       # inputs the stream may still read
        self._lib = L.lib()   # the library that made the plan releases it

    def _stream_handle(self):
        return ctypes.c_void_p(self.stream.cuda_stream)

    def close(self):
        if self.handle and self.handle.value:
            with torch.cuda.device(self.device):
                self._lib.rbf_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p()
        self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _make_allocator(device: torch.device, stream: torch.cuda.Stream):
    def _alloc(nbytes, _ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device=device, stream=stream)
        except Exception:
            return None

    def _release(ptr, _nbytes, _ctx):
        torch.cuda.caching_allocator_delete(ptr)

    a = L.Allocator(L.ALLOC_FN(_alloc), L.RELEASE_FN(_release), None)
    return a


def rbf_fit_plan(points: torch.Tensor, centers: torch.Tensor, rho: Optional[float] = None,
                 rho_per_center: Optional[torch.Tensor] = None, min_support: int = 1,
                 lambda_rel: float = 0.0, stream: Optional[torch.cuda.Stream] = None,
                 polynomial: bool = False, staging: bool = True,
                 row_assembly: bool = False) -> Plan:
    """Hash, support counts and the sparsity pattern of B (rbf_fit_plan).

    polynomial: linear polynomial reproduction (coefficients c, then k = (a, a_0)).
    staging: False sets RBF_PLAN_NO_STAGING (the CG iteration gathers from
    global memory; same results).
    row_assembly: True sets RBF_PLAN_ROW_ASSEMBLY (pattern and B formed row by
    row instead of by point tiles; same pattern, same values up to the order
    of the sums).
    """
    _need(points, "points")
    if points.dim() != 2:
        raise ValueError("points must be (dim, N)")
    dim, n = points.shape
    _need(centers, "centers")
    if centers.dim() != 2 or centers.shape[0] != dim:
        raise ValueError("centers must be (dim, M)")
    m = centers.shape[1]
    if rho_per_center is not None:
        _need(rho_per_center, "rho_per_center", (m,))
    elif rho is None:
        raise ValueError("give rho or rho_per_center")
    plan = Plan()
    plan.dim, plan.n, plan.m = int(dim), int(n), int(m)
    plan.n_poly = int(dim) + 1 if polynomial else 0
    plan.device = points.device
    plan.stream = stream if stream is not None else torch.cuda.current_stream(points.device)
    plan._alloc = _make_allocator(plan.device, plan.stream)
    desc = L.PlanDesc(int(dim), int(n), int(m), points.data_ptr(), centers.data_ptr(),
                      float(rho) if rho is not None else 0.0,
                      rho_per_center.data_ptr() if rho_per_center is not None else None,
                      int(min_support), float(lambda_rel), int(bool(polynomial)),
                      (0 if staging else L.PLAN_NO_STAGING)
                      | (L.PLAN_ROW_ASSEMBLY if row_assembly else 0))
    with torch.cuda.device(plan.device):
        st = L.lib().rbf_fit_plan(ctypes.byref(desc), ctypes.byref(plan._alloc),
                                  plan._stream_handle(), ctypes.byref(plan.handle))
    L.check(st, "rbf_fit_plan")
    return plan


def rbf_plan_info(plan: Plan) -> dict:
    s = L.PlanStats()
    with torch.cuda.device(plan.device):
        L.check(L.lib().rbf_plan_info(plan.handle, ctypes.byref(s)), "rbf_plan_info")
    out = {k: getattr(s, k) for k, _ in L.PlanStats._fields_}
    out["grid"] = list(s.grid)
    out.pop("pad_", None)
    return out


def rbf_plan_pattern(plan: Plan):
    """(row_ptr int64 [M+1], col int32 [nnz_upper], support int32 [M]) on the host."""
    info = rbf_plan_info(plan)
    rp = np.zeros(plan.m + 1, np.int64)
    col = np.zeros(max(1, info["nnz_upper"]), np.int32)
    sup = np.zeros(plan.m, np.int32)
    with torch.cuda.device(plan.device):
        L.check(L.lib().rbf_plan_pattern(plan.handle, rp.ctypes.data, col.ctypes.data,
                                         sup.ctypes.data), "rbf_plan_pattern")
    return rp, col[:info["nnz_upper"]], sup


def rbf_stream_begin(centers: torch.Tensor, max_chunk: int, rho: Optional[float] = None,
                     rho_per_center: Optional[torch.Tensor] = None, phi: str = "w31",
                     prec: str = "fp64", min_support: int = 1, lambda_rel: float = 0.0,
                     stream: Optional[torch.cuda.Stream] = None, staging: bool = True) -> Plan:
    """Stream plan from the centres alone (rbf_stream_begin): points then come
    in chunks of at most max_chunk (rbf_stream_add) and rbf_stream_finish
    forms the system, as rbf_fit_plan + rbf_assemble would for all of them."""
    _need(centers, "centers")
    if centers.dim() != 2:
        raise ValueError("centers must be (dim, M)")
    dim, m = centers.shape
    if rho_per_center is not None:
        _need(rho_per_center, "rho_per_center", (m,))
    elif rho is None:
        raise ValueError("give rho or rho_per_center")
    plan = Plan()
    plan.dim, plan.n, plan.m = int(dim), 0, int(m)
    plan.device = centers.device
    plan.stream = stream if stream is not None else torch.cuda.current_stream(centers.device)
    plan._alloc = _make_allocator(plan.device, plan.stream)
    desc = L.StreamDesc(int(dim), int(m), centers.data_ptr(),
                        float(rho) if rho is not None else 0.0,
                        rho_per_center.data_ptr() if rho_per_center is not None else None,
                        int(min_support), float(lambda_rel), L.PHI[phi], L.PREC[prec],
                        int(max_chunk), 0 if staging else L.PLAN_NO_STAGING)
    with torch.cuda.device(plan.device):
        st = L.lib().rbf_stream_begin(ctypes.byref(desc), ctypes.byref(plan._alloc),
                                      plan._stream_handle(), ctypes.byref(plan.handle))
    L.check(st, "rbf_stream_begin")
    return plan


def rbf_stream_add(plan: Plan, points: torch.Tensor, values: torch.Tensor) -> None:
    """Add a chunk (rbf_stream_add): points (dim, n) and values (n,) float64,
    contiguous, both on the GPU or both in host memory (pinned for an
    asynchronous copy that overlaps the previous chunk's accumulation)."""
    on_host = not points.is_cuda
    for t, name in ((points, "points"), (values, "values")):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 tensor")
        if t.is_cuda == on_host:
            raise ValueError("points and values must both be on the GPU or both on the host")
    if points.dim() != 2 or points.shape[0] != plan.dim:
        raise ValueError(f"points must be ({plan.dim}, n)")
    n = int(points.shape[1])
    if tuple(values.shape) != (n,):
        raise ValueError(f"values has shape {tuple(values.shape)}, expected ({n},)")
    with torch.cuda.device(plan.device):
        st = L.lib().rbf_stream_add(plan.handle, n, points.data_ptr() if n else None,
                                    values.data_ptr() if n else None, int(on_host))
    L.check(st, "rbf_stream_add")
    plan.n += n
    # inputs the streams may still read: device chunks until the finish, host
    # chunks until the next call has returned
    if on_host:
        plan._keep = [t for t in plan._keep if t.is_cuda] + [points, values]
    else:
        plan._keep += [points, values]


def rbf_stream_finish(plan: Plan) -> None:
    """Form the system of all chunks added (rbf_stream_finish); blocks."""
    with torch.cuda.device(plan.device):
        st = L.lib().rbf_stream_finish(plan.handle)
    L.check(st, "rbf_stream_finish")
    plan._keep = []


def rbf_assemble(plan: Plan, phi: str, prec: str, values: torch.Tensor) -> None:
    """Values of B (+ ridge) and g = A^T h in precision 'fp64' or 'fp32' (rbf_assemble)."""
    _need(values, "values", (plan.n,))
    with torch.cuda.device(plan.device):
        st = L.lib().rbf_assemble(plan.handle, L.PHI[phi], L.PREC[prec], values.data_ptr())
    L.check(st, "rbf_assemble")
    plan._keep = [values]


def rbf_set_values(plan: Plan, values: torch.Tensor) -> None:
    """New sample values for the assembled system: g = A^T h (and P^T h) only,
    B kept (rbf_set_values); one call per component of vector-valued data."""
    _need(values, "values", (plan.n,))
    with torch.cuda.device(plan.device):
        st = L.lib().rbf_set_values(plan.handle, values.data_ptr())
    L.check(st, "rbf_set_values")
    plan._keep = [values]


def rbf_system_export(plan: Plan):
    """(upper values of B + lambda I [nnz_upper], g [M], lambda) on the host."""
    info = rbf_plan_info(plan)
    val = np.zeros(max(1, info["nnz_upper"]))
    g = np.zeros(plan.m)
    lam = ctypes.c_double()
    with torch.cuda.device(plan.device):
        L.check(L.lib().rbf_system_export(plan.handle, val.ctypes.data, g.ctypes.data,
                                          ctypes.byref(lam)), "rbf_system_export")
    return val[:info["nnz_upper"]], g, lam.value


def rbf_poly_export(plan: Plan):
    """(A^T P [M][d+1], P^T P, P^T h) of eq. 10 on the host, basis P_i = (x_i^T, 1)."""
    k = plan.n_poly
    q = np.zeros((plan.m, k))
    c = np.zeros((k, k))
    e = np.zeros(k)
    with torch.cuda.device(plan.device):
        L.check(L.lib().rbf_poly_export(plan.handle, q.ctypes.data, c.ctypes.data,
                                        e.ctypes.data), "rbf_poly_export")
    return q, c, e


def rbf_solve(plan: Plan, coeffs: Optional[torch.Tensor] = None, rtol: float = 1e-10,
              max_iter: int = 100000, warm_start: bool = False, check_every: int = 32,
              reliable_delta: float = 0.1, stall_limit: int = 0):
    """Jacobi-PCG solve of (B + lambda I) c = g, or of the bordered system of eq. 10
    with a polynomial (rbf_solve).  Returns (coeffs [M + n_poly], info)."""
    if coeffs is None:
        coeffs = torch.zeros(plan.m + plan.n_poly, dtype=torch.float64, device=plan.device)
    _need(coeffs, "coeffs", (plan.m + plan.n_poly,))
    opts = L.SolveOpts(float(rtol), int(max_iter), int(bool(warm_start)), int(check_every),
                       float(reliable_delta), int(stall_limit))
    info = L.SolveInfo()
    with torch.cuda.device(plan.device):
        st = L.lib().rbf_solve(plan.handle, ctypes.byref(opts), coeffs.data_ptr(),
                               ctypes.byref(info))
    L.check(st, "rbf_solve")
    return coeffs, {"iterations": info.iterations, "reliable_updates": info.reliable_updates,
                    "rel_residual": info.rel_residual, "lambda": info.lambda_,
                    "precision": "fp64" if info.precision == 0 else "fp32",
                    "status": info.status}


def rbf_solve_lsqr(plan: Plan, coeffs: Optional[torch.Tensor] = None, rtol: float = 1e-12,
                   max_iter: int = 100000, warm_start: bool = False):
    """The least-squares fit by LSQR on A itself (rbf_solve_lsqr): for dense,
    ill-conditioned A where CG on A^T A cannot reach float64 accuracy.  Returns
    (coeffs [M + n_poly], info)."""
    if coeffs is None:
        coeffs = torch.zeros(plan.m + plan.n_poly, dtype=torch.float64, device=plan.device)
    _need(coeffs, "coeffs", (plan.m + plan.n_poly,))
    opts = L.SolveOpts(float(rtol), int(max_iter), int(bool(warm_start)), 1, 0.1, 0)
    info = L.SolveInfo()
    with torch.cuda.device(plan.device):
        st = L.lib().rbf_solve_lsqr(plan.handle, ctypes.byref(opts), coeffs.data_ptr(),
                                    ctypes.byref(info))
    L.check(st, "rbf_solve_lsqr")
    return coeffs, {"iterations": info.iterations, "rel_residual": info.rel_residual,
                    "lambda": info.lambda_, "precision": "fp64", "status": info.status}


def rbf_solve_batch(plan: Plan, values: torch.Tensor, coeffs: Optional[torch.Tensor] = None,
                    rtol: float = 1e-10, max_iter: int = 100000, warm_start: bool = False,
                    check_every: int = 32, reliable_delta: float = 0.1):
    """All components of vector-valued data at once (rbf_solve_batch): values
    (p, N) with 2 <= p <= 4.  Returns (coeffs (p, M), [info per component])."""
    _need(values, "values")
    if values.dim() != 2 or values.shape[1] != plan.n:
        raise ValueError("values must be (p, N)")
    nr = int(values.shape[0])
    if coeffs is None:
        coeffs = torch.zeros((nr, plan.m), dtype=torch.float64, device=plan.device)
    _need(coeffs, "coeffs", (nr, plan.m))
    opts = L.SolveOpts(float(rtol), int(max_iter), int(bool(warm_start)), int(check_every),
                       float(reliable_delta))
    infos = (L.SolveInfo * max(nr, 1))()
    with torch.cuda.device(plan.device):
        st = L.lib().rbf_solve_batch(plan.handle, nr, values.data_ptr(), ctypes.byref(opts),
                                     coeffs.data_ptr(), infos)
    L.check(st, "rbf_solve_batch")
    plan._keep = [values]
    out = [{"iterations": f.iterations, "reliable_updates": f.reliable_updates,
            "rel_residual": f.rel_residual, "lambda": f.lambda_,
            "precision": "fp64" if f.precision == 0 else "fp32", "status": f.status}
           for f in infos[:nr]]
    return coeffs, out


def rbf_eval(plan: Plan, queries: torch.Tensor, coeffs: torch.Tensor,
             out: Optional[torch.Tensor] = None, values: Optional[torch.Tensor] = None):
    """f at the query points (eq. 3, or eq. 6 with a polynomial), and the RMSE
    against `values` when given."""
    _need(queries, "queries")
    if queries.dim() != 2 or queries.shape[0] != plan.dim:
        raise ValueError("queries must be (dim, Q)")
    nq = int(queries.shape[1])
    _need(coeffs, "coeffs", (plan.m + plan.n_poly,))
    if out is None:
        out = torch.empty(nq, dtype=torch.float64, device=plan.device)
    _need(out, "out", (nq,))
    rmse = ctypes.c_double(float("nan"))
    if values is not None:
        _need(values, "values", (nq,))
    with torch.cuda.device(plan.device):
        st = L.lib().rbf_eval(plan.handle, nq, queries.data_ptr(), coeffs.data_ptr(),
                              out.data_ptr(), values.data_ptr() if values is not None else None,
                              ctypes.byref(rmse))
    L.check(st, "rbf_eval")
    plan._keep = [queries, coeffs]
    return out, (rmse.value if values is not None else None)


def rbf_eval_noalloc(plan: Plan, queries: torch.Tensor, coeffs: torch.Tensor,
                     out: torch.Tensor, values: Optional[torch.Tensor] = None):
    """rbf_eval without any device allocation (rbf_eval_noalloc): the library's
    static workspace replaces the plan's; `out` (Q,) float64 is the caller's."""
    _need(queries, "queries")
    if queries.dim() != 2 or queries.shape[0] != plan.dim:
        raise ValueError("queries must be (dim, Q)")
    nq = int(queries.shape[1])
    _need(coeffs, "coeffs", (plan.m + plan.n_poly,))
    _need(out, "out", (nq,))
    rmse = ctypes.c_double(float("nan"))
    if values is not None:
        _need(values, "values", (nq,))
    with torch.cuda.device(plan.device):
        st = L.lib().rbf_eval_noalloc(plan.handle, nq, queries.data_ptr(), coeffs.data_ptr(),
                                      out.data_ptr(),
                                      values.data_ptr() if values is not None else None,
                                      ctypes.byref(rmse))
    L.check(st, "rbf_eval_noalloc")
    return out, (rmse.value if values is not None else None)


def rbf_profile(plan: Plan, enable: bool) -> None:
    """Start (reset) or stop event timing of the assembly and CG iteration launches."""
    with torch.cuda.device(plan.device):
        L.check(L.lib().rbf_profile(plan.handle, int(bool(enable))), "rbf_profile")


def rbf_profile_read(plan: Plan, kernel: str):
    """(timed launches, summed milliseconds) of 'cg_iter' or 'assemble'."""
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    with torch.cuda.device(plan.device):
        L.check(L.lib().rbf_profile_read(plan.handle, L.KERNEL[kernel], ctypes.byref(n),
                                         ctypes.byref(ms)), "rbf_profile_read")
    return n.value, ms.value


def _need32(t, name, shape=None):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_cuda \
            or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 GPU tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


def rbf_density_features(plan: Plan, radii, blocks_per_dim: int) -> torch.Tensor:
    """Per-block density features [nblocks, 2 len(radii)] (float32, on the GPU)."""
    r = np.ascontiguousarray(np.asarray(radii, dtype=np.float64))
    nblk = blocks_per_dim ** plan.dim
    out = torch.empty((nblk, 2 * len(r)), dtype=torch.float32, device=plan.device)
    with torch.cuda.device(plan.device):
        L.check(L.lib().rbf_density_features(plan.handle, len(r), r.ctypes.data, blocks_per_dim,
                                             out.data_ptr()), "rbf_density_features")
    return out


def rbf_block_sq_err(plan: Plan, queries: torch.Tensor, f: torch.Tensor, h: torch.Tensor,
                     blocks_per_dim: int):
    """(sum of squared errors, count) per block of the centres' box, on the host."""
    _need(queries, "queries")
    nq = int(queries.shape[1])
    _need(f, "f", (nq,))
    _need(h, "h", (nq,))
    nblk = blocks_per_dim ** plan.dim
    sums = np.zeros(nblk)
    cnt = np.zeros(nblk, np.int64)
    with torch.cuda.device(plan.device):
        L.check(L.lib().rbf_block_sq_err(plan.handle, nq, queries.data_ptr(), f.data_ptr(),
                                         h.data_ptr(), blocks_per_dim, sums.ctypes.data,
                                         cnt.ctypes.data), "rbf_block_sq_err")
    return sums, cnt


def rbf_radius_broadcast(plan: Plan, pred_log: torch.Tensor, blocks_per_dim: int, spacing: float,
                         rho_min: float, rho_max: float, rho_fallback: float) -> torch.Tensor:
    """Per-centre radii (float64 [M] on the GPU) from per-block log-radius predictions."""
    nblk = blocks_per_dim ** plan.dim
    _need32(pred_log, "pred_log", (nblk,))
    out = torch.empty(plan.m, dtype=torch.float64, device=plan.device)
    with torch.cuda.device(plan.device):
        L.check(L.lib().rbf_radius_broadcast(plan.handle, pred_log.data_ptr(), blocks_per_dim,
                                             float(spacing), float(rho_min), float(rho_max),
                                             float(rho_fallback), out.data_ptr()),
                "rbf_radius_broadcast")
    return out


class Mlp:
    """Owner of an rbf_mlp handle (the 16-64-64-1 radius network)."""

    def __init__(self, params, device=None, stream=None):
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        if p.shape != (L.MLP_PARAMS,):
            raise ValueError(f"params must have {L.MLP_PARAMS} entries")
        self.device = torch.device(device) if device is not None else torch.device("cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            L.check(L.lib().rbf_mlp_create(p.ctypes.data, ctypes.c_void_p(self.stream.cuda_stream),
                                           ctypes.byref(self.handle)), "rbf_mlp_create")

    def params(self) -> np.ndarray:
        out = np.zeros(L.MLP_PARAMS, np.float32)
        with torch.cuda.device(self.device):
            L.check(L.lib().rbf_mlp_params(self.handle, out.ctypes.data), "rbf_mlp_params")
        return out

    def grad(self, x: torch.Tensor, y: torch.Tensor):
        n = int(x.shape[0])
        _need32(x, "x", (n, L.MLP_INPUTS))
        _need32(y, "y", (n,))
        g = np.zeros(L.MLP_PARAMS, np.float32)
        loss = ctypes.c_float()
        with torch.cuda.device(self.device):
            L.check(L.lib().rbf_mlp_grad(self.handle, x.data_ptr(), y.data_ptr(), n, g.ctypes.data,
                                         ctypes.byref(loss)), "rbf_mlp_grad")
        return float(loss.value), g

    def train(self, x: torch.Tensor, y: torch.Tensor, order, batch: int, lr: float):
        n = int(x.shape[0])
        _need32(x, "x", (n, L.MLP_INPUTS))
        _need32(y, "y", (n,))
        o = torch.as_tensor(np.ascontiguousarray(np.asarray(order, dtype=np.int32)),
                            device=self.device)
        steps = int(o.numel()) // batch
        losses = np.zeros(max(steps, 1), np.float32)
        with torch.cuda.device(self.device):
            L.check(L.lib().rbf_mlp_train(self.handle, x.data_ptr(), y.data_ptr(), n, o.data_ptr(),
                                          steps, batch, float(lr), losses.ctypes.data),
                    "rbf_mlp_train")
        return losses[:steps]

    def infer_bf16(self, x: torch.Tensor) -> torch.Tensor:
        n = int(x.shape[0])
        _need32(x, "x", (n, L.MLP_INPUTS))
        out = torch.empty(n, dtype=torch.float32, device=self.device)
        with torch.cuda.device(self.device):
            L.check(L.lib().rbf_mlp_infer_bf16(self.handle, x.data_ptr(), n, out.data_ptr()),
                    "rbf_mlp_infer_bf16")
        return out

    def set_input_scaling(self, mean, std) -> None:
        """Inputs are standardised as (x - mean) / std (float32, per input) by
        the training, gradient and inference kernels."""
        m = np.ascontiguousarray(np.asarray(mean, dtype=np.float32).reshape(L.MLP_INPUTS))
        s = np.ascontiguousarray(np.asarray(std, dtype=np.float32).reshape(L.MLP_INPUTS))
        with torch.cuda.device(self.device):
            L.check(L.lib().rbf_mlp_set_input_scaling(self.handle, m.ctypes.data, s.ctypes.data),
                    "rbf_mlp_set_input_scaling")

    def state(self) -> dict:
        """Everything training continues from: parameters, Adam moments and
        step count, input scaling (rbf_mlp_state)."""
        out = {k: np.zeros(L.MLP_PARAMS, np.float32) for k in ("params", "m1", "m2")}
        out["mean"] = np.zeros(L.MLP_INPUTS, np.float32)
        out["std"] = np.zeros(L.MLP_INPUTS, np.float32)
        step = ctypes.c_int64()
        with torch.cuda.device(self.device):
            L.check(L.lib().rbf_mlp_state(self.handle, out["params"].ctypes.data,
                                          out["m1"].ctypes.data, out["m2"].ctypes.data,
                                          ctypes.byref(step), out["mean"].ctypes.data,
                                          out["std"].ctypes.data), "rbf_mlp_state")
        out["step"] = int(step.value)
        return out

    def load_state(self, st: dict) -> None:
        """Resume from a state() dictionary (rbf_mlp_load_state)."""
        arr = {k: np.ascontiguousarray(np.asarray(st[k], dtype=np.float32))
               for k in ("params", "m1", "m2", "mean", "std")}
        with torch.cuda.device(self.device):
            L.check(L.lib().rbf_mlp_load_state(self.handle, arr["params"].ctypes.data,
                                               arr["m1"].ctypes.data, arr["m2"].ctypes.data,
                                               int(st["step"]), arr["mean"].ctypes.data,
                                               arr["std"].ctypes.data), "rbf_mlp_load_state")

    def close(self):
        if self.handle and self.handle.value:
            with torch.cuda.device(self.device):
                L.lib().rbf_mlp_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rbf_plan_destroy(plan: Plan) -> None:
    plan.close()
