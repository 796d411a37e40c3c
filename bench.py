#!/usr/bin/env python3
"""Fit throughput of the CS-RBF normal-equation path on one MI355X.

Workload "terrain2d": N = 2^20 clustered points (64 anisotropic Gaussians,
scanline-thinned) carrying a 256-mode fractal height field plus noise
(sigma 1e-3), 1 % held out; 256 x 256 grid of reference points; Wendland
phi_{3,1} with a radius covering ~40 centres; ridge lambda_rel = 1e-4; solved
to a relative residual of 1e-10.

One step = one whole fit on inputs already resident in HBM: hash + pattern
(rbf_fit_plan), assembly of B and g (rbf_assemble), Jacobi-PCG (rbf_solve) and
evaluation of the held-out RMSE (rbf_eval).  The headline value is the
mixed-precision path (float32 basis/assembly/CG with float64 reliable
updates); the float64 path is timed the same way and reported beside it,
with both held-out RMSEs (matched when they agree to 0.1 %).  The ridge
lambda_rel = 1e-4 is the largest of the swept values whose held-out RMSE lies
within 1 % of the sweep's best; the same fits at lambda_rel = 1e-5 (the
sweep's best RMSE, twice the iterations) are timed too and reported under
"lambda_1e-5".

roofline: the CG iteration kernel's algorithmic bytes per launch (8 bytes per
nonzero of B plus ten float32 vector passes) over its average duration,
timed live with start/stop events on one launch in 128 (a stamped launch reads
about 1 us longer than the same launch in a kernel trace); the bytes the
int16-delta layout moves (6 bytes per nonzero plus twelve vector passes) are
reported beside it, and so is the bandwidth of a plain 2 GiB device copy.

``--workload terrain2d_big`` (N = 2^24, 1024 x 1024 centres, phi_{3,2}) and
``--workload field3d`` (N = 2^22 in 3D, 64^3 centres, scored at 10^6
uniform queries against the clean field) time the same step on the larger
workloads; the oracle baseline is taken for terrain2d only.
``--polynomial`` fits with linear polynomial reproduction (Section 3).
``--components p`` fits vector-valued data (p terrain fields of the same
points): one plan and assembly, then rbf_set_values and rbf_solve per
component (or, with ``--batch``, rbf_solve_batch: all components in one CG
kernel per iteration); throughput counts N points per fit of all p
components.  ``--stream K`` assembles from K point chunks (rbf_stream_begin,
rbf_stream_add per chunk, rbf_stream_finish: B and g as sums over the chunks)
instead of one resident plan; the timed fits read the chunks from HBM, and
one more fit from pinned host memory is reported beside (PCIe included).

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fit throughput (data pts/s, assembly+CG) at matched RMSE; FP32-mixed vs FP64"
HBM_PEAK = 8.0e12  # MI355X HBM3E, bytes/s
LAMBDA_REL = 1e-4
RTOL = 1e-10


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def iter_bytes(nnz_full: int, m: int, val_bytes: int, col_bytes: int, vec_bytes: int,
               n_poly: int = 0) -> int:
    """HBM bytes one CG iteration launch of this layout moves at least: every
    nonzero of B once (value and column index as stored, padding excluded)
    and, per solver row (an active centre), its state record (r, w, s, d)
    read and written plus p and x read and written, and with a polynomial its
    n_poly entries of A^T P."""
    return nnz_full * (val_bytes + col_bytes) + (12 + n_poly) * m * vec_bytes


def algorithmic_iter_bytes(nnz_full: int, m: int, vec_bytes: int) -> int:
    """Algorithmic bytes of one CG iteration, the per-unit figure of the
    mixed-precision solve: one pass over B at 8 bytes per nonzero (a float32
    value and a 32-bit column index) plus about ten passes over float32
    vectors of the solver's size."""
    return nnz_full * 8 + 10 * m * vec_bytes


def copy_peak(gib: float = 2.0, reps: int = 5) -> float:
    """Achievable HBM bandwidth: a plain device-to-device copy of `gib` GiB
    (read + write bytes over the copy time, best of `reps`), in bytes/s."""
    import torch
    n = int(gib * (1 << 30)) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * n * 4 / best


def kernel_digest() -> str:
    """Digest of the CG iteration kernel's source (its device code and layouts)."""
    csrc = os.path.join(ROOT, "paper_1806_07884_amd", "csrc")
    src = open(os.path.join(csrc, "cg_kernels.hip")).read()
    a = src.index("// Row sum over one slice of the wave")
    b = src.index("// x_hi += x_lo; x_lo = 0")
    hdr = open(os.path.join(csrc, "solver.h")).read()
    c = hdr.index("template <typename XT>\nstruct alignas")
    d = hdr.index("__host__ __device__ inline int64_t sell_pos")
    return hashlib.sha256((src[a:b] + hdr[c:d]).encode()).hexdigest()[:16]


def cpu_baseline(prob, frac: float):
    """The oracle (as it stands) on a bounded window of the same workload."""
    import numpy as np
    from oracle import rbf_oracle as orc
    try:
        import threadpoolctl
        threads = max([i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()] + [1])
    except Exception:
        threads = 1
    cores = len(os.sched_getaffinity(0))
    w = frac
    ctr = prob.centers
    keep_c = np.all(ctr <= w + 1e-12, axis=0)
    c_win = np.ascontiguousarray(ctr[:, keep_c])
    keep_p = np.all(prob.points <= w + prob.rho, axis=0)
    p_win = np.ascontiguousarray(prob.points[:, keep_p])
    h_win = np.ascontiguousarray(prob.values[keep_p])
    t0 = time.perf_counter()
    ne = orc.normal_equations(p_win, h_win, c_win, prob.rho, prob.phi, lambda_rel=LAMBDA_REL)
    orc.solve(ne)
    dt = time.perf_counter() - t0
    n_used = p_win.shape[1]
    return {"value": n_used / dt, "unit": "pts/s", "cores": int(cores), "kind": "oracle",
            "blas_threads": int(threads),
            "sample": (f"window [0,{w}]^2 of the same workload: {c_win.shape[1]} centres, "
                       f"{n_used} points (those within rho of the window), assembly of "
                       f"A, B = A^T A, g = A^T h (single-threaded NumPy/SciPy) plus the "
                       f"Cholesky solve (LAPACK, {threads} threads); {dt:.1f} s"),
            "seconds": dt}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="terrain2d",
                    choices=["terrain2d", "terrain2d_big", "field3d"])
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=None,
                    help="timed float64 fits for the comparison (default: --steps)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-window", type=float, default=0.75)
    ap.add_argument("--scale", type=float, default=1.0, help=argparse.SUPPRESS)
    ap.add_argument("--polynomial", action="store_true",
                    help="linear polynomial reproduction (bordered system of eq. 10)")
    ap.add_argument("--components", type=int, default=1,
                    help="vector-valued data: components sharing the points (B assembled once)")
    ap.add_argument("--batch", action="store_true",
                    help="with --components 2..4: solve all components in one batched CG")
    ap.add_argument("--stream", type=int, default=0, metavar="K",
                    help="assemble from K point chunks (rbf_stream_*) instead of one resident "
                         "plan; the chunks sit in HBM for the timed fits, and one more fit takes "
                         "them from pinned host memory (PCIe-inclusive, reported beside)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration) and exit")
    ap.add_argument("--no-lambda-leg", action="store_true",
                    help="skip the extra fits at lambda_rel = 1e-5 (the sweep's best held-out RMSE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); "
              "the library has no multi-GPU path", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copied {args.copy_calibration} MiB three times")
        return 0

    import paper_1806_07884_amd as rbf
    import synthdata as sd

    wl = args.workload
    log(f"generating {wl} inputs")
    prob = sd.make_problem(wl, scale=args.scale)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    pts, vals, ctr = dev(prob.points), dev(prob.values), dev(prob.centers)
    q, qh = sd.scoring_queries(prob)
    tpts, tvals = dev(q), dev(qh)
    # the 3D field is scored at uniform queries; its held-out points and the
    # queries inside some support are reported as second scores
    second = prob.score == "uniform" and prob.test_points.shape[1] > 0
    hpts, hvals = (dev(prob.test_points), dev(prob.test_values)) if second else (None, None)
    scores = {}

    def score2(plan, c, fq):
        if not second:
            return
        cov = fq != 0
        scores["covered_fraction"] = float(cov.double().mean().item())
        scores["covered_rmse"] = float(torch.sqrt(torch.mean((fq[cov] - tvals[cov]) ** 2)).item())
        _, scores["heldout_rmse"] = rbf.rbf_eval(plan, hpts, c, values=hvals)
    n_train = prob.points.shape[1]
    torch.cuda.synchronize()

    # further components of vector-valued data: other terrain fields of the same points
    extra = []
    for k in range(1, max(1, args.components)):
        r = sd.streams(7000 + k, 2)
        modes = sd.terrain_modes(r[0], 256 if prob.dim == 2 else 128, prob.dim)
        hk = sd.terrain_values(modes, prob.points) + 1e-3 * r[1].standard_normal(n_train)
        qk = sd.terrain_values(modes, q)
        extra.append((dev(hk), dev(qk)))
    stacked = torch.stack([vals] + [hk for hk, _ in extra]) if args.batch and extra else None
    # point chunks of the streamed assembly: contiguous (dim, n_c) copies, in
    # HBM and in pinned host memory
    chunks_dev, chunks_host = [], []
    if args.stream:
        if args.polynomial or args.components > 1:
            log("--stream takes neither --polynomial nor --components")
            return 2
        bounds = np.linspace(0, n_train, args.stream + 1).astype(np.int64)
        for a, b in zip(bounds[:-1], bounds[1:]):
            xc = np.ascontiguousarray(prob.points[:, a:b])
            hc = np.ascontiguousarray(prob.values[a:b])
            chunks_dev.append((dev(xc), dev(hc)))
            chunks_host.append((torch.from_numpy(xc).pin_memory(),
                                torch.from_numpy(hc).pin_memory()))
        max_chunk = int(np.max(np.diff(bounds)))
    source = {"chunks": chunks_dev}
    torch.cuda.synchronize()

    def fit(prec: str, profile: bool = False, lam: float = LAMBDA_REL):
        if args.stream:
            plan = rbf.rbf_stream_begin(ctr, max_chunk, rho=prob.rho, phi=prob.phi, prec=prec,
                                        lambda_rel=lam)
            if profile:
                rbf.rbf_profile(plan, True)
            for xc, hc in source["chunks"]:
                rbf.rbf_stream_add(plan, xc, hc)
            rbf.rbf_stream_finish(plan)
            c, info = rbf.rbf_solve(plan, rtol=RTOL, max_iter=200000)
            fq, rmse = rbf.rbf_eval(plan, tpts, c, values=tvals)
            score2(plan, c, fq)
            return plan, info, rmse
        plan = rbf.rbf_fit_plan(pts, ctr, rho=prob.rho, lambda_rel=lam,
                                polynomial=args.polynomial)
        if profile:
            rbf.rbf_profile(plan, True)
        rbf.rbf_assemble(plan, prob.phi, prec, vals)
        if stacked is not None:
            C, infos = rbf.rbf_solve_batch(plan, stacked, rtol=RTOL, max_iter=200000)
            _, rmse = rbf.rbf_eval(plan, tpts, C[0].contiguous(), values=tvals)
            for k in range(1, C.shape[0]):
                rbf.rbf_eval(plan, tpts, C[k].contiguous())
            return plan, infos[0], rmse
        c, info = rbf.rbf_solve(plan, rtol=RTOL, max_iter=200000)
        fq, rmse = rbf.rbf_eval(plan, tpts, c, values=tvals)
        score2(plan, c, fq)
        for hk, qk in extra:
            rbf.rbf_set_values(plan, hk)
            ck, _ = rbf.rbf_solve(plan, rtol=RTOL, max_iter=200000)
            rbf.rbf_eval(plan, tpts, ck)
        return plan, info, rmse

    def timed(prec: str, steps: int, warm: int, lam: float = LAMBDA_REL):
        for _ in range(warm):
            plan, info, rmse = fit(prec, lam=lam)
            plan.close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        per = []
        spmv_n, spmv_ms, asm_ms = 0, 0.0, 0.0
        for _ in range(steps):
            plan, info, rmse = fit(prec, profile=True, lam=lam)
            sc = dict(scores)
            n, ms = rbf.rbf_profile_read(plan, "cg_iter_batch" if stacked is not None else "cg_iter")
            _, ams = rbf.rbf_profile_read(plan, "assemble")
            spmv_n += n
            spmv_ms += ms
            asm_ms += ams
            per.append((info, rmse, sc))
            stats = rbf.rbf_plan_info(plan)
            plan.close()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        avg = spmv_ms / max(spmv_n, 1) * 1e3
        log(f"{prec}: {dt * 1e3:.1f} ms/fit, iters {per[-1][0]['iterations']}, "
            f"rmse {per[-1][1]:.6e}, cg iteration kernel {avg:.2f} us")
        return dt, per, stats, spmv_n, avg, asm_ms / steps

    steps = max(1, args.steps)
    dt32, per32, stats, n32, avg32, asm32 = timed("fp32", steps, args.warmup)
    dt64, per64, _, n64, avg64, asm64 = timed("fp64", args.fp64_steps or steps, args.warmup)
    value = n_train / dt32
    pcie = None
    if args.stream:
        # the same fit with the chunks coming from pinned host memory
        source["chunks"] = chunks_host
        dth, perh, _, _, _, _ = timed("fp32", 1, 0)
        pcie = {"ms_per_fit": dth * 1e3, "value": n_train / dth,
                "scoring_rmse": perh[-1][1], "chunks": args.stream}
        source["chunks"] = chunks_dev
    rmse32, rmse64 = per32[-1][1], per64[-1][1]
    matched = abs(rmse32 - rmse64) <= 1e-3 * rmse64
    second_scores = None
    if second:
        s32, s64 = per32[-1][2], per64[-1][2]
        second_scores = {"heldout_points": int(prob.test_points.shape[1]),
                         "mixed": s32, "fp64": s64,
                         "heldout_matched": bool(abs(s32["heldout_rmse"] - s64["heldout_rmse"])
                                                 <= 1e-3 * s64["heldout_rmse"])}
        matched = matched and second_scores["heldout_matched"]

    # the solver's rows are the active centres
    nnz, m, cb = stats["nnz_full"], stats["n_active"], stats["solver_col_bytes"]
    npoly = stats["n_poly"]
    # kernel time from start/stop events of sampled launches on the plan's stream
    kern32 = max(avg32, 1e-3) * 1e-6
    bytes32 = iter_bytes(nnz, m, 4, cb, 4, npoly)
    algo32 = algorithmic_iter_bytes(nnz, m, 4)
    achieved = algo32 / kern32
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"cg_iter_fp32_{wl}_traffic.json")
    if os.path.exists(tfile) and not npoly:
        with open(tfile) as fh:
            t = json.load(fh)
        if t.get("kernel_digest") == kernel_digest():
            traffic = t.get("bytes_per_launch")
    log("timing a plain device copy (achievable HBM bandwidth)")
    copy_bw = copy_peak()
    roofline = {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9,
                "unit": "GB/s", "frac": achieved / HBM_PEAK, "traffic": traffic,
                "kernel": "k_cg_iter<float,float,int16,L>",
                "algorithmic_bytes_per_launch": algo32,
                "layout_bytes_per_launch": bytes32,
                "frac_layout_bytes": bytes32 / kern32 / HBM_PEAK,
                "measured_copy_peak": copy_bw / 1e9,
                "frac_of_copy_peak": achieved / copy_bw,
                "avg_kernel_us": kern32 * 1e6, "timed_launches": n32,
                "solver_entries": stats["solver_entries"], "solver_lanes": stats["solver_lanes"]}
    kern64 = max(avg64, 1e-3) * 1e-6
    b64 = iter_bytes(nnz, m, 8, cb, 8, npoly)

    # the same fits at lambda_rel = 1e-5, the ridge with the best held-out RMSE
    # of the sweep: throughput not bought with regularisation
    lam_leg = None
    if (not args.no_lambda_leg and wl == "terrain2d" and not args.stream and not args.polynomial
            and args.components == 1):
        lam5 = 1e-5
        d5, p5, _, _, a5, _ = timed("fp32", 1, 0, lam=lam5)
        d5b, p5b, _, _, _, _ = timed("fp64", 1, 0, lam=lam5)
        lam_leg = {"lambda_rel": lam5, "value": n_train / d5, "ms_per_fit": d5 * 1e3,
                   "iterations": p5[-1][0]["iterations"], "scoring_rmse": p5[-1][1],
                   "cg_iter_kernel_us": a5,
                   "fp64": {"value": n_train / d5b, "ms_per_fit": d5b * 1e3,
                            "iterations": p5b[-1][0]["iterations"],
                            "scoring_rmse": p5b[-1][1]},
                   "rmse_matched": bool(abs(p5[-1][1] - p5b[-1][1]) <= 1e-3 * p5b[-1][1])}

    cpu = None
    if not args.no_cpu_baseline and wl == "terrain2d" and not args.polynomial:
        log("timing the oracle on a window of the workload")
        cpu = cpu_baseline(prob, args.cpu_window)
        log(f"oracle: {cpu['value']:.0f} pts/s ({cpu['seconds']:.1f} s)")

    out = {
        "metric": METRIC, "value": value, "unit": "pts/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": dt32 * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": wl, "dim": prob.dim,
                   "n_points": int(prob.points.shape[1] + prob.test_points.shape[1]),
                   "n_train": int(n_train), "n_centers": int(stats["n_centers"]),
                   "n_active": int(m), "grid": prob.grid,
                   "phi": prob.phi, "rho": prob.rho, "lambda_rel": LAMBDA_REL, "rtol": RTOL,
                   "nnz_full": int(nnz), "precision": "fp32 assembly/CG + fp64 reliable updates",
                   "polynomial": "linear" if npoly else "none",
                   "components": max(1, args.components),
                   "batched_solve": stacked is not None,
                   "stream_chunks": int(args.stream)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "mixed": {"ms_per_fit": dt32 * 1e3, "iterations": per32[-1][0]["iterations"],
                  "reliable_updates": per32[-1][0]["reliable_updates"],
                  "rel_residual": per32[-1][0]["rel_residual"], "scoring_rmse": rmse32,
                  "assembly_ms": asm32},
        "fp64": {"value": n_train / dt64, "ms_per_fit": dt64 * 1e3,
                 "iterations": per64[-1][0]["iterations"],
                 "rel_residual": per64[-1][0]["rel_residual"], "scoring_rmse": rmse64,
                 "assembly_ms": asm64, "cg_iter_kernel_us": kern64 * 1e6,
                 "cg_iter_gbps": b64 / kern64 / 1e9},
        "speedup_mixed_vs_fp64": dt64 / dt32,
        "lambda_1e-5": lam_leg,
        "stream_from_host": pcie,
        "rmse_matched": bool(matched),
        "second_scores": second_scores,
        "scoring": (f"{q.shape[1]} held-out points vs noisy samples" if prob.score == "heldout"
                    else f"{q.shape[1]} uniform queries vs the noise-free field"),
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
