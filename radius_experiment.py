#!/usr/bin/env python3
"""Learned support radius on synthetic terrain sets, end to end on one MI355X.

The workload: `--sets` synthetic clustered terrain sets (N log-uniform in
2^lo..2^hi, 1..`--clusters` anisotropic Gaussian clusters, a `--modes`-mode
fractal height field plus noise 1e-3, 10 % held out), centres on a regular
grid of `--grid`^dim points cut into `--blocks`^dim blocks, Wendland
phi_{3,1}, ridge lambda_rel 1e-4, mixed-precision fits.

For every set the library fits once per sweep radius (balls covering 10..113
centres) and scores every block by the held-out RMSE of its queries; the
label of a block is the best radius, its features the density statistics of
rbf_density_features.  The first sets train the MLP 16-64-64-1 with the
library's Adam kernel; the last `--test` sets are fitted with the radii it
predicts (BF16 inference, broadcast per block) and compared with the best
fixed sweep radius whose fit costs no more CG work (stored entries x
iterations, deterministic; wall times are reported too).

Prints progress to stderr and one JSON summary line on stdout.

    python radius_experiment.py                       # 2D: 256 sets, 256^2 centres
    python radius_experiment.py --dim 3 --grid 64 --sets 64 --test 16 --lo 18 --hi 21 \\
        --clusters 32 --modes 128 --apply field3d     # 3D, then the 3D field workload
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def log(*a):
    print("[radius]", *a, file=sys.stderr, flush=True)


def make_set(sd, seed: int, dim: int, lo: float, hi: float, clusters: int, modes: int):
    import numpy as np
    r = sd.streams(seed, 6)
    n = int(2 ** r[0].uniform(lo, hi))
    k = int(r[0].integers(1, clusters + 1))
    pts = sd.gaussian_mixture_points(r[1], n, dim, k)
    clean = sd.terrain_values(sd.terrain_modes(r[2], modes, dim), pts)
    h = clean + 1e-3 * r[3].standard_normal(n)
    tr, te = sd.heldout_split(r[4], n, 0.1)
    return (np.ascontiguousarray(pts[:, tr]), np.ascontiguousarray(h[tr]),
            np.ascontiguousarray(pts[:, te]), np.ascontiguousarray(h[te]))


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--dim", type=int, default=2)
    ap.add_argument("--sets", type=int, default=256)
    ap.add_argument("--test", type=int, default=32)
    ap.add_argument("--grid", type=int, default=256)
    ap.add_argument("--blocks", type=int, default=4, help="blocks per dimension")
    ap.add_argument("--lo", type=float, default=16.0, help="log2 of the smallest N")
    ap.add_argument("--hi", type=float, default=20.0, help="log2 of the largest N")
    ap.add_argument("--clusters", type=int, default=64)
    ap.add_argument("--modes", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--apply", default=None, choices=[None, "field3d", "terrain2d"],
                    help="after training, fit this workload with the learned radii")
    args = ap.parse_args()
    if args.test >= args.sets:
        log("--test must be smaller than --sets")
        return 2

    import numpy as np
    import torch

    import paper_1806_07884_amd as rbf
    from paper_1806_07884_amd import radius
    import synthdata as sd

    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    dim, G, NB = args.dim, args.grid, args.blocks
    ctr = sd.grid_centers(G, dim)
    dc = dev(ctr)
    spacing = 1.0 / (G - 1)
    radii = radius.sweep_radii(spacing, dim)
    t_start = time.time()
    feats, labels, keep, sweeps = [], [], [], []
    gen_s = 0.0
    for s in range(args.sets):
        tg = time.time()
        p, h, tp, th = make_set(sd, args.seed * 100003 + s, dim, args.lo, args.hi, args.clusters,
                                args.modes)
        gen_s += time.time() - tg
        dp, dh, dtp, dth = dev(p), dev(h), dev(tp), dev(th)
        feats.append(radius.block_features(dp, dc, radii, NB).cpu().numpy())
        sw = radius.sweep_labels(dp, dh, dtp, dth, dc, radii, spacing, NB)
        labels.append(sw.labels)
        keep.append(sw.block_count >= 5)
        sweeps.append(sw)
        if s % 8 == 0 or s == args.sets - 1:
            log(f"set {s + 1}/{args.sets}: N {p.shape[1]}, sweep fits {sw.seconds.sum():.2f} s, "
                f"elapsed {time.time() - t_start:.0f} s")
    n_train = args.sets - args.test
    F = np.concatenate([f[k] for f, k in zip(feats[:n_train], keep[:n_train])])
    Y = np.concatenate([l[k] for l, k in zip(labels[:n_train], keep[:n_train])])
    rng = np.random.default_rng(args.seed)
    tt = time.time()
    model, losses = radius.train(F, Y, radius.initial_params(rng), epochs=args.epochs, batch=32,
                                 lr=args.lr, rng=rng)
    train_s = time.time() - tt
    log(f"trained on {F.shape[0]} blocks of {n_train} sets in {train_s:.2f} s; loss "
        f"{losses[:5].mean():.4f} -> {losses[-5:].mean():.4f}")
    rows = []
    for s in range(n_train, args.sets):
        p, h, tp, th = make_set(sd, args.seed * 100003 + s, dim, args.lo, args.hi, args.clusters,
                                args.modes)
        dp, dh, dtp, dth = dev(p), dev(h), dev(tp), dev(th)
        fplan = rbf.rbf_fit_plan(dp, dc, rho=float(radii.max()))
        rho = radius.predict_radii(model, fplan, dev(feats[s]), NB, spacing, float(radii.min()),
                                   float(radii.max()), float(radii[4]))
        fplan.close()
        torch.cuda.synchronize()
        ta = time.perf_counter()
        plan, c, info = radius.fit_once(dp, dh, dc, None, "w31", "fp32", 1e-4, rho_per_center=rho)
        torch.cuda.synchronize()
        t_l = time.perf_counter() - ta
        w_l = radius.fit_work(plan, info)
        _, r_l = rbf.rbf_eval(plan, dtp, c, values=dth)
        plan.close()
        sw = sweeps[s]
        ok = sw.work <= w_l
        i_eq = int(np.argmin(np.where(ok, sw.rmse, np.inf))) if np.any(ok) else 0
        i_best = int(np.argmin(sw.rmse))
        blk = np.sqrt((sw.block_rmse.min(axis=0) ** 2 * sw.block_count).sum() /
                      max(sw.block_count.sum(), 1))
        rows.append(dict(n=int(p.shape[1]), learned_rmse=float(r_l), learned_work=w_l,
                         learned_s=t_l, equal_work_rmse=float(sw.rmse[i_eq]),
                         equal_work_radius=float(radii[i_eq]), equal_work_s=float(sw.seconds[i_eq]),
                         best_fixed_rmse=float(sw.rmse[i_best]),
                         best_fixed_work=float(sw.work[i_best]),
                         best_fixed_s=float(sw.seconds[i_best]), per_block_best_rmse=float(blk)))
    L = np.array([r["learned_rmse"] for r in rows])
    E = np.array([r["equal_work_rmse"] for r in rows])
    B = np.array([r["best_fixed_rmse"] for r in rows])
    wins = int(np.sum(L < E))
    out = {
        "experiment": "learned support radius", "dim": dim, "sets": args.sets,
        "test_sets": args.test, "grid": G, "blocks_per_dim": NB,
        "n_log2_range": [args.lo, args.hi], "clusters_max": args.clusters, "modes": args.modes,
        "train_blocks": int(F.shape[0]), "epochs": args.epochs,
        "loss_first": float(losses[:5].mean()), "loss_last": float(losses[-5:].mean()),
        "train_seconds": train_s, "generation_seconds": gen_s,
        "mean_heldout_rmse": {"learned": float(L.mean()), "fixed_at_equal_work": float(E.mean()),
                              "best_fixed_any_cost": float(B.mean())},
        "learned_beats_equal_work": f"{wins}/{len(rows)}",
        "mean_work_ratio_learned_vs_best_fixed": float(np.mean(
            [r["learned_work"] / r["best_fixed_work"] for r in rows])),
        "mean_seconds": {"learned": float(np.mean([r["learned_s"] for r in rows])),
                         "best_fixed": float(np.mean([r["best_fixed_s"] for r in rows]))},
        "wall_seconds": time.time() - t_start,
    }
    log(f"test: learned {L.mean():.4e}, fixed at equal work {E.mean():.4e}, best fixed "
        f"{B.mean():.4e}; learned better in {wins}/{len(rows)}")

    if args.apply:
        p = sd.make_problem(args.apply)
        q, qh = sd.scoring_queries(p)
        if p.grid != G:
            log(f"--apply {args.apply}: its grid ({p.grid}) differs from --grid; skipped")
        else:
            dp, dh, dq, dqh = dev(p.points), dev(p.values), dev(q), dev(qh)
            fplan = rbf.rbf_fit_plan(dp, dc, rho=float(radii.max()))
            f = rbf.rbf_density_features(fplan, radii, NB)
            rho = radius.predict_radii(model, fplan, f, NB, spacing, float(radii.min()),
                                       float(radii.max()), float(p.rho))
            fplan.close()
            has_ho = p.test_points.shape[1] > 0
            dtp, dth = (dev(p.test_points), dev(p.test_values)) if has_ho else (None, None)

            def one(rho_fixed, kw):
                torch.cuda.synchronize()
                ta = time.perf_counter()
                plan, c, info = radius.fit_once(dp, dh, dc, rho_fixed, p.phi, "fp32", 1e-4, **kw)
                torch.cuda.synchronize()
                dt = time.perf_counter() - ta
                fq, r = rbf.rbf_eval(plan, dq, c, values=dqh)
                cov = fq != 0
                d = dict(query_rmse=float(r), seconds=dt, work=radius.fit_work(plan, info),
                         iterations=int(info["iterations"]),
                         covered_fraction=float(cov.double().mean().item()),
                         covered_rmse=float(torch.sqrt(torch.mean(
                             (fq[cov] - dqh[cov]) ** 2)).item()))
                if has_ho:
                    _, d["heldout_rmse"] = rbf.rbf_eval(plan, dtp, c, values=dth)
                plan.close()
                return d

            res = {"learned": one(None, dict(rho_per_center=rho)), "fixed": one(p.rho, {})}
            # every sweep radius as a fixed radius: the best held-out RMSE at no more
            # CG work than the learned fit, and at any cost
            sweep = [dict(radius=float(rr), **one(float(rr), {})) for rr in radii]
            res["sweep"] = sweep
            key = "heldout_rmse" if has_ho else "query_rmse"
            ok = [s for s in sweep if s["work"] <= res["learned"]["work"]]
            if ok:
                res["fixed_at_equal_work"] = min(ok, key=lambda s: s[key])
            res["best_fixed_any_cost"] = min(sweep, key=lambda s: s[key])
            res["score"] = key
            out["apply"] = {"workload": args.apply, **res}
            log(f"{args.apply}: learned {res['learned']}, fixed {res['fixed']}, at equal work "
                f"{res.get('fixed_at_equal_work')}, best {res['best_fixed_any_cost']}")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
