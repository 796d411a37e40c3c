"""Learned support radius: label sweeps, training and prediction.

Host-side orchestration of C-ABI calls (every numeric step runs in librbf):

* ``sweep_labels``: for one data set, fit with each of the sweep radii and
  score every block of centres by the held-out RMSE of its queries
  (rbf_block_sq_err); the label of a block is log(rho / spacing) of the
  radius with the smallest block RMSE (ties to the smaller radius).
* ``block_features``: the network's inputs for a data set (rbf_density_features).
* ``train``: Adam on (features, labels) with rbf_mlp_train.
* ``predict_radii``: BF16 inference per block and broadcast to the centres
  (rbf_mlp_infer_bf16, rbf_radius_broadcast); a non-finite prediction falls
  back to the fixed radius.

Features are standardised with the training set's mean and deviation (stored
with the model), so the network sees O(1) inputs.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L
from . import binding as B

# sweep radii: balls covering c_s grid centres on average
SWEEP_COVER = (10.0, 14.0, 20.0, 28.0, 40.0, 57.0, 80.0, 113.0)


def sweep_radii(spacing: float, dim: int, cover: Sequence[float] = SWEEP_COVER) -> np.ndarray:
    if dim == 2:
        return np.array([spacing * math.sqrt(c / math.pi) for c in cover])
    return np.array([spacing * (3.0 * c / (4.0 * math.pi)) ** (1.0 / 3.0) for c in cover])


def initial_params(rng: np.random.Generator) -> np.ndarray:
    """Glorot-uniform weights and zero biases for the 16-64-64-1 network, in
    the parameter layout of the library (W1 input-major, b1, W2, b2, W3, b3);
    the draw is host-side and handed to the kernels as their input."""
    n_in, n_h = L.MLP_INPUTS, 64

    def glorot(fan_in, fan_out, count):
        a = math.sqrt(6.0 / (fan_in + fan_out))
        return rng.uniform(-a, a, size=count)
    parts = [glorot(n_in, n_h, n_in * n_h), np.zeros(n_h), glorot(n_h, n_h, n_h * n_h),
             np.zeros(n_h), glorot(n_h, 1, n_h), np.zeros(1)]
    theta = np.concatenate(parts)
    assert theta.size == L.MLP_PARAMS
    return theta


def _dev(a) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def fit_once(points, values, centers, rho, phi: str, prec: str, lambda_rel: float,
             rho_per_center: Optional[torch.Tensor] = None, rtol: float = 1e-8,
             max_iter: int = 50000):
    """Plan, assemble and solve; returns (plan, coefficients, solve info)."""
    plan = B.rbf_fit_plan(points, centers, rho=rho, rho_per_center=rho_per_center,
                          lambda_rel=lambda_rel)
    B.rbf_assemble(plan, phi, prec, values)
    c, info = B.rbf_solve(plan, rtol=rtol, max_iter=max_iter)
    return plan, c, info


def block_features(points: torch.Tensor, centers: torch.Tensor, radii, blocks_per_dim: int):
    """[nblocks, 16] density features (float32, GPU) of one data set."""
    plan = B.rbf_fit_plan(points, centers, rho=float(np.max(radii)))
    f = B.rbf_density_features(plan, radii, blocks_per_dim)
    plan.close()
    return f


@dataclasses.dataclass
class SweepResult:
    labels: np.ndarray        # [nblocks] log(rho_best / spacing)
    block_rmse: np.ndarray    # [n_radii, nblocks] held-out RMSE per radius and block
    block_count: np.ndarray   # [nblocks] held-out queries per block
    rmse: np.ndarray          # [n_radii] held-out RMSE of the whole set
    seconds: np.ndarray       # [n_radii] wall time of each fit (plan + assembly + solve)
    work: np.ndarray          # [n_radii] CG work of each fit: stored entries x iterations


def fit_work(plan: B.Plan, info: dict) -> float:
    """Deterministic cost figure of a fit: entries of B times CG iterations
    (the matrix products dominate a fit's time)."""
    return float(B.rbf_plan_info(plan)["nnz_full"]) * float(info["iterations"])


def sweep_labels(points, values, test_points, test_values, centers, radii, spacing: float,
                 blocks_per_dim: int, phi: str = "w31", prec: str = "fp32",
                 lambda_rel: float = 1e-4) -> SweepResult:
    nr = len(radii)
    nblk = blocks_per_dim ** int(centers.shape[0])
    brmse = np.zeros((nr, nblk))
    rmse = np.zeros(nr)
    secs = np.zeros(nr)
    work = np.zeros(nr)
    cnt = None
    for s, rho in enumerate(radii):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan, c, info = fit_once(points, values, centers, float(rho), phi, prec, lambda_rel)
        torch.cuda.synchronize()
        secs[s] = time.perf_counter() - t0
        work[s] = fit_work(plan, info)
        f, r = B.rbf_eval(plan, test_points, c, values=test_values)
        sums, cnt = B.rbf_block_sq_err(plan, test_points, f, test_values, blocks_per_dim)
        brmse[s] = np.sqrt(sums / np.maximum(cnt, 1))
        rmse[s] = r
        plan.close()
    best = np.argmin(brmse, axis=0)           # first minimum: ties go to the smaller radius
    labels = np.log(np.asarray(radii)[best] / spacing)
    return SweepResult(labels=labels, block_rmse=brmse, block_count=cnt, rmse=rmse, seconds=secs,
                       work=work)


@dataclasses.dataclass
class RadiusModel:
    mlp: B.Mlp        # carries the input standardisation of its training features
    mean: np.ndarray
    std: np.ndarray


def train(features: np.ndarray, labels: np.ndarray, init_params: np.ndarray, epochs: int,
          batch: int, lr: float, rng: np.random.Generator) -> tuple[RadiusModel, np.ndarray]:
    """Adam over shuffled mini-batches (the shuffles are drawn here, on the host,
    and passed to the kernel as row indices)."""
    mean = features.mean(axis=0).astype(np.float32)
    std = (features.std(axis=0) + 1e-6).astype(np.float32)
    x = _dev(features.astype(np.float32))
    y = _dev(labels.astype(np.float32))
    n = features.shape[0]
    per_epoch = max(1, n // batch)
    order = np.concatenate([rng.permutation(n)[:per_epoch * batch] for _ in range(epochs)])
    mlp = B.Mlp(init_params.astype(np.float32))
    mlp.set_input_scaling(mean, std)      # the kernels standardise as they load
    losses = mlp.train(x, y, order, batch, lr)
    return RadiusModel(mlp=mlp, mean=mean, std=std), losses


def predict_radii(model: RadiusModel, plan_for_centres: B.Plan, feats: torch.Tensor,
                  blocks_per_dim: int, spacing: float, rho_min: float, rho_max: float,
                  rho_fallback: float) -> torch.Tensor:
    """Per-centre radii (float64 [M], GPU) from the BF16 network."""
    pred = model.mlp.infer_bf16(feats.contiguous())
    return B.rbf_radius_broadcast(plan_for_centres, pred, blocks_per_dim, spacing, rho_min,
                                  rho_max, rho_fallback)
