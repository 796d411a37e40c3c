"""FP64 oracle of the learned support radius (test infrastructure only).

The paper notes that CS-RBF approximation is sensitive to data density and to
the shape parameter, chooses alpha = 1/rho experimentally (Section 6,
Table 3), and names the computation of optimal shape parameters as future work
(Section 7).  The learned radius predicts, per block of reference points, the
radius that minimises held-out error from the local density of the data:

* density features per block: for each sweep radius rho_s the mean and the
  standard deviation, over the block's centres, of log(1 + n_j(rho_s)), with
  n_j(rho) the number of points in the support of centre j (Algorithm 1's
  strict range query, eq. 18);
* an MLP 16-64-64-1 with tanh hidden units regressing log(rho / spacing);
* Adam on the mean squared error;
* the prediction clamped to the sweep range and broadcast to every centre of
  the block (a non-finite prediction falls back to a fixed radius).

Parameter layout (5313 floats): W1[16][64] (input-major), b1[64],
W2[64][64], b2[64], W3[64], b3.

bfloat16 inference reference: weights, inputs and hidden activations
rounded to bfloat16 (nearest even), sums in float64.

Parity: pinned.  Gradients against central finite differences, the first Adam
step against its closed form, features against brute-force support counts,
block assignment against integer grid arithmetic, per-block squared errors
against a per-query search over the blocks' boxes, the bfloat16 rounding
against torch's bfloat16 conversion and the bfloat16 network against a
single-path network written out with that conversion (tests/test_oracle_mlp.py).
"""
from __future__ import annotations

import math

import numpy as np

N_IN, N_H = 16, 64
N_PARAMS = N_IN * N_H + N_H + N_H * N_H + N_H + N_H + 1  # 5313


def unpack(theta: np.ndarray):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (N_PARAMS,)
    o = 0
    W1 = theta[o:o + N_IN * N_H].reshape(N_IN, N_H); o += N_IN * N_H
    b1 = theta[o:o + N_H]; o += N_H
    W2 = theta[o:o + N_H * N_H].reshape(N_H, N_H); o += N_H * N_H
    b2 = theta[o:o + N_H]; o += N_H
    W3 = theta[o:o + N_H]; o += N_H
    b3 = theta[o]
    return W1, b1, W2, b2, W3, b3


def init_params(rng: np.random.Generator) -> np.ndarray:
    """Glorot-uniform weights, zero biases (the draw is an input of both paths)."""
    def glorot(fan_in, fan_out, shape):
        a = math.sqrt(6.0 / (fan_in + fan_out))
        return rng.uniform(-a, a, size=shape)
    parts = [glorot(N_IN, N_H, N_IN * N_H), np.zeros(N_H), glorot(N_H, N_H, N_H * N_H),
             np.zeros(N_H), glorot(N_H, 1, N_H), np.zeros(1)]
    return np.concatenate(parts)


def forward(theta, X):
    """Predictions for the rows of X (n, 16); also the hidden activations."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    H1 = np.tanh(X @ W1 + b1)
    H2 = np.tanh(H1 @ W2 + b2)
    out = H2 @ W3 + b3
    return out, (X, H1, H2)


def loss_and_grad(theta, X, y):
    """Mean squared error over the batch and its gradient (backpropagation)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    out, (X, H1, H2) = forward(theta, X)
    n = X.shape[0]
    r = out - np.asarray(y, dtype=np.float64)
    loss = float(np.mean(r * r))
    d_out = 2.0 * r / n
    gW3 = H2.T @ d_out
    gb3 = np.sum(d_out)
    dZ2 = np.outer(d_out, W3) * (1.0 - H2 * H2)
    gW2 = H1.T @ dZ2
    gb2 = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ W2.T) * (1.0 - H1 * H1)
    gW1 = X.T @ dZ1
    gb1 = dZ1.sum(axis=0)
    grad = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3, [gb3]])
    return loss, grad


class Adam:
    """Adam (Kingma & Ba) with bias correction."""

    def __init__(self, n, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, theta, g):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return theta - self.lr * mh / (np.sqrt(vh) + self.eps)


def train(theta, X, y, order, batch, lr):
    """Adam steps over mini-batches X[order[k*batch:(k+1)*batch]]; returns
    the parameters and the loss of every step."""
    opt = Adam(theta.size, lr=lr)
    losses = []
    steps = len(order) // batch
    for k in range(steps):
        idx = order[k * batch:(k + 1) * batch]
        loss, g = loss_and_grad(theta, X[idx], y[idx])
        losses.append(loss)
        theta = opt.step(theta, g)
    return theta, np.asarray(losses)


# ---------------------------------------------------------------- blocks
def block_index(coords: np.ndarray, centers: np.ndarray, blocks_per_dim: int) -> np.ndarray:
    """Block index of every column of coords (SoA [dim][n]) in a uniform
    nb^dim partition of the centres' bounding box: per dimension
    t = (x - min) / (max - min) and b = floor(t nb) clipped to [0, nb - 1]
    (coordinates outside the box go to the nearest block), first coordinate
    fastest."""
    dim, n = coords.shape
    nb = blocks_per_dim
    idx = np.zeros(n, dtype=np.int64)
    mul = 1
    for d in range(dim):
        lo, hi = centers[d].min(), centers[d].max()
        ext = hi - lo
        t = (coords[d] - lo) / ext if ext > 0 else np.zeros(n)
        b = np.clip(np.floor(t * nb), 0, nb - 1).astype(np.int64)
        idx += b * mul
        mul *= nb
    return idx


def block_of(centers: np.ndarray, blocks_per_dim: int) -> np.ndarray:
    """Block index of every centre (t lies in [0, 1], so only t = 1 clips)."""
    return block_index(centers, centers, blocks_per_dim)


def density_features(points, centers, radii, blocks_per_dim):
    """[nblocks, 2 * len(radii)]: per block and radius, mean and standard
    deviation (population) of log(1 + n_j(rho)) over the block's centres."""
    from .rbf_oracle import supports
    blk = block_of(centers, blocks_per_dim)
    nblocks = blocks_per_dim ** centers.shape[0]
    feats = np.zeros((nblocks, 2 * len(radii)))
    for s, rho in enumerate(radii):
        cnt = np.array([len(x) for x in supports(points, centers, rho)], dtype=np.float64)
        lc = np.log1p(cnt)
        for b in range(nblocks):
            sel = lc[blk == b]
            if sel.size:
                feats[b, 2 * s] = sel.mean()
                feats[b, 2 * s + 1] = np.sqrt(np.mean((sel - sel.mean()) ** 2))
    return feats


def broadcast_radius(pred_log, centers, blocks_per_dim, spacing, rho_min, rho_max, rho_fallback):
    """rho_j = clamp(spacing exp(pred[block(j)]), rho_min, rho_max), or the
    fallback radius where the prediction is not finite."""
    blk = block_of(centers, blocks_per_dim)
    p = np.asarray(pred_log, dtype=np.float64)[blk]
    rho = np.clip(spacing * np.exp(p), rho_min, rho_max)
    return np.where(np.isfinite(p), rho, rho_fallback)


def block_sq_err(queries, f, h, centers, blocks_per_dim):
    """Per block of the centres' box (block_index): sum of (f - h)^2 over the
    queries in the block and their count."""
    idx = block_index(np.asarray(queries, dtype=np.float64), centers, blocks_per_dim)
    nblk = blocks_per_dim ** centers.shape[0]
    e = (np.asarray(f, dtype=np.float64) - np.asarray(h, dtype=np.float64)) ** 2
    return np.bincount(idx, weights=e, minlength=nblk), np.bincount(idx, minlength=nblk)


# ---------------------------------------------------------------- bfloat16
def bf16_round(a) -> np.ndarray:
    """Values rounded to bfloat16 and returned as float64: first to float32
    (nearest even), then the 32-bit pattern to its upper 16 bits, nearest with
    ties to even (add 0x7FFF plus the lowest kept bit, drop the low half)."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    keep_lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + keep_lsb) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_forward(theta, X) -> np.ndarray:
    """The network with bfloat16 weights, inputs and hidden activations:
    every parameter and input rounded to bfloat16, each layer's affine map
    summed in float64, tanh in float64 and its output rounded to bfloat16; the
    output layer's sum is not rounded."""
    W1, b1, W2, b2, W3, b3 = unpack(bf16_round(np.asarray(theta, np.float64)))
    x = bf16_round(X)
    h1 = bf16_round(np.tanh(x @ W1 + b1))
    h2 = bf16_round(np.tanh(h1 @ W2 + b2))
    return h2 @ W3 + b3
