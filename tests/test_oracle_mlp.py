"""Pins of the learned-radius oracle: gradients, Adam, features, blocks."""
import math

import numpy as np
import pytest

from oracle import mlp_oracle as mo
from oracle import rbf_oracle as orc
import synthdata as sd


def test_param_count():
    assert mo.N_PARAMS == 5313


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    theta = mo.init_params(rng)
    theta[[1024 + 3, 1024 + 64 + 4096 + 5, -1]] = [0.1, -0.2, 0.3]  # non-zero biases
    X = rng.standard_normal((37, 16))
    y = rng.standard_normal(37)
    _, g = mo.loss_and_grad(theta, X, y)
    h = 1e-6
    idx = list(rng.choice(mo.N_PARAMS, size=60, replace=False)) + [0, 1023, 1024, 5311, 5312]
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mo.loss_and_grad(tp, X, y)[0] - mo.loss_and_grad(tm, X, y)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_dropped_chain_rule_term_would_be_caught():
    # sanity of the pin: forgetting the tanh derivative changes the gradient
    rng = np.random.default_rng(1)
    theta = mo.init_params(rng)
    X = rng.standard_normal((20, 16))
    y = rng.standard_normal(20)
    W1, b1, W2, b2, W3, b3 = mo.unpack(theta)
    out, (_, H1, H2) = mo.forward(theta, X)
    d_out = 2 * (out - y) / 20
    wrong_gW2 = H1.T @ np.outer(d_out, W3)          # no (1 - H2^2)
    _, g = mo.loss_and_grad(theta, X, y)
    gW2 = g[1024 + 64:1024 + 64 + 4096].reshape(64, 64)
    assert np.max(np.abs(wrong_gW2 - gW2)) > 1e-3 * np.max(np.abs(gW2))


def test_first_adam_step_closed_form():
    # at t = 1 the bias-corrected moments are g and g^2, so the step is
    # -lr g / (|g| + eps)
    rng = np.random.default_rng(2)
    theta = rng.standard_normal(50)
    g = rng.standard_normal(50)
    opt = mo.Adam(50, lr=0.01)
    new = opt.step(theta, g)
    assert np.allclose(new, theta - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_training_reduces_loss():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((256, 16))
    y = np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2]
    theta = mo.init_params(rng)
    order = np.concatenate([rng.permutation(256) for _ in range(40)])
    _, losses = mo.train(theta, X, y, order, 64, 3e-3)
    assert losses[-10:].mean() < 0.3 * losses[:10].mean()


def test_block_of_grid_centres():
    c = sd.grid_centers(256, 2)
    b = mo.block_of(c, 4)
    i = np.arange(256)
    expect = (np.repeat(i[None, :] // 64, 256, 0) + 4 * np.repeat(i[:, None] // 64, 256, 1)).ravel()
    assert np.array_equal(b, expect)
    c3 = sd.grid_centers(64, 3)
    b3 = mo.block_of(c3, 4)
    assert np.bincount(b3).tolist() == [16 ** 3] * 64


def test_density_features_from_counts():
    rng = np.random.default_rng(4)
    pts = rng.random((2, 3000))
    ctr = sd.grid_centers(8, 2)
    radii = [0.05, 0.1]
    f = mo.density_features(pts, ctr, radii, 2)
    blk = mo.block_of(ctr, 2)
    for s, rho in enumerate(radii):
        cnt = np.array([np.sum(orc.sqdist(pts, ctr[:, j]) < rho * rho) for j in range(64)])
        for b in range(4):
            lc = np.log1p(cnt[blk == b])
            assert math.isclose(f[b, 2 * s], lc.mean(), rel_tol=1e-14)
            assert math.isclose(f[b, 2 * s + 1], lc.std(), rel_tol=1e-12, abs_tol=1e-15)


def test_broadcast_clamps_and_falls_back():
    ctr = sd.grid_centers(4, 2)
    pred = np.array([0.0, 10.0, -10.0, np.nan])
    rho = mo.broadcast_radius(pred, ctr, 2, 0.1, 0.05, 0.5, 0.2)
    blk = mo.block_of(ctr, 2)
    assert np.allclose(rho[blk == 0], 0.1)
    assert np.allclose(rho[blk == 1], 0.5)
    assert np.allclose(rho[blk == 2], 0.05)
    assert np.allclose(rho[blk == 3], 0.2)


# ------------------------------------------------------ per-block squared errors
def _block_boxes_brute(queries, centers, nb):
    """Block of every query by search: the query, clamped into the centres'
    box, lies in block (k_0, .., k_{d-1}) iff lo_d + k_d ext_d / nb <= x_d <
    lo_d + (k_d + 1) ext_d / nb for each d (the last block closed above); the
    flat index takes the first coordinate fastest."""
    dim, n = queries.shape
    lo = centers.min(axis=1)
    hi = centers.max(axis=1)
    out = np.full(n, -1, dtype=np.int64)
    for q in range(n):
        x = np.minimum(np.maximum(queries[:, q], lo), hi)
        ks = []
        for d in range(dim):
            ext = hi[d] - lo[d]
            for k in range(nb):
                a = lo[d] + k * ext / nb
                b = lo[d] + (k + 1) * ext / nb
                if a <= x[d] and (x[d] < b or k == nb - 1):
                    ks.append(k)
                    break
        flat, mul = 0, 1
        for d in range(dim):
            flat += ks[d] * mul
            mul *= nb
        out[q] = flat
    return out


@pytest.mark.parametrize("dim", [2, 3])
def test_block_sq_err_equals_per_query_search(dim):
    # a grid with a different extent, offset and count per axis, so that a
    # swapped axis or stride changes the blocks; no grid line falls on a
    # block boundary inside the box
    rng = np.random.default_rng(60 + dim)
    axes = ([np.linspace(0.0, 2.0, 16), np.linspace(0.5, 1.0, 8)] if dim == 2 else
            [np.linspace(-1.0, 0.0, 6), np.linspace(0.25, 3.25, 8), np.linspace(0.0, 0.3, 4)])
    mesh = np.meshgrid(*axes, indexing="ij")
    ctr = np.stack([g.ravel(order="F") for g in mesh])
    nb = 4
    lo, hi = ctr.min(axis=1), ctr.max(axis=1)
    pad = 0.3 * (hi - lo)
    q = lo[:, None] - pad[:, None] + rng.random((dim, 1500)) * (hi - lo + 2 * pad)[:, None]
    q = np.concatenate([q, ctr], axis=1)            # the centres themselves too
    f = rng.standard_normal(q.shape[1])
    h = rng.standard_normal(q.shape[1])
    idx = _block_boxes_brute(q, ctr, nb)
    sums, cnt = mo.block_sq_err(q, f, h, ctr, nb)
    nblk = nb ** dim
    assert cnt.tolist() == [int(np.sum(idx == b)) for b in range(nblk)]
    for b in range(nblk):
        sel = idx == b
        assert math.isclose(sums[b], float(np.sum((f[sel] - h[sel]) ** 2)), rel_tol=1e-13)
    # queries at the centres fall in the centres' own blocks
    m = ctr.shape[1]
    assert np.array_equal(mo.block_index(ctr, ctr, nb), mo.block_of(ctr, nb))
    assert np.array_equal(idx[-m:], mo.block_of(ctr, nb))
    # and the axes are not interchangeable on this grid
    swapped = _block_boxes_brute(q[::-1], ctr[::-1], nb)
    assert not np.array_equal(swapped, idx)


# ---------------------------------------------------------------------- bfloat16
def test_bf16_round_equals_torch_conversion():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(70)
    hi = rng.integers(0, 1 << 16, size=4000, dtype=np.uint64)
    ties = (hi << 16) | 0x8000                        # exact halfway cases, both parities
    near = np.concatenate([(hi << 16) | 0x7FFF, (hi << 16) | 0x8001, (hi << 16) | 0x0001])
    pats = np.concatenate([ties, near]).astype(np.uint32)
    vals = pats.view(np.float32)
    vals = vals[np.isfinite(vals)]
    extra = np.array([0.0, -0.0, 1.0, -1.0, 3.0e38, -3.3e38, 1e-40, -1e-42, np.inf, -np.inf],
                     dtype=np.float32)
    vals = np.concatenate([vals, extra, rng.standard_normal(2000).astype(np.float32)])
    want = torch.from_numpy(vals).to(torch.bfloat16).to(torch.float64).numpy()
    got = mo.bf16_round(vals.astype(np.float64))
    assert np.array_equal(got, want)
    assert np.sum((pats & 0xFFFF) == 0x8000) >= 4000  # the ties were exercised
    # float64 inputs round through float32 first (the GPU holds float32 values)
    x = rng.standard_normal(500)
    assert np.array_equal(mo.bf16_round(x), torch.from_numpy(x.astype(np.float32))
                          .to(torch.bfloat16).to(torch.float64).numpy())
    assert np.isnan(mo.bf16_round(np.array([np.nan]))[0])


def test_bf16_forward_single_path_network():
    # one input i -> one hidden unit k -> one hidden unit k2 -> output, every
    # other weight 0: out = w3 bf(tanh(w2 bf(tanh(w1 bf(x_i) + b1)) + b2)) + b3
    # with bf the bfloat16 rounding (via float32) of torch
    torch = pytest.importorskip("torch")
    bf = lambda v: float(torch.tensor(np.float32(v)).to(torch.bfloat16).to(torch.float64))
    rng = np.random.default_rng(71)
    for (i, k, k2) in [(3, 5, 9), (15, 0, 63), (0, 63, 1)]:
        w1, b1, w2, b2, w3, b3 = 0.75, 0.125, -1.5, 0.0625, 2.0, -0.25
        theta = np.zeros(mo.N_PARAMS)
        o = 0
        theta[o + i * mo.N_H + k] = w1; o += mo.N_IN * mo.N_H
        theta[o + k] = b1; o += mo.N_H
        theta[o + k * mo.N_H + k2] = w2; o += mo.N_H * mo.N_H
        theta[o + k2] = b2; o += mo.N_H
        theta[o + k2] = w3; o += mo.N_H
        theta[o] = b3
        X = rng.standard_normal((40, 16)) * 1.7
        out = mo.bf16_forward(theta, X)
        for r in range(40):
            a1 = bf(math.tanh(w1 * bf(X[r, i]) + b1))
            a2 = bf(math.tanh(w2 * a1 + b2))
            assert out[r] == w3 * a2 + b3
        # the same network in float64 differs (the roundings are there)
        full, _ = mo.forward(theta, X)
        assert np.max(np.abs(full - out)) > 1e-4
