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
