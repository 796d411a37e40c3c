"""Parity of the learned-radius kernels with the FP64 oracle.

* density features: float32 storage of float64 statistics of exact counts:
  |f - f*| <= 1e-6 (1 + |f*|);
* block squared errors: counts exact, sums within 1e-12 relative;
* broadcast: within 1e-14 relative (the exponential in float64 on both sides);
* MLP gradient (float32 arithmetic, sums of <= 64 terms then chunk sums):
  |g - g*| <= 1e-4 max|g*| + 1e-5 |g*|, loss within 1e-5 relative;
* Adam: five steps of float32 training against float64 training from the
  same parameters and batches: losses within 1e-4 relative, and all but a
  handful of parameters within 1e-5 (a gradient component whose sign differs
  between float32 and float64 moves its parameter by 2 lr in the first step);
* BF16 inference against the oracle's bfloat16 emulation (round to nearest
  even of weights, inputs and hidden activations, float64 accumulation):
  within 2^-7 (1 + |out|) -- one bfloat16 ulp of a hidden activation may
  round the other way because tanh is evaluated in float32 on the GPU.
"""
import sys

import numpy as np
import pytest
import torch

import synthdata as sd
from oracle import mlp_oracle as mo
from oracle import rbf_oracle as orc

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rbf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1806_07884_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("dim", [2, 3])
def test_density_features(rbf, dim):
    from paper_1806_07884_amd import radius
    rng = np.random.default_rng(30 + dim)
    g = 32 if dim == 2 else 12
    ctr = sd.grid_centers(g, dim)
    pts = sd.gaussian_mixture_points(rng, 12000, dim, 6)
    spacing = 1.0 / (g - 1)
    radii = radius.sweep_radii(spacing, dim)
    say("features", dim, radii)
    f = radius.block_features(dev(pts), dev(ctr), radii, 4).cpu().numpy()
    ref = mo.density_features(pts, ctr, radii, 4)
    assert f.shape == ref.shape
    assert np.all(np.abs(f - ref) <= 1e-6 * (1 + np.abs(ref)))


def test_block_sq_err_and_broadcast(rbf):
    rng = np.random.default_rng(40)
    ctr = sd.grid_centers(16, 2)
    pts = rng.random((2, 2000))
    plan = rbf.rbf_fit_plan(dev(pts), dev(ctr), rho=0.15)
    q = rng.random((2, 3000)) * 1.2 - 0.1
    f = rng.standard_normal(3000)
    h = rng.standard_normal(3000)
    sums, cnt = rbf.rbf_block_sq_err(plan, dev(q), dev(f), dev(h), 4)
    rs, rc = mo.block_sq_err(q, f, h, ctr, 4)
    assert np.array_equal(cnt, rc)
    assert np.allclose(sums, rs, rtol=1e-12, atol=0)
    pred = np.array([0.1 * k - 0.8 for k in range(16)], dtype=np.float32)
    pred[5] = np.nan
    rho = rbf.rbf_radius_broadcast(plan, dev(pred), 4, 1 / 15, 0.05, 0.2, 0.1).cpu().numpy()
    ref = mo.broadcast_radius(pred.astype(np.float64), ctr, 4, 1 / 15, 0.05, 0.2, 0.1)
    assert np.allclose(rho, ref, rtol=1e-14, atol=0)


def test_mlp_gradient(rbf):
    rng = np.random.default_rng(50)
    theta = mo.init_params(rng).astype(np.float32).astype(np.float64)
    X = rng.standard_normal((200, 16)).astype(np.float32)
    y = rng.standard_normal(200).astype(np.float32)
    mlp = rbf.Mlp(theta)
    loss, g = mlp.grad(dev(X), dev(y))
    ref_loss, ref_g = mo.loss_and_grad(theta, X.astype(np.float64), y.astype(np.float64))
    say("loss", loss, ref_loss)
    assert abs(loss - ref_loss) <= 1e-5 * ref_loss
    assert np.all(np.abs(g - ref_g) <= 1e-4 * np.abs(ref_g).max() + 1e-5 * np.abs(ref_g))
    mlp.close()


def test_mlp_adam_steps(rbf):
    rng = np.random.default_rng(51)
    theta = mo.init_params(rng).astype(np.float32).astype(np.float64)
    X = rng.standard_normal((320, 16)).astype(np.float32)
    y = (np.sin(X[:, 0]) + 0.3 * X[:, 1]).astype(np.float32)
    order = np.concatenate([rng.permutation(320)[:256] for _ in range(2)])[:5 * 64]
    mlp = rbf.Mlp(theta)
    losses = mlp.train(dev(X), dev(y), order, 64, 1e-3)
    new = mlp.params().astype(np.float64)
    ref, ref_losses = mo.train(theta, X.astype(np.float64), y.astype(np.float64), order, 64, 1e-3)
    say("losses", losses, ref_losses)
    assert np.allclose(losses, ref_losses, rtol=1e-4, atol=0)
    far = np.abs(new - ref) > 1e-5
    assert far.sum() <= 0.01 * far.size, int(far.sum())
    assert np.all(np.abs(new - ref) <= 2 * 5 * 1e-3 + 1e-6)
    mlp.close()


def test_mlp_bf16_inference(rbf):
    rng = np.random.default_rng(52)
    theta = mo.init_params(rng)
    X = rng.standard_normal((777, 16)).astype(np.float32)
    mlp = rbf.Mlp(theta)
    out = mlp.infer_bf16(dev(X)).cpu().numpy().astype(np.float64)
    ref = mo.bf16_forward(theta, X.astype(np.float64))
    full, _ = mo.forward(theta, X.astype(np.float64))
    say("bf16 vs emulation max", np.max(np.abs(out - ref)), "vs float64 net max",
        np.max(np.abs(out - full)))
    assert np.all(np.abs(out - ref) <= 2.0 ** -7 * (1 + np.abs(ref)))
    mlp.close()


def test_mlp_input_scaling(rbf):
    # the kernels standardise the inputs as they load them: gradient and
    # inference on raw inputs equal the oracle's on (x - mean) / std formed in
    # float32
    rng = np.random.default_rng(53)
    theta = mo.init_params(rng).astype(np.float32).astype(np.float64)
    X = (rng.standard_normal((300, 16)) * 3.0 + 5.0).astype(np.float32)
    y = rng.standard_normal(300).astype(np.float32)
    mean = X.mean(axis=0).astype(np.float32)
    std = (X.std(axis=0) + 1e-6).astype(np.float32)
    Xs = ((X - mean) / std).astype(np.float32).astype(np.float64)
    mlp = rbf.Mlp(theta)
    mlp.set_input_scaling(mean, std)
    loss, g = mlp.grad(dev(X), dev(y))
    ref_loss, ref_g = mo.loss_and_grad(theta, Xs, y.astype(np.float64))
    assert abs(loss - ref_loss) <= 1e-5 * ref_loss
    assert np.all(np.abs(g - ref_g) <= 1e-4 * np.abs(ref_g).max() + 1e-5 * np.abs(ref_g))
    out = mlp.infer_bf16(dev(X)).cpu().numpy().astype(np.float64)
    ref = mo.bf16_forward(theta, Xs)
    assert np.all(np.abs(out - ref) <= 2.0 ** -7 * (1 + np.abs(ref)))
    st = mlp.state()
    assert np.array_equal(st["mean"], mean) and np.array_equal(st["std"], std)
    from paper_1806_07884_amd._lib import RbfError
    with pytest.raises(RbfError):
        mlp.set_input_scaling(mean, np.zeros(16, np.float32))
    mlp.close()


def test_mlp_checkpoint_resume_is_bit_exact(rbf):
    # 3 + 4 Adam steps with a checkpoint in between (restored into a fresh MLP)
    # give the bits of 7 steps in one go: parameters, both moments, step count
    rng = np.random.default_rng(54)
    theta = mo.init_params(rng)
    X = rng.standard_normal((256, 16)).astype(np.float32)
    y = (np.sin(X[:, 0]) - 0.5 * X[:, 3]).astype(np.float32)
    order = np.concatenate([rng.permutation(256) for _ in range(2)])[:7 * 64]
    mean = X.mean(axis=0).astype(np.float32)
    std = X.std(axis=0).astype(np.float32)
    whole = rbf.Mlp(theta)
    whole.set_input_scaling(mean, std)
    l_whole = whole.train(dev(X), dev(y), order, 64, 2e-3)
    a = rbf.Mlp(theta)
    a.set_input_scaling(mean, std)
    l_a = a.train(dev(X), dev(y), order[:3 * 64], 64, 2e-3)
    ck = a.state()
    assert ck["step"] == 3
    a.close()
    b = rbf.Mlp(np.zeros(mo.N_PARAMS))
    b.load_state(ck)
    l_b = b.train(dev(X), dev(y), order[3 * 64:], 64, 2e-3)
    sw, sb = whole.state(), b.state()
    say("losses", l_whole, l_a, l_b)
    assert np.array_equal(np.concatenate([l_a, l_b]), l_whole)
    for k in ("params", "m1", "m2", "mean", "std"):
        assert sw[k].tobytes() == sb[k].tobytes(), k
    assert sw["step"] == sb["step"] == 7
    whole.close()
    b.close()
