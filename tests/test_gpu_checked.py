"""The checked build (librbf_checked.so: device index checks in the plan,
assembly and evaluation kernels) against the normal build, in one process.

Each case runs the same calls through both libraries on the same inputs: the
checks must never trip on a correct plan, and, since they only guard
accesses, every result (pattern, B and g, coefficients, evaluation) must be
bit for bit the normal build's.  Cases cover the tile paths in 2D and 3D,
the row paths (per-lane and grouped), a stream plan and the allocation-free
evaluation.
"""
import sys

import numpy as np
import pytest
import torch

import synthdata as sd

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def libs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1806_07884_amd as rbf
    from paper_1806_07884_amd import _lib
    prev = _lib.lib()  # the checked one too when RBF_LIBRARY=checked
    normal = _lib.load(_lib.LIB_PATH)
    checked = _lib.load(_lib.CHECKED_LIB_PATH)
    assert normal.rbf_build_checked() == 0 and checked.rbf_build_checked() == 1
    yield rbf, _lib, normal, checked
    _lib.use(prev)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def fit_all(rbf, pts, ctr, h, q, rho, phi, prec, **kw):
    """Pattern, system, coefficients and evaluation of one fit."""
    plan = rbf.rbf_fit_plan(dev(pts), dev(ctr), rho=rho, lambda_rel=1e-5, **kw)
    rp, col, _ = rbf.rbf_plan_pattern(plan)
    rbf.rbf_assemble(plan, phi, prec, dev(h))
    val, g, lam = rbf.rbf_system_export(plan)
    c, info = rbf.rbf_solve(plan, rtol=1e-10)
    f, rmse = rbf.rbf_eval(plan, dev(q), c)
    f2, _ = rbf.rbf_eval_noalloc(plan, dev(q), c, torch.empty_like(f))
    out = dict(rp=rp, col=col, val=val, g=g, lam=np.array([lam]), c=c.cpu().numpy(),
               f=f.cpu().numpy(), f2=f2.cpu().numpy(), info=rbf.rbf_plan_info(plan))
    plan.close()
    return out


def both(libs, fn):
    rbf, _lib, normal, checked = libs
    _lib.use(normal)
    a = fn(rbf)
    _lib.use(checked)
    try:
        b = fn(rbf)
    finally:
        _lib.use(normal)
    return a, b


def same(a, b):
    for k in a:
        if k == "info":
            continue
        assert np.array_equal(a[k], b[k]), k


CASES = [
    # dim, grid, radius in centre spacings, points, plan flags
    (2, 24, 2.6, 30000, {}),                        # tile pattern and tile assembly
    (3, 9, 1.9, 30000, {}),
    (2, 24, 2.6, 30000, {"row_assembly": True}),    # rows, one lane per column
    (2, 16, 9.0, 12000, {}),                        # wide windows: grouped rows
]


@pytest.mark.parametrize("dim,g,rc,n,kw", CASES)
def test_checked_build_matches(libs, dim, g, rc, n, kw):
    rng = np.random.default_rng(700 + dim + int(rc * 10))
    ctr = sd.grid_centers(g, dim)
    pts = np.concatenate([rng.random((dim, n // 2)),
                          sd.gaussian_mixture_points(rng, n - n // 2, dim, 4)], axis=1)
    h = np.cos(5 * pts[0]) * pts[1]
    q = rng.random((dim, 5000))
    rho = rc / (g - 1)
    for prec in ("fp64", "fp32"):
        say("checked", dim, g, rc, n, kw, prec)
        a, b = both(libs, lambda rbf: fit_all(rbf, pts, ctr, h, q, rho, "w31", prec, **kw))
        say("tiles", a["info"]["assembly_tiles"], "window", a["info"]["tile_window"])
        same(a, b)


def test_checked_build_radii_support_polynomial(libs):
    # per-centre radii, a support threshold and the linear polynomial (the
    # bordered system's moments are assembled too)
    rng = np.random.default_rng(720)
    g = 20
    ctr = sd.grid_centers(g, 2)
    m = ctr.shape[1]
    rho_vec = (0.6 + 0.8 * rng.random(m)) * 2.4 / (g - 1)
    pts = np.concatenate([rng.random((2, 12000)),
                          sd.gaussian_mixture_points(rng, 12000, 2, 4)], axis=1)
    h = 3.0 + 2.0 * pts[0] - pts[1] + 0.1 * np.sin(6 * pts[0])
    q = rng.random((2, 4000))

    def run(rbf):
        plan = rbf.rbf_fit_plan(dev(pts), dev(ctr), rho_per_center=dev(rho_vec), min_support=8,
                                lambda_rel=1e-5, polynomial=True)
        rp, col, sup = rbf.rbf_plan_pattern(plan)
        rbf.rbf_assemble(plan, "w32", "fp64", dev(h))
        val, gv, lam = rbf.rbf_system_export(plan)
        c, _ = rbf.rbf_solve(plan, rtol=1e-10)
        f, _ = rbf.rbf_eval(plan, dev(q), c)
        torch.cuda.synchronize()
        out = dict(rp=rp, col=col, sup=sup, val=val, g=gv, c=c.cpu().numpy(), f=f.cpu().numpy())
        plan.close()
        return out

    say("checked radii, min_support 8, polynomial")
    a, b = both(libs, run)
    same(a, b)


def test_checked_build_stream(libs):
    rng = np.random.default_rng(710)
    ctr = sd.grid_centers(20, 2)
    pts = np.concatenate([rng.random((2, 15000)),
                          sd.gaussian_mixture_points(rng, 15000, 2, 4)], axis=1)
    h = np.sin(4 * pts[0]) + pts[1]
    q = rng.random((2, 3000))

    def run(rbf):
        plan = rbf.rbf_stream_begin(dev(ctr), max_chunk=8000, rho=2.4 / 19, phi="w31",
                                    prec="fp64", lambda_rel=1e-5)
        for k in range(0, pts.shape[1], 8000):
            rbf.rbf_stream_add(plan, dev(pts[:, k:k + 8000]), dev(h[k:k + 8000]))
        rbf.rbf_stream_finish(plan)
        val, g, lam = rbf.rbf_system_export(plan)
        c, _ = rbf.rbf_solve(plan, rtol=1e-10)
        f, _ = rbf.rbf_eval(plan, dev(q), c)
        torch.cuda.synchronize()
        out = dict(val=val, g=g, c=c.cpu().numpy(), f=f.cpu().numpy())
        plan.close()
        return out

    say("checked stream")
    a, b = both(libs, run)
    same(a, b)
