"""Assembly of B by point tiles against the FP64 oracle and the row assembly.

The tile path (the default) evaluates each basis function once per (point,
window centre) pair, forms every tile's products on the matrix cores in
float64 and adds the tiles' shares as fixed-point integers; the row path
(RBF_PLAN_ROW_ASSEMBLY) streams each row's support.  Bars as in
test_gpu_parity: |b - b*| <= 1e-12 sqrt(b*_jj b*_ll) in float64 and 2e-6 in
float32; g is the rows' sum in both paths (bit for bit).  Cases cover both
dimensions, all four basis functions, variable radii, cells with more points
than one tile holds, windows that need several passes over a tile's points,
and windows too wide for the tiles (the plan then assembles by rows).
"""
import sys

import numpy as np
import pytest
import torch

import synthdata as sd
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


def scaled_error(rbf, plan, ne):
    """max over stored entries of |b - b*| / sqrt(b*_jj b*_ll), and g's error
    relative to sum |phi h| (both with the ridge added on the diagonal)."""
    val, g, lam = rbf.rbf_system_export(plan)
    ref = ne.val.copy()
    ref[ne.row_ptr[:-1][ne.active]] += ne.lam
    m = ne.m
    diag = np.zeros(m)
    for j in range(m):
        if ne.row_ptr[j + 1] > ne.row_ptr[j]:
            diag[j] = ne.val[ne.row_ptr[j]]
    r = np.repeat(np.arange(m), np.diff(ne.row_ptr))
    scale = np.sqrt(diag[r] * diag[ne.col])
    return float(np.max(np.abs(val - ref) / (scale + 1e-300))), val, g


def problem(rng, dim, g, rho_cells, n, clustered=True):
    ctr = sd.grid_centers(g, dim)
    rho = rho_cells / (g - 1)
    parts = [rng.random((dim, n // 2))]
    if clustered:
        parts.append(sd.gaussian_mixture_points(rng, n - n // 2, dim, 4))
    else:
        parts.append(rng.random((dim, n - n // 2)))
    pts = np.concatenate(parts, axis=1)
    h = np.cos(5 * pts[0]) * pts[1] + 0.1 * rng.standard_normal(pts.shape[1])
    return pts, ctr, rho, h


@pytest.mark.parametrize("phi", ["w30", "w31", "w32", "w33"])
@pytest.mark.parametrize("dim", [2, 3])
def test_tiles_against_oracle_and_rows(rbf, dim, phi):
    rng = np.random.default_rng(300 + dim)
    pts, ctr, rho, h = problem(rng, dim, 14 if dim == 2 else 7, 2.6 if dim == 2 else 1.9, 8000)
    say("tiles", dim, phi)
    ne = orc.normal_equations(pts, h, ctr, rho, phi, lambda_rel=1e-5)
    for prec, bar in (("fp64", 1e-12), ("fp32", 2e-6)):
        tile = rbf.rbf_fit_plan(dev(pts), dev(ctr), rho=rho, lambda_rel=1e-5)
        rows = rbf.rbf_fit_plan(dev(pts), dev(ctr), rho=rho, lambda_rel=1e-5, row_assembly=True)
        rbf.rbf_assemble(tile, phi, prec, dev(h))
        rbf.rbf_assemble(rows, phi, prec, dev(h))
        it, ir = rbf.rbf_plan_info(tile), rbf.rbf_plan_info(rows)
        assert it["assembly_tiles"] == 1 and ir["assembly_tiles"] == 0
        et, vt, gt = scaled_error(rbf, tile, ne)
        er, vr, gr = scaled_error(rbf, rows, ne)
        say(prec, "window", it["tile_window"], f"tiles {et:.2e} rows {er:.2e}")
        assert et <= bar and er <= bar
        assert np.array_equal(gt, gr)          # g: the rows' sums on both paths
        tile.close()
        rows.close()


@pytest.mark.parametrize("dim,g,rho_cells,n", [
    (2, 24, 5.2, 20000),   # windows of ~200 centres: several passes over a tile
    (3, 10, 2.6, 20000),   # ~300 centres in 3D: several passes
])
def test_tiles_several_passes(rbf, dim, g, rho_cells, n):
    rng = np.random.default_rng(310 + dim)
    pts, ctr, rho, h = problem(rng, dim, g, rho_cells, n)
    say("passes", dim, g, rho_cells)
    ne = orc.normal_equations(pts, h, ctr, rho, "w31", lambda_rel=1e-5)
    plan = rbf.rbf_fit_plan(dev(pts), dev(ctr), rho=rho, lambda_rel=1e-5)
    for prec, bar in (("fp64", 1e-12), ("fp32", 2e-6)):
        rbf.rbf_assemble(plan, "w31", prec, dev(h))
        info = rbf.rbf_plan_info(plan)
        e, _, _ = scaled_error(rbf, plan, ne)
        say(prec, "window", info["tile_window"], f"{e:.2e}")
        assert info["assembly_tiles"] == 1
        assert info["tile_window"] > (128 if dim == 2 else 192)
        assert e <= bar
    plan.close()


def test_tiles_dense_cells_and_variable_radii(rbf):
    # one tight cluster puts thousands of points into a few cells (several
    # tiles per cell); radii vary per centre
    rng = np.random.default_rng(320)
    ctr = sd.grid_centers(16, 2)
    m = ctr.shape[1]
    rho_vec = (0.7 + 0.6 * rng.random(m)) * 2.5 / 15
    pts = np.concatenate([rng.random((2, 4000)),
                          0.5 + 0.004 * rng.standard_normal((2, 6000))], axis=1)
    h = np.sin(4 * pts[0]) + pts[1] ** 2
    say("dense cells")
    ne = orc.normal_equations(pts, h, ctr, rho_vec, "w32", lambda_rel=1e-6)
    plan = rbf.rbf_fit_plan(dev(pts), dev(ctr), rho_per_center=dev(rho_vec), lambda_rel=1e-6)
    for prec, bar in (("fp64", 1e-12), ("fp32", 2e-6)):
        rbf.rbf_assemble(plan, "w32", prec, dev(h))
        assert rbf.rbf_plan_info(plan)["assembly_tiles"] == 1
        e, _, _ = scaled_error(rbf, plan, ne)
        say(prec, f"{e:.2e}")
        assert e <= bar
    plan.close()


def test_tiles_deterministic(rbf):
    p = sd.make_problem("terrain2d", scale=1 / 64)
    plan = rbf.rbf_fit_plan(dev(p.points), dev(p.centers), rho=p.rho, lambda_rel=1e-4)
    for prec in ("fp64", "fp32"):
        out = []
        for _ in range(2):
            rbf.rbf_assemble(plan, p.phi, prec, dev(p.values))
            val, g, lam = rbf.rbf_system_export(plan)
            out.append((val.tobytes(), g.tobytes(), lam))
        assert out[0] == out[1], prec
    plan.close()


def test_wide_windows_assemble_by_rows(rbf):
    # ~9 centre spacings of radius: ~650 centres within reach of a cell, more
    # than a tile's window holds; the plan assembles by rows instead
    rng = np.random.default_rng(330)
    pts, ctr, rho, h = problem(rng, 2, 20, 9.0, 6000, clustered=False)
    say("wide windows")
    ne = orc.normal_equations(pts, h, ctr, rho, "w31")
    plan = rbf.rbf_fit_plan(dev(pts), dev(ctr), rho=rho)
    rbf.rbf_assemble(plan, "w31", "fp64", dev(h))
    info = rbf.rbf_plan_info(plan)
    say("window", info["tile_window"])
    assert info["tile_window"] > 256 and info["assembly_tiles"] == 0
    e, _, _ = scaled_error(rbf, plan, ne)
    assert e <= 1e-12
    plan.close()


@pytest.mark.parametrize("dim,min_support", [(2, 1), (2, 20), (3, 1), (3, 8)])
def test_tile_pattern_equals_rows_pattern(rbf, dim, min_support):
    # the pattern by point tiles (marks over each row's walk of cells) and row
    # by row (RBF_PLAN_ROW_ASSEMBLY) on clustered points with per-centre radii
    rng = np.random.default_rng(340 + dim + min_support)
    g = 20 if dim == 2 else 8
    ctr = sd.grid_centers(g, dim)
    m = ctr.shape[1]
    rho_vec = (0.6 + 0.8 * rng.random(m)) * 2.4 / (g - 1)
    pts = np.concatenate([rng.random((dim, 6000)),
                          sd.gaussian_mixture_points(rng, 9000, dim, 5)], axis=1)
    say("tile pattern", dim, min_support)
    a = rbf.rbf_fit_plan(dev(pts), dev(ctr), rho_per_center=dev(rho_vec), min_support=min_support)
    b = rbf.rbf_fit_plan(dev(pts), dev(ctr), rho_per_center=dev(rho_vec), min_support=min_support,
                         row_assembly=True)
    ia, ib = rbf.rbf_plan_info(a), rbf.rbf_plan_info(b)
    assert ia["tile_window"] > 0 and ib["tile_window"] == 0
    for x, y in zip(rbf.rbf_plan_pattern(a), rbf.rbf_plan_pattern(b)):
        assert np.array_equal(x, y)
    ne = orc.normal_equations(pts, pts[0], ctr, rho_vec, "w31", min_support=min_support)
    rp, col, sup = rbf.rbf_plan_pattern(a)
    assert np.array_equal(rp, ne.row_ptr) and np.array_equal(col, ne.col)
    a.close()
    b.close()
