"""Parity of the HIP path (through the C-ABI) with the FP64 CPU oracle.

Bars
----
* supports, active set and the upper-CSR pattern of B: bit-exact;
* values of B (FP64): |b - b*| <= 1e-12 sqrt(b*_jj b*_ll) (the Cauchy-Schwarz
  scale of the entry; each of the n_jl products carries a few rounding errors
  of phi and of the sum, bounded well below that);
* values of B (FP32 + Kahan): |b - b*| <= 2e-6 sqrt(b*_jj b*_ll);
* g: |g - g*| <= 1e-12 sum_k |phi_kj h_k| (FP64) or 2e-6 (FP32);
* FP64 solve (to relative residual 1e-13): fitted values
  ||A (c - c*)|| / ||A c*|| <= 1e-10 (relative 1e-10 of the fitted surface);
  coefficients <= max(1e-10, kappa (rel_residual + 10 u)), the perturbation
  bound of the solve plus the oracle's Cholesky error;
* mixed solve: held-out RMSE within 0.1 % of the FP64 oracle's;
* evaluation: |f - f*| <= 1e-12 (sum_j |c_j phi_j| + 1e-300).
"""
import sys

import numpy as np
import pytest
import torch

import synthdata as sd
from oracle import rbf_oracle as orc
from tolerances import FIT_FP64, FP64_RTOL

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53


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


def entry_scale(ne, rows=None):
    """sqrt(b_jj b_ll) for every stored upper entry."""
    m = ne.m
    diag = np.zeros(m)
    for j in range(m):
        a, b = ne.row_ptr[j], ne.row_ptr[j + 1]
        if b > a:
            diag[j] = ne.val[a]  # first upper entry of a row is its diagonal
    r = np.repeat(np.arange(m), np.diff(ne.row_ptr))
    return np.sqrt(diag[r] * diag[ne.col])


def check_pattern(rbf, plan, ne):
    rp, col, sup = rbf.rbf_plan_pattern(plan)
    assert np.array_equal(sup, ne.support_count)
    assert np.array_equal(rp, ne.row_ptr)
    assert np.array_equal(col, ne.col)
    info = rbf.rbf_plan_info(plan)
    assert info["nnz_upper"] == ne.nnz_upper
    assert info["nnz_full"] == ne.nnz_full
    assert info["n_active"] == int(ne.active.sum())


def check_values(rbf, plan, ne, h, tol):
    val, g, lam = rbf.rbf_system_export(plan)
    ref = ne.val.copy()
    diag_pos = ne.row_ptr[:-1][ne.active]
    ref[diag_pos] += ne.lam
    # a stored diagonal is b_jj + lambda: its scale includes the ridge, whose
    # own rounding (a float64 mean over the diagonals) is relative to lambda
    # (a centre with one far point in its support has b_jj ~ 1e-26 << lambda)
    scale = entry_scale(ne)
    scale[diag_pos] += ne.lam
    err = np.abs(val - ref)
    assert np.all(err <= tol * scale + 1e-300), float(np.max(err / (scale + 1e-300)))
    gscale = np.abs(ne.A).T @ np.abs(h)
    assert np.all(np.abs(g - ne.g) <= tol * gscale + 1e-300)
    assert abs(lam - ne.lam) <= 1e-10 * max(ne.lam, 1e-300) or (lam == 0.0 and ne.lam == 0.0) \
        or abs(lam - ne.lam) <= tol * ne.lam * 10
    return float(np.max(err / (scale + 1e-300)))


def boundary_stress_points(ctr, rho, rng, n):
    """Points exactly at distance rho from centres along the axes, and just inside."""
    dim, m = ctr.shape
    js = rng.integers(0, m, size=n)
    ax = rng.integers(0, dim, size=n)
    sgn = rng.choice([-1.0, 1.0], size=n)
    p = ctr[:, js].copy()
    inside = rng.random(n) < 0.5
    step = np.where(inside, np.nextafter(rho, 0.0), rho)
    p[ax, np.arange(n)] += sgn * step
    return p


# ----------------------------------------------------------------- patterns
@pytest.mark.parametrize("dim,n,g,rho,seed", [
    (2, 1, 3, 0.3, 0),            # one point
    (2, 777, 7, 0.21, 1),         # ragged, several tiles
    (2, 5000, 23, 0.09, 2),
    (3, 1999, 5, 0.31, 3),
    (3, 4000, 8, 0.2, 4),
])
def test_pattern_bit_exact_random(rbf, dim, n, g, rho, seed):
    rng = np.random.default_rng(seed)
    ctr = sd.grid_centers(g, dim)
    pts = rng.random((dim, n)) * 1.2 - 0.1          # some points outside every support
    if n > 10:
        pts = np.concatenate([pts, boundary_stress_points(ctr, rho, rng, n // 5)], axis=1)
    h = np.sin(7 * pts[0]) + pts[-1]
    say("pattern", dim, pts.shape[1], ctr.shape[1], rho)
    ne = orc.normal_equations(pts, h, ctr, rho, "w31")
    plan = rbf.rbf_fit_plan(dev(pts), dev(ctr), rho=rho)
    check_pattern(rbf, plan, ne)


@pytest.mark.parametrize("dim,min_support", [(2, 1), (2, 25), (3, 6)])
def test_pattern_variable_radius_and_min_support(rbf, dim, min_support):
    rng = np.random.default_rng(10 + dim)
    g = 9 if dim == 2 else 5
    ctr = sd.grid_centers(g, dim)
    m = ctr.shape[1]
    rho_vec = (0.6 + 0.8 * rng.random(m)) * 1.8 / (g - 1)
    pts = sd.gaussian_mixture_points(rng, 3000, dim, 4)
    h = pts[0] * 2 - pts[-1]
    say("variable-radius", dim, min_support)
    ne = orc.normal_equations(pts, h, ctr, rho_vec, "w32", min_support=min_support)
    plan = rbf.rbf_fit_plan(dev(pts), dev(ctr), rho_per_center=dev(rho_vec),
                            min_support=min_support)
    check_pattern(rbf, plan, ne)
    rbf.rbf_assemble(plan, "w32", "fp64", dev(h))
    check_values(rbf, plan, ne, h, 1e-12)


def test_pattern_franke_config(rbf):
    p = sd.make_problem("franke2d")
    say("franke2d pattern", p.points.shape, p.centers.shape)
    ne = orc.normal_equations(p.points, p.values, p.centers, p.rho, p.phi)
    plan = rbf.rbf_fit_plan(dev(p.points), dev(p.centers), rho=p.rho)
    check_pattern(rbf, plan, ne)


# ------------------------------------------------------------------- values
@pytest.mark.parametrize("phi", ["w30", "w31", "w32", "w33"])
@pytest.mark.parametrize("dim", [2, 3])
def test_values_fp64_and_fp32(rbf, phi, dim):
    rng = np.random.default_rng(20 + dim)
    g = 12 if dim == 2 else 6
    ctr = sd.grid_centers(g, dim)
    rho = 2.2 / (g - 1)
    pts = rng.random((dim, 6000))
    h = np.cos(5 * pts[0]) * pts[1]
    say("values", phi, dim)
    ne = orc.normal_equations(pts, h, ctr, rho, phi, lambda_rel=1e-5)
    plan = rbf.rbf_fit_plan(dev(pts), dev(ctr), rho=rho, lambda_rel=1e-5)
    rbf.rbf_assemble(plan, phi, "fp64", dev(h))
    e64 = check_values(rbf, plan, ne, h, 1e-12)
    rbf.rbf_assemble(plan, phi, "fp32", dev(h))
    e32 = check_values(rbf, plan, ne, h, 2e-6)
    say(f"max scaled error fp64 {e64:.2e} fp32 {e32:.2e}")


# Rows wider than one wave take the assembly's grouped path (columns listed
# per group of 64 spatially ordered points); two cases pass the row in more
# than one block of 256 columns.
@pytest.mark.parametrize("dim,g,rho_cells,n,seed", [
    (2, 24, 5.5, 20000, 0),   # upper rows 121 columns on average, up to 187
    (2, 24, 8.0, 12000, 1),   # 202 on average, up to 342: two column blocks
    (3, 10, 3.0, 20000, 2),   # 199 on average, up to 404
])
def test_values_grouped_path(rbf, dim, g, rho_cells, n, seed):
    rng = np.random.default_rng(60 + seed)
    ctr = sd.grid_centers(g, dim)
    rho = rho_cells / (g - 1)
    pts = np.concatenate([rng.random((dim, n // 2)),
                          sd.gaussian_mixture_points(rng, n - n // 2, dim, 4)], axis=1)
    h = np.cos(5 * pts[0]) * pts[1] + 0.1 * rng.standard_normal(n)
    say("grouped values", dim, g, rho_cells, n)
    ne = orc.normal_equations(pts, h, ctr, rho, "w31", lambda_rel=1e-5)
    plan = rbf.rbf_fit_plan(dev(pts), dev(ctr), rho=rho, lambda_rel=1e-5)
    check_pattern(rbf, plan, ne)
    info = rbf.rbf_plan_info(plan)
    upper_mean = (info["nnz_full"] + info["n_active"]) / (2 * info["n_active"])
    say("upper row mean", upper_mean)
    assert upper_mean > 64
    rbf.rbf_assemble(plan, "w31", "fp64", dev(h))
    e64 = check_values(rbf, plan, ne, h, 1e-12)
    rbf.rbf_assemble(plan, "w31", "fp32", dev(h))
    e32 = check_values(rbf, plan, ne, h, 2e-6)
    say(f"max scaled error fp64 {e64:.2e} fp32 {e32:.2e}")


def test_deterministic(rbf):
    p = sd.make_problem("terrain2d", scale=1 / 64)
    outs = []
    for _ in range(2):
        plan = rbf.rbf_fit_plan(dev(p.points), dev(p.centers), rho=p.rho, lambda_rel=1e-4)
        rbf.rbf_assemble(plan, p.phi, "fp64", dev(p.values))
        val, g, lam = rbf.rbf_system_export(plan)
        c, info = rbf.rbf_solve(plan, rtol=1e-10)
        outs.append((val.tobytes(), g.tobytes(), c.cpu().numpy().tobytes(), info["iterations"]))
        plan.close()
    assert outs[0] == outs[1]


# -------------------------------------------------------------------- solve
def test_solve_fp64_franke(rbf):
    p = sd.make_problem("franke2d")
    say("franke2d fp64 solve")
    ne = orc.normal_equations(p.points, p.values, p.centers, p.rho, p.phi)
    c_ref = orc.solve(ne)
    plan = rbf.rbf_fit_plan(dev(p.points), dev(p.centers), rho=p.rho)
    rbf.rbf_assemble(plan, p.phi, "fp64", dev(p.values))
    check_values(rbf, plan, ne, p.values, 1e-12)
    c, info = rbf.rbf_solve(plan, rtol=1e-13, max_iter=50000)
    say("info", info)
    assert info["status"] == 0 and info["rel_residual"] <= 1e-13
    c = c.cpu().numpy()
    A = ne.A
    fit = np.linalg.norm(A @ (c - c_ref)) / np.linalg.norm(A @ c_ref)
    B = ne.full_matrix().toarray()
    kappa = np.linalg.cond(B)
    coef = np.linalg.norm(c - c_ref) / np.linalg.norm(c_ref)
    say(f"fit {fit:.2e} coef {coef:.2e} kappa {kappa:.2e}")
    assert fit <= FIT_FP64
    # ||c - c*|| / ||c*|| <= kappa (||r|| / ||g||) for the GPU's residual r, plus
    # the oracle's own error (Cholesky is backward stable: a few kappa u)
    assert coef <= max(1e-10, kappa * (info["rel_residual"] + 10 * U64))
    # evaluation at the data points and at random queries (some outside the grid box)
    q = np.concatenate([p.points[:, :500], np.random.default_rng(5).random((2, 500)) * 1.6 - 0.3],
                       axis=1)
    f, _ = rbf.rbf_eval(plan, dev(q), dev(c))
    f_ref = orc.evaluate(q, p.centers, p.rho, p.phi, c)
    absum = orc.evaluate(q, p.centers, p.rho, p.phi, np.abs(c))
    assert np.all(np.abs(f.cpu().numpy() - f_ref) <= 1e-12 * absum + 1e-300)
    # RMSE reduction on the GPU
    _, rmse = rbf.rbf_eval(plan, dev(p.points), dev(c), values=dev(p.values))
    ref_rmse = orc.rmse(A @ c, p.values)
    assert abs(rmse - ref_rmse) <= 1e-12 * ref_rmse


def test_solve_mixed_matches_rmse(rbf):
    p = sd.make_problem("terrain2d", scale=1 / 64)
    say("terrain2d/64 mixed solve")
    lam = 1e-4
    ne = orc.normal_equations(p.points, p.values, p.centers, p.rho, p.phi, lambda_rel=lam)
    c_ref = orc.solve(ne)
    r_ref = orc.rmse(orc.evaluate(p.test_points, p.centers, p.rho, p.phi, c_ref), p.test_values)
    plan = rbf.rbf_fit_plan(dev(p.points), dev(p.centers), rho=p.rho, lambda_rel=lam)
    res = {}
    for prec in ("fp64", "fp32"):
        rbf.rbf_assemble(plan, p.phi, prec, dev(p.values))
        c, info = rbf.rbf_solve(plan, rtol=FP64_RTOL if prec == "fp64" else 1e-10)
        _, r = rbf.rbf_eval(plan, dev(p.test_points), c, values=dev(p.test_values))
        res[prec] = (r, info, c.cpu().numpy())
        say(prec, info, r, r_ref)
    assert abs(res["fp64"][0] - r_ref) <= 1e-6 * r_ref
    assert abs(res["fp32"][0] - r_ref) <= 1e-3 * r_ref
    assert res["fp32"][1]["status"] == 0 and res["fp32"][1]["precision"] == "fp32"
    A = ne.A
    fit = np.linalg.norm(A @ (res["fp64"][2] - c_ref)) / np.linalg.norm(A @ c_ref)
    say(f"fp64 fit {fit:.2e}")
    assert fit <= FIT_FP64


def test_profile_counts(rbf):
    # Timing on: the assembly launch and one CG iteration launch in 128 are
    # stamped; launches queued past convergence are not counted.
    p = sd.make_problem("terrain2d", scale=1 / 64)
    plan = rbf.rbf_fit_plan(dev(p.points), dev(p.centers), rho=p.rho, lambda_rel=1e-4)
    for prec in ("fp32", "fp64"):
        rbf.rbf_profile(plan, True)
        rbf.rbf_assemble(plan, p.phi, prec, dev(p.values))
        c, info = rbf.rbf_solve(plan, rtol=1e-10)
        n_cg, ms_cg = rbf.rbf_profile_read(plan, "cg_iter")
        n_asm, ms_asm = rbf.rbf_profile_read(plan, "assemble")
        rbf.rbf_profile(plan, False)
        it = info["iterations"]
        say(prec, "iterations", it, "timed", n_cg, "avg us", 1e3 * ms_cg / max(n_cg, 1))
        assert info["status"] == 0
        assert n_asm == 1 and ms_asm > 0.0
        assert abs(n_cg - it / 128) <= 2 + info["reliable_updates"]
        assert 1e-4 < ms_cg / n_cg < 1.0


def test_warm_start_and_maxiter(rbf):
    p = sd.make_problem("franke2d", scale=0.25)
    plan = rbf.rbf_fit_plan(dev(p.points), dev(p.centers), rho=p.rho)
    rbf.rbf_assemble(plan, p.phi, "fp64", dev(p.values))
    c, info = rbf.rbf_solve(plan, rtol=1e-12, max_iter=5)
    assert info["status"] == 1 and info["iterations"] == 5
    c2, info2 = rbf.rbf_solve(plan, coeffs=c.clone(), warm_start=True, rtol=1e-12)
    assert info2["status"] == 0 and info2["rel_residual"] <= 1e-12
    c3, info3 = rbf.rbf_solve(plan, coeffs=c2.clone(), warm_start=True, rtol=1e-12)
    assert info3["iterations"] <= 1


# --------------------------------------------------------------- edge cases
def test_single_centre_and_empty_supports(rbf):
    rng = np.random.default_rng(3)
    pts = rng.random((2, 400)) * 0.5                    # lower-left quarter only
    ctr = sd.grid_centers(6, 2)
    h = pts[0] + 1.0
    ne = orc.normal_equations(pts, h, ctr, 0.15, "w31")
    assert np.any(~ne.active)
    plan = rbf.rbf_fit_plan(dev(pts), dev(ctr), rho=0.15)
    check_pattern(rbf, plan, ne)
    rbf.rbf_assemble(plan, "w31", "fp64", dev(h))
    c, info = rbf.rbf_solve(plan, rtol=FP64_RTOL)
    c = c.cpu().numpy()
    assert np.all(c[~ne.active] == 0.0)
    c_ref = orc.solve(ne)
    fit = np.linalg.norm(ne.A @ (c - c_ref)) / np.linalg.norm(ne.A @ c_ref)
    say(f"fit {fit:.2e}")
    assert fit <= FIT_FP64
    one = np.array([[0.5], [0.5]])
    plan1 = rbf.rbf_fit_plan(dev(pts), dev(one), rho=0.2)
    ne1 = orc.normal_equations(pts, h, one, 0.2, "w31")
    check_pattern(rbf, plan1, ne1)
    rbf.rbf_assemble(plan1, "w31", "fp64", dev(h))
    c1, _ = rbf.rbf_solve(plan1, rtol=1e-14)
    assert abs(c1.item() - orc.solve(ne1)[0]) <= 1e-12 * abs(orc.solve(ne1)[0])


def test_no_point_in_any_support(rbf):
    pts = np.array([[5.0, 6.0], [5.0, 6.0]])
    ctr = sd.grid_centers(4, 2)
    plan = rbf.rbf_fit_plan(dev(pts), dev(ctr), rho=0.2)
    info = rbf.rbf_plan_info(plan)
    assert info["nnz_upper"] == 0 and info["n_active"] == 0
    rbf.rbf_assemble(plan, "w31", "fp64", dev(np.array([1.0, 2.0])))
    c, inf = rbf.rbf_solve(plan)
    assert inf["status"] == 0 and np.all(c.cpu().numpy() == 0.0)


def test_invalid_inputs_raise(rbf):
    from paper_1806_07884_amd._lib import RbfError
    ctr = dev(sd.grid_centers(4, 2))
    bad = dev(np.array([[0.1, np.nan], [0.2, 0.3]]))
    with pytest.raises(RbfError, match="non-finite"):
        rbf.rbf_fit_plan(bad, ctr, rho=0.2)
    with pytest.raises(RbfError):
        rbf.rbf_fit_plan(dev(np.random.rand(2, 10)), ctr, rho=0.2, min_support=0)
    plan = rbf.rbf_fit_plan(dev(np.random.rand(2, 10)), ctr, rho=0.2)
    with pytest.raises(RbfError, match="assemble"):
        rbf.rbf_solve(plan)


@pytest.mark.parametrize("name,scale", [("terrain2d", 1 / 64), ("franke2d", 1.0), ("terrain2d", 1 / 4),
                                        ("field3d", 1 / 512)])
def test_staged_iteration_is_bit_identical(rbf, name, scale):
    # the float64 CG iteration staging each slice's neighbourhood in LDS
    # computes the same numbers as the one gathering from global memory
    p = sd.make_problem(name, scale=scale)
    lam = 0.0 if name == "franke2d" else 1e-4
    res = {}
    for staging in (True, False):
        plan = rbf.rbf_fit_plan(dev(p.points), dev(p.centers), rho=p.rho, lambda_rel=lam,
                                staging=staging)
        rbf.rbf_assemble(plan, p.phi, "fp64", dev(p.values))
        c, info = rbf.rbf_solve(plan, rtol=1e-10)
        staged = rbf.rbf_plan_info(plan)["solver_staged"]
        say(name, scale, "staging", staging, "staged columns per slice <=", staged)
        assert (staged > 0) == staging
        res[staging] = (c.cpu().numpy().tobytes(), info["iterations"])
        plan.close()
    assert res[True] == res[False]


def _unsorted_padding(ne, lanes):
    """Stored entries over nonzeros of the solver layout with the rows in
    centre order (slices of 64 / lanes rows padded to their longest row)."""
    fl = np.diff(ne.full_matrix().tocsr().indptr)[ne.active]
    s = 64 // lanes
    tot = sum(int(np.ceil(fl[k:k + s].max() / lanes) * lanes) * s for k in range(0, len(fl), s))
    return tot / fl.sum()


@pytest.mark.parametrize("n_uniform,rvar,sorted_rows", [(1000, 0.8, 1), (3000, 0.0, 0)])
def test_sorted_solver_rows(rbf, n_uniform, rvar, sorted_rows):
    # clustered 3D points with (optionally) per-centre radii: row lengths vary
    # enough for the layout to pad by more than 1.3x, and the plan reorders
    # the rows within windows of 64; values, solve and evaluation stay the
    # oracle's, with the rows in either order
    rng = np.random.default_rng(910)
    g = 14
    ctr = sd.grid_centers(g, 3)
    pts = np.concatenate([rng.random((3, n_uniform)),
                          sd.gaussian_mixture_points(rng, 12000, 3, 3)], axis=1)
    h = np.sin(3 * pts[0]) + pts[1] * pts[2]
    m = ctr.shape[1]
    rho = 1.9 / (g - 1) * (1 + rvar * (rng.random(m) - 0.5)) if rvar else 1.9 / (g - 1)
    say("sorted rows", n_uniform, rvar)
    ne = orc.normal_equations(pts, h, ctr, rho, "w31", lambda_rel=1e-4)
    kw = {"rho_per_center": dev(rho)} if rvar else {"rho": rho}
    plan = rbf.rbf_fit_plan(dev(pts), dev(ctr), lambda_rel=1e-4, **kw)
    check_pattern(rbf, plan, ne)
    info = rbf.rbf_plan_info(plan)
    pad = _unsorted_padding(ne, info["solver_lanes"])
    say("padding in centre order", round(pad, 3), "sorted", info["solver_rows_sorted"],
        "stored", info["solver_entries"])
    assert (pad > 1.3) == bool(sorted_rows)
    assert info["solver_rows_sorted"] == sorted_rows
    if sorted_rows:
        assert info["solver_entries"] < pad * info["nnz_full"]
    rbf.rbf_assemble(plan, "w31", "fp64", dev(h))
    check_values(rbf, plan, ne, h, 1e-12)
    c_ref = orc.solve(ne)
    c, sinfo = rbf.rbf_solve(plan, rtol=1e-13, max_iter=50000)
    assert sinfo["status"] == 0
    c = c.cpu().numpy()
    A = ne.A
    assert np.linalg.norm(A @ (c - c_ref)) <= FIT_FP64 * np.linalg.norm(A @ c_ref)
    q = rng.random((3, 2000))
    f, _ = rbf.rbf_eval(plan, dev(q), dev(c))
    f_ref = orc.evaluate(q, ctr, rho, "w31", c)
    absum = orc.evaluate(q, ctr, rho, "w31", np.abs(c))
    assert np.all(np.abs(f.cpu().numpy() - f_ref) <= 1e-12 * absum + 1e-300)
    # the mixed solve on the same plan
    rbf.rbf_assemble(plan, "w31", "fp32", dev(h))
    c32, i32 = rbf.rbf_solve(plan, rtol=1e-10)
    assert i32["status"] in (0, 2)
    r32 = np.linalg.norm(A @ c32.cpu().numpy() - h) / np.sqrt(len(h))
    r64 = np.linalg.norm(A @ c - h) / np.sqrt(len(h))
    assert abs(r32 - r64) <= 1e-3 * r64
    plan.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_chunking_does_not_change_iterates(rbf, prec):
    # the host only decides how many launches it queues between checks (and
    # stops queueing at a flag the iteration raises); which iteration raises
    # a flag, and every iterate, are the device's: any chunk length gives the
    # same bits, the same iteration count and the same reliable updates
    p = sd.make_problem("terrain2d", scale=1 / 64)
    plan = rbf.rbf_fit_plan(dev(p.points), dev(p.centers), rho=p.rho, lambda_rel=1e-5)
    rbf.rbf_assemble(plan, p.phi, prec, dev(p.values))
    out = []
    for ce in (1, 5, 32, 200):
        c, info = rbf.rbf_solve(plan, rtol=1e-10, check_every=ce)
        say(prec, "check_every", ce, "iterations", info["iterations"], "updates",
            info["reliable_updates"])
        out.append((c.cpu().numpy().tobytes(), info["iterations"], info["reliable_updates"]))
    assert all(o == out[0] for o in out)
    plan.close()
