"""Linear polynomial reproduction (Section 3, eq. 6-10) on the HIP path, through
the C-ABI, against the FP64 CPU oracle.

Bars
----
* blocks of eq. 10 in the paper's basis P_i = (x_i^T, 1):
  |Q - Q*| <= 1e-12 |A|^T (|P| + 1), |C - C*| <= 1e-12 (|P| + 1)^T (|P| + 1),
  |e - e*| <= 1e-12 (|P| + 1)^T |h| (the library sums in a scaled basis and
  converts, which costs a few roundings of those magnitudes);
* FP64 solve (to relative residual 1e-13): fitted values
  ||A (c - c*) + P (k - k*)|| / ||A c* + P k*|| <= 1e-10;
* mixed solve: held-out RMSE within 0.1 % of the FP64 oracle's;
* evaluation: |f - f*| <= 1e-12 (sum_j |c_j phi_j| + |a^T y| + |a_0|);
* exact linear data: the fitted surface within 1e-10 max |h| of the plane
  (FP64; 1e-5 mixed), k = (a, a_0) to 1e-9 and |c| <= 1e-6 (FP64).
"""
import sys

import numpy as np
import pytest
import torch

import synthdata as sd
from oracle import rbf_oracle as orc
from tolerances import FIT_FP64, FP64_RTOL

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


def check_blocks(rbf, plan, ne, pts, h):
    ps = orc.poly_system(ne, pts, h)
    q, c, e = rbf.rbf_poly_export(plan)
    P1 = np.abs(orc.poly_basis(pts)) + 1.0
    qs = np.abs(ne.A).T @ P1
    assert np.all(np.abs(q - ps.Q) <= 1e-12 * qs + 1e-300), float(np.max(np.abs(q - ps.Q) / qs))
    assert np.all(np.abs(c - ps.C) <= 1e-12 * (P1.T @ P1))
    assert np.all(np.abs(e - ps.e) <= 1e-12 * (P1.T @ np.abs(h)))
    return ps


def fitted_error(ne, pts, c, k, c_ref, k_ref):
    P = orc.poly_basis(pts)
    ref = ne.A @ c_ref + P @ k_ref
    return np.linalg.norm(ne.A @ (c - c_ref) + P @ (k - k_ref)) / np.linalg.norm(ref)


@pytest.mark.parametrize("name,scale,shift,lam", [
    ("franke2d", 1.0, 0.0, 0.0),
    ("franke2d", 0.25, 250.0, 1e-6),     # coordinates far from the origin
    ("field3d", 1 / 512, 0.0, 1e-5),
])
def test_poly_fp64_parity(rbf, name, scale, shift, lam):
    p = sd.make_problem(name, scale=scale)
    pts, ctr = p.points + shift, p.centers + shift
    say("poly fp64", name, scale, shift, lam, pts.shape, ctr.shape)
    ne = orc.normal_equations(pts, p.values, ctr, p.rho, p.phi, lambda_rel=lam)
    plan = rbf.rbf_fit_plan(dev(pts), dev(ctr), rho=p.rho, lambda_rel=lam, polynomial=True)
    assert rbf.rbf_plan_info(plan)["n_poly"] == p.dim + 1
    rbf.rbf_assemble(plan, p.phi, "fp64", dev(p.values))
    ps = check_blocks(rbf, plan, ne, pts, p.values)
    if shift == 0.0:
        c_ref, k_ref = orc.solve_poly(ne, ps)
    else:
        # far from the origin P^T P dwarfs A^T A (the paper's caveat after eq. 10)
        # and the raw-basis normal equations lose digits: QR of eq. 9 instead
        c_ref, k_ref = orc.lstsq_dense_poly(pts, p.values, ctr, p.rho, p.phi, lam=ne.lam)
    ck, info = rbf.rbf_solve(plan, rtol=1e-13, max_iter=100000)
    say("info", info)
    assert info["status"] == 0 and info["rel_residual"] <= 1e-13
    ck = ck.cpu().numpy()
    c, k = ck[:ne.m], ck[ne.m:]
    assert np.all(c[~ne.active] == 0.0)
    fit = fitted_error(ne, pts, c, k, c_ref, k_ref)
    say(f"fit {fit:.2e} k {k} k* {k_ref}")
    assert fit <= FIT_FP64
    # evaluation: data points and random queries, some outside every support
    rng = np.random.default_rng(8)
    q = np.concatenate([pts[:, :400], shift + rng.random((p.dim, 400)) * 1.6 - 0.3], axis=1)
    f, _ = rbf.rbf_eval(plan, dev(q), dev(ck))
    f_ref = orc.evaluate_poly(q, ctr, p.rho, p.phi, c, k)
    absum = (orc.evaluate(q, ctr, p.rho, p.phi, np.abs(c)) + np.abs(k[:-1]) @ np.abs(q)
             + abs(k[-1]))
    assert np.all(np.abs(f.cpu().numpy() - f_ref) <= 1e-12 * absum)
    plan.close()


def test_poly_mixed_matches_rmse(rbf):
    p = sd.make_problem("terrain2d", scale=1 / 64)
    lam = 1e-4
    say("poly mixed terrain2d/64")
    ne = orc.normal_equations(p.points, p.values, p.centers, p.rho, p.phi, lambda_rel=lam)
    c_ref, k_ref = orc.solve_poly(ne, orc.poly_system(ne, p.points, p.values))
    r_ref = orc.rmse(orc.evaluate_poly(p.test_points, p.centers, p.rho, p.phi, c_ref, k_ref),
                     p.test_values)
    plan = rbf.rbf_fit_plan(dev(p.points), dev(p.centers), rho=p.rho, lambda_rel=lam,
                            polynomial=True)
    res = {}
    for prec in ("fp64", "fp32"):
        rbf.rbf_assemble(plan, p.phi, prec, dev(p.values))
        ck, info = rbf.rbf_solve(plan, rtol=FP64_RTOL if prec == "fp64" else 1e-10)
        _, r = rbf.rbf_eval(plan, dev(p.test_points), ck, values=dev(p.test_values))
        res[prec] = (r, info, ck.cpu().numpy())
        say(prec, info, r, r_ref)
    assert abs(res["fp64"][0] - r_ref) <= 1e-6 * r_ref
    assert abs(res["fp32"][0] - r_ref) <= 1e-3 * r_ref
    assert res["fp32"][1]["status"] == 0 and res["fp32"][1]["precision"] == "fp32"
    ck = res["fp64"][2]
    fit = fitted_error(ne, p.points, ck[:ne.m], ck[ne.m:], c_ref, k_ref)
    say(f"fp64 fit {fit:.2e}")
    assert fit <= FIT_FP64
    plan.close()


@pytest.mark.parametrize("dim,prec", [(2, "fp64"), (2, "fp32"), (3, "fp64")])
def test_linear_data_reproduced(rbf, dim, prec):
    rng = np.random.default_rng(31 + dim)
    n = 6000 if dim == 2 else 9000
    pts = rng.random((dim, n))
    ctr = sd.grid_centers(20 if dim == 2 else 7, dim)
    rho = sd.support_radius_for_k(20 if dim == 2 else 7, dim, 30.0)
    a = np.array([1.75, -0.625, 2.5][:dim])
    a0 = -3.25
    h = a @ pts + a0
    say("linear data", dim, prec)
    plan = rbf.rbf_fit_plan(dev(pts), dev(ctr), rho=rho, lambda_rel=1e-4, polynomial=True)
    rbf.rbf_assemble(plan, "w31", prec, dev(h))
    ck, info = rbf.rbf_solve(plan, rtol=FP64_RTOL if prec == "fp64" else 1e-12)
    m = ctr.shape[1]
    say("info", info, "k", ck[m:].cpu().numpy())
    # the fitted surface at fresh points is the plane (float32 accuracy for the
    # mixed path: float32 basis values and samples)
    q = rng.random((dim, 2000))
    f, _ = rbf.rbf_eval(plan, dev(q), ck)
    err = np.max(np.abs(f.cpu().numpy() - (a @ q + a0)))
    say(prec, "plane error", err)
    assert err <= (FIT_FP64 if prec == "fp64" else 1e-5) * np.max(np.abs(h))
    if prec == "fp64":
        # k itself; c is 0 up to the solver's residual (rtol times the
        # conditioning of the bordered system)
        ck = ck.cpu().numpy()
        np.testing.assert_allclose(ck[m:], np.concatenate([a, [a0]]), rtol=0, atol=1e-9)
        assert np.max(np.abs(ck[:m])) <= 1e-6
    plan.close()


def test_warm_start_and_determinism(rbf):
    p = sd.make_problem("franke2d", scale=0.25)
    plan = rbf.rbf_fit_plan(dev(p.points), dev(p.centers), rho=p.rho, polynomial=True)
    rbf.rbf_assemble(plan, p.phi, "fp64", dev(p.values))
    ck, info = rbf.rbf_solve(plan, rtol=1e-12, max_iter=5)
    assert info["status"] == 1 and info["iterations"] == 5
    ck2, info2 = rbf.rbf_solve(plan, coeffs=ck.clone(), warm_start=True, rtol=1e-12)
    assert info2["status"] == 0 and info2["rel_residual"] <= 1e-12
    ck3, info3 = rbf.rbf_solve(plan, coeffs=ck2.clone(), warm_start=True, rtol=1e-12)
    assert info3["iterations"] <= 1
    a, _ = rbf.rbf_solve(plan, rtol=1e-12)
    b, _ = rbf.rbf_solve(plan, rtol=1e-12)
    assert torch.equal(a, b)
    plan.close()


def test_no_active_centre_fits_plane(rbf):
    rng = np.random.default_rng(4)
    pts = 5.0 + rng.random((2, 300))              # far from every centre
    h = 2.0 * pts[0] - 0.5 * pts[1] + 1.0 + 0.01 * rng.standard_normal(300)
    ctr = sd.grid_centers(4, 2)
    plan = rbf.rbf_fit_plan(dev(pts), dev(ctr), rho=0.2, polynomial=True)
    assert rbf.rbf_plan_info(plan)["n_active"] == 0
    rbf.rbf_assemble(plan, "w31", "fp64", dev(h))
    ck, info = rbf.rbf_solve(plan)
    ck = ck.cpu().numpy()
    k_ref = np.linalg.lstsq(orc.poly_basis(pts), h, rcond=None)[0]
    assert info["status"] == 0 and np.all(ck[:16] == 0.0)
    np.testing.assert_allclose(ck[16:], k_ref, rtol=1e-9, atol=1e-10)


def test_poly_errors(rbf):
    from paper_1806_07884_amd._lib import RbfError
    ctr = dev(sd.grid_centers(4, 2))
    plan = rbf.rbf_fit_plan(dev(np.random.rand(2, 50)), ctr, rho=0.3)
    rbf.rbf_assemble(plan, "w31", "fp64", dev(np.random.rand(50)))
    with pytest.raises(RbfError, match="polynomial"):
        rbf.rbf_poly_export(plan)
    # every point on one line: P^T P is singular
    t = np.random.rand(50)
    line = np.stack([t, 0.5 * t + 0.1])
    plan2 = rbf.rbf_fit_plan(dev(line), ctr, rho=0.3, polynomial=True)
    rbf.rbf_assemble(plan2, "w31", "fp64", dev(t))
    with pytest.raises(RbfError, match="singular"):
        rbf.rbf_solve(plan2)
