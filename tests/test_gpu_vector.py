"""Vector-valued data (Section 2: values h_i in E^p) through rbf_set_values and
rbf_solve_batch.

A and B depend on the points and reference points only, so the components of
vector-valued data share them: the library assembles once and replaces g = A^T h
(and P^T h) per component.

Bars: g after rbf_set_values is bit for bit g of a fresh rbf_assemble with the
same values (both assembly paths, float64 and float32), the coefficients of a
component then equal those of a fresh fit bit for bit (the solver is
deterministic), and each component's fit matches the oracle's Cholesky fit of
that component (fitted values within 1e-10, as in test_gpu_parity).  The
batched solve (all components in one CG kernel per iteration) meets the same
oracle bar in float64, and in the mixed path its held-out values agree with
the sequential solves' to 1e-5 of their size (both stop at the same float64
residual; their float32 arithmetic differs in summation order and in when
the reliable updates fall).
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


def components(p):
    return [sd.franke(p), np.sin(4 * p[0]) * np.cos(3 * p[1]), 2.0 * p[0] - p[1] + 0.5]


@pytest.mark.parametrize("k_cover,prec", [(10.0, "fp64"), (10.0, "fp32"), (40.0, "fp64"),
                                          (40.0, "fp32")])
def test_set_values_equals_assembly(rbf, k_cover, prec):
    rng = np.random.default_rng(12)
    p = rng.random((2, 20000))
    g_side = 40
    ctr = sd.grid_centers(g_side, 2)
    rho = sd.support_radius_for_k(g_side, 2, k_cover)
    h1, h2, _ = components(p)
    plan = rbf.rbf_fit_plan(dev(p), dev(ctr), rho=rho, lambda_rel=1e-6)
    info = rbf.rbf_plan_info(plan)
    upper_mean = (info["nnz_full"] + info["n_active"]) / (2 * info["n_active"])
    say("set_values", k_cover, prec, "upper row mean", upper_mean)
    assert (upper_mean > 64) == (k_cover > 20)      # both assembly paths are covered
    rbf.rbf_assemble(plan, "w31", prec, dev(h1))
    rbf.rbf_set_values(plan, dev(h2))
    val_a, g_a, lam_a = rbf.rbf_system_export(plan)
    c_a, _ = rbf.rbf_solve(plan, rtol=1e-10)
    rbf.rbf_assemble(plan, "w31", prec, dev(h2))
    val_b, g_b, lam_b = rbf.rbf_system_export(plan)
    c_b, _ = rbf.rbf_solve(plan, rtol=1e-10)
    assert np.array_equal(g_a, g_b) and np.array_equal(val_a, val_b) and lam_a == lam_b
    assert torch.equal(c_a, c_b)
    plan.close()


@pytest.mark.parametrize("poly", [False, True])
def test_vector_valued_fit(rbf, poly):
    prob = sd.make_problem("franke2d", scale=0.5)
    p, ctr, rho = prob.points, prob.centers, prob.rho
    H = components(p)
    say("vector-valued", len(H), "components", "poly" if poly else "")
    plan = rbf.rbf_fit_plan(dev(p), dev(ctr), rho=rho, polynomial=poly)
    rbf.rbf_assemble(plan, "w31", "fp64", dev(H[0]))
    m = ctr.shape[1]
    for i, h in enumerate(H):
        if i > 0:
            rbf.rbf_set_values(plan, dev(h))
        ck, info = rbf.rbf_solve(plan, rtol=1e-13, max_iter=50000)
        assert info["status"] == 0
        ck = ck.cpu().numpy()
        ne = orc.normal_equations(p, h, ctr, rho, "w31")
        if poly:
            ps = orc.poly_system(ne, p, h)
            q, cmat, e = rbf.rbf_poly_export(plan)
            P1 = np.abs(orc.poly_basis(p)) + 1.0
            assert np.all(np.abs(e - ps.e) <= 1e-12 * (P1.T @ np.abs(h)))
            c_ref, k_ref = orc.solve_poly(ne, ps)
            P = orc.poly_basis(p)
            ref = ne.A @ c_ref + P @ k_ref
            fit = np.linalg.norm(ne.A @ ck[:m] + P @ ck[m:] - ref) / np.linalg.norm(ref)
        else:
            c_ref = orc.solve(ne)
            ref = ne.A @ c_ref
            fit = np.linalg.norm(ne.A @ ck - ref) / np.linalg.norm(ref)
        say(f"component {i}: fit {fit:.2e}, iterations {info['iterations']}")
        assert fit <= FIT_FP64
    plan.close()


def test_set_values_needs_assembly(rbf):
    from paper_1806_07884_amd._lib import RbfError
    plan = rbf.rbf_fit_plan(dev(np.random.rand(2, 50)), dev(sd.grid_centers(4, 2)), rho=0.3)
    with pytest.raises(RbfError, match="assemble"):
        rbf.rbf_set_values(plan, dev(np.random.rand(50)))


# ------------------------------------------------------------- batched solve
@pytest.mark.parametrize("nr", [2, 3, 4])
def test_batch_fp64_matches_oracle(rbf, nr):
    prob = sd.make_problem("franke2d", scale=0.5)
    p, ctr, rho = prob.points, prob.centers, prob.rho
    H = components(p) + [np.cos(5 * p[0] + 2 * p[1])]
    H = H[:nr]
    say("batched fp64", nr)
    plan = rbf.rbf_fit_plan(dev(p), dev(ctr), rho=rho)
    rbf.rbf_assemble(plan, "w31", "fp64", dev(H[0]))
    C, infos = rbf.rbf_solve_batch(plan, dev(np.stack(H)), rtol=1e-13, max_iter=50000)
    C = C.cpu().numpy()
    for k, h in enumerate(H):
        say(k, infos[k])
        assert infos[k]["status"] == 0 and infos[k]["rel_residual"] <= 1e-13
        ne = orc.normal_equations(p, h, ctr, rho, "w31")
        c_ref = orc.solve(ne)
        fit = np.linalg.norm(ne.A @ (C[k] - c_ref)) / np.linalg.norm(ne.A @ c_ref)
        say(k, "fit", fit)
        assert fit <= FIT_FP64, (k, fit)
    # the plan is left holding the last component's values
    _, g, _ = rbf.rbf_system_export(plan)
    rbf.rbf_set_values(plan, dev(H[-1]))
    _, g2, _ = rbf.rbf_system_export(plan)
    assert np.array_equal(g, g2)
    plan.close()


@pytest.mark.parametrize("nr", [2, 4])
def test_batch_mixed_matches_sequential(rbf, nr):
    prob = sd.make_problem("terrain2d", scale=1 / 64)
    p, ctr, rho = prob.points, prob.centers, prob.rho
    rng = np.random.default_rng(9)
    H = [prob.values] + [sd.terrain_values(sd.terrain_modes(rng, 64, 2), p) for _ in range(nr - 1)]
    Q = [prob.test_values] + [None] * (nr - 1)
    plan = rbf.rbf_fit_plan(dev(p), dev(ctr), rho=rho, lambda_rel=1e-4)
    rbf.rbf_assemble(plan, prob.phi, "fp32", dev(H[0]))
    C, infos = rbf.rbf_solve_batch(plan, dev(np.stack(H)), rtol=1e-10)
    say("batched mixed", nr, [i["iterations"] for i in infos])
    for k, h in enumerate(H):
        assert infos[k]["status"] == 0 and infos[k]["precision"] == "fp32"
        rbf.rbf_set_values(plan, dev(h))
        c1, i1 = rbf.rbf_solve(plan, rtol=1e-10)
        f_b, _ = rbf.rbf_eval(plan, dev(prob.test_points), C[k].contiguous())
        f_1, _ = rbf.rbf_eval(plan, dev(prob.test_points), c1)
        ref = orc.rmse(f_1.cpu().numpy(), 0.0)
        d = orc.rmse(f_b.cpu().numpy(), f_1.cpu().numpy())
        say(k, "batch vs sequential held-out values", d, "scale", ref, i1["iterations"])
        assert d <= 1e-5 * ref
    plan.close()


def test_batch_warm_start_and_errors(rbf):
    from paper_1806_07884_amd._lib import RbfError
    prob = sd.make_problem("franke2d", scale=0.25)
    p, ctr, rho = prob.points, prob.centers, prob.rho
    H = np.stack(components(p)[:2])
    plan = rbf.rbf_fit_plan(dev(p), dev(ctr), rho=rho)
    with pytest.raises(RbfError, match="assemble"):
        rbf.rbf_solve_batch(plan, dev(H))
    rbf.rbf_assemble(plan, "w31", "fp64", dev(H[0]))
    C, infos = rbf.rbf_solve_batch(plan, dev(H), rtol=1e-12, max_iter=5)
    assert all(i["status"] == 1 for i in infos)
    C2, infos2 = rbf.rbf_solve_batch(plan, dev(H), coeffs=C.clone(), warm_start=True, rtol=1e-12)
    assert all(i["status"] == 0 and i["rel_residual"] <= 1e-12 for i in infos2)
    with pytest.raises(RbfError, match="nrhs"):
        rbf.rbf_solve_batch(plan, dev(np.stack([H[0]] * 5)))
    pplan = rbf.rbf_fit_plan(dev(p), dev(ctr), rho=rho, polynomial=True)
    rbf.rbf_assemble(pplan, "w31", "fp64", dev(H[0]))
    with pytest.raises(RbfError, match="polynomial"):
        rbf.rbf_solve_batch(pplan, dev(H))
    # no active centre: zeros
    far = 5.0 + np.random.default_rng(1).random((2, 100))
    zplan = rbf.rbf_fit_plan(dev(far), dev(ctr), rho=rho)
    rbf.rbf_assemble(zplan, "w31", "fp64", dev(far[0]))
    Z, zi = rbf.rbf_solve_batch(zplan, dev(np.stack([far[0], far[1]])))
    assert torch.count_nonzero(Z).item() == 0 and zi[0]["status"] == 0


@pytest.mark.parametrize("prec,nr", [("fp32", 2), ("fp32", 4), ("fp64", 2)])
def test_batch_staged_is_bit_identical(rbf, prec, nr):
    # the batched iteration staging the slices' neighbourhoods in LDS computes
    # the same numbers as the one gathering every record from global memory
    prob = sd.make_problem("terrain2d", scale=1 / 64)
    rng = np.random.default_rng(2)
    H = np.stack([prob.values] + [sd.terrain_values(sd.terrain_modes(rng, 64, 2), prob.points)
                                  for _ in range(nr - 1)])
    out = {}
    for staging in (True, False):
        plan = rbf.rbf_fit_plan(dev(prob.points), dev(prob.centers), rho=prob.rho,
                                lambda_rel=1e-4, staging=staging)
        rbf.rbf_assemble(plan, prob.phi, prec, dev(H[0]))
        C, infos = rbf.rbf_solve_batch(plan, dev(H), rtol=1e-10)
        staged = rbf.rbf_plan_info(plan)["solver_staged"]
        say("batch", prec, nr, "staging", staging, "staged", staged,
            [i["iterations"] for i in infos])
        assert (staged > 0) == staging
        out[staging] = (C.cpu().numpy().tobytes(), [i["iterations"] for i in infos])
        plan.close()
    assert out[True] == out[False]


def test_batch_3d(rbf):
    prob = sd.make_problem("field3d", scale=1 / 512)
    p, ctr, rho = prob.points, prob.centers, prob.rho
    H = [prob.values, np.sin(3 * p[0]) * np.cos(2 * p[2]) + p[1]]
    plan = rbf.rbf_fit_plan(dev(p), dev(ctr), rho=rho, lambda_rel=1e-5)
    rbf.rbf_assemble(plan, prob.phi, "fp64", dev(H[0]))
    C, infos = rbf.rbf_solve_batch(plan, dev(np.stack(H)), rtol=FP64_RTOL, max_iter=50000)
    say("batched 3D", rbf.rbf_plan_info(plan)["solver_staged"], [i["iterations"] for i in infos])
    C = C.cpu().numpy()
    for k, h in enumerate(H):
        assert infos[k]["status"] == 0
        ne = orc.normal_equations(p, h, ctr, rho, prob.phi, lambda_rel=1e-5)
        c_ref = orc.solve(ne)
        fit = np.linalg.norm(ne.A @ (C[k] - c_ref)) / np.linalg.norm(ne.A @ c_ref)
        say(k, "fit", fit)
        assert fit <= FIT_FP64
    plan.close()
