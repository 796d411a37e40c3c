"""Linear polynomial reproduction at the full size of the terrain workload
(N = 2^20 clustered points, 256 x 256 centres, the configuration bench.py
times with --polynomial), on outputs the oracle recomputes one by one:

* P^T P and P^T h over all points (paper's basis P_i = (x_i^T, 1)):
  1e-12 of (|P| + 1)^T (|P| + 1) and (|P| + 1)^T |h|;
* sampled rows of A^T P (float64 assembly): 1e-12 of |A|^T (|P| + 1);
* the solution (float64 and mixed): the bordered normal equations of eq. 10
  with the oracle's blocks and the GPU coefficients, at sampled rows of B and
  at the d + 1 polynomial rows, stay below the requested relative residual
  times ||(g*, e*)|| (plus, for the mixed path, the float32 assembly bounds of
  test_gpu_fullsize);
* evaluation at held-out points equals the oracle's evaluation of the same
  coefficients; mixed and float64 held-out RMSE agree to 0.1 %.
"""
import sys

import numpy as np
import pytest
import torch

import synthdata as sd
from oracle import rbf_oracle as orc

pytestmark = pytest.mark.gpu
LAM = 1e-4
RTOL = 1e-10


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def prob():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return sd.make_problem("terrain2d")


@pytest.fixture(scope="module")
def rbf():
    import paper_1806_07884_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.fixture(scope="module")
def ref(prob):
    say("oracle blocks at full size")
    A = orc.design_matrix(prob.points, prob.centers, prob.rho, prob.phi)
    P = orc.poly_basis(prob.points)
    P1 = np.abs(P) + 1.0
    return dict(A=A, P=P, P1=P1, Q=np.asarray(A.T @ P), C=P.T @ P, e=P.T @ prob.values,
                g=A.T @ prob.values, Qs=np.asarray(abs(A).T @ P1))


@pytest.fixture(scope="module")
def plan(prob, rbf):
    say("terrain2d full plan with polynomial")
    p = rbf.rbf_fit_plan(dev(prob.points), dev(prob.centers), rho=prob.rho, lambda_rel=LAM,
                         polynomial=True)
    yield p
    p.close()


RES = {}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_poly_fullsize(prob, rbf, plan, ref, prec):
    rbf.rbf_assemble(plan, prob.phi, prec, dev(prob.values))
    q, cmat, e = rbf.rbf_poly_export(plan)
    P1, h = ref["P1"], prob.values
    assert np.all(np.abs(cmat - ref["C"]) <= 1e-12 * (P1.T @ P1))
    assert np.all(np.abs(e - ref["e"]) <= 1e-12 * (P1.T @ np.abs(h)))
    rng = np.random.default_rng(3)
    m = prob.centers.shape[1]
    rows = sorted(set([0, m // 2, m - 1] + list(rng.integers(0, m, size=12))))
    if prec == "fp64":
        for j in rows:
            assert np.all(np.abs(q[j] - ref["Q"][j]) <= 1e-12 * ref["Qs"][j] + 1e-300), j
    rp, col, _ = rbf.rbf_plan_pattern(plan)
    val, g, lam = rbf.rbf_system_export(plan)
    ck, info = rbf.rbf_solve(plan, rtol=RTOL, max_iter=200000)
    say(prec, "solve", info)
    assert info["status"] == 0 and info["precision"] == prec
    ck = ck.cpu().numpy()
    c, k = ck[:m], ck[m:]
    A = ref["A"]
    diag_ref = np.asarray(A.multiply(A).sum(axis=0)).ravel()
    lam_ref = LAM * diag_ref[diag_ref > 0].mean()
    norm = np.linalg.norm(np.concatenate([ref["g"], ref["e"]]))
    a_tol, n_tol = (0.0, 0.0) if prec == "fp64" else (1e-5, 3e-6)
    for j in rows:
        row = orc.sample_row(prob.points, prob.values, prob.centers, prob.rho, prob.phi, j,
                             lower=True)
        if row.support.size == 0:
            assert c[j] == 0.0
            continue
        r = row.g - np.dot(row.vals, c[row.cols]) - lam_ref * c[j] - ref["Q"][j] @ k
        gscale = np.sum(np.abs(A[:, j].toarray().ravel() * h))
        hsum = np.sum(np.abs(h[row.support]))
        bound = RTOL * norm * 1.01
        if prec == "fp32":
            # float32 values of B, g and Q (phi rounded to float32 in all three)
            bound += (a_tol * np.dot(np.abs(row.vals), np.abs(c[row.cols]))
                      + n_tol * np.dot(row.pair_count, np.abs(c[row.cols]))
                      + a_tol * gscale + n_tol * hsum
                      + (a_tol + n_tol) * (ref["Qs"][j] @ np.abs(k)))
        assert abs(r) <= bound, (j, r, bound)
    # the d + 1 polynomial rows of eq. 10
    rpoly = ref["e"] - ref["Q"].T @ c - ref["C"] @ k
    bound = RTOL * norm * 1.01
    if prec == "fp32":
        bound += (a_tol + n_tol) * (ref["Qs"].T @ np.abs(c))
    say(prec, "polynomial rows residual", rpoly, bound)
    assert np.all(np.abs(rpoly) <= bound)
    # evaluation at held-out points
    f, rmse = rbf.rbf_eval(plan, dev(prob.test_points), dev(ck), values=dev(prob.test_values))
    qq = slice(0, 2000)
    f_ref = orc.evaluate_poly(prob.test_points[:, qq], prob.centers, prob.rho, prob.phi, c, k)
    absf = (orc.evaluate(prob.test_points[:, qq], prob.centers, prob.rho, prob.phi, np.abs(c))
            + np.abs(k[:-1]) @ np.abs(prob.test_points[:, qq]) + abs(k[-1]))
    assert np.all(np.abs(f.cpu().numpy()[qq] - f_ref) <= 1e-12 * absf)
    say(prec, "held-out rmse", rmse)
    RES[prec] = rmse


def test_poly_fullsize_matched_rmse():
    if len(RES) < 2:
        pytest.skip("needs both precisions")
    assert abs(RES["fp32"] - RES["fp64"]) <= 1e-3 * RES["fp64"]
