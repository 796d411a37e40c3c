"""Parity at the full size of the terrain workload (N = 2^20 clustered points,
256 x 256 centres, the launch configuration bench.py times), on outputs the
oracle recomputes one by one:

* support counts of sampled centres (brute force over all points): exact;
* sampled rows of the upper pattern of B: exact; their values and g_j within
  1e-13 (b* + n_jl phi(0)^2) for FP64 and 1e-5 b* + 3e-6 n_jl phi(0)^2 for FP32
  (phi is evaluated from a scaled distance that carries a few roundings; near
  the edge of the support its absolute error is bounded by a small multiple of
  u phi(0), hence the n_jl phi(0)^2 term);
* the solution: at sampled rows the normal-equation residual
  g*_j - sum_l b*_jl c_l - lambda c_j (oracle row, GPU coefficients) stays
  below the requested relative residual times ||g*||;
* evaluation: GPU values at held-out points equal the oracle's evaluation of
  the same coefficients; mixed and FP64 held-out RMSE agree to 0.1 %.
"""
import sys

import numpy as np
import pytest
import torch

import synthdata as sd
from oracle import rbf_oracle as orc

pytestmark = pytest.mark.gpu
LAM = 1e-4


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


def sample_rows(prob, k=12, seed=0):
    rng = np.random.default_rng(seed)
    m = prob.centers.shape[1]
    return sorted(set([0, m - 1, m // 2] + list(rng.integers(0, m, size=k))))


@pytest.fixture(scope="module")
def plan(prob, rbf):
    say("terrain2d full plan", prob.points.shape, prob.centers.shape, prob.rho)
    p = rbf.rbf_fit_plan(dev(prob.points), dev(prob.centers), rho=prob.rho, lambda_rel=LAM)
    yield p
    p.close()


def test_fullsize_pattern_sampled(prob, rbf, plan):
    rp, col, sup = rbf.rbf_plan_pattern(plan)
    rows = sample_rows(prob)
    for j in rows:
        s = orc.sqdist(prob.points, prob.centers[:, j])
        assert sup[j] == int(np.sum(s < prob.rho * prob.rho))
        row = orc.sample_row(prob.points, prob.values, prob.centers, prob.rho, prob.phi, j)
        got = col[rp[j]:rp[j + 1]]
        assert np.array_equal(got, row.cols), j
    info = rbf.rbf_plan_info(plan)
    say("info", info)
    assert info["nnz_upper"] == len(col)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fullsize_values_and_solve(prob, rbf, plan, prec):
    say("assemble + solve", prec)
    rbf.rbf_assemble(plan, prob.phi, prec, dev(prob.values))
    rp, col, _ = rbf.rbf_plan_pattern(plan)
    val, g, lam = rbf.rbf_system_export(plan)
    rows = sample_rows(prob, seed=1)
    c, info = rbf.rbf_solve(plan, rtol=1e-10, max_iter=200000)
    say("solve", info)
    assert info["status"] == 0 and info["precision"] == prec
    c = c.cpu().numpy()
    # oracle pieces: g* for every centre (for ||g*||), sampled full rows
    A = orc.design_matrix(prob.points, prob.centers, prob.rho, prob.phi)
    g_ref = A.T @ prob.values
    diag_ref = np.asarray(A.multiply(A).sum(axis=0)).ravel()
    lam_ref = LAM * diag_ref[diag_ref > 0].mean()
    # lambda is a mean of assembled diagonals: float64 or float32-Kahan accurate
    assert abs(lam - lam_ref) <= (1e-9 if prec == "fp64" else 1e-6) * lam_ref
    gnorm = np.linalg.norm(g_ref)
    a_tol, n_tol = (1e-13, 1e-13) if prec == "fp64" else (1e-5, 3e-6)
    for j in rows:
        row = orc.sample_row(prob.points, prob.values, prob.centers, prob.rho, prob.phi, j,
                             lower=True)
        if row.support.size == 0:
            assert c[j] == 0.0
            continue
        up = row.cols >= j
        got = val[rp[j]:rp[j + 1]]
        ref = row.vals[up].copy()
        ref[0] += lam_ref
        tol = a_tol * ref + n_tol * row.pair_count[up] + 1e-12 * lam_ref
        assert np.all(np.abs(got - ref) <= tol), (j, float(np.max(np.abs(got - ref) / tol)))
        gscale = np.sum(np.abs(A[:, j].toarray().ravel() * prob.values))
        hsum = np.sum(np.abs(prob.values[row.support]))
        assert abs(g[j] - row.g) <= a_tol * gscale + n_tol * hsum
        # residual of the normal equations at row j with the oracle's row; the
        # mixed path solves the float32-stored system, whose entries differ from
        # the oracle's by the assembly bound above
        r = row.g - np.dot(row.vals, c[row.cols]) - lam_ref * c[j]
        bound = 1e-10 * gnorm
        if prec == "fp32":
            bound += (a_tol * np.dot(np.abs(row.vals), np.abs(c[row.cols]))
                      + n_tol * np.dot(row.pair_count, np.abs(c[row.cols]))
                      + a_tol * gscale + n_tol * hsum)
        assert abs(r) <= bound, (j, r, bound)
    # evaluation at held-out points
    f, rmse = rbf.rbf_eval(plan, dev(prob.test_points), dev(c), values=dev(prob.test_values))
    q = slice(0, 2000)
    f_ref = orc.evaluate(prob.test_points[:, q], prob.centers, prob.rho, prob.phi, c)
    absf = orc.evaluate(prob.test_points[:, q], prob.centers, prob.rho, prob.phi, np.abs(c))
    assert np.all(np.abs(f.cpu().numpy()[q] - f_ref) <= 1e-12 * absf + 1e-300)
    say(prec, "heldout rmse", rmse)
    test_fullsize_values_and_solve.rmse[prec] = rmse


test_fullsize_values_and_solve.rmse = {}


def test_fullsize_matched_rmse():
    r = test_fullsize_values_and_solve.rmse
    if len(r) < 2:
        pytest.skip("needs both precisions")
    assert abs(r["fp32"] - r["fp64"]) <= 1e-3 * r["fp64"]
