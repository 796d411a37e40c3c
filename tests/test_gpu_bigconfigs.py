"""Parity at the two largest workloads, on outputs the oracle recomputes one
by one (the whole system is far beyond a dense or banded CPU solve):

* terrain2d_big: N = 2^24 clustered points, 1024 x 1024 centres, phi_{3,2},
  radius covering ~40 centres, float32 assembly with compensated sums,
  float32 Jacobi-PCG with float64 reliable updates to 1e-10, 1 % held out;
* field3d: N = 2^22 points in [0,1]^3 from 32 clusters, 64^3 centres,
  phi_{3,1}, mixed and float64 solves, evaluation at 10^6 uniform queries
  scored against the noise-free field.

Checked, for each:

* support counts of sampled centres (brute force over all points): exact;
* sampled rows of the upper pattern of B: exact;
* sampled values of B and g_j within 1e-13 (b* + n_jl phi(0)^2) (float64)
  or 1e-5 b* + 3e-6 n_jl phi(0)^2 (float32; the terms of a float32 sum each
  carry a few roundings of phi, bounded relative to phi(0));
* lambda: the stored diagonals satisfy lambda = lambda_rel mean(b_jj) over
  the active centres (a property of the whole matrix, checked in float64 on
  the exported values);
* the solution: at sampled rows the normal-equation residual with the
  oracle's row and the GPU coefficients stays below the requested relative
  residual times ||g|| plus, for float32, the assembly bound applied to the
  row (||g|| from the exported g, whose sampled entries were checked);
* evaluation: at sampled queries the GPU value equals the oracle's
  evaluation of the GPU coefficients within 1e-12 sum |c_j phi|;
* field3d: mixed and float64 RMSE agree to 0.1 %, both against the clean
  field at the uniform queries and against the noisy samples at its 1 %
  held-out points (the queries reach beyond the data, so the held-out score
  is the one that measures the fit itself).
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
N_QUERIES = 1_000_000


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.fixture(scope="module")
def rbf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1806_07884_amd as m
    return m


class Case:
    def __init__(self, name, rbf):
        say("generating", name)
        self.name = name
        self.prob = p = sd.make_problem(name)
        say(name, "points", p.points.shape, "centres", p.centers.shape, "rho", p.rho, p.phi)
        self.q, self.qh = sd.scoring_queries(p, N_QUERIES)
        self.dp, self.dc = dev(p.points), dev(p.centers)
        say(name, "plan")
        self.plan = rbf.rbf_fit_plan(self.dp, self.dc, rho=p.rho, lambda_rel=LAM)
        self.rmse = {}
        self.heldout = {}
        self.pattern = None

    def rows(self, k, seed):
        rng = np.random.default_rng(seed)
        m = self.prob.centers.shape[1]
        return sorted(set([0, m - 1, m // 2] + list(rng.integers(0, m, size=k))))


@pytest.fixture(scope="module", params=["terrain2d_big", "field3d"])
def case(request, rbf):
    c = Case(request.param, rbf)
    yield c
    c.plan.close()


@pytest.mark.timeout(600)
def test_big_pattern_sampled(case, rbf):
    p = case.prob
    rp, col, sup = rbf.rbf_plan_pattern(case.plan)
    case.pattern = (rp, col)
    info = rbf.rbf_plan_info(case.plan)
    say(case.name, "info", info)
    assert info["nnz_upper"] == len(col) == rp[-1]
    for j in case.rows(8, 0):
        s = orc.sqdist(p.points, p.centers[:, j])
        assert sup[j] == int(np.sum(s < p.rho * p.rho)), j
        row = orc.sample_row(p.points, p.values, p.centers, p.rho, p.phi, j)
        assert np.array_equal(col[rp[j]:rp[j + 1]], row.cols), j


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_big_values_solve_eval(case, rbf, prec):
    p = case.prob
    if case.name == "terrain2d_big" and prec == "fp64":
        pytest.skip("the 2^24-point workload is specified for the mixed path only")
    say(case.name, prec, "assemble")
    rbf.rbf_assemble(case.plan, p.phi, prec, dev(p.values))
    if case.pattern is None:
        rp, col, _ = rbf.rbf_plan_pattern(case.plan)
        case.pattern = (rp, col)
    rp, col = case.pattern
    val, g, lam = rbf.rbf_system_export(case.plan)
    # lambda = lambda_rel mean(b_jj) over active rows (stored diagonal = b_jj + lambda)
    m = p.centers.shape[1]
    rows_nonempty = rp[1:] > rp[:-1]
    jj = np.nonzero(rows_nonempty)[0]
    assert np.all(col[rp[jj]] == jj)
    diag = val[rp[jj]] - lam
    lam_prop = LAM * diag.mean()
    say(case.name, prec, "lambda", lam, "property", lam_prop)
    assert abs(lam - lam_prop) <= (1e-12 if prec == "fp64" else 1e-6) * lam_prop
    phi0sq = float(orc.wendland(p.phi, np.array([0.0]))[0]) ** 2
    a_tol, n_tol = (1e-13, 1e-13) if prec == "fp64" else (1e-5, 3e-6)
    say(case.name, prec, "solve")
    c, info = rbf.rbf_solve(case.plan, rtol=RTOL, max_iter=200000)
    say(case.name, prec, "solve info", info)
    assert info["status"] == 0 and info["precision"] == prec
    assert info["rel_residual"] <= RTOL
    c = c.cpu().numpy()
    gnorm = np.linalg.norm(g)
    for j in case.rows(8, 1):
        row = orc.sample_row(p.points, p.values, p.centers, p.rho, p.phi, j, lower=True)
        if row.support.size == 0:
            assert rp[j + 1] == rp[j] and c[j] == 0.0
            continue
        up = row.cols >= j
        got = val[rp[j]:rp[j + 1]]
        ref = row.vals[up].copy()
        ref[0] += lam
        tol = a_tol * ref + n_tol * phi0sq * row.pair_count[up] + 1e-12 * lam
        assert np.all(np.abs(got - ref) <= tol), (j, float(np.max(np.abs(got - ref) / tol)))
        hsum = np.sum(np.abs(p.values[row.support]))
        gtol = (a_tol + n_tol) * np.sqrt(phi0sq) * hsum
        assert abs(g[j] - row.g) <= gtol, (j, g[j], row.g)
        r = row.g - np.dot(row.vals, c[row.cols]) - lam * c[j]
        bound = 1.01 * RTOL * gnorm + gtol
        if prec == "fp32":
            bound += (a_tol * np.dot(np.abs(row.vals), np.abs(c[row.cols]))
                      + n_tol * phi0sq * np.dot(row.pair_count, np.abs(c[row.cols])))
        assert abs(r) <= bound, (j, r, bound)
    say(case.name, prec, "eval", case.q.shape)
    f, rmse = rbf.rbf_eval(case.plan, dev(case.q), dev(c), values=dev(case.qh))
    f = f.cpu().numpy()
    rng = np.random.default_rng(5)
    for i in rng.integers(0, case.q.shape[1], size=200):
        y = case.q[:, i]
        ref = orc.evaluate_one(y, p.centers, p.rho, p.phi, c)
        absf = orc.evaluate_one(y, p.centers, p.rho, p.phi, np.abs(c))
        assert abs(f[i] - ref) <= 1e-12 * absf + 1e-300, (i, f[i], ref)
    cov = f != 0.0
    say(case.name, prec, "rmse", rmse, "covered queries", float(cov.mean()),
        "rmse there", float(np.sqrt(np.mean((f[cov] - case.qh[cov]) ** 2))))
    case.rmse[prec] = rmse
    assert np.isfinite(rmse)
    if p.score == "uniform" and p.test_points.shape[1]:
        _, hr = rbf.rbf_eval(case.plan, dev(p.test_points), dev(c), values=dev(p.test_values))
        say(case.name, prec, "held-out rmse", hr, "points", p.test_points.shape[1])
        case.heldout[prec] = hr
        assert np.isfinite(hr)


def test_big_matched_rmse(case):
    if len(case.rmse) < 2:
        pytest.skip("needs both precisions")
    assert abs(case.rmse["fp32"] - case.rmse["fp64"]) <= 1e-3 * case.rmse["fp64"]
    if case.heldout:
        assert abs(case.heldout["fp32"] - case.heldout["fp64"]) <= 1e-3 * case.heldout["fp64"]


@pytest.mark.timeout(900)
def test_big_stream_equals_resident(case, rbf):
    # the same points streamed in 8 chunks (rbf_stream_*, float32): pattern
    # and support counts equal to the resident plan's, sampled values and g_j
    # within the float32 bars of the oracle's rows, the same RMSE
    p = case.prob
    n = p.points.shape[1]
    bounds = np.linspace(0, n, 9).astype(np.int64)
    say(case.name, "stream in 8 chunks")
    st = rbf.rbf_stream_begin(case.dc, int(np.max(np.diff(bounds))), rho=p.rho, phi=p.phi,
                              prec="fp32", lambda_rel=LAM)
    for a, b in zip(bounds[:-1], bounds[1:]):
        rbf.rbf_stream_add(st, dev(p.points[:, a:b]), dev(p.values[a:b]))
    rbf.rbf_stream_finish(st)
    rp, col, sup = rbf.rbf_plan_pattern(st)
    rp0, col0, sup0 = rbf.rbf_plan_pattern(case.plan)
    assert np.array_equal(rp, rp0) and np.array_equal(col, col0) and np.array_equal(sup, sup0)
    val, g, lam = rbf.rbf_system_export(st)
    phi0sq = float(orc.wendland(p.phi, np.array([0.0]))[0]) ** 2
    a_tol, n_tol = 1e-5, 3e-6
    for j in case.rows(4, 2):
        row = orc.sample_row(p.points, p.values, p.centers, p.rho, p.phi, j)
        if row.support.size == 0:
            continue
        got = val[rp[j]:rp[j + 1]]
        ref = row.vals.copy()
        ref[0] += lam
        tol = a_tol * ref + n_tol * phi0sq * row.pair_count + 1e-12 * lam
        assert np.all(np.abs(got - ref) <= tol), (j, float(np.max(np.abs(got - ref) / tol)))
        hsum = np.sum(np.abs(p.values[row.support]))
        assert abs(g[j] - row.g) <= (a_tol + n_tol) * np.sqrt(phi0sq) * hsum
    c, info = rbf.rbf_solve(st, rtol=RTOL, max_iter=200000)
    assert info["status"] == 0
    _, rmse = rbf.rbf_eval(st, dev(case.q), c, values=dev(case.qh))
    say(case.name, "streamed rmse", rmse, "resident", case.rmse.get("fp32"))
    if "fp32" in case.rmse:
        assert abs(rmse - case.rmse["fp32"]) <= 1e-3 * case.rmse["fp32"]
    st.close()
