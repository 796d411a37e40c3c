"""Chunked assembly at the full size of the terrain workload (N = 2^20
clustered points, 256 x 256 centres, eight chunks from pinned host memory, as
``bench.py --stream 8`` runs it), on outputs the oracle recomputes one by one:

* support counts of sampled centres (brute force over all points): exact;
* sampled rows of the upper pattern: exact; their values and g_j within the
  bars of the resident full-size test (FP32: 1e-5 b* + 3e-6 n_jl phi(0)^2);
* the whole pattern equals the resident plan's bit for bit;
* the mixed solve reaches the same held-out RMSE as the resident fit (0.1 %).
"""
import sys

import numpy as np
import pytest
import torch

import synthdata as sd
from oracle import rbf_oracle as orc

pytestmark = pytest.mark.gpu
LAM = 1e-4
CHUNKS = 8


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


def test_stream_fullsize(rbf):
    prob = sd.make_problem("terrain2d")
    n = prob.points.shape[1]
    bounds = np.linspace(0, n, CHUNKS + 1).astype(np.int64)
    say("terrain2d full, streamed in", CHUNKS, "host chunks")
    plan = rbf.rbf_stream_begin(dev(prob.centers), int(np.max(np.diff(bounds))), rho=prob.rho,
                                phi=prob.phi, prec="fp32", lambda_rel=LAM)
    for a, b in zip(bounds[:-1], bounds[1:]):
        xc = torch.from_numpy(np.ascontiguousarray(prob.points[:, a:b])).pin_memory()
        hc = torch.from_numpy(np.ascontiguousarray(prob.values[a:b])).pin_memory()
        rbf.rbf_stream_add(plan, xc, hc)
    rbf.rbf_stream_finish(plan)
    rp, col, sup = rbf.rbf_plan_pattern(plan)
    val, g, lam = rbf.rbf_system_export(plan)

    # the resident plan of the same points: the same pattern
    res = rbf.rbf_fit_plan(dev(prob.points), dev(prob.centers), rho=prob.rho, lambda_rel=LAM)
    rp0, col0, sup0 = rbf.rbf_plan_pattern(res)
    assert np.array_equal(rp, rp0) and np.array_equal(col, col0) and np.array_equal(sup, sup0)

    rng = np.random.default_rng(3)
    m = prob.centers.shape[1]
    rows = sorted(set([0, m - 1, m // 2] + list(rng.integers(0, m, size=12))))
    A = orc.design_matrix(prob.points, prob.centers, prob.rho, prob.phi)
    diag_ref = np.asarray(A.multiply(A).sum(axis=0)).ravel()
    lam_ref = LAM * diag_ref[diag_ref > 0].mean()
    assert abs(lam - lam_ref) <= 1e-6 * lam_ref
    a_tol, n_tol = 1e-5, 3e-6
    for j in rows:
        s = orc.sqdist(prob.points, prob.centers[:, j])
        assert sup[j] == int(np.sum(s < prob.rho * prob.rho))
        row = orc.sample_row(prob.points, prob.values, prob.centers, prob.rho, prob.phi, j)
        assert np.array_equal(col[rp[j]:rp[j + 1]], row.cols), j
        if row.support.size == 0:
            continue
        got = val[rp[j]:rp[j + 1]]
        ref = row.vals.copy()
        ref[0] += lam_ref
        tol = a_tol * ref + n_tol * row.pair_count + 1e-12 * lam_ref
        assert np.all(np.abs(got - ref) <= tol), (j, float(np.max(np.abs(got - ref) / tol)))
        gscale = np.sum(np.abs(A[:, j].toarray().ravel() * prob.values))
        hsum = np.sum(np.abs(prob.values[row.support]))
        assert abs(g[j] - row.g) <= a_tol * gscale + n_tol * hsum

    out = {}
    rbf.rbf_assemble(res, prob.phi, "fp32", dev(prob.values))
    for name, p in (("stream", plan), ("resident", res)):
        c, info = rbf.rbf_solve(p, rtol=1e-10, max_iter=200000)
        assert info["status"] == 0
        _, r = rbf.rbf_eval(p, dev(prob.test_points), c, values=dev(prob.test_values))
        out[name] = r
    say("held-out rmse", out)
    assert abs(out["stream"] - out["resident"]) <= 1e-3 * out["resident"]
