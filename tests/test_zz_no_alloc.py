"""rbf_eval_noalloc (the allocation-free evaluation) against rbf_eval, through
the C-ABI: the same kernels, so outputs and RMSE agree bit for bit, on two
calls in a row where the second has fewer centres and fewer queries (stale
workspace contents from the first call must not leak into the second), on a
polynomial plan, with no queries, and the size limit is refused."""
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
def rbf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1806_07884_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def fit(rbf, p, poly=False):
    plan = rbf.rbf_fit_plan(dev(p.points), dev(p.centers), rho=p.rho, lambda_rel=1e-5,
                            polynomial=poly)
    rbf.rbf_assemble(plan, p.phi, "fp64", dev(p.values))
    c, _ = rbf.rbf_solve(plan, rtol=1e-10)
    return plan, c


def same(rbf, plan, q, c, h):
    ref, r_ref = rbf.rbf_eval(plan, q, c, values=h)
    out = torch.full_like(ref, float("nan"))
    got, r = rbf.rbf_eval_noalloc(plan, q, c, out, values=h)
    assert got.data_ptr() == out.data_ptr()
    assert torch.equal(got, ref)
    assert r == r_ref
    return r


def test_noalloc_matches_eval_two_calls(rbf):
    big = sd.make_problem("terrain2d", scale=1 / 16)         # 64^2 centres
    small = sd.make_problem("franke2d", scale=0.25)          # 16^2 centres
    say("noalloc", big.centers.shape, small.centers.shape)
    pb, cb = fit(rbf, big)
    ps, cs = fit(rbf, small)
    rng = np.random.default_rng(5)
    qb = dev(rng.random((2, 20000)))
    qs = dev(rng.random((2, 700)) * 1.2 - 0.1)
    hb = dev(rng.standard_normal(20000))
    hs = dev(rng.standard_normal(700))
    r1 = same(rbf, pb, qb, cb, hb)
    r2 = same(rbf, ps, qs, cs, hs)
    say("rmse", r1, r2)
    # and back to the larger plan, then without values
    same(rbf, pb, qb, cb, hb)
    out = torch.empty(700, dtype=torch.float64, device="cuda")
    got, r = rbf.rbf_eval_noalloc(ps, qs, cs, out)
    assert r is None and torch.equal(got, rbf.rbf_eval(ps, qs, cs)[0])
    # no queries: nothing launched, the same answer as rbf_eval (an empty
    # tensor hands the library a null pointer, so no RMSE is asked for)
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    _, r0 = rbf.rbf_eval_noalloc(ps, dev(np.zeros((2, 0))), cs, e, values=e)
    _, r0_ref = rbf.rbf_eval(ps, dev(np.zeros((2, 0))), cs, values=e)
    assert r0 == r0_ref or (np.isnan(r0) and np.isnan(r0_ref))
    pb.close()
    ps.close()


def test_noalloc_polynomial_and_3d(rbf):
    p3 = sd.make_problem("field3d", scale=1 / 512)
    plan, c = fit(rbf, p3, poly=True)
    q = dev(np.random.default_rng(6).random((3, 5000)))
    same(rbf, plan, q, c, dev(np.zeros(5000)))
    plan.close()


def test_noalloc_size_limit(rbf):
    from paper_1806_07884_amd._lib import RbfError
    ctr = sd.grid_centers(1025, 2)                           # 1,050,625 > 2^20 centres
    pts = np.random.default_rng(7).random((2, 1000))
    plan = rbf.rbf_fit_plan(dev(pts), dev(ctr), rho=0.003)
    c = torch.zeros(ctr.shape[1], dtype=torch.float64, device="cuda")
    out = torch.empty(10, dtype=torch.float64, device="cuda")
    with pytest.raises(RbfError, match="at most 1048576 centres"):
        rbf.rbf_eval_noalloc(plan, dev(pts[:, :10]), c, out)
    plan.close()
