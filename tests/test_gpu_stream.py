"""Parity of the chunked assembly (rbf_stream_begin / rbf_stream_add /
rbf_stream_finish) with the FP64 CPU oracle, through the C-ABI.

B = A^T A and g = A^T h are sums over the points (the point-block form of the
decomposition of Section 5, eq. 13-16), so the system formed from chunks is the
oracle's system of all points:

* supports, active set and the pattern of B: bit-exact, whatever the chunks;
* values of B and g: the bars of the resident assembly (|b - b*| <= 1e-12
  sqrt(b*_jj b*_ll) in FP64, 2e-6 in FP32; g alike);
* the solve: fitted values within 1e-10 of the oracle's (FP64), held-out RMSE
  equal to the resident fit's;
* the same chunks in the same order give the same bits; another order the same
  pattern and values within rounding.

Chunks are taken from device memory and from pinned host memory (staged by the
library on its own copy stream).
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


def host(a):
    return torch.from_numpy(np.ascontiguousarray(a)).pin_memory()


def entry_scale(ne):
    m = ne.m
    diag = np.zeros(m)
    for j in range(m):
        a, b = ne.row_ptr[j], ne.row_ptr[j + 1]
        if b > a:
            diag[j] = ne.val[a]
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
    return info


def check_values(rbf, plan, ne, h, tol):
    val, g, lam = rbf.rbf_system_export(plan)
    ref = ne.val.copy()
    ref[ne.row_ptr[:-1][ne.active]] += ne.lam
    scale = entry_scale(ne)
    err = np.abs(val - ref)
    assert np.all(err <= tol * scale + 1e-300), float(np.max(err / (scale + 1e-300)))
    gscale = np.abs(ne.A).T @ np.abs(h)
    assert np.all(np.abs(g - ne.g) <= tol * gscale + 1e-300)
    assert abs(lam - ne.lam) <= 10 * tol * ne.lam or (lam == 0.0 and ne.lam == 0.0)
    return float(np.max(err / (scale + 1e-300)))


def cuts(n, k, rng):
    """k ragged contiguous chunks of [0, n) (some may be empty)."""
    c = np.sort(rng.integers(0, n + 1, size=k - 1))
    return list(zip(np.r_[0, c], np.r_[c, n]))


def stream(rbf, pts, h, ctr, rho, phi, prec, parts, on_host, lam=1e-5, min_support=1,
           rho_per_center=None, max_chunk=None):
    mc = max_chunk or max(1, max(b - a for a, b in parts))
    plan = rbf.rbf_stream_begin(dev(ctr), mc, rho=rho, phi=phi, prec=prec, lambda_rel=lam,
                                min_support=min_support,
                                rho_per_center=None if rho_per_center is None
                                else dev(rho_per_center))
    put = host if on_host else dev
    for a, b in parts:
        rbf.rbf_stream_add(plan, put(pts[:, a:b]), put(h[a:b]))
    rbf.rbf_stream_finish(plan)
    return plan


@pytest.mark.parametrize("dim,phi,prec,k,on_host", [
    (2, "w31", "fp64", 1, False),
    (2, "w31", "fp64", 6, False),
    (2, "w32", "fp32", 5, True),
    (2, "w30", "fp32", 3, False),
    (3, "w31", "fp64", 4, True),
    (3, "w33", "fp32", 3, False),
])
def test_stream_matches_oracle(rbf, dim, phi, prec, k, on_host):
    rng = np.random.default_rng(70 + 10 * dim + k)
    g = 14 if dim == 2 else 7
    ctr = sd.grid_centers(g, dim)
    rho = 2.3 / (g - 1)
    n = 9000
    pts = np.concatenate([rng.random((dim, n // 2)),
                          sd.gaussian_mixture_points(rng, n - n // 2, dim, 3)], axis=1)
    h = np.cos(5 * pts[0]) * pts[1] + 0.05 * rng.standard_normal(n)
    parts = cuts(n, k, rng)
    say("stream", dim, phi, prec, "chunks", [b - a for a, b in parts], "host" if on_host else "device")
    ne = orc.normal_equations(pts, h, ctr, rho, phi, lambda_rel=1e-5)
    plan = stream(rbf, pts, h, ctr, rho, phi, prec, parts, on_host)
    info = check_pattern(rbf, plan, ne)
    assert info["n_points"] == n
    err = check_values(rbf, plan, ne, h, 1e-12 if prec == "fp64" else 2e-6)
    say("max scaled error", err)
    c, sinfo = rbf.rbf_solve(plan, rtol=FP64_RTOL if prec == "fp64" else 1e-10)
    assert sinfo["status"] == 0 and sinfo["precision"] == prec
    c = c.cpu().numpy()
    assert np.all(c[~ne.active] == 0.0)
    if prec == "fp64":
        c_ref = orc.solve(ne)
        fit = np.linalg.norm(ne.A @ (c - c_ref)) / np.linalg.norm(ne.A @ c_ref)
        say("fit", fit)
        assert fit <= FIT_FP64


def test_stream_equals_resident(rbf):
    # terrain-shaped data at 1/64 scale, points shuffled into 7 chunks: the
    # streamed system is the resident one (pattern bit for bit, values within
    # the summation bound) and so is the fit
    p = sd.make_problem("terrain2d", scale=1 / 64)
    rng = np.random.default_rng(5)
    n = p.points.shape[1]
    order = rng.permutation(n)
    pts, h = p.points[:, order], p.values[order]
    parts = cuts(n, 7, rng)
    for prec, tol in (("fp64", 1e-12), ("fp32", 2e-6)):
        res = rbf.rbf_fit_plan(dev(p.points), dev(p.centers), rho=p.rho, lambda_rel=1e-4)
        rbf.rbf_assemble(res, p.phi, prec, dev(p.values))
        st = stream(rbf, pts, h, p.centers, p.rho, p.phi, prec, parts, on_host=True, lam=1e-4)
        rp0, col0, sup0 = rbf.rbf_plan_pattern(res)
        rp1, col1, sup1 = rbf.rbf_plan_pattern(st)
        assert np.array_equal(rp0, rp1) and np.array_equal(col0, col1)
        assert np.array_equal(sup0, sup1)
        i0, i1 = rbf.rbf_plan_info(res), rbf.rbf_plan_info(st)
        for key in ("n_active", "nnz_full", "support_total", "n_points_in_box", "solver_entries",
                    "solver_lanes", "solver_col_bytes"):
            assert i0[key] == i1[key], key
        v0, g0, l0 = rbf.rbf_system_export(res)
        v1, g1, l1 = rbf.rbf_system_export(st)
        m = len(rp0) - 1
        diag = np.zeros(m)
        has = np.diff(rp0) > 0
        diag[has] = v0[rp0[:-1][has]]   # the first upper entry of a row is its diagonal
        scale = np.sqrt(np.repeat(diag, np.diff(rp0)) * diag[col0])
        assert np.all(np.abs(v1 - v0) <= tol * scale + 1e-300)
        gs = np.abs(g0).max()
        assert np.all(np.abs(g1 - g0) <= tol * gs)
        assert abs(l1 - l0) <= tol * l0
        out = {}
        for name, plan in (("resident", res), ("stream", st)):
            c, info = rbf.rbf_solve(plan, rtol=1e-10, max_iter=200000)
            assert info["status"] == 0
            _, r = rbf.rbf_eval(plan, dev(p.test_points), c, values=dev(p.test_values))
            out[name] = (r, info["iterations"])
        say(prec, out)
        # two solves to a relative residual of 1e-10 of systems equal to within
        # the summation bound (the resident-vs-oracle bar of the float64 fit is
        # the same 1e-6); FP32: two float32-stored systems that differ by the
        # assembly's rounding
        rtol = 1e-6 if prec == "fp64" else 1e-4
        assert abs(out["stream"][0] - out["resident"][0]) <= rtol * out["resident"][0]
        res.close()
        st.close()


def test_stream_deterministic_and_order(rbf):
    rng = np.random.default_rng(11)
    ctr = sd.grid_centers(10, 2)
    rho = 0.3
    pts = sd.gaussian_mixture_points(rng, 6000, 2, 4)
    h = np.sin(4 * pts[0]) + pts[1]
    parts = cuts(6000, 5, rng)
    a = stream(rbf, pts, h, ctr, rho, "w31", "fp32", parts, on_host=False)
    b = stream(rbf, pts, h, ctr, rho, "w31", "fp32", parts, on_host=True)
    va, ga, la = rbf.rbf_system_export(a)
    vb, gb, lb = rbf.rbf_system_export(b)
    assert np.array_equal(va, vb) and np.array_equal(ga, gb) and la == lb
    # host chunks in pageable memory (a synchronous copy): the same bits
    c = rbf.rbf_stream_begin(dev(ctr), max(b1 - a1 for a1, b1 in parts), rho=rho, phi="w31",
                             prec="fp32", lambda_rel=1e-5)
    for a1, b1 in parts:
        rbf.rbf_stream_add(c, torch.from_numpy(np.ascontiguousarray(pts[:, a1:b1])),
                           torch.from_numpy(np.ascontiguousarray(h[a1:b1])))
    rbf.rbf_stream_finish(c)
    vc, gc, lc = rbf.rbf_system_export(c)
    assert np.array_equal(va, vc) and np.array_equal(ga, gc) and la == lc
    rev = stream(rbf, pts, h, ctr, rho, "w31", "fp64", parts[::-1], on_host=False)
    fwd = stream(rbf, pts, h, ctr, rho, "w31", "fp64", parts, on_host=False)
    assert np.array_equal(rbf.rbf_plan_pattern(rev)[1], rbf.rbf_plan_pattern(fwd)[1])
    vr, gr, _ = rbf.rbf_system_export(rev)
    vf, gf, _ = rbf.rbf_system_export(fwd)
    assert np.all(np.abs(vr - vf) <= 1e-13 * np.abs(vf).max())
    assert np.all(np.abs(gr - gf) <= 1e-13 * np.abs(gf).max())


def test_stream_edge_cases(rbf):
    rng = np.random.default_rng(12)
    ctr = sd.grid_centers(8, 2)
    rho = 0.25
    pts = rng.random((2, 3000)) * 0.6          # lower-left part only: empty supports
    h = pts[0] - 2 * pts[1]
    far = np.full((2, 50), 7.0)                # outside the centres' grid
    # empty chunks, a chunk of far points, min_support applied at the finish,
    # per-centre radii
    rpc = rho * (0.8 + 0.4 * rng.random(ctr.shape[1]))
    ne = orc.normal_equations(pts, h, ctr, rpc, "w31", min_support=25, lambda_rel=1e-6)
    plan = rbf.rbf_stream_begin(dev(ctr), 2000, rho_per_center=dev(rpc), phi="w31",
                                prec="fp64", lambda_rel=1e-6, min_support=25)
    rbf.rbf_stream_add(plan, dev(np.zeros((2, 0))), dev(np.zeros(0)))
    rbf.rbf_stream_add(plan, dev(pts[:, :1700]), dev(h[:1700]))
    rbf.rbf_stream_add(plan, host(far), host(np.ones(50)))
    rbf.rbf_stream_add(plan, host(np.zeros((2, 0))), host(np.zeros(0)))
    rbf.rbf_stream_add(plan, dev(pts[:, 1700:]), dev(h[1700:]))
    rbf.rbf_stream_finish(plan)
    assert np.any(~ne.active) and np.any(ne.support_count[~ne.active] > 0)
    info = check_pattern(rbf, plan, ne)
    assert info["n_points"] == 3050 and info["n_points_in_box"] == 3000
    check_values(rbf, plan, ne, h, 1e-12)
    c, sinfo = rbf.rbf_solve(plan, rtol=FP64_RTOL)
    c = c.cpu().numpy()
    assert np.all(c[~ne.active] == 0.0)
    c_ref = orc.solve(ne)
    fit = np.linalg.norm(ne.A @ (c - c_ref)) / np.linalg.norm(ne.A @ c_ref)
    say("fit", fit)
    assert fit <= FIT_FP64
    # no chunk at all: nothing active, the solve gives zeros
    empty = rbf.rbf_stream_begin(dev(ctr), 10, rho=rho)
    rbf.rbf_stream_finish(empty)
    assert rbf.rbf_plan_info(empty)["n_active"] == 0
    c0, inf0 = rbf.rbf_solve(empty)
    assert inf0["status"] == 0 and np.all(c0.cpu().numpy() == 0.0)


def test_stream_errors(rbf):
    from paper_1806_07884_amd._lib import RbfError
    ctr = sd.grid_centers(6, 2)
    pts = np.random.default_rng(1).random((2, 100))
    h = pts[0].copy()
    plan = rbf.rbf_stream_begin(dev(ctr), 64, rho=0.3)
    with pytest.raises(RbfError, match="max_chunk"):
        rbf.rbf_stream_add(plan, dev(pts), dev(h))
    with pytest.raises(RbfError, match="finish"):
        rbf.rbf_plan_info(plan)
    with pytest.raises(RbfError, match="must precede"):
        rbf.rbf_solve(plan)
    with pytest.raises(RbfError, match="no points"):
        rbf.rbf_assemble(plan, "w31", "fp64", dev(h[:0]))
    rbf.rbf_stream_add(plan, dev(pts[:, :64]), dev(h[:64]))
    rbf.rbf_stream_finish(plan)
    with pytest.raises(RbfError, match="finished"):
        rbf.rbf_stream_add(plan, dev(pts[:, :10]), dev(h[:10]))
    with pytest.raises(RbfError, match="finished"):
        rbf.rbf_stream_finish(plan)
    with pytest.raises(RbfError, match="no points"):
        rbf.rbf_set_values(plan, dev(h[:64]))
    resident = rbf.rbf_fit_plan(dev(pts), dev(ctr), rho=0.3)
    with pytest.raises(RbfError, match="not a stream plan"):
        rbf.rbf_stream_add(resident, dev(pts[:, :10]), dev(h[:10]))
    bad = pts[:, :20].copy()
    bad[1, 7] = np.nan
    p2 = rbf.rbf_stream_begin(dev(ctr), 64, rho=0.3)
    rbf.rbf_stream_add(p2, host(bad), host(h[:20]))
    with pytest.raises(RbfError, match="non-finite"):
        rbf.rbf_stream_finish(p2)
    with pytest.raises(RbfError, match="max_chunk"):
        rbf.rbf_stream_begin(dev(ctr), 0, rho=0.3)
