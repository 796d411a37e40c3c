"""FP64 oracle of the CS-RBF least-squares approximation (test infrastructure only).

What it computes, after Majdisova & Skala, "Big Geo Data Surface Approximation
using Radial Basis Functions: A Comparative Study":

* the approximant f(x) = sum_j c_j phi(||x - xi_j|| / rho_j)           (Section 2, eq. 3)
* the overdetermined system A c = h, A_ij = phi(||x_i - xi_j|| / rho_j) (Section 2, eq. 4-5)
* its least-squares solution through the normal equations
  A^T A c = A^T h                                                      (Section 2, end)
* B = A^T A entry by entry, b_jl = sum_k phi_kj phi_kl                  (Section 5, eq. 11-12)
  of which only the upper triangle is kept                              (Section 5, eq. 13 and Fig. 2)
* the Wendland basis functions with truncated power (1 - r)_+          (Table 2, eq. 18)
* support found by a strict range query ||x_q - xi_j|| < 1/alpha       (Algorithm 1)
* the COO sparse product y[row] += data * x[col]                        (Section 4)
* linear polynomial reproduction: f(x) = sum_j c_j phi_j(x) + a^T x + a_0 and
  the bordered normal equations [[A^T A, A^T P], [P^T A, P^T P]] (c, k) =
  (A^T h, P^T h) with P_i = (x_i^T, 1)                                   (Section 3, eq. 6-10)

Every routine is the plain definition: the design matrix is built explicitly,
B and g are library sparse products of it, and the solve is a Cholesky
factorisation.  There is no blocking, fusion or reordering of the method.

Readings where the paper is silent (each is listed with its reason in the
design notes of the repository):

* radius: rho = 1/alpha, so phi(r / rho) is the tabulated (1 - alpha r)_+ form;
* predicate: s = (dx*dx + dy*dy) [+ dz*dz], every product and sum rounded
  separately in FP64 (no fused multiply-add), dx = x - xi in FP64; a point is
  in the support of centre j iff s < rho_j * rho_j (strict, the product rounded
  once).  The HIP path evaluates the very same expression, so supports and the
  sparsity pattern agree bit for bit;
* pattern of B: structural, (j, l) is stored iff some point lies in both
  supports, whatever the value;
* empty or thin supports: a centre with fewer than ``min_support`` points is
  inactive, its row and column are removed and its coefficient is zero;
* ridge: the solved system is (B + lambda I) c = g with
  lambda = lambda_rel * mean(diag B over active centres);
* phi_{3,2} = (1-r)^6 (35 r^2 + 18 r + 3) completes the Wendland family of
  Table 2 (same family, smoothness C^4);
* polynomial with ridge: the ridge is added to the A^T A block only (the
  polynomial coefficients are not penalised); inactive centres have no row in
  Q = A^T P, every point is a row of P.

Parity: pinned.  Basis closed forms, brute-force supports, dense least
squares (QR), symmetry / positive definiteness, the normal-equation invariant,
the interpolation special case, the worked COO example of Section 4 and, for
the RMSE, closed forms and the noise level of the Franke fit (a least-squares
fit leaves sigma sqrt(1 - M/N) of N(0, sigma^2) noise) pin every function here; the polynomial part is pinned by exact reproduction of
linear data, the QR solution of eq. 9 and the Table 4 density with a
polynomial (see tests/test_oracle_*.py).
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
from scipy.spatial import cKDTree

PHI_KINDS = ("w30", "w31", "w32", "w33")


# ---------------------------------------------------------------------------
# Basis functions (Table 2; phi_{3,2} from the same Wendland family)
# ---------------------------------------------------------------------------
def wendland(kind: str, r):
    """Wendland CS-RBF of the scaled distance r = ||x - xi|| / rho.

    (1 - r)_+ is the truncated power of eq. 18: zero for r > 1.
      w30: (1-r)^2_+                                   C^0
      w31: (1-r)^4_+ (4 r + 1)                         C^2
      w32: (1-r)^6_+ (35 r^2 + 18 r + 3)               C^4
      w33: (1-r)^8_+ (32 r^3 + 25 r^2 + 8 r + 1)       C^6
    """
    r = np.asarray(r, dtype=np.float64)
    t = np.where(r <= 1.0, 1.0 - r, 0.0)
    if kind == "w30":
        return t ** 2
    if kind == "w31":
        return t ** 4 * (4.0 * r + 1.0)
    if kind == "w32":
        return t ** 6 * (35.0 * r ** 2 + 18.0 * r + 3.0)
    if kind == "w33":
        return t ** 8 * (32.0 * r ** 3 + 25.0 * r ** 2 + 8.0 * r + 1.0)
    raise ValueError(f"unknown basis {kind!r}")


# ---------------------------------------------------------------------------
# Support predicate (Algorithm 1, strict inequality; eq. 18)
# ---------------------------------------------------------------------------
def sqdist(points: np.ndarray, center: np.ndarray) -> np.ndarray:
    """Canonical squared distance of SoA ``points`` (dim, n) to one centre.

    s = (dx*dx + dy*dy) + dz*dz, each operation rounded on its own (NumPy never
    fuses a multiply with an add), evaluated left to right.
    """
    dim = points.shape[0]
    d0 = points[0] - center[0]
    s = d0 * d0
    for k in range(1, dim):
        dk = points[k] - center[k]
        s = s + dk * dk
    return s


def rho_squared(rho: np.ndarray) -> np.ndarray:
    return np.asarray(rho, dtype=np.float64) * np.asarray(rho, dtype=np.float64)


def _rho_vec(rho, m: int) -> np.ndarray:
    rho = np.asarray(rho, dtype=np.float64)
    if rho.ndim == 0:
        return np.full(m, float(rho))
    assert rho.shape == (m,)
    return rho


def supports(points: np.ndarray, centers: np.ndarray, rho,
             brute_limit: int = 50_000_000) -> list[np.ndarray]:
    """For every centre j the ascending point indices q with s_qj < rho_j^2.

    Small problems are brute force over all pairs; larger ones take candidates
    from a k-d tree query with 1e-6 relative slack (the range query of
    Algorithm 1) and let the exact predicate decide.
    """
    dim, n = points.shape
    m = centers.shape[1]
    rv = _rho_vec(rho, m)
    r2 = rho_squared(rv)
    out: list[np.ndarray] = []
    if n * m <= brute_limit:
        for j in range(m):
            s = sqdist(points, centers[:, j])
            out.append(np.nonzero(s < r2[j])[0].astype(np.int64))
        return out
    tree = cKDTree(points.T)
    for j in range(m):
        cand = np.asarray(tree.query_ball_point(centers[:, j], rv[j] * (1.0 + 1e-6)),
                          dtype=np.int64)
        cand.sort()
        s = sqdist(points[:, cand], centers[:, j])
        out.append(cand[s < r2[j]])
    return out


def design_matrix(points, centers, rho, phi: str, supp: Optional[list] = None) -> sp.csc_matrix:
    """A (N x M, CSC): A_qj = phi(sqrt(s_qj) / rho_j) for q in supp(j) (eq. 4-5)."""
    n = points.shape[1]
    m = centers.shape[1]
    rv = _rho_vec(rho, m)
    if supp is None:
        supp = supports(points, centers, rv)
    indptr = np.zeros(m + 1, dtype=np.int64)
    indptr[1:] = np.cumsum([len(s) for s in supp])
    indices = np.concatenate(supp) if m else np.zeros(0, np.int64)
    data = np.empty(indices.shape[0])
    for j in range(m):
        q = supp[j]
        s = sqdist(points[:, q], centers[:, j])
        data[indptr[j]:indptr[j + 1]] = wendland(phi, np.sqrt(s) / rv[j])
    return sp.csc_matrix((data, indices, indptr), shape=(n, m))


@dataclasses.dataclass
class NormalEquations:
    """Upper-triangular CSR of B = A^T A (active rows/cols only) and g = A^T h."""
    m: int
    support_count: np.ndarray   # int32 [M], n_j
    active: np.ndarray          # bool  [M]
    row_ptr: np.ndarray         # int64 [M+1], upper CSR (diagonal included)
    col: np.ndarray             # int32 [nnz_u], ascending within each row
    val: np.ndarray             # float64 [nnz_u]
    pair_count: np.ndarray      # int64 [nnz_u], points shared by the two supports
    g: np.ndarray               # float64 [M], zero on inactive centres
    lam: float                  # ridge actually added to the diagonal
    A: sp.csc_matrix            # the design matrix itself

    @property
    def nnz_upper(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def nnz_full(self) -> int:
        diag = int(np.sum(self.active))
        return 2 * self.nnz_upper - diag

    def full_matrix(self, with_ridge: bool = True) -> sp.csr_matrix:
        up = sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.m, self.m))
        full = up + sp.triu(up, k=1).T
        if with_ridge and self.lam != 0.0:
            full = full + sp.diags(np.where(self.active, self.lam, 0.0))
        return full.tocsr()


def normal_equations(points, values, centers, rho, phi: str, min_support: int = 1,
                     lambda_rel: float = 0.0, supp: Optional[list] = None) -> NormalEquations:
    """B = A^T A (eq. 11-12, upper triangle as in eq. 13) and g = A^T h."""
    m = centers.shape[1]
    A = design_matrix(points, centers, rho, phi, supp)
    counts = np.diff(A.indptr).astype(np.int32)
    active = counts >= max(1, int(min_support))
    act_idx = np.nonzero(active)[0]
    Aa = A[:, act_idx].tocsc()
    # structural pattern: integer counts of shared points, S^T S with S = pattern(A)
    S = sp.csc_matrix((np.ones_like(Aa.data, dtype=np.int64), Aa.indices, Aa.indptr),
                      shape=Aa.shape)
    shared = sp.triu((S.T @ S).tocsr()).tocsr()
    shared.sort_indices()
    vals = sp.triu((Aa.T @ Aa).tocsr()).tocsr()
    vals.sort_indices()
    # align values to the structural pattern (a product of positive numbers is never 0,
    # but take values by position anyway so a dropped entry would show up as 0)
    val_aligned = np.zeros(shared.nnz)
    for r in range(shared.shape[0]):
        a, b = shared.indptr[r], shared.indptr[r + 1]
        va, vb = vals.indptr[r], vals.indptr[r + 1]
        pos = np.searchsorted(shared.indices[a:b], vals.indices[va:vb])
        val_aligned[a + pos] = vals.data[va:vb]
    # scatter back to the original centre numbering
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    row_len = np.zeros(m, dtype=np.int64)
    row_len[act_idx] = np.diff(shared.indptr)
    row_ptr[1:] = np.cumsum(row_len)
    col = act_idx[shared.indices].astype(np.int32)
    g = np.zeros(m)
    g[act_idx] = Aa.T @ np.asarray(values, dtype=np.float64)
    diag = np.zeros(m)
    full_diag = (Aa.multiply(Aa)).sum(axis=0).A1
    diag[act_idx] = full_diag
    lam = float(lambda_rel) * (float(np.mean(full_diag)) if act_idx.size else 0.0)
    return NormalEquations(m=m, support_count=counts, active=active, row_ptr=row_ptr,
                           col=col, val=val_aligned, pair_count=shared.data.astype(np.int64),
                           g=g, lam=lam, A=A)


# ---------------------------------------------------------------------------
# Direct solve (the paper leaves the solver open; the oracle takes Cholesky)
# ---------------------------------------------------------------------------
def _active_solver(ne: NormalEquations, dense_limit: int):
    """Cholesky of (B + lambda I) on the active set; returns a solve(rhs) function.

    Dense up to ``dense_limit`` active centres, banded above (band taken from
    the pattern in the original centre order).
    """
    act = np.nonzero(ne.active)[0]
    full = ne.full_matrix(with_ridge=True)[act][:, act].tocsr()
    if act.size <= dense_limit:
        cf = sla.cho_factor(full.toarray(), lower=False)
        return lambda rhs: sla.cho_solve(cf, rhs)
    coo = full.tocoo()
    up = coo.col >= coo.row
    bw = int(np.max(coo.col[up] - coo.row[up]))
    ab = np.zeros((bw + 1, act.size))
    ab[bw + coo.row[up] - coo.col[up], coo.col[up]] = coo.data[up]
    cb = sla.cholesky_banded(ab, lower=False, check_finite=False)
    return lambda rhs: sla.cho_solve_banded((cb, False), rhs, check_finite=False)


def solve(ne: NormalEquations, dense_limit: int = 4096) -> np.ndarray:
    """c solving (B + lambda I) c = g on the active set by Cholesky; 0 elsewhere."""
    act = np.nonzero(ne.active)[0]
    c = np.zeros(ne.m)
    if act.size == 0:
        return c
    c[act] = _active_solver(ne, dense_limit)(ne.g[act])
    return c


# ---------------------------------------------------------------------------
# Linear polynomial reproduction (Section 3, eq. 6-10)
# ---------------------------------------------------------------------------
def poly_basis(points) -> np.ndarray:
    """P (N x (d+1)): row i is (x_i^T, 1), the linear polynomial basis of eq. 9."""
    pts = np.asarray(points, dtype=np.float64)
    return np.vstack([pts, np.ones(pts.shape[1])]).T


@dataclasses.dataclass
class PolySystem:
    """The blocks that eq. 10 adds to the normal equations.

    Q = A^T P restricted to active centres (inactive rows are zero), C = P^T P,
    e = P^T h.  The bordered matrix is [[B + lambda I, Q], [Q^T, C]] and the
    unknown vector (c, k) with k = (a, a_0) of eq. 7.
    """
    Q: np.ndarray   # float64 [M][d+1]
    C: np.ndarray   # float64 [d+1][d+1]
    e: np.ndarray   # float64 [d+1]

    def bordered_matrix(self, ne: NormalEquations) -> sp.csr_matrix:
        """The full matrix of eq. 10 over the active centres, ridge included."""
        act = np.nonzero(ne.active)[0]
        B = ne.full_matrix(with_ridge=True)[act][:, act]
        Qa = sp.csr_matrix(self.Q[act])
        return sp.bmat([[B, Qa], [Qa.T, sp.csr_matrix(self.C)]]).tocsr()


def poly_system(ne: NormalEquations, points, values) -> PolySystem:
    """Q = A^T P, C = P^T P and e = P^T h (eq. 10) as plain products."""
    P = poly_basis(points)
    h = np.asarray(values, dtype=np.float64)
    Q = np.zeros((ne.m, P.shape[1]))
    act = np.nonzero(ne.active)[0]
    if act.size:
        Q[act] = ne.A[:, act].T @ P
    return PolySystem(Q=Q, C=P.T @ P, e=P.T @ h)


def solve_poly(ne: NormalEquations, ps: PolySystem, dense_limit: int = 4096):
    """(c, k) solving eq. 10 with the ridge on the A^T A block; c is 0 off the active set.

    Small systems: Cholesky of the whole bordered matrix.  Large ones: the same
    system by block elimination, (B + lambda I) Y = [g, Q] by Cholesky, then the
    (d+1) x (d+1) Schur complement C - Q^T Y_Q for k, and c = Y_g - Y_Q k.
    """
    act = np.nonzero(ne.active)[0]
    nk = ps.C.shape[0]
    c = np.zeros(ne.m)
    if act.size == 0:
        return c, np.linalg.solve(ps.C, ps.e)
    if act.size + nk <= dense_limit:
        K = ps.bordered_matrix(ne).toarray()
        z = sla.cho_solve(sla.cho_factor(K, lower=False), np.concatenate([ne.g[act], ps.e]))
        c[act] = z[:act.size]
        return c, z[act.size:]
    Qa = ps.Q[act]
    Y = _active_solver(ne, dense_limit)(np.column_stack([ne.g[act], Qa]))
    S = ps.C - Qa.T @ Y[:, 1:]
    k = np.linalg.solve(S, ps.e - Qa.T @ Y[:, 0])
    c[act] = Y[:, 0] - Y[:, 1:] @ k
    return c, k


def lstsq_dense_poly(points, values, centers, rho, phi: str, lam: float = 0.0):
    """min ||A c + P k - h||^2 + lam ||c||^2 by dense QR of [A P] (eq. 9, no normal equations)."""
    A = design_matrix(points, centers, rho, phi).toarray()
    P = poly_basis(points)
    m = A.shape[1]
    AP = np.hstack([A, P])
    h = np.asarray(values, dtype=np.float64)
    if lam != 0.0:
        AP = np.vstack([AP, np.hstack([np.sqrt(lam) * np.eye(m), np.zeros((m, P.shape[1]))])])
        h = np.concatenate([h, np.zeros(m)])
    q, r = np.linalg.qr(AP)
    z = sla.solve_triangular(r, q.T @ h)
    return z[:m], z[m:]


def evaluate_poly(queries, centers, rho, phi: str, coeffs, k) -> np.ndarray:
    """f(y) of eq. 6 with the linear polynomial of eq. 7: the RBF sum plus a^T y + a_0."""
    return evaluate(queries, centers, rho, phi, coeffs) + poly_basis(queries) @ np.asarray(k)


def lstsq_dense(points, values, centers, rho, phi: str, lam: float = 0.0) -> np.ndarray:
    """min ||A c - h||^2 + lam ||c||^2 by dense QR (no normal equations)."""
    A = design_matrix(points, centers, rho, phi).toarray()
    h = np.asarray(values, dtype=np.float64)
    if lam != 0.0:
        A = np.vstack([A, np.sqrt(lam) * np.eye(A.shape[1])])
        h = np.concatenate([h, np.zeros(A.shape[1])])
    q, r = np.linalg.qr(A)
    return sla.solve_triangular(r, q.T @ h)


# ---------------------------------------------------------------------------
# Evaluation (eq. 3) and error measures
# ---------------------------------------------------------------------------
def evaluate(queries, centers, rho, phi: str, coeffs, brute_limit: int = 50_000_000) -> np.ndarray:
    """f(y) = sum_j c_j phi(sqrt(s_yj) / rho_j), same strict predicate as the fit."""
    m = centers.shape[1]
    rv = _rho_vec(rho, m)
    r2 = rho_squared(rv)
    nq = queries.shape[1]
    f = np.zeros(nq)
    c = np.asarray(coeffs, dtype=np.float64)
    if nq * m <= brute_limit:
        for j in range(m):
            s = sqdist(queries, centers[:, j])
            hit = s < r2[j]
            f[hit] += c[j] * wendland(phi, np.sqrt(s[hit]) / rv[j])
        return f
    tree = cKDTree(queries.T)
    for j in range(m):
        cand = np.asarray(tree.query_ball_point(centers[:, j], rv[j] * (1.0 + 1e-6)),
                          dtype=np.int64)
        if cand.size == 0:
            continue
        s = sqdist(queries[:, cand], centers[:, j])
        hit = s < r2[j]
        f[cand[hit]] += c[j] * wendland(phi, np.sqrt(s[hit]) / rv[j])
    return f


def evaluate_one(query, centers, rho, phi: str, coeffs) -> float:
    """f at a single point, summed over centres in increasing index.

    (xi - y)^2 equals (y - xi)^2 exactly (negation is exact), so the canonical
    squared distance may take the centres as the moving operand.
    """
    m = centers.shape[1]
    rv = _rho_vec(rho, m)
    s = sqdist(centers, np.asarray(query, dtype=np.float64))
    hit = np.nonzero(s < rho_squared(rv))[0]
    return float(np.sum(np.asarray(coeffs)[hit] * wendland(phi, np.sqrt(s[hit]) / rv[hit])))


def rmse(f, h) -> float:
    d = np.asarray(f, dtype=np.float64) - np.asarray(h, dtype=np.float64)
    return float(np.sqrt(np.mean(d * d))) if d.size else 0.0


# ---------------------------------------------------------------------------
# One row of B recomputed on its own (for checks at sizes where B is too big)
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Row:
    j: int
    support: np.ndarray       # ascending point indices in supp(j)
    cols: np.ndarray          # ascending upper columns l >= j
    vals: np.ndarray          # b_jl, each summed over points in increasing index
    pair_count: np.ndarray
    g: float                  # g_j = sum_q phi_qj h_q


def sample_row(points, values, centers, rho, phi: str, j: int, lower: bool = False) -> Row:
    """Row j of the pattern and values of B, plus g_j, straight from eq. 12.

    Columns l >= j (the stored upper triangle), or every column when ``lower``.
    Active set is taken as min_support = 1: a column l that shares a point with
    row j has a nonempty support, so every column found here is active.
    """
    m = centers.shape[1]
    rv = _rho_vec(rho, m)
    r2 = rho_squared(rv)
    sj = sqdist(points, centers[:, j])
    q = np.nonzero(sj < r2[j])[0]
    phij = wendland(phi, np.sqrt(sj[q]) / rv[j])
    g = float(np.sum(phij * np.asarray(values)[q]))
    if q.size == 0:
        return Row(j, q, np.zeros(0, np.int32), np.zeros(0), np.zeros(0, np.int64), 0.0)
    # any column sharing a point lies within rho_j + rho_l of centre j
    cdist2 = sqdist(centers, centers[:, j])
    reach = (rv[j] + rv) * (1.0 + 1e-6)
    cand = np.nonzero((cdist2 <= reach * reach) & ((np.arange(m) >= j) | lower))[0]
    pts = points[:, q]
    cols, vals, cnt = [], [], []
    for l in cand:
        sl = sqdist(pts, centers[:, l])
        hit = sl < r2[l]
        if np.any(hit):
            cols.append(l)
            vals.append(float(np.sum(phij[hit] * wendland(phi, np.sqrt(sl[hit]) / rv[l]))))
            cnt.append(int(np.sum(hit)))
    return Row(j, q, np.asarray(cols, np.int32), np.asarray(vals), np.asarray(cnt, np.int64), g)


# ---------------------------------------------------------------------------
# COO sparse product (Section 4)
# ---------------------------------------------------------------------------
def coo_spmv(n_rows: int, row: Sequence[int], col: Sequence[int], data, x) -> np.ndarray:
    """y = Q x for Q in coordinate format: y[row[i]] += data[i] * x[col[i]]."""
    y = np.zeros(n_rows, dtype=np.result_type(np.asarray(data), np.asarray(x)))
    for i in range(len(data)):
        y[row[i]] = y[row[i]] + data[i] * x[col[i]]
    return y


def coo_to_csr(n_rows: int, row, col, data):
    """Row pointer, column and value arrays of the same matrix, columns ascending."""
    row = np.asarray(row, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    data = np.asarray(data)
    order = np.lexsort((col, row))
    ptr = np.zeros(n_rows + 1, dtype=np.int64)
    np.add.at(ptr, row + 1, 1)
    return np.cumsum(ptr), col[order], data[order]
