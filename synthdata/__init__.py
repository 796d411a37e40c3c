"""Seeded synthetic inputs for the CS-RBF fit: point clouds, sampled values, grids.

This module only *draws inputs*: it holds none of the approximation method's
arithmetic (no basis function, no distance predicate, no system assembly), so
both the CPU oracle and the HIP path may take their inputs from it.

The paper measures on real LiDAR terrain (Serpent Mound, Mount St. Helens;
Section 6, Table 1) and on Franke's function sampled at Halton points
(Section 6, eq. 17).  The LiDAR sets are not available, so the generators
below stand in for them with terrain-like synthetic clouds of the same
character: clustered, anisotropic, scanline-thinned point densities carrying a
fractal height field.

All randomness comes from ``numpy.random.Generator(PCG64)`` streams spawned
from one ``SeedSequence(seed)``, so a (recipe, seed) pair fixes every byte.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = [
    "streams", "uniform_points", "gaussian_mixture_points", "franke",
    "terrain_modes", "terrain_values", "grid_centers", "heldout_split",
    "Problem", "make_problem", "CONFIGS", "support_radius_for_k", "scoring_queries",
    "halton_points",
]


def streams(seed: int, n: int) -> list[np.random.Generator]:
    """``n`` independent PCG64 generators spawned from ``SeedSequence(seed)``."""
    return [np.random.Generator(np.random.PCG64(s))
            for s in np.random.SeedSequence(seed).spawn(n)]


def uniform_points(rng: np.random.Generator, n: int, dim: int) -> np.ndarray:
    """``n`` points uniform in [0,1]^dim, returned SoA as ``(dim, n)`` float64."""
    return np.ascontiguousarray(rng.random((dim, n)))


def _random_rotation(rng: np.random.Generator, dim: int) -> np.ndarray:
    if dim == 2:
        t = rng.uniform(0.0, 2.0 * math.pi)
        return np.array([[math.cos(t), -math.sin(t)], [math.sin(t), math.cos(t)]])
    q, r = np.linalg.qr(rng.standard_normal((dim, dim)))
    return q * np.sign(np.diag(r))


def gaussian_mixture_points(rng: np.random.Generator, n: int, dim: int,
                            n_clusters: int, scanlines: bool = True) -> np.ndarray:
    """Clustered, scanline-like cloud in [0,1]^dim, SoA ``(dim, n)`` float64.

    Recipe: ``n_clusters`` Gaussians with means U[0.05,0.95]^dim; major standard
    deviation log-uniform in [0.01, 0.1]; every minor axis shorter by a
    log-uniform factor in [1, 16] (elongated strips); random orientation;
    mixture weights Dirichlet(1).  Samples outside the unit cube are rejected.
    With ``scanlines`` the density is striped like airborne LiDAR swaths: a
    point whose ``frac(512 * x_last)`` is >= 0.5 is kept with probability 0.25.
    """
    means = rng.uniform(0.05, 0.95, size=(n_clusters, dim))
    major = np.exp(rng.uniform(math.log(0.01), math.log(0.1), size=n_clusters))
    aspect = np.exp(rng.uniform(0.0, math.log(16.0), size=(n_clusters, dim - 1)))
    rot = [_random_rotation(rng, dim) for _ in range(n_clusters)]
    weights = rng.dirichlet(np.ones(n_clusters))
    out = np.empty((dim, n))
    filled = 0
    while filled < n:
        batch = max(1024, int(1.3 * (n - filled)) * (3 if scanlines else 1))
        comp = rng.choice(n_clusters, size=batch, p=weights)
        z = rng.standard_normal((batch, dim))
        sig = np.empty((n_clusters, dim))
        sig[:, 0] = major
        sig[:, 1:] = major[:, None] / aspect
        # group the batch by component once (a stable sort keeps each group in
        # draw order), transform every group as one contiguous slice, scatter back
        key = comp.astype(np.uint8) if n_clusters <= 256 else comp
        order = np.argsort(key, kind="stable")
        ends = np.cumsum(np.bincount(comp, minlength=n_clusters))
        zs = z[order]
        ps = np.empty((batch, dim))
        start = 0
        for c in range(n_clusters):
            if ends[c] > start:
                ps[start:ends[c]] = (zs[start:ends[c]] * sig[c]) @ rot[c].T + means[c]
            start = ends[c]
        pts = np.empty((batch, dim))
        pts[order] = ps
        keep = np.all((pts >= 0.0) & (pts <= 1.0), axis=1)
        if scanlines:
            stripe = np.mod(pts[:, -1] * 512.0, 1.0) >= 0.5
            keep &= ~stripe | (rng.random(batch) < 0.25)
        pts = pts[keep]
        take = min(n - filled, pts.shape[0])
        out[:, filled:filled + take] = pts[:take].T
        filled += take
    return np.ascontiguousarray(out)


def franke(p: np.ndarray) -> np.ndarray:
    """Franke's test function exactly as printed in the paper (Section 6, eq. 17).

    Note the second exponent: the printed form squares ``(9 x2 + 1)`` and
    divides by 10, which differs from the textbook linear term; the relief
    the paper lists for its synthetic set (Table 1, 1.238) matches the printed
    form, so that form is used.  ``p`` is SoA ``(2, n)``.
    """
    x1, x2 = p[0], p[1]
    f1 = 0.75 * np.exp(-((9 * x1 - 2) ** 2) / 4 - ((9 * x2 - 2) ** 2) / 4)
    f2 = 0.75 * np.exp(-((9 * x1 + 1) ** 2) / 49 - ((9 * x2 + 1) ** 2) / 10)
    f3 = 0.50 * np.exp(-((9 * x1 - 7) ** 2) / 4 - ((9 * x2 - 3) ** 2) / 4)
    f4 = 0.20 * np.exp(-((9 * x1 - 4) ** 2) - ((9 * x2 - 7) ** 2))
    return f1 + f2 + f3 - f4


def halton_points(n: int, dim: int = 2, bases=(2, 3, 5)) -> np.ndarray:
    """The first ``n`` Halton points in [0,1]^dim (radical inverses of 1..n in
    the first ``dim`` primes), SoA ``(dim, n)``: the point set of the paper's
    synthetic experiment (Section 6, Table 1: 1089 Halton points).  The start
    index is not printed; 1 is taken."""
    out = np.empty((dim, n))
    for d in range(dim):
        b = bases[d]
        for i in range(n):
            f, r, k = 1.0, 0.0, i + 1
            while k > 0:
                f /= b
                r += f * (k % b)
                k //= b
            out[d, i] = r
    return out


@dataclasses.dataclass
class TerrainModes:
    wavevec: np.ndarray   # (n_modes, dim)
    amp: np.ndarray       # (n_modes,)
    phase: np.ndarray     # (n_modes,)


def terrain_modes(rng: np.random.Generator, n_modes: int, dim: int,
                  kmin: float = 1.0, kmax: float = 64.0) -> TerrainModes:
    """Random Fourier modes of a fractal height field.

    |k| log-uniform in [kmin, kmax], direction uniform, phase U[0, 2 pi),
    amplitude |k|^-2 (a k^-2 spectrum, rough like terrain).
    """
    kmag = np.exp(rng.uniform(math.log(kmin), math.log(kmax), size=n_modes))
    d = rng.standard_normal((n_modes, dim))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    phase = rng.uniform(0.0, 2.0 * math.pi, size=n_modes)
    return TerrainModes(wavevec=d * kmag[:, None], amp=kmag ** -2.0, phase=phase)


def terrain_values(modes: TerrainModes, p: np.ndarray, chunk: int = 1 << 16) -> np.ndarray:
    """h(x) = sum_m amp_m cos(2 pi k_m . x + phase_m) at SoA points ``p``.

    Chunks are independent and run on a thread pool (NumPy releases the GIL
    in these loops); every chunk does the same operations whatever the pool
    size, so the result does not depend on the thread count.
    """
    import concurrent.futures as cf
    import os
    n = p.shape[1]
    out = np.empty(n)
    two_pi_k = 2.0 * math.pi * modes.wavevec          # (m, dim)

    def run(s):
        arg = two_pi_k @ p[:, s:s + chunk] + modes.phase[:, None]
        out[s:s + chunk] = modes.amp @ np.cos(arg)

    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    with cf.ThreadPoolExecutor(workers) as ex:
        list(ex.map(run, range(0, n, chunk)))
    return out


def grid_centers(g: int, dim: int) -> np.ndarray:
    """Regular g^dim grid of reference points at i/(g-1), boundaries included.

    Index order is row-major with the first coordinate fastest, returned SoA
    ``(dim, g^dim)`` float64.
    """
    t = np.arange(g, dtype=np.float64) / (g - 1)
    mesh = np.meshgrid(*([t] * dim), indexing="ij")
    # first coordinate fastest: transpose axes so that axis order is (x_dim-1, ..., x_0)
    cols = [m.transpose(tuple(range(dim))[::-1]).reshape(-1) for m in mesh]
    return np.ascontiguousarray(np.stack(cols))


def support_radius_for_k(g: int, dim: int, k: float) -> float:
    """Radius whose ball covers ``k`` grid centres on average (spacing 1/(g-1))."""
    delta = 1.0 / (g - 1)
    if dim == 2:
        return delta * math.sqrt(k / math.pi)
    return delta * (3.0 * k / (4.0 * math.pi)) ** (1.0 / 3.0)


def heldout_split(rng: np.random.Generator, n: int, frac: float):
    """Seeded permutation split: (train_idx, test_idx), both sorted ascending."""
    n_test = int(round(frac * n))
    perm = rng.permutation(n)
    return np.sort(perm[n_test:]), np.sort(perm[:n_test])


@dataclasses.dataclass
class Problem:
    name: str
    dim: int
    points: np.ndarray        # (dim, n_train) SoA float64, training points
    values: np.ndarray        # (n_train,) noisy samples
    test_points: np.ndarray   # (dim, n_test)
    test_values: np.ndarray   # (n_test,) noisy samples at held-out points
    test_clean: np.ndarray    # (n_test,) noise-free field at held-out points
    centers: np.ndarray       # (dim, M) SoA float64
    rho: float
    phi: str                  # "w30" | "w31" | "w32" | "w33"
    grid: int
    modes: Optional[TerrainModes] = None   # the terrain field's modes (clean values anywhere)
    score: str = "heldout"    # "heldout": held-out points vs noisy samples;
                              # "uniform": uniform queries vs the noise-free field


# The five workloads (sizes, densities, fields, basis and radius).  A radius
# "covering ~40 centres" is the ball holding 40 grid centres on average.
CONFIGS = {
    "franke2d": dict(dim=2, n=10_000, cloud="uniform", field="franke", noise=0.01,
                     grid=32, phi="w31", rho=0.12, holdout=0.0, seed=1),
    "terrain2d": dict(dim=2, n=1 << 20, cloud="mixture", clusters=64, field="terrain",
                      modes=256, noise=1e-3, grid=256, phi="w31", k_cover=40.0,
                      holdout=0.01, seed=2),
    "terrain2d_big": dict(dim=2, n=1 << 24, cloud="mixture", clusters=64, field="terrain",
                          modes=256, noise=1e-3, grid=1024, phi="w32", k_cover=40.0,
                          holdout=0.01, seed=3),
    "field3d": dict(dim=3, n=1 << 22, cloud="mixture", clusters=32, field="terrain",
                    modes=128, noise=1e-3, grid=64, phi="w31", k_cover=40.0,
                    holdout=0.01, seed=5, score="uniform"),
}


def make_problem(name: str, scale: float = 1.0, seed: Optional[int] = None,
                 **override) -> Problem:
    """Build one named workload.  ``scale`` shrinks N and the grid together
    (N by ``scale``, grid side by ``scale ** (1/dim)``) for quick tests while
    keeping the points-per-centre ratio and the radius in grid units."""
    cfg = dict(CONFIGS[name])
    cfg.update(override)
    dim = cfg["dim"]
    seed = cfg["seed"] if seed is None else seed
    r_cloud, r_field, r_noise, r_split, r_noise_t = streams(seed, 5)
    n_total = max(16, int(round(cfg["n"] * scale)))
    g = max(4, int(round(cfg["grid"] * scale ** (1.0 / dim))))
    if cfg["cloud"] == "uniform":
        pts = uniform_points(r_cloud, n_total, dim)
    else:
        pts = gaussian_mixture_points(r_cloud, n_total, dim, cfg["clusters"])
    modes = None
    if cfg["field"] == "franke":
        clean = franke(pts)
    else:
        modes = terrain_modes(r_field, cfg["modes"], dim)
        clean = terrain_values(modes, pts)
    noisy = clean + cfg["noise"] * r_noise.standard_normal(n_total)
    if cfg["holdout"] > 0:
        tr, te = heldout_split(r_split, n_total, cfg["holdout"])
    else:
        tr, te = np.arange(n_total), np.arange(0)
    if "rho" in cfg and cfg.get("rho") is not None and scale == 1.0:
        rho = float(cfg["rho"])
    elif "rho" in cfg and cfg.get("rho") is not None:
        rho = float(cfg["rho"]) * (cfg["grid"] - 1) / (g - 1)
    else:
        rho = support_radius_for_k(g, dim, cfg["k_cover"])
    return Problem(
        name=name, dim=dim,
        points=np.ascontiguousarray(pts[:, tr]), values=np.ascontiguousarray(noisy[tr]),
        test_points=np.ascontiguousarray(pts[:, te]),
        test_values=np.ascontiguousarray(noisy[te]),
        test_clean=np.ascontiguousarray(clean[te]),
        centers=grid_centers(g, dim), rho=rho, phi=cfg["phi"], grid=g, modes=modes,
        score=cfg.get("score", "heldout"))


def scoring_queries(prob: Problem, n: int = 1_000_000, seed: Optional[int] = None):
    """Points at which a fit of ``prob`` is scored, with the values to score against.

    A workload scored on held-out points is scored there against the noisy
    samples.  The 3D field (and any workload without held-out points) is
    scored at ``n`` points uniform in the unit cube against the noise-free
    field; the stream is seeded by ``1000 + dim`` unless ``seed`` is given.
    Its held-out points (``prob.test_points``) are a second score.
    """
    if prob.score == "heldout" and prob.test_points.shape[1] > 0:
        return prob.test_points, prob.test_values
    if prob.modes is None:
        raise ValueError("workload has neither held-out points nor a terrain field")
    rng = streams(1000 + prob.dim if seed is None else seed, 1)[0]
    q = uniform_points(rng, n, prob.dim)
    return q, terrain_values(prob.modes, q)
