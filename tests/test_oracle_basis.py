"""Pins of the oracle's Wendland basis (Table 2, eq. 18) against mathematics.

None of these tests retypes the closed forms: they check what the table's
caption states about the functions (compact support, polynomial degree,
smoothness, positive definiteness up to dimension 3) and Wendland's
construction of phi_{d,s} by repeated integration of a truncated power.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import rbf_oracle as orc

S_OF = {"w30": 0, "w31": 1, "w32": 2, "w33": 3}


@pytest.mark.parametrize("kind", orc.PHI_KINDS)
def test_compact_support(kind):
    r = np.array([1.0, 1.0 + 1e-12, 1.5, 3.0, 100.0])
    assert np.all(orc.wendland(kind, r) == 0.0)
    inside = np.linspace(0.0, 1.0 - 1e-9, 257)
    assert np.all(orc.wendland(kind, inside) > 0.0)


@pytest.mark.parametrize("kind", orc.PHI_KINDS)
def test_polynomial_degree(kind):
    # Table 2 caption: degree floor(d/2) + 3s + 1 with d = 3
    s = S_OF[kind]
    deg = 1 + 3 * s + 1
    r = np.linspace(0.0, 1.0, 200)
    y = orc.wendland(kind, r)
    fit = np.polynomial.polynomial.Polynomial.fit(r, y, deg)
    assert np.max(np.abs(fit(r) - y)) < 1e-10 * max(1.0, np.max(y))
    low = np.polynomial.polynomial.Polynomial.fit(r, y, deg - 1)
    assert np.max(np.abs(low(r) - y)) > 1e-6 * np.max(y)


def _wendland_by_integration(s: int, r: float, d: int = 3) -> float:
    """Wendland's construction: phi_{d,s} = I^s (1-t)^l_+ with l = floor(d/2)+s+1,
    (I f)(r) = int_r^1 t f(t) dt, evaluated by nested numerical quadrature."""
    ell = d // 2 + s + 1

    def base(t):
        return (1.0 - t) ** ell if t < 1.0 else 0.0

    f = base
    for _ in range(s):
        prev = f

        def f(x, prev=prev):
            return integrate.quad(lambda t: t * prev(t), x, 1.0, epsabs=1e-14, epsrel=1e-12)[0]
    return f(r)


@pytest.mark.parametrize("kind", ["w30", "w31", "w32"])
def test_matches_wendland_construction(kind):
    """Up to a positive constant, the table's form equals the integral construction."""
    s = S_OF[kind]
    rs = [0.0, 0.2, 0.45, 0.7, 0.9]
    ref = np.array([_wendland_by_integration(s, r) for r in rs])
    got = orc.wendland(kind, np.array(rs))
    ratio = got / ref
    assert np.all(ratio > 0)
    assert np.allclose(ratio, ratio[0], rtol=1e-7, atol=0)


def test_w33_matches_wendland_construction():
    # three nested quadratures are slow; fewer sample points
    rs = [0.1, 0.5, 0.8]
    ref = np.array([_wendland_by_integration(3, r) for r in rs])
    got = orc.wendland("w33", np.array(rs))
    ratio = got / ref
    assert np.allclose(ratio, ratio[0], rtol=1e-6, atol=0)


@pytest.mark.parametrize("kind", ["w31", "w32", "w33"])
def test_smooth_at_origin(kind):
    # C^{2s} radial smoothness needs phi'(0) = 0 for s >= 1
    h = 1e-6
    d = (orc.wendland(kind, h) - orc.wendland(kind, 0.0)) / h
    assert abs(d) < 1e-4 * orc.wendland(kind, 0.0)


@pytest.mark.parametrize("kind", orc.PHI_KINDS)
def test_smoothness_at_support_edge(kind):
    # phi has a zero of order l+s = 2s+2 (+1 for d=3 rounding) at r = 1: derivatives up to 2s
    # vanish there, so phi is C^{2s} across the edge of its support
    s = S_OF[kind]
    p = np.polynomial.polynomial.Polynomial.fit(np.linspace(0, 1, 400),
                                                orc.wendland(kind, np.linspace(0, 1, 400)),
                                                1 + 3 * s + 1)
    for k in range(0, 2 * s + 1):
        assert abs(p.deriv(k)(1.0)) < 1e-6 * max(1.0, abs(p.deriv(k)(0.0)))


@pytest.mark.parametrize("kind", orc.PHI_KINDS)
def test_positive_definite_in_3d(kind):
    # Table 2 caption: positive definite up to dimension d = 3
    rng = np.random.default_rng(7)
    x = rng.random((3, 120))
    rho = 0.6
    K = np.empty((120, 120))
    for j in range(120):
        K[:, j] = orc.wendland(kind, np.sqrt(orc.sqdist(x, x[:, j])) / rho)
    assert np.allclose(K, K.T)
    assert np.linalg.eigvalsh(K).min() > 0


def test_w31_sign_error_would_break_pd():
    # sanity of the PD pin: a plausible typo (4r - 1 instead of 4r + 1) is not PD
    rng = np.random.default_rng(3)
    x = rng.random((3, 150))
    rho = 0.6
    K = np.empty((150, 150))
    for j in range(150):
        r = np.sqrt(orc.sqdist(x, x[:, j])) / rho
        K[:, j] = np.where(r < 1, (1 - r) ** 4 * (4 * r - 1), 0.0)
    assert np.linalg.eigvalsh(K).min() < 0
