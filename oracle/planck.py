"""Planck group emission coefficients by adaptive high-precision quadrature.

TEST INFRASTRUCTURE ONLY (part of the CPU oracle; never called by the GPU
path).

Section 2, the group emission coefficient: eps_f = (c / 4 pi) times the
integral of the Planck function B(nu, T) = 8 pi h nu^3 / c^3 / (exp(h nu / k T) - 1)
over the group [nu_{f-1}, nu_f).  In units with h = k = c = 1 this is

    eps_f(T) = 2 T^4  int_{nu_{f-1}/T}^{nu_f/T}  x^3 / (e^x - 1) dx,

and the gray sum over all groups is 2 pi^4 T^4 / 15 = c a T^4 / (4 pi) with
a = 8 pi^5 / 15 (the gray limit stated right after the Planck function).

The integral is evaluated with mpmath's tanh-sinh quadrature at 60 digits,
an implementation independent of the library's series evaluation.
`group_emission_quad` evaluates the same integrals in double precision with
QUADPACK (scipy.integrate.quad); it serves the coupled-temperature oracle,
which needs many evaluations at varying T.
"""
from __future__ import annotations

import functools
import math

import mpmath
import numpy as np
from scipy import integrate

_DPS = 60


def _shifted_integrand(a):
    """u -> (a+u)^3 e^{-u} / (1 - e^{-(a+u)}), so that
    int_a^b x^3/(e^x - 1) dx = e^{-a} int_0^{b-a} (this) du.  Factoring e^{-a}
    out keeps the integrand O(1) wherever the group sits, which matters
    because the quadrature's error control is absolute."""
    def f(u):
        x = a + u
        if x == 0:
            return mpmath.mpf(0)
        return x ** 3 * mpmath.exp(-u) / (-mpmath.expm1(-x))
    return f


@functools.lru_cache(maxsize=None)
def planck_integral(xa: float, xb: float) -> float:
    """int_{xa}^{xb} x^3/(e^x - 1) dx for 0 <= xa < xb <= inf (float in, float out)."""
    with mpmath.workdps(_DPS):
        a = mpmath.mpf(xa)
        w = mpmath.inf if math.isinf(xb) else mpmath.mpf(xb) - a
        if not (w > 0):
            return 0.0
        # split where the shifted integrand changes character (unit-scale decay
        # in u, and the Rayleigh-Jeans / Wien crossover near x ~ 1..10)
        cuts = {mpmath.mpf(d) for d in (0.25, 0.5, 1, 2, 4, 8, 16, 32, 64, 128)}
        cuts |= {mpmath.mpf(s) - a for s in (1, 3, 10, 30)}
        pts = [mpmath.mpf(0)] + sorted(c for c in cuts if 0 < c < w) + [w]
        val = mpmath.exp(-a) * mpmath.quad(_shifted_integrand(a), pts)
        return float(val)


def group_emission(edges, T: float) -> np.ndarray:
    """eps_g(T) for every group, h = k = c = 1 (Section 2, group emission)."""
    edges = np.asarray(edges, dtype=float)
    G = len(edges) - 1
    out = np.zeros(G)
    if T <= 0.0:
        return out
    for g in range(G):
        xa = edges[g] / T
        xb = edges[g + 1] / T
        out[g] = 2.0 * T ** 4 * planck_integral(float(xa), float(xb))
    return out


def emission_field(edges, T_cell) -> np.ndarray:
    """(N_X, N_nu) emission coefficients for a per-cell temperature field."""
    T_cell = np.asarray(T_cell, dtype=float)
    uniq, inv = np.unique(T_cell, return_inverse=True)
    table = np.stack([group_emission(edges, float(t)) for t in uniq])
    return table[inv]


def gray_emission(T: float) -> float:
    """Sum over all groups: 2 pi^4 T^4 / 15 (the single-group limit)."""
    return 2.0 * math.pi ** 4 * T ** 4 / 15.0


def _x3_over_expm1(x: float) -> float:
    """x^3 / (e^x - 1), written as x^3 e^{-x} / (1 - e^{-x}) (no overflow)."""
    if x == 0.0:
        return 0.0
    return x ** 3 * math.exp(-x) / -math.expm1(-x)


def group_emission_quad(edges, T: float) -> np.ndarray:
    """eps_g(T) for every group by double-precision adaptive quadrature
    (QUADPACK), h = k = c = 1; the integrand x^3 / (e^x - 1) is integrated
    over each group's [nu_{g-1} / T, nu_g / T), split at x = 1, 4, 16, 64
    and cut at x = 800 (beyond which it underflows)."""
    edges = np.asarray(edges, dtype=float)
    G = len(edges) - 1
    out = np.zeros(G)
    if T <= 0.0:
        return out
    for g in range(G):
        xa = edges[g] / T
        xb = min(edges[g + 1] / T, 800.0)
        if not xb > xa:
            continue
        pts = [xa] + [c for c in (1.0, 4.0, 16.0, 64.0) if xa < c < xb] + [xb]
        tot = 0.0
        for lo, hi in zip(pts[:-1], pts[1:]):
            tot += integrate.quad(_x3_over_expm1, lo, hi, epsabs=0.0, epsrel=1e-13, limit=200)[0]
        out[g] = 2.0 * T ** 4 * tot
    return out
