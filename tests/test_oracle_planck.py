"""Pins of the oracle's Planck group integrals (Section 2, group emission).

Every check here compares against something other than the oracle's own
quadrature: values the paper prints, closed forms, and textbook limits.
"""
import math

import numpy as np
import pytest

from oracle import planck

# cgs constants, used only to restate the paper's thermal-relaxation setup
H_CGS = 6.62607015e-27
KB_CGS = 1.380649e-16


def _fraction_table(edges_x):
    """Fraction of the Planck integral in [x_a, x_b) for consecutive x edges."""
    tot = math.pi ** 4 / 15.0
    return np.array([planck.planck_integral(edges_x[i], edges_x[i + 1]) / tot
                     for i in range(len(edges_x) - 1)])


def test_gray_sum_closed_form():
    # summing every group covers [0, inf): 2 pi^4 T^4 / 15 (gray limit, Section 2)
    for T in (0.1, 1.0, 2.5):
        for edges in (np.array([0.0, 0.5, 1.3, 7.0, np.inf]),
                      np.concatenate([[0.0], np.geomspace(0.01, 10, 7), [np.inf]])):
            s = planck.group_emission(edges, T).sum()
            assert s == pytest.approx(planck.gray_emission(T), rel=1e-13)


def test_equilibrium_temperature_reading():
    # Thermal relaxation test: rho c_v T + a T^4 conserved with c_v = 8, T = 10,
    # T_r = 1, a = c = 1; the paper prints T_eq ~ 2.77.
    f = lambda T: 8.0 * T + T ** 4 - (8.0 * 10.0 + 1.0)
    lo, hi = 0.0, 10.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if f(mid) < 0 else (lo, mid)
    assert round(lo, 2) == 2.77


def test_paper_relaxation_group_fractions():
    # Thermal relaxation, N_nu = 3 with nu_1 = k, nu_2 = 2k, k = 1.5e11 (cgs).
    # The paper prints the equilibrium fractions E_f / (a T_eq^4) = 0.31, 0.47, 0.22.
    f = lambda T: 8.0 * T + T ** 4 - 81.0
    lo, hi = 0.0, 10.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if f(mid) < 0 else (lo, mid)
    T_eq = lo
    k = 1.5e11
    x = [0.0, H_CGS * k / (KB_CGS * T_eq), H_CGS * 2 * k / (KB_CGS * T_eq), np.inf]
    fr = _fraction_table(x)
    np.testing.assert_allclose(fr, [0.31, 0.47, 0.22], atol=0.006)
    assert fr.sum() == pytest.approx(1.0, abs=1e-14)


def test_rayleigh_jeans_series():
    # small x: int_0^x t^3/(e^t-1) dt = x^3/3 - x^4/8 + x^5/60 - x^7/5040 + ...
    for x in (1e-3, 1e-2):
        ref = x ** 3 / 3 - x ** 4 / 8 + x ** 5 / 60 - x ** 7 / 5040
        assert planck.planck_integral(0.0, x) == pytest.approx(ref, rel=1e-12)


def test_wien_tail_closed_form():
    # large x: int_x^inf t^3 e^{-t} dt = e^{-x}(x^3 + 3x^2 + 6x + 6); the Bose
    # correction sum_{k>=2} is O(e^{-2x}), far below double precision at x = 60
    for x in (40.0, 60.0, 105.0, 333.0, 650.0):
        ref = math.exp(-x) * (x ** 3 + 3 * x ** 2 + 6 * x + 6)
        assert planck.planck_integral(x, math.inf) == pytest.approx(ref, rel=1e-14)
    # a finite group far in the tail: difference of the two closed-form tails
    a, b = 105.0, 333.0
    ref = (math.exp(-a) * (a ** 3 + 3 * a ** 2 + 6 * a + 6) - math.exp(-b) * (b ** 3 + 3 * b ** 2 + 6 * b + 6))
    assert planck.planck_integral(a, b) == pytest.approx(ref, rel=1e-14)


def test_zero_temperature_and_homogeneity():
    edges = np.array([0.0, 0.3, 1.0, 4.0, np.inf])
    assert np.all(planck.group_emission(edges, 0.0) == 0.0)
    # eps_g(s T) on edges s*nu equals s^4 eps_g(T): x = nu/T is scale free
    e1 = planck.group_emission(edges, 0.7)
    e2 = planck.group_emission(edges * 3.0, 2.1)
    np.testing.assert_allclose(e2, 81.0 * e1, rtol=1e-13)
