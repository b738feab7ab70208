"""Pins of the coupled-temperature oracle (Section 2.1, the coupled source
stage; Section 4, thermal relaxation).  CPU only."""
import math
import os

import numpy as np
import pytest

import tt_inputs as ti
from oracle import dense, planck

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "thermal_relax_3group.txt")


def _golden():
    vals = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        k, *v = line.split()
        vals[k] = [float(x) for x in v]
    return vals


def test_quadpack_planck_matches_mpmath():
    rng = np.random.default_rng(3)
    edges = np.concatenate([[0.0], np.sort(rng.uniform(0.005, 40.0, 9)), [np.inf]])
    for T in (0.02, 0.1, 0.7, 2.77, 10.0, 55.0):
        a = planck.group_emission(edges, T)
        b = planck.group_emission_quad(edges, T)
        big = a > 1e-250
        assert np.allclose(b[big], a[big], rtol=2e-13, atol=0.0), T
        assert np.all(np.abs(b[~big]) < 1e-200)


def _cell_problem(edges, kappas, C, T=1.0):
    p = ti.thermal_relax(n_cells=1)
    return p.copy(edges=np.asarray(edges, float), kappa_scale=np.asarray(kappas, float), heat_capacity=C,
                  T_cell=np.array([T]))


def test_gray_stage_temperature_is_quartic_root():
    # one group [0, inf): eps = 2 pi^4 T^4 / 15, so the stage equation is a
    # quartic in T+ once J^{m+1}(T+) is substituted
    for (T_m, J, kap, C) in ((10.0, 0.001, 10.0, 1305.7), (0.3, 5.0, 0.5, 2.0), (2.0, 2.0, 100.0, 1e-2)):
        p = _cell_problem([0.0, np.inf], [kap], C, T_m)
        dt = dense.time_step(p)
        cdt = p.c * dt
        d = 1.0 / (1.0 + cdt * kap)
        coef = 4.0 * math.pi * dt * kap * d / C
        s = 2.0 * math.pi ** 4 / 15.0
        roots = np.roots([-coef * s, 0.0, 0.0, -1.0, T_m + coef * J])
        real = [r.real for r in roots if abs(r.imag) < 1e-9 * abs(r) and r.real > 0]
        assert len(real) == 1
        Tp = dense.stage_temperature(p, T_m, np.array([J]), np.array([kap]), dt)
        assert Tp == pytest.approx(real[0], rel=1e-13)


def _periodic_problem(n_cells=6, C=3.0):
    p = ti.thermal_relax(n_cells=n_cells, n_theta=4)
    rng = np.random.default_rng(7)
    edges = np.array([0.0, 0.3, 1.2, 4.0, np.inf])
    return p.copy(edges=edges, kappa_scale=np.array([5.0, 1.0, 0.2, 0.05]), kappa0=rng.uniform(0.5, 2.0, n_cells),
                  T_cell=rng.uniform(0.3, 2.0, n_cells), T_rad0=rng.uniform(0.2, 1.5, n_cells), heat_capacity=C,
                  cfl=0.4)


def test_large_heat_capacity_reduces_to_fixed_temperature():
    p = _periodic_problem(C=1e16)
    I = dense.initial_dense(p)
    Is = dense.transport(p, I)
    I_new, T_new = dense.coupled_source(p, Is, p.T_cell)
    ref = dense.source(p, Is)
    assert np.allclose(I_new, ref, rtol=1e-12, atol=0.0)
    assert np.allclose(T_new, p.T_cell, rtol=1e-12, atol=0.0)


def test_energy_conserved_and_new_temperature_is_stage_root():
    # periodic medium: streaming moves energy between cells only, the source
    # stage exchanges it between radiation and medium; and without rounding the
    # energy-conserving update gives back the stage root itself
    p = _periodic_problem()
    I = dense.initial_dense(p)
    T = p.T_cell.copy()
    U0 = dense.total_energy(p, I, T)
    dt = dense.time_step(p)
    kap = dense.kappa_field(p)
    for _ in range(5):
        Is = dense.transport(p, I)
        Js = dense.mean_intensity(p, Is)
        roots = np.array([dense.stage_temperature(p, float(T[x]), Js[x], kap[x], dt) for x in range(p.n_x)])
        I, T = dense.coupled_source(p, Is, T)
        assert np.allclose(T, roots, rtol=1e-12, atol=0.0)
        assert dense.total_energy(p, I, T) == pytest.approx(U0, rel=1e-13)
    assert not np.allclose(T, p.T_cell)


def test_thermal_relaxation_reaches_printed_equilibrium():
    gold = _golden()
    p = ti.thermal_relax(n_cells=1, t_final=80.0)
    I, T = dense.march_coupled(p, dense.initial_dense(p), p.T_cell, p.n_steps)
    # equilibrium from total energy: C_v T + a T^4 = C_v T0 + a T_r0^4 (a = c = 1 units: 8 T + T^4 = 81)
    T_eq = [r.real for r in np.roots([1.0, 0, 0, 8.0, -81.0]) if abs(r.imag) < 1e-12 and r.real > 0][0]
    assert round(T_eq, 2) == gold["T_eq"][0]
    assert T[0] == pytest.approx(T_eq, rel=1e-6)
    a = ti.radiation_constant(p.c)
    E_bar = 4.0 * math.pi / p.c * dense.mean_intensity(p, I)[0] / (a * T_eq ** 4)
    assert np.round(E_bar, 2).tolist() == gold["E_bar"]
    assert float(np.sum(E_bar)) == pytest.approx(1.0, rel=1e-5)
