"""Pins of the oracle's Rusanov flux and isotropic scattering (Section 2.1:
the three flux stencils and the backward-Euler source update with the
scattering opacity; Appendix A, "Value of n"; the Gaussian diffusion test of
Section 4, eq. diffusion)."""
import numpy as np
import pytest

import tt_inputs as ti
from oracle import dense, tt as ott


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_rusanov_with_unit_speed_on_unit_directions_is_upwind():
    # For n = +-1 and S+ = c the Rusanov interface flux is the upwind flux:
    # (c n / 2)(I_L + I_R) - (c / 2)(I_R - I_L) = c I_L for n = 1.
    p = ti.slab1d(n_cells=23, n_groups=3, n_theta=2, T=0.2)
    p = p.copy(mu=np.array([-1.0, 1.0]), w_theta=np.array([1.0, 1.0]),
               bc=(ti.BC_INFLOW_PLANCK, ti.BC_INFLOW_VALUES, 0, 0, 0, 0),
               bc_values=np.full((6, 3), 0.3))
    rng = np.random.default_rng(0)
    I = rng.uniform(0.5, 1.5, (p.M, 2, 1))
    up = dense.transport(p, I)
    ru = dense.transport(p.copy(flux=ti.FLUX_RUSANOV, rusanov_s=1.0), I)
    np.testing.assert_allclose(ru, up, rtol=1e-14, atol=1e-15)
    Z, Th, Ph = ti.random_tt(p.M, 2, 1, 3, 1, seed=1)
    a = ott.full(*ott.apply_transport(p, Z, Th, Ph))
    b = ott.full(*ott.apply_transport(p.copy(flux=ti.FLUX_RUSANOV, rusanov_s=1.0), Z, Th, Ph))
    np.testing.assert_allclose(b, a, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("s_rus", [1.0, 0.6, 0.0])
def test_rusanov_and_scattering_conserve_energy_on_a_periodic_domain(s_rus):
    # flux form: the interface fluxes telescope on a periodic grid; scattering
    # keeps the angle mean of every row (kappa_a = 0)
    p = ti.plane2d(n=9, n_groups=3, n_theta=4, n_phi=6)
    p.n_cells = (9, 7, 1)
    p = p.copy(kappa0=np.zeros(63), T_cell=np.zeros(63), bc=(ti.BC_PERIODIC,) * 4 + (0, 0),
               flux=ti.FLUX_RUSANOV, rusanov_s=s_rus,
               kappa_s_full=np.random.default_rng(1).uniform(0.5, 5.0, (63, 3)))
    rng = np.random.default_rng(2)
    I = rng.uniform(0.1, 1.0, (p.M, 4, 6))
    E0 = dense.energy(p, I)
    I = dense.march(p, I, 6)
    assert dense.energy(p, I) == pytest.approx(E0, rel=1e-13)


def test_homogeneous_medium_scattering_and_absorption_closed_form():
    # uniform in space: streaming does nothing, and per step the angle mean
    # follows J <- (J + a eps) / (1 + a) while the anisotropic part I - J
    # decays by 1 / (1 + a + b)
    p = ti.slab1d(n_cells=8, n_groups=2, n_theta=6, T=0.5)
    ka, ks = np.array([0.3, 2.0]), np.array([4.0, 0.7])
    p = p.copy(bc=(ti.BC_PERIODIC, ti.BC_PERIODIC, 0, 0, 0, 0), kappa_full=np.tile(ka, (8, 1)),
               kappa_s_full=np.tile(ks, (8, 1)), flux=ti.FLUX_RUSANOV, rusanov_s=1.0)
    rng = np.random.default_rng(3)
    ang = rng.uniform(0.2, 1.0, (2, 6))                           # per group and direction
    I0 = np.tile(ang[None, :, :, None], (8, 1, 1, 1)).reshape(p.M, 6, 1)
    m = 7
    I = dense.march(p, I0, m)
    cdt = p.c * dense.time_step(p)
    a, b = cdt * ka, cdt * ks
    eps = dense.emission(p)[0]
    J0 = ang @ p.w_theta * p.w_phi[0] / (4 * np.pi)
    Jm = eps + (J0 - eps) * (1.0 + a) ** (-m)
    expect = Jm[:, None] + (ang - J0[:, None]) * ((1.0 + a + b) ** (-m))[:, None]
    np.testing.assert_allclose(I.reshape(8, 2, 6), np.broadcast_to(expect, (8, 2, 6)), rtol=1e-13)
    # the TT oracle from the same state: Z one-hot in the group, Theta = ang
    Z = np.tile(np.eye(2), (8, 1))
    Th = ang[:, :, None]
    (Zm, Tm, Pm), _ = ott.solve(p, m, cores=(Z, Th, np.ones((1, 1))), tol=1e-14, cap=20)
    np.testing.assert_allclose(ott.full(Zm, Tm, Pm).reshape(8, 2, 6), np.broadcast_to(expect, (8, 2, 6)),
                               rtol=1e-12)


def _diffusion_error(n_cells, t_end=187.5):
    p = ti.gaussian_diffusion(n_cells=n_cells, n_groups=3)
    dt = dense.time_step(p)
    steps = int(round(t_end / dt))
    J0 = ti.gaussian_profile(p, 0.0).reshape(-1)
    I0 = np.broadcast_to(J0[:, None, None], (p.M, p.n_theta, 1)).copy()
    I = dense.march(p, I0, steps)
    J = dense.mean_intensity(p, I)
    ref = ti.gaussian_profile(p, steps * dt)
    return np.max(np.abs(J - ref)) / np.max(ref), p


def test_gaussian_diffusion_follows_the_closed_form_and_converges():
    # eq. diffusion: E_g(t, x) = A / sqrt(4 pi D_g (t0 + t)) exp(-x^2 / (4 D_g (t0 + t))),
    # D_g = c / (3 kappa_s,g); Rusanov with S+ = 0 and pure scattering.  The
    # scheme is second order in space for this smooth pulse (central
    # differences over a two-cell stencil: ~(2 dx)^2 / (12 sigma^2) ~ 2 % at
    # 128 cells), so the error must stay at that level and drop ~4x when the
    # grid is refined.
    e128, p = _diffusion_error(128)
    e256, _ = _diffusion_error(256)
    assert e128 < 0.05
    assert e256 < e128 / 3.0
    # the groups have separated: their diffusion coefficients differ
    ks = p.kappa_s_full[0]
    assert ks[-1] / ks[0] > 1.2


@pytest.mark.parametrize("dim,s_rus", [(1, 1.0), (1, 0.0), (2, 0.5), (3, 1.0)])
def test_tt_oracle_equals_dense_with_rusanov_and_scattering(dim, s_rus):
    if dim == 1:
        p = ti.slab1d(n_cells=13, n_groups=3, n_theta=6, T=0.3, tol=1e-14, rank_cap=60)
    elif dim == 2:
        p = ti.plane2d(n=6, n_groups=2, n_theta=4, n_phi=6, T=0.3, tol=1e-14, rank_cap=60)
        p.n_cells = (6, 5, 1)
        p.T_cell = np.full(30, 0.3)
        p.kappa0 = np.random.default_rng(0).uniform(0.5, 2.0, 30)
    else:
        p = ti.clumps3d(n=4, n_groups=2, n_theta=2, n_phi=4, T=0.3, tol=1e-14, rank_cap=60)
        p.n_cells = (4, 3, 3)
        p.T_cell = np.full(36, 0.3)
        p.kappa0 = np.random.default_rng(0).uniform(0.5, 2.0, 36)
    rng = np.random.default_rng(5)
    p = p.copy(flux=ti.FLUX_RUSANOV, rusanov_s=s_rus, kappa_s_full=rng.uniform(0.0, 3.0, (p.n_x, p.n_groups)))
    if dim == 3:
        p = p.copy(bc=(ti.BC_INFLOW_PLANCK, 0, ti.BC_INFLOW_PLANCK, 0, 0, ti.BC_INFLOW_PLANCK), bc_T=(1.0,) * 6)
    steps = 5
    (Z, Th, Ph), _ = ott.solve(p, steps)
    ref = dense.march(p, dense.initial_dense(p), steps)
    assert _rel(ott.full(Z, Th, Ph), ref) < 1e-11


def test_coupled_temperature_with_scattering_conserves_total_energy():
    p = ti.slab1d(n_cells=12, n_groups=3, n_theta=6)
    rng = np.random.default_rng(4)
    p = p.copy(bc=(ti.BC_PERIODIC, ti.BC_PERIODIC, 0, 0, 0, 0), flux=ti.FLUX_RUSANOV, rusanov_s=1.0,
               kappa_s_full=rng.uniform(0.5, 4.0, (12, 3)), T_cell=rng.uniform(0.3, 1.0, 12),
               T_rad0=rng.uniform(0.1, 0.6, 12), heat_capacity=5.0)
    I0 = dense.initial_dense(p)
    E0 = dense.total_energy(p, I0, p.T_cell)
    I, T = dense.march_coupled(p, I0, p.T_cell, 4)
    assert dense.total_energy(p, I, T) == pytest.approx(E0, rel=1e-12)
