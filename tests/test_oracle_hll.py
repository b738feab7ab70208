"""Pins of the oracle's HLL flux (Section 2.1: the asymptotic-preserving
stencil, whose only multigroup change is a per-group optical depth; Appendix
A: upwind-structured with spatially varying coefficients, two rank-1
operators per axis).  CPU only.

* Optically thin limit: with no opacity every interface factor is 1 and the
  HLL step is the upwind step, for the dense march and the TT terms.
* Optically thick limit: with the optical-depth factor beta -> inf every
  factor tends to 0 and the HLL step is central differences, i.e. the
  Rusanov step with S+ = 0 (itself pinned by the Gaussian diffusion closed
  form).
* Conservation: on a periodic domain with pure scattering the flux form and
  the scattering source keep the quadrature-weighted energy to round-off.
* Asymptotic preservation (the property the paper picks the flux for): on the
  Gaussian diffusion problem (eq. diffusion, kappa_s ~ 1000-2000) the HLL
  flux with beta = 20 follows the closed form to < 1 % at 128 cells, where
  the upwind flux's numerical diffusion puts it off by > 50 %; with beta = 1
  the error is several times the beta = 20 one.
* The TT operator terms (per-row coefficients, two Dirichlet columns per
  inflow face) reconstruct to exactly the dense HLL step in 1D, 2D and 3D,
  with inflow, vacuum and periodic faces; ranks (n + 1) r + n_bc.
"""
import numpy as np
import pytest

import tt_inputs as ti
from oracle import dense, tt as ott


def _case(dim, scatter=True, seed=0):
    rng = np.random.default_rng(seed)
    if dim == 1:
        p = ti.slab1d(n_cells=13, n_groups=3, n_theta=6, tol=1e-12, rank_cap=32)
        p = p.copy(bc=(1, 1, 0, 0, 0, 0), bc_T=(1.0, 0.4, 0, 0, 0, 0), kappa0=rng.uniform(0.1, 60.0, 13))
    elif dim == 2:
        p = ti.plane2d(n=6, n_groups=3, n_theta=4, n_phi=4, tol=1e-12, rank_cap=64, precision=0)
        p = p.copy(n_cells=(6, 5, 1), kappa0=rng.uniform(0.1, 50.0, 30), T_cell=np.full(30, 0.2),
                   bc=(1, 0, 2, 2, 0, 0))
    else:
        p = ti.clumps3d(n=4, n_groups=2, n_theta=4, n_phi=4, tol=1e-12, rank_cap=64, precision=0)
        p = p.copy(n_cells=(4, 3, 3), kappa0=rng.uniform(0.1, 80.0, 36), T_cell=np.full(36, 0.2),
                   bc=(1, 0, 0, 1, 2, 2))
    ks = rng.uniform(0.0, 5.0, (p.n_x, p.n_groups)) if scatter else None
    return p.copy(flux=ti.FLUX_HLL, hll_beta=20.0, kappa_s_full=ks)


def _dense_state(p, seed=3):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, (p.M, p.n_theta, p.n_phi))


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_thin_limit_is_the_upwind_step(dim):
    p = _case(dim, scatter=False)
    p = p.copy(kappa0=np.zeros(p.n_x))
    I = _dense_state(p)
    hll = dense.transport(p, I)
    up = dense.transport(p.copy(flux=ti.FLUX_UPWIND), I)
    np.testing.assert_allclose(hll, up, rtol=0, atol=1e-15 * np.abs(up).max())
    Z, Th, Ph = ti.random_tt(p.M, p.n_theta, p.n_phi, 3, min(2, p.n_phi), seed=1)
    a = ott.full(*ott.apply_transport(p, Z, Th, Ph))
    b = ott.full(*ott.apply_transport(p.copy(flux=ti.FLUX_UPWIND), Z, Th, Ph))
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-14 * np.abs(b).max())


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_thick_limit_is_central_differences(dim):
    p = _case(dim).copy(hll_beta=1e30)
    I = _dense_state(p)
    hll = dense.transport(p, I)
    central = dense.transport(p.copy(flux=ti.FLUX_RUSANOV, rusanov_s=0.0), I)
    np.testing.assert_allclose(hll, central, rtol=0, atol=1e-13 * np.abs(central).max())


@pytest.mark.parametrize("dim", [1, 2])
def test_periodic_pure_scattering_conserves_energy(dim):
    p = _case(dim)
    p = p.copy(bc=(2, 2, 2, 2, 0, 0), kappa0=np.zeros(p.n_x))
    I = _dense_state(p)
    E0 = dense.energy(p, I)
    I1 = dense.march(p, I, 7)
    assert dense.energy(p, I1) == pytest.approx(E0, rel=1e-13)
    # the opacity does vary across the faces, so the interface factors differ
    eL, eR = ott.hll_eps(p, 0)
    assert eL.min() < 0.5 * eL.max()


def _diffusion_error(flux, beta=20.0, n_cells=128, t_end=187.5):
    p = ti.gaussian_diffusion(n_cells=n_cells, n_groups=3).copy(flux=flux, hll_beta=beta)
    dt = dense.time_step(p)
    steps = int(round(t_end / dt))
    J0 = ti.gaussian_profile(p, 0.0).reshape(-1)
    I0 = np.broadcast_to(J0[:, None, None], (p.M, p.n_theta, 1)).copy()
    J = dense.mean_intensity(p, dense.march(p, I0, steps))
    ref = ti.gaussian_profile(p, steps * dt)
    return np.max(np.abs(J - ref)) / np.max(ref)


def test_asymptotic_preserving_in_the_diffusion_limit():
    e20 = _diffusion_error(ti.FLUX_HLL, 20.0)
    e1 = _diffusion_error(ti.FLUX_HLL, 1.0)
    eup = _diffusion_error(ti.FLUX_UPWIND)
    assert e20 < 0.01
    assert eup > 0.5
    assert e1 > 5 * e20


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_tt_terms_equal_the_dense_hll_step(dim):
    p = _case(dim)
    Z, Th, Ph = ti.random_tt(p.M, p.n_theta, p.n_phi, 3, min(2, p.n_phi), seed=4)
    Zs, Ts, Ps = ott.apply_transport(p, Z, Th, Ph)
    ref = dense.transport(p, ott.full(Z, Th, Ph))
    assert np.linalg.norm(ott.full(Zs, Ts, Ps) - ref) <= 1e-14 * np.linalg.norm(ref)
    n_in = sum(1 for f in range(2 * dim) if p.bc[f] in (ti.BC_INFLOW_PLANCK, ti.BC_INFLOW_VALUES))
    assert Zs.shape[1] == (2 * dim + 1) * 3 + 2 * n_in
    # one full step (transport, then scattering and absorption/emission)
    Zf, Tf, Pf = ott.apply_step(p, Z, Th, Ph)
    ref2 = dense.source(p, ref)
    assert np.linalg.norm(ott.full(Zf, Tf, Pf) - ref2) <= 1e-13 * np.linalg.norm(ref2)
