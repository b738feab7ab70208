"""Pins of the dense FP64 oracle (Section 2.1 numerics, upwind flux, implicit
source at fixed T) against closed forms of the discrete scheme.

(i)   infinite homogeneous medium relaxes as eps + (I0 - eps)(1 + c dt kappa)^-m
(ii)  beam in a pure absorber: the steady state (1 + kappa dx / mu)^-(i+1) is a
      fixed point of the step, and marching converges to it
(iii) energy balance of one step, exact to round-off; with kappa = 0 and
      periodic faces the content is conserved
(iv)  exact translation at lambda |n| = 1 (direction and index convention)
(v)   a y-uniform 2D field with periodic y evolves like the 1D scheme fed with
      the n_x of each 2D direction
"""
import math

import numpy as np
import pytest

import tt_inputs as ti
from oracle import dense, planck


def _problem(dim, n, G=3, nt=4, nphi=4, bc=None, kappa=1.0, T=0.5, cfl=0.5, seed=0, bc_T=None):
    nc = tuple(list(n) + [1] * (3 - len(n)))
    nx = int(np.prod(nc))
    edges = np.array([0.0] + list(np.geomspace(0.2, 3.0, G - 1)) + [np.inf])
    if dim == 1:
        mu, wt = ti.gauss_legendre_mu(nt)
        phi, wp = np.zeros(1), np.full(1, 2 * math.pi)
    else:
        mu, wt = ti.midpoint_mu(nt)
        phi, wp = ti.midpoint_phi(nphi)
    return ti.Problem(name="t", dim=dim, n_cells=nc, extent=(1.0, 0.7, 1.3), edges=edges,
                      kappa0=np.full(nx, kappa), kappa_scale=np.linspace(1.0, 2.0, G),
                      T_cell=np.full(nx, T), mu=mu, w_theta=wt, phi=phi, w_phi=wp,
                      bc=bc or (0,) * 6, bc_T=bc_T or (0.0,) * 6, cfl=cfl)


@pytest.mark.parametrize("dim,n", [(1, (7,)), (2, (5, 4)), (3, (3, 4, 2))])
def test_homogeneous_relaxation_closed_form(dim, n):
    p = _problem(dim, n, bc=(2,) * 6, kappa=2.0, T=0.8)
    G = p.n_groups
    I0 = np.full((p.M, p.n_theta, p.n_phi), 0.37)
    m = 9
    I = dense.march(p, I0, m)
    dt = dense.time_step(p)
    eps = planck.group_emission(p.edges, 0.8)
    kap = 2.0 * p.kappa_scale
    fac = (1.0 + p.c * dt * kap) ** (-m)
    ref_g = eps + (0.37 - eps) * fac
    ref = np.broadcast_to(np.tile(ref_g, p.n_x)[:, None, None], I.shape)
    np.testing.assert_allclose(I, ref, rtol=1e-13)


def _beam_steady(p, I_in):
    dx = p.extent[0] / p.n_cells[0]
    N = p.n_cells[0]
    G = p.n_groups
    kap = p.kappa0[0] * p.kappa_scale
    out = np.zeros((N, G, p.n_theta, 1))
    for l, mu in enumerate(p.mu):
        if mu <= 0:
            continue
        for i in range(N):
            out[i, :, l, 0] = I_in * (1.0 + kap * dx / mu) ** (-(i + 1))
    return out.reshape(p.M, p.n_theta, 1)


def test_beam_pure_absorber_fixed_point_and_convergence():
    p = _problem(1, (12,), nt=6, bc=(1, 0, 0, 0, 0, 0), bc_T=(1.0,) + (0.0,) * 5, kappa=3.0,
                 T=0.0, cfl=0.9)
    I_in = planck.group_emission(p.edges, 1.0)
    ss = _beam_steady(p, I_in)
    one = dense.march(p, ss, 1)
    np.testing.assert_allclose(one, ss, rtol=1e-13, atol=1e-15 * ss.max())
    I = dense.march(p, np.zeros_like(ss), 4000)
    np.testing.assert_allclose(I, ss, rtol=1e-9, atol=1e-13 * ss.max())
    # the continuum limit: (1 + k dx/mu)^-(i+1) -> exp(-k x/mu) at the outflow
    # face as dx -> 0 (first order)
    mu, k = 0.7, 1.0
    errs = []
    for N in (100, 200, 400):
        dx = 1.0 / N
        errs.append(abs((1 + k * dx / mu) ** (-N) - math.exp(-k / mu)))
    assert errs[1] < 0.55 * errs[0] and errs[2] < 0.55 * errs[1]


def _stream_energy_change(p, I, ghost, dt):
    """c dt * sum over faces of (inflow - outflow) for the upwind scheme."""
    G, NT, NP = p.n_groups, p.n_theta, p.n_phi
    N = [p.n_cells[d] if d < p.dim else 1 for d in range(3)]
    X = I.reshape(N[2], N[1], N[0], G, NT, NP)
    w = np.outer(p.w_theta, p.w_phi)
    dV = float(np.prod([p.extent[d] / p.n_cells[d] for d in range(p.dim)]))
    mu = np.asarray(p.mu)
    tot = 0.0
    for d in range(p.dim):
        lam = p.c * dt / (p.extent[d] / p.n_cells[d])
        if p.dim == 1:
            nd = np.repeat(mu[:, None], NP, axis=1)
        else:
            st = np.sqrt(1 - mu ** 2)[:, None]
            nd = [st * np.cos(p.phi)[None, :], st * np.sin(p.phi)[None, :],
                  np.repeat(mu[:, None], NP, axis=1)][d]
        npos, nneg = np.maximum(nd, 0), np.minimum(nd, 0)
        ax = 2 - d
        first = np.take(X, 0, axis=ax)
        last = np.take(X, N[d] - 1, axis=ax)
        glo = ghost[2 * d][:, None, None] if p.bc[2 * d] in (1, 3) else 0.0
        ghi = ghost[2 * d + 1][:, None, None] if p.bc[2 * d + 1] in (1, 3) else 0.0
        # telescoped sums of the two one-sided differences along the axis
        s = -(npos * (last - glo) + nneg * (ghi - first))
        tot += lam * dV * float(np.einsum("...glp,lp->...", s, w).sum())
    return tot


@pytest.mark.parametrize("dim,n", [(1, (9,)), (2, (6, 5)), (3, (4, 3, 5))])
def test_energy_balance_exact(dim, n):
    rng = np.random.default_rng(3)
    bc = (1, 0, 0, 1, 0, 0)
    bc_T = (1.0, 0.0, 0.0, 0.6, 0.0, 0.0)
    p = _problem(dim, n, bc=bc, bc_T=bc_T, T=0.4)
    p.kappa0 = rng.uniform(0.1, 5.0, p.n_x)
    I0 = rng.uniform(0.0, 1.0, (p.M, p.n_theta, p.n_phi))
    dt = dense.time_step(p)
    I1 = dense.march(p, I0, 1)
    ghost = dense.ghost_values(p)
    E0, E1 = dense.energy(p, I0), dense.energy(p, I1)
    kap = dense.kappa_field(p).reshape(-1)
    eps = dense.emission(p).reshape(-1)
    dV = float(np.prod([p.extent[d] / p.n_cells[d] for d in range(p.dim)]))
    w = np.outer(p.w_theta, p.w_phi)
    src = p.c * dt * dV * float(np.einsum("k,klp,lp->", kap, eps[:, None, None] - I1, w))
    pred = _stream_energy_change(p, I0, ghost, dt) + src
    assert E1 - E0 == pytest.approx(pred, abs=1e-12 * E0)


def test_energy_conserved_periodic_no_absorption():
    rng = np.random.default_rng(5)
    p = _problem(2, (6, 7), bc=(2,) * 6, kappa=0.0)
    I0 = rng.uniform(0.0, 1.0, (p.M, p.n_theta, p.n_phi))
    I = dense.march(p, I0, 25)
    assert dense.energy(p, I) == pytest.approx(dense.energy(p, I0), rel=1e-13)


def test_exact_translation_lambda_one():
    # 1D, directions mu = -1 and +1 only, CFL 1 so lambda |mu| = 1, no absorption:
    # each step moves the profile exactly one cell along mu (vacuum faces)
    p = _problem(1, (10,), G=2, kappa=0.0, T=0.0, cfl=1.0)
    p.mu = np.array([-1.0, 1.0])
    p.w_theta = np.array([1.0, 1.0])
    rng = np.random.default_rng(0)
    prof = rng.uniform(0.5, 1.0, (10, 2))
    I0 = np.repeat(prof.reshape(20, 1, 1), 2, axis=1)
    I = dense.march(p, I0, 3).reshape(10, 2, 2)
    right = np.zeros((10, 2)); right[3:] = prof[:-3]
    left = np.zeros((10, 2)); left[:-3] = prof[3:]
    np.testing.assert_array_equal(I[:, :, 1], right)
    np.testing.assert_array_equal(I[:, :, 0], left)


def test_2d_y_uniform_matches_1d_with_projected_directions():
    rng = np.random.default_rng(7)
    Nx, Ny = 8, 3
    p2 = _problem(2, (Nx, Ny), nt=4, nphi=4, bc=(1, 0, 2, 2, 0, 0), bc_T=(1.0,) + (0.0,) * 5,
                  T=0.3)
    k0 = rng.uniform(0.2, 3.0, Nx)
    p2.kappa0 = np.tile(k0, Ny)
    G = p2.n_groups
    prof = rng.uniform(0.0, 1.0, (Nx, G, p2.n_theta, p2.n_phi))
    I2 = np.broadcast_to(prof[None], (Ny, Nx, G, p2.n_theta, p2.n_phi)).reshape(p2.M, p2.n_theta,
                                                                                  p2.n_phi)
    dt = dense.time_step(p2)
    out2 = dense.march(p2, I2, 3, dt=dt).reshape(Ny, Nx, G, p2.n_theta, p2.n_phi)
    # 1D problem whose "mu" list is n_x of every 2D direction
    st = np.sqrt(1 - p2.mu ** 2)
    nx = (st[:, None] * np.cos(p2.phi)[None, :]).ravel()
    p1 = _problem(1, (Nx,), nt=len(nx), bc=(1, 0, 0, 0, 0, 0), bc_T=(1.0,) + (0.0,) * 5, T=0.3)
    p1.mu = nx
    p1.w_theta = np.ones(len(nx))
    p1.kappa0 = k0
    p1.extent = p2.extent
    I1 = prof.reshape(Nx * G, -1, 1)
    out1 = dense.march(p1, I1, 3, dt=dt).reshape(Nx, G, p2.n_theta, p2.n_phi)
    for j in range(Ny):
        np.testing.assert_allclose(out2[j], out1, rtol=1e-14, atol=1e-16)


def test_mirror_symmetry():
    # inflow on x+ with mirrored medium equals the mirrored x- inflow solution
    rng = np.random.default_rng(11)
    pa = _problem(1, (9,), nt=6, bc=(1, 0, 0, 0, 0, 0), bc_T=(1.0,) + (0.0,) * 5, T=0.2)
    pa.kappa0 = rng.uniform(0.5, 2.0, 9)
    pb = _problem(1, (9,), nt=6, bc=(0, 1, 0, 0, 0, 0), bc_T=(0.0, 1.0) + (0.0,) * 4, T=0.2)
    pb.kappa0 = pa.kappa0[::-1].copy()
    G = pa.n_groups
    I0 = rng.uniform(0, 1, (9, G, 6))
    Ia = dense.march(pa, I0.reshape(-1, 6, 1), 5).reshape(9, G, 6)
    # GL nodes are symmetric: index l <-> 5 - l flips mu
    Ib = dense.march(pb, I0[::-1, :, ::-1].reshape(-1, 6, 1), 5).reshape(9, G, 6)
    np.testing.assert_allclose(Ib[::-1, :, ::-1], Ia, rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("n_mat", [1, 3, 5])
def test_multi_material_kappa_has_rank_of_material_count(n_mat):
    # the opacity matrix of n materials on a partition has rank n (n <= N_nu)
    edges = ti.log_group_edges(8, 0.01, 10.0)
    K = ti.multi_material_kappa((9, 7, 1), (1.0, 1.0, 1.0), edges, n_mat, seed=n_mat)
    assert K.shape == (63, 8) and np.all(K > 0)
    assert np.linalg.matrix_rank(K) == n_mat
    assert len(np.unique(K[:, 0])) == n_mat


def test_kappa_full_of_a_factored_field_equals_the_factored_march():
    p = ti.slab1d(n_cells=16, n_groups=4, n_theta=6)
    p.kappa0 = ti.lognormal_kappa0(p.n_cells, p.extent, 1, seed=2)
    q = p.copy(kappa_full=np.outer(p.kappa0, p.kappa_scale), kappa0=None, kappa_scale=None)
    a = dense.march(p, dense.initial_dense(p), 5)
    b = dense.march(q, dense.initial_dense(q), 5)
    assert np.array_equal(a, b)


def test_kappa_full_rows_follow_cell_major_order():
    # kappa = "infinity" on rows (cell, g) with cell + g even, 0 elsewhere: after
    # one step the former hold eps_g(T_cell) and the latter the pure streaming
    # result, which fixes the row order cell * N_nu + g of kappa_full.
    p = ti.slab1d(n_cells=15, n_groups=4, n_theta=6, T=0.4)
    cell, g = np.meshgrid(np.arange(15), np.arange(4), indexing="ij")
    thick = (cell + g) % 2 == 0
    q = p.copy(kappa_full=np.where(thick, 1e300, 0.0))
    I0 = dense.initial_dense(q) * 0.25
    got = dense.march(q, I0, 1).reshape(15, 4, -1)
    stream = dense.march(p.copy(kappa0=np.zeros(15)), I0, 1).reshape(15, 4, -1)
    eps = dense.emission(p).reshape(15, 4)
    np.testing.assert_allclose(got[thick], np.broadcast_to(eps[thick][:, None], got[thick].shape), rtol=1e-14)
    np.testing.assert_array_equal(got[~thick], stream[~thick])
