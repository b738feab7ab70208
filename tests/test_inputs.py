"""The seeded input generators (the synthetic stand-ins for the paper's
workloads): shapes, seeding and the structure each one promises."""
import numpy as np

import tt_inputs as ti


def test_generators_are_seeded():
    a, b = ti.plane2d(n=16, seed=3), ti.plane2d(n=16, seed=3)
    assert np.array_equal(a.kappa0, b.kappa0)
    assert not np.array_equal(a.kappa0, ti.plane2d(n=16, seed=4).kappa0)


def test_lognormal_field_has_unit_log_variance():
    k0 = ti.lognormal_kappa0((64, 64, 1), (1.0, 1.0, 1.0), 2, sigma=1.0, seed=1)
    g = np.log(k0)
    assert abs(g.mean()) < 1e-12 and abs(g.std() - 1.0) < 1e-12


def test_spike_slab_is_the_cube_field_cut_along_z():
    # one GPU's share of the spike cube: the cube's opacity restricted to
    # z-planes [slab * nz, (slab + 1) * nz), with the cube's cell size
    n, nz = 16, 4
    cube = ti.spikes3d(n=n, n_groups=8, n_theta=2, n_phi=4, rank_cap=4)
    for slab in (0, 2):
        p = ti.spikes3d_slab(n=n, nz=nz, slab=slab, n_groups=8, n_theta=2, n_phi=4, rank_cap=4)
        assert p.n_cells == (n, n, nz) and p.n_x == n * n * nz
        assert np.array_equal(p.kappa0, cube.kappa0.reshape(n, n, n)[slab * nz:(slab + 1) * nz].ravel())
        assert np.allclose([p.extent[d] / p.n_cells[d] for d in range(3)], 1.0 / n)
        assert np.array_equal(p.kappa_scale, cube.kappa_scale)
        assert p.bc[4] == ti.BC_VACUUM and p.bc[5] == ti.BC_VACUUM


def test_gaussian_diffusion_set_up():
    p = ti.gaussian_diffusion(n_cells=64, n_groups=5)
    ks = p.kappa_s_full.reshape(p.n_x, p.n_groups)
    assert np.all(ks == ks[0]) and np.all((ks[0] >= 1000.0) & (ks[0] <= 2000.0))
    assert p.flux == ti.FLUX_RUSANOV and p.rusanov_s == 0.0 and np.all(p.kappa0 == 0.0)
    J0 = ti.gaussian_profile(p, 0.0)
    # identical initial profile in every group, unit area (A = 1) on the grid
    assert np.allclose(J0, J0[:, :1])
    assert abs(J0[:, 0].sum() * p.extent[0] / p.n_cells[0] - 1.0) < 1e-9
    # later the groups differ: the larger D (smaller kappa_s) has spread more
    J = ti.gaussian_profile(p, 100.0)
    assert J[:, int(np.argmin(ks[0]))].max() < J[:, int(np.argmax(ks[0]))].max()


def test_multi_material_opacity_is_piecewise_constant_per_material():
    edges = ti.log_group_edges(6, 0.01, 10.0)
    K = ti.multi_material_kappa((12, 10, 1), (1.0, 1.0, 1.0), edges, 4, seed=2)
    rows = {tuple(r) for r in np.round(K, 12)}
    assert len(rows) == 4
