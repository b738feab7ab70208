"""GPU parity of the coupled medium temperature (Section 2.1, the coupled
source stage) through the C ABI against the coupled dense oracle, and the
thermal relaxation test of Section 4.

Tolerances: FP64 with tol 1e-13 and caps that never bind, the TT solve is the
dense scheme up to rounding, so intensity and temperature agree to 1e-9 after
tens of steps; FP32 (fused path, tol 1e-6): 5e-4 for the intensity, 1e-4 for
the temperature.  Total energy (medium + radiation) is conserved by
construction against the rounded state, so on a periodic domain it holds to
round-off.

The paper's step order (Section 3.1: transport, round, source stage, round)
takes the source stage's J* from the rounded state after transport.  The dense
scheme has no rounding, so at tol 1e-13 both orders equal it to the same
bounds."""
import math
import os

import numpy as np
import pytest

import tt_inputs as ti
from oracle import dense

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "thermal_relax_3group.txt")


@pytest.fixture(scope="module")
def tt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_00290_amd as tt
    return tt


def full(Z, Th, Ph):
    return np.einsum("ka,alb,bp->klp", Z, Th, Ph, optimize=True)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _coupled(dim, prec=ti.PREC_FP64, tol=1e-13, cap=24, C=20.0, seed=0):
    rng = np.random.default_rng(seed)
    if dim == 1:
        p = ti.slab1d(n_cells=24, n_groups=5, n_theta=8, tol=tol, rank_cap=cap, precision=prec, seed=seed)
    else:
        p = ti.plane2d(n=7, n_groups=4, n_theta=4, n_phi=6, tol=tol, rank_cap=cap, precision=prec, seed=seed)
        p.n_cells = (7, 5, 1)
    p.kappa0 = ti.lognormal_kappa0(p.n_cells, p.extent, dim, seed=seed)
    n = p.n_x
    return p.copy(T_cell=rng.uniform(0.3, 1.2, n), T_rad0=rng.uniform(0.1, 0.8, n), heat_capacity=C)


def _run(tt, p, steps):
    s = tt.Solver(p)
    st = s.solve(steps)
    Z, Th, Ph = s.get_cores()
    T = s.get_temperature()
    s.destroy()
    return full(Z, Th, Ph), T, st


@pytest.mark.parametrize("dim", [1, 2])
def test_coupled_fp64_matches_dense_oracle(tt, dim):
    p = _coupled(dim)
    steps = 12
    I, T, st = _run(tt, p, steps)
    I_ref, T_ref = dense.march_coupled(p, dense.initial_dense(p), p.T_cell, steps)
    assert rel(I, I_ref) < 1e-9
    np.testing.assert_allclose(T, T_ref, rtol=1e-9, atol=0.0)
    assert np.max(np.abs(T - p.T_cell) / p.T_cell) > 1e-3   # the temperature did move


def test_coupled_fp32_fused_matches_dense_oracle(tt):
    p = _coupled(2, prec=ti.PREC_FP32, tol=1e-6, cap=16)
    steps = 10
    I, T, st = _run(tt, p, steps)
    I_ref, T_ref = dense.march_coupled(p, dense.initial_dense(p), p.T_cell, steps)
    assert rel(I, I_ref) < 5e-4
    np.testing.assert_allclose(T, T_ref, rtol=1e-4, atol=0.0)


@pytest.mark.parametrize("dim", [1, 2])
def test_coupled_paper_step_order_fp64_matches_dense_oracle(tt, dim):
    p = _coupled(dim).copy(step_order=1)
    steps = 12
    print(f"couple: paper order fp64 dim={dim}", flush=True)
    I, T, st = _run(tt, p, steps)
    I_ref, T_ref = dense.march_coupled(p, dense.initial_dense(p), p.T_cell, steps)
    assert rel(I, I_ref) < 1e-9
    np.testing.assert_allclose(T, T_ref, rtol=1e-9, atol=0.0)
    assert np.max(np.abs(T - p.T_cell) / p.T_cell) > 1e-3


def test_coupled_paper_step_order_fp32_fused_matches_dense_oracle(tt):
    p = _coupled(2, prec=ti.PREC_FP32, tol=1e-6, cap=16).copy(step_order=1)
    steps = 10
    I, T, st = _run(tt, p, steps)
    I_ref, T_ref = dense.march_coupled(p, dense.initial_dense(p), p.T_cell, steps)
    assert rel(I, I_ref) < 5e-4
    np.testing.assert_allclose(T, T_ref, rtol=1e-4, atol=0.0)


def test_coupled_paper_step_order_energy_on_periodic_domain(tt):
    # the source stage conserves the total against the rounded states; the
    # transport round in between is exact to the tolerance
    p = _coupled(2).copy(bc=(2, 2, 2, 2, 0, 0), step_order=1)
    s = tt.Solver(p)
    st0 = s.get_stats()
    U0 = st0["energy"] / p.c + st0["medium_energy"]
    st = s.solve(20)
    U = st["energy"] / p.c + st["medium_energy"]
    assert U == pytest.approx(U0, rel=1e-10)
    s.destroy()


def test_coupled_energy_conserved_on_periodic_domain(tt):
    p = _coupled(2).copy(bc=(2, 2, 2, 2, 0, 0))
    s = tt.Solver(p)
    st0 = s.get_stats()
    U0 = st0["energy"] / p.c + st0["medium_energy"]
    for _ in range(4):
        st = s.solve(5)
        U = st["energy"] / p.c + st["medium_energy"]
        assert U == pytest.approx(U0, rel=1e-11)
    assert abs(st["medium_energy"] - st0["medium_energy"]) > 1e-3 * abs(st0["medium_energy"])
    s.destroy()


def test_thermal_relaxation_reaches_printed_equilibrium_on_gpu(tt):
    gold = {}
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            k, *v = line.split()
            gold[k] = [float(x) for x in v]
    p = ti.thermal_relax(n_cells=4, t_final=80.0)
    s = tt.Solver(p)
    s.solve(p.n_steps)
    T = s.get_temperature()
    Z, Th, Ph = s.get_cores()
    s.destroy()
    T_eq = [r.real for r in np.roots([1.0, 0, 0, 8.0, -81.0]) if abs(r.imag) < 1e-12 and r.real > 0][0]
    assert round(T_eq, 2) == gold["T_eq"][0]
    np.testing.assert_allclose(T, T_eq, rtol=1e-6)
    I = full(Z, Th, Ph)
    J = dense.mean_intensity(p, I)                        # (N_X, 3)
    E_bar = 4.0 * math.pi / p.c * J / (ti.radiation_constant(p.c) * T_eq ** 4)
    for x in range(p.n_x):
        assert np.round(E_bar[x], 2).tolist() == gold["E_bar"]


def test_coupled_problem_rejects_apply_op(tt):
    p = _coupled(1)
    s = tt.Solver(p)
    with pytest.raises(tt.TTError) as e:
        s.apply_op()
    assert e.value.status == tt.TT_ERR_STATE
    s.destroy()
