"""The projection in direction space (Y = Z W over the state's rank, then
the operator's stencil on Y, per direction) through the C ABI.

Once both small-core factors are square (k2 = N_phi and k1 = N_theta N_phi),
the columns of L_Theta are the directions, and each block of the pending
sum's angular core (Section 3.1: the TT sum of the streaming terms, Appendix
A: its rank-r blocks and rank-1 columns) is the state's angular matrix
Theta x_3 Phi scaled by the term's angular factors.  The library then forms
the projected first core from one contraction over r1 instead of the
gathered one over the sum's rank R1, for FP64 data with 128-column cores.
Every case below checks that it ran (or, for the cases it does not cover,
that it did not) through the stats' direction_space_rounds, and compares the
result with the oracle:

* 8 x 16 directions on a 4 x 3 x 2-cell cube with 2 or 4 groups and
  inflow, periodic and vacuum faces; the first steps (sum ranks below the
  angle counts) take the gathered projection, the later ones the
  direction-space one (the oracle's ranks of these cases reach R1 > 128);
* upwind with Householder QR rounding at tol 1e-13 against the dense march
  (1e-9; 2 groups, so the cap cannot bind), and with Gram rounding against
  the oracle's TT solve (1e-7, equal ranks);
* the Rusanov flux with isotropic scattering (seven rank-1 blocks; the
  oracle's ranks stay below the cap) and the coupled medium temperature (2
  groups) against the dense march (1e-9), the paper's step order against the
  oracle's TT solve (1e-10);
* HLL and a Rusanov case with more rank-1 blocks than the path holds: the
  gathered projection, against the oracle's TT solve (1e-10, equal ranks);
* one step of the 3D workload's shape from a seeded rank-(64, 16) state
  (R1 = 450), QR route, against the oracle's step (1e-12, equal ranks);
* one step on 8 x 8 x 5 cells, where an x-y plane is a whole number of
  64-row batches and each stencil block takes one batch position in up to 16
  consecutive planes (five here, so most of its waves idle), with z periodic,
  with inflow on both z faces, or with x periodic (the taps reused along an
  x-line stop at its wrapped ends): against the oracle's step (1e-12, equal
  ranks);
* FP32 data (Y = Z W on FP32 MFMA, FP32 Y and B, FP64 sums in the stencil):
  one step of the 3D shape at the cap (Gram and Householder TSQR rounding)
  and of the plane-tiled cube against the oracle's step (2e-6, the FP32
  bound), and a 12-step Gram solve on the cube against the oracle's TT solve
  (1e-4).
"""
import numpy as np
import pytest

import tt_inputs as ti
from oracle import dense, tt as ott

pytestmark = pytest.mark.gpu


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


def _cube(seed=0, tol=1e-13, cap=48, groups=4, bc=None, bc_T=None, **kw):
    rng = np.random.default_rng(seed)
    p = ti.clumps3d(n=4, n_groups=groups, n_theta=8, n_phi=16, tol=tol, rank_cap=cap, precision=ti.PREC_FP64,
                    T=0.3)
    p.n_cells = (4, 3, 2)
    p.kappa0 = rng.uniform(0.3, 3.0, 24)
    p.T_cell = np.full(24, 0.3)
    p.bc = bc or (ti.BC_INFLOW_PLANCK, ti.BC_INFLOW_PLANCK, ti.BC_PERIODIC, ti.BC_PERIODIC, 0, ti.BC_INFLOW_PLANCK)
    p.bc_T = bc_T or (1.0, 0.5, 0.0, 0.0, 0.0, 0.8)
    return p.copy(**kw) if kw else p


def _solve(tt, p, steps, method):
    s = tt.Solver(p, round_method=method)
    st = s.solve(steps)
    out = full(*s.get_cores())
    s.destroy()
    return out, st


STEPS = 12


def test_upwind_qr_matches_dense_march(tt):
    p = _cube(groups=2)                    # M = 48 rows: the cap 48 cannot bind
    print(f"stencil: upwind qr M={p.M}", flush=True)
    I, st = _solve(tt, p, STEPS, tt.TT_ROUND_QR)
    assert 0 < st["direction_space_rounds"] < STEPS
    assert rel(I, dense.march(p, dense.initial_dense(p), STEPS)) < 1e-9


def test_upwind_gram_matches_oracle_tt_solve(tt):
    p = _cube(tol=1e-6, cap=40)
    print(f"stencil: upwind gram M={p.M}", flush=True)
    s = tt.Solver(p, round_method=tt.TT_ROUND_GRAM)
    st = s.solve(STEPS)
    (Zo, To, Po), infos = ott.solve(p, STEPS)
    assert st["direction_space_rounds"] > 0
    assert (st["r1"], st["r2"]) == (infos[-1]["r1"], infos[-1]["r2"])
    assert rel(full(*s.get_cores()), full(Zo, To, Po)) < 1e-7
    s.destroy()


def test_rusanov_scattering_matches_dense_march(tt):
    rng = np.random.default_rng(3)
    p = _cube(flux=ti.FLUX_RUSANOV, rusanov_s=0.7)
    p = p.copy(kappa_s_full=rng.uniform(0.0, 4.0, (p.n_x, p.n_groups)))
    print(f"stencil: rusanov + scattering M={p.M}", flush=True)
    I, st = _solve(tt, p, STEPS, tt.TT_ROUND_QR)
    assert st["direction_space_rounds"] > 0
    assert rel(I, dense.march(p, dense.initial_dense(p), STEPS)) < 1e-9


def test_paper_step_order_matches_oracle_tt_solve(tt):
    p = _cube(tol=1e-11, cap=48, step_order=1)
    print(f"stencil: paper step order M={p.M}", flush=True)
    s = tt.Solver(p, round_method=tt.TT_ROUND_QR)
    st = s.solve(8)
    (Zo, To, Po), _ = ott.solve(p, 8)
    assert st["direction_space_rounds"] > 0
    assert rel(full(*s.get_cores()), full(Zo, To, Po)) < 1e-10
    s.destroy()


def test_coupled_temperature_matches_dense_march(tt):
    rng = np.random.default_rng(4)
    p = _cube(groups=2)
    p = p.copy(T_cell=rng.uniform(0.3, 1.2, p.n_x), T_rad0=rng.uniform(0.1, 0.8, p.n_x), heat_capacity=20.0)
    print(f"stencil: coupled temperature M={p.M}", flush=True)
    s = tt.Solver(p, round_method=tt.TT_ROUND_QR)
    st = s.solve(STEPS)
    I = full(*s.get_cores())
    T = s.get_temperature()
    s.destroy()
    I_ref, T_ref = dense.march_coupled(p, dense.initial_dense(p), p.T_cell, STEPS)
    assert st["direction_space_rounds"] > 0
    assert rel(I, I_ref) < 1e-9
    np.testing.assert_allclose(T, T_ref, rtol=1e-9, atol=0.0)


@pytest.mark.parametrize("case", ["hll", "many_rank1"])
def test_gathered_projection_where_the_path_does_not_apply(tt, case):
    if case == "hll":
        p = _cube(flux=ti.FLUX_HLL)
    else:
        # Rusanov: two rank-1 columns per inflow face, five faces, plus the
        # emission: eleven rank-1 blocks
        p = _cube(flux=ti.FLUX_RUSANOV, rusanov_s=1.0,
                  bc=(ti.BC_INFLOW_PLANCK,) * 5 + (0,), bc_T=(1.0, 0.5, 0.7, 0.3, 0.9, 0.0))
    print(f"stencil: fallback {case} M={p.M}", flush=True)
    I, st = _solve(tt, p, STEPS, tt.TT_ROUND_QR)
    (Zo, To, Po), infos = ott.solve(p, STEPS)
    assert st["direction_space_rounds"] == 0
    assert (st["r1"], st["r2"]) == (infos[-1]["r1"], infos[-1]["r2"])
    assert rel(I, full(Zo, To, Po)) < 1e-10


def test_one_step_of_the_3d_shape_at_the_cap(tt):
    p = ti.clumps3d(n=12, n_groups=8, n_theta=8, n_phi=16, tol=1e-5, rank_cap=64, precision=ti.PREC_FP64)
    print(f"stencil: 3D shape one step M={p.M}", flush=True)
    s = tt.Solver(p, round_method=tt.TT_ROUND_QR)
    Z, Th, Ph = ti.random_tt(p.M, 8, 16, 64, 16, seed=31, decay=0.9)
    s.set_cores(Z, Th, Ph)
    st = s.solve(1)
    Zo, To, Po, info = ott.step(p, Z, Th, Ph)
    assert st["max_R1"] == 450 and st["direction_space_rounds"] == 1
    assert s.get_ranks() == (info["r1"], info["r2"])
    assert rel(full(*s.get_cores()), full(Zo, To, Po)) < 1e-12
    s.destroy()


@pytest.mark.parametrize("zbc", ["periodic", "inflow", "x_periodic"])
def test_one_step_with_plane_tiles(tt, zbc):
    p = ti.clumps3d(n=8, n_groups=4, n_theta=8, n_phi=16, tol=1e-9, rank_cap=48, precision=ti.PREC_FP64, T=0.3)
    p.n_cells = (8, 8, 5)
    rng = np.random.default_rng(9)
    p.kappa0 = rng.uniform(0.3, 3.0, 320)
    p.T_cell = np.full(320, 0.3)
    if zbc == "periodic":
        p.bc = (ti.BC_INFLOW_PLANCK, 0, 0, 0, ti.BC_PERIODIC, ti.BC_PERIODIC)
        p.bc_T = (1.0, 0.0, 0.0, 0.0, 0.0, 0.0)
    elif zbc == "x_periodic":
        # x-lines wrap: the stencil's reuse of the previous row's taps must
        # stop at each line's ends
        p.bc = (ti.BC_PERIODIC, ti.BC_PERIODIC, ti.BC_INFLOW_PLANCK, 0, 0, ti.BC_INFLOW_PLANCK)
        p.bc_T = (0.0, 0.0, 1.0, 0.0, 0.0, 0.6)
    else:
        p.bc = (ti.BC_INFLOW_PLANCK, 0, 0, 0, ti.BC_INFLOW_PLANCK, ti.BC_INFLOW_PLANCK)
        p.bc_T = (1.0, 0.0, 0.0, 0.0, 0.7, 0.4)
    print(f"stencil: plane tiles z {zbc} M={p.M}", flush=True)
    s = tt.Solver(p, round_method=tt.TT_ROUND_QR)
    Z, Th, Ph = ti.random_tt(p.M, 8, 16, 24, 16, seed=41, decay=0.8)
    s.set_cores(Z, Th, Ph)
    st = s.solve(1)
    Zo, To, Po, info = ott.step(p, Z, Th, Ph)
    assert st["direction_space_rounds"] == 1
    assert s.get_ranks() == (info["r1"], info["r2"])
    assert rel(full(*s.get_cores()), full(Zo, To, Po)) < 1e-12
    s.destroy()


@pytest.mark.parametrize("case", ["3d_shape", "3d_shape_qr", "plane_tiles"])
def test_fp32_one_step(tt, case):
    if case.startswith("3d_shape"):
        p = ti.clumps3d(n=12, n_groups=8, n_theta=8, n_phi=16, tol=1e-5, rank_cap=64, precision=ti.PREC_FP32)
        Z, Th, Ph = ti.random_tt(p.M, 8, 16, 64, 16, seed=31, decay=0.9)
    else:
        p = ti.clumps3d(n=8, n_groups=4, n_theta=8, n_phi=16, tol=1e-5, rank_cap=48, precision=ti.PREC_FP32, T=0.3)
        p.n_cells = (8, 8, 5)
        rng = np.random.default_rng(9)
        p.kappa0 = rng.uniform(0.3, 3.0, 320)
        p.T_cell = np.full(320, 0.3)
        p.bc = (ti.BC_INFLOW_PLANCK, 0, 0, 0, ti.BC_PERIODIC, ti.BC_PERIODIC)
        p.bc_T = (1.0, 0.0, 0.0, 0.0, 0.0, 0.0)
        Z, Th, Ph = ti.random_tt(p.M, 8, 16, 24, 16, seed=41, decay=0.8)
    print(f"stencil: fp32 one step {case} M={p.M}", flush=True)
    s = tt.Solver(p, round_method=tt.TT_ROUND_QR) if case.endswith("_qr") else tt.Solver(p)
    s.set_cores(Z, Th, Ph)
    st = s.solve(1)
    Zo, To, Po, info = ott.step(p, Z, Th, Ph)
    assert st["direction_space_rounds"] == 1
    r1, r2 = s.get_ranks()
    assert abs(r1 - info["r1"]) <= 1 and abs(r2 - info["r2"]) <= 1
    slack = 2 * p.tol * ((r1, r2) != (info["r1"], info["r2"]))
    assert rel(full(*s.get_cores()), full(Zo, To, Po)) < 2e-6 + slack
    s.destroy()


def test_fp32_gram_solve_matches_oracle_tt_solve(tt):
    p = _cube(tol=1e-6, cap=40, precision=ti.PREC_FP32)
    print(f"stencil: fp32 gram solve M={p.M}", flush=True)
    s = tt.Solver(p, round_method=tt.TT_ROUND_GRAM)
    st = s.solve(STEPS)
    (Zo, To, Po), infos = ott.solve(p, STEPS)
    assert st["direction_space_rounds"] > 0
    assert rel(full(*s.get_cores()), full(Zo, To, Po)) < 1e-4
    s.destroy()
