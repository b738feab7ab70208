"""GPU parity of the HLL flux (Section 2.1: the asymptotic-preserving stencil
with a per-group optical depth; Appendix A: two rank-1 operators per axis
whose spatial parts vary per row) through the C ABI against the oracle.

* The pending TT sum equals the oracle's explicit Appendix-A sum elementwise
  (1e-13) in 1D, 2D and 3D with inflow faces on both sides.
* FP64 solves at a tolerance that never truncates equal the dense HLL march
  (1e-9); at working tolerances they equal the oracle's TT solve (1e-10, the
  FP64 bound, same ranks), with QR and Gram rounding (1e-8 per step for Gram)
  and in the paper's step order.
* With no opacity the HLL solve is the upwind solve (1e-13).
* Problems the build does not provide it for (FP32 data, scattering) are
  refused with TT_ERR_INVALID_ARG.
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


def _case(dim, tol=1e-7, cap=24, seed=0, beta=20.0):
    rng = np.random.default_rng(seed)
    if dim == 1:
        p = ti.slab1d(n_cells=29, n_groups=4, n_theta=8, tol=tol, rank_cap=cap, T=0.3)
        p = p.copy(bc=(1, 3, 0, 0, 0, 0), bc_values=np.full((6, 4), 0.05), kappa0=rng.uniform(0.05, 40.0, 29))
    elif dim == 2:
        p = ti.plane2d(n=9, n_groups=3, n_theta=4, n_phi=6, tol=tol, rank_cap=cap, precision=ti.PREC_FP64, T=0.3)
        p = p.copy(n_cells=(9, 7, 1), kappa0=rng.uniform(0.05, 40.0, 63), T_cell=np.full(63, 0.3),
                   bc=(1, 0, 2, 2, 0, 0))
    else:
        p = ti.clumps3d(n=5, n_groups=2, n_theta=4, n_phi=4, tol=tol, rank_cap=cap, precision=ti.PREC_FP64, T=0.3)
        p = p.copy(n_cells=(5, 4, 3), kappa0=rng.uniform(0.05, 40.0, 60), T_cell=np.full(60, 0.3),
                   bc=(1, 1, 0, 0, 2, 2), bc_T=(1.0, 0.5, 0, 0, 0, 0))
    return p.copy(flux=ti.FLUX_HLL, hll_beta=beta, precision=ti.PREC_FP64)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_hll_explicit_sum_matches_oracle(tt, dim):
    p = _case(dim)
    s = tt.Solver(p)
    Z, Th, Ph = ti.random_tt(p.M, p.n_theta, p.n_phi, 3, min(2, p.n_phi), seed=dim)
    s.set_cores(Z, Th, Ph)
    s.apply_op()
    Zr, Tr, Pr = ott.apply_step(p, Z, Th, Ph)
    Zg, Tg, Pg = s.get_cores(pending_shape=(Zr.shape[1], Pr.shape[0]))
    np.testing.assert_allclose(Zg, Zr, rtol=1e-13, atol=1e-15 * np.abs(Zr).max())
    np.testing.assert_allclose(Tg, Tr, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(Pg, Pr, rtol=1e-14, atol=1e-15)
    s.round(p.tol, p.rank_cap)
    Zo, To, Po, info = ott.round_tt(Zr, Tr, Pr, p.tol, p.rank_cap)
    assert s.get_ranks() == (info["r1"], info["r2"])
    assert rel(full(*s.get_cores()), full(Zo, To, Po)) < 1e-12
    s.destroy()


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_hll_solve_equals_dense_march(tt, dim):
    p = _case(dim, tol=1e-13, cap=48)
    steps = 10
    print(f"hll dense dim={dim}", flush=True)
    s = tt.Solver(p, round_method=tt.TT_ROUND_QR)
    st = s.solve(steps)
    ref = dense.march(p, dense.initial_dense(p), steps)
    assert rel(full(*s.get_cores()), ref) < 1e-9
    assert st["nan_flag"] == 0
    s.destroy()


@pytest.mark.parametrize("dim,method", [(1, "qr"), (2, "qr"), (3, "qr"), (2, "gram")])
def test_hll_solve_matches_oracle_tt_solve(tt, dim, method):
    p = _case(dim, tol=1e-6, cap=10)
    K = 15
    s = tt.Solver(p, round_method=tt.TT_ROUND_QR if method == "qr" else tt.TT_ROUND_GRAM)
    st = s.solve(K)
    (Zo, To, Po), infos = ott.solve(p, K)
    if method == "qr":
        assert (st["r1"], st["r2"]) == (infos[-1]["r1"], infos[-1]["r2"])
    assert rel(full(*s.get_cores()), full(Zo, To, Po)) < (1e-10 if method == "qr" else 1e-7)
    s.destroy()


def test_hll_paper_step_order(tt):
    p = _case(2, tol=1e-7, cap=12).copy(step_order=1)
    s = tt.Solver(p)
    s.solve(8)
    (Zo, To, Po), _ = ott.solve(p, 8)
    assert rel(full(*s.get_cores()), full(Zo, To, Po)) < 1e-10
    s.destroy()


def test_hll_thin_limit_is_upwind_on_the_gpu(tt):
    p = _case(2, tol=1e-8, cap=16)
    p = p.copy(kappa0=np.zeros(p.n_x))
    a = tt.Solver(p)
    a.solve(6)
    b = tt.Solver(p.copy(flux=ti.FLUX_UPWIND))
    b.solve(6)
    assert rel(full(*a.get_cores()), full(*b.get_cores())) < 1e-13


def test_hll_refusals(tt):
    p = _case(1)
    with pytest.raises(tt.TTError) as e:
        tt.Solver(p.copy(precision=ti.PREC_FP32))
    assert e.value.status == tt.TT_ERR_INVALID_ARG
    with pytest.raises(tt.TTError) as e:
        tt.Solver(p.copy(kappa_s_full=np.ones((p.n_x, p.n_groups))))
    assert e.value.status == tt.TT_ERR_INVALID_ARG
    with pytest.raises(tt.TTError) as e:
        tt.Solver(p.copy(hll_beta=0.0))
    assert e.value.status == tt.TT_ERR_INVALID_ARG
