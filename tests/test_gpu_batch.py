"""The persistent ragged small-solve kernel (tt_transport_solve_small_batch):
many small FP64 requests of different grids, group counts, rank caps and
step counts advanced in one launch, one workgroup per request.

* Each request equals the oracle's TT solve (1e-10, the FP64 bound, with
  equal ranks) and the launched per-kernel path (1e-12: the gather
  projection sums in another order).
* A request's result does not depend on the batch: bitwise equal alone and
  inside a mixed batch, in any position.
* Ineligible handles (FP32 data, a projected core wider than 16 columns) are
  refused with TT_ERR_INVALID_ARG, and a handle continues correctly with the
  launched path after a batch (odd step counts flip the core buffers).
"""
import numpy as np
import pytest

import tt_inputs as ti
from oracle import tt as ott

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


def _requests():
    # 1D slabs (16 or 8 Gauss-Legendre directions, so k1 <= 16) of different
    # sizes, group counts, caps, tolerances and opacity fields
    out = []
    for i, (nc, G, nt, cap, tol, steps) in enumerate(
            [(64, 8, 16, 8, 1e-8, 40), (37, 5, 8, 6, 1e-7, 23), (200, 16, 16, 12, 1e-6, 31),
             (90, 12, 16, 4, 1e-5, 17), (512, 4, 16, 10, 1e-8, 9)]):
        p = ti.slab1d(n_cells=nc, n_groups=G, n_theta=nt, tol=tol, rank_cap=cap, n_steps=steps, seed=i)
        p.kappa0 = ti.lognormal_kappa0(p.n_cells, p.extent, 1, seed=i)
        if i % 2:
            p.bc = (ti.BC_INFLOW_PLANCK, ti.BC_INFLOW_PLANCK, 0, 0, 0, 0)
            p.bc_T = (1.0, 0.5, 0, 0, 0, 0)
        out.append(p)
    return out


def test_small_batch_matches_oracle_and_launched_path(tt):
    probs = _requests()
    solvers = [tt.Solver(p, round_method=tt.TT_ROUND_QR) for p in probs]
    print("small batch: ragged solve", flush=True)
    stats = tt.solve_small_batch(solvers, [p.n_steps for p in probs])
    for p, s, st in zip(probs, solvers, stats):
        got = full(*s.get_cores())
        (Zo, To, Po), infos = ott.solve(p, p.n_steps)
        assert (st["r1"], st["r2"]) == (infos[-1]["r1"], infos[-1]["r2"])
        assert rel(got, full(Zo, To, Po)) < 1e-10
        ref = tt.Solver(p, round_method=tt.TT_ROUND_QR)
        ref.solve(p.n_steps)
        assert rel(got, full(*ref.get_cores())) < 1e-12
        ref.destroy()
        assert st["nan_flag"] == 0 and st["steps"] == p.n_steps


def test_small_batch_result_independent_of_the_batch(tt):
    probs = _requests()
    alone = []
    for p in probs:
        s = tt.Solver(p, round_method=tt.TT_ROUND_QR)
        tt.solve_small_batch([s], p.n_steps)
        alone.append(s.get_cores())
        s.destroy()
    order = [3, 0, 4, 1, 2]
    solvers = [tt.Solver(probs[i], round_method=tt.TT_ROUND_QR) for i in order]
    print("small batch: mixed order", flush=True)
    tt.solve_small_batch(solvers, [probs[i].n_steps for i in order])
    for i, s in zip(order, solvers):
        for a, b in zip(s.get_cores(), alone[i]):
            np.testing.assert_array_equal(a, b)


def test_small_batch_then_launched_steps_and_refusals(tt):
    p = _requests()[1]
    s = tt.Solver(p, round_method=tt.TT_ROUND_QR)
    tt.solve_small_batch([s], 7)          # odd: the ping-pong buffers flip
    s.solve(5)
    (Zo, To, Po), _ = ott.solve(p, 12)
    assert rel(full(*s.get_cores()), full(Zo, To, Po)) < 1e-10
    bad32 = tt.Solver(p.copy(precision=ti.PREC_FP32))
    with pytest.raises(tt.TTError) as e:
        tt.solve_small_batch([s, bad32], 2)
    assert e.value.status == tt.TT_ERR_INVALID_ARG
    wide = tt.Solver(ti.plane2d(n=8, n_groups=2, n_theta=4, n_phi=8, precision=ti.PREC_FP64),
                     round_method=tt.TT_ROUND_QR)
    with pytest.raises(tt.TTError) as e:
        tt.solve_small_batch([wide], 2)
    assert e.value.status == tt.TT_ERR_INVALID_ARG
