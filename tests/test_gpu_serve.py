"""Serving loop on the GPU: requests admitted by memory, overlapping on the
device, give the same result as when run alone (bitwise: the kernels are
deterministic and no reduction crosses requests)."""
import numpy as np
import pytest

import tt_inputs as ti

pytestmark = pytest.mark.gpu


def _mix():
    reqs = []
    # 1D and 2D, FP64 (QR rounding) and FP32 (fused Gram rounding), different caps and sizes
    reqs.append(ti.slab1d(n_cells=40, n_groups=6, rank_cap=6, precision=ti.PREC_FP64, n_steps=5))
    reqs.append(ti.plane2d(n=24, n_groups=8, rank_cap=12, precision=ti.PREC_FP32, n_steps=7, seed=3))
    reqs.append(ti.plane2d(n=19, n_groups=5, rank_cap=7, precision=ti.PREC_FP64, n_steps=6, seed=4))
    reqs.append(ti.slab1d(n_cells=33, n_groups=9, rank_cap=5, precision=ti.PREC_FP32, n_steps=8))
    reqs.append(ti.plane2d(n=30, n_groups=6, rank_cap=16, precision=ti.PREC_FP32, n_steps=5, seed=5))
    reqs.append(ti.plane2d(n=17, n_groups=7, rank_cap=9, precision=ti.PREC_FP32, n_steps=9, seed=6))
    return reqs


def test_served_results_equal_alone():
    import torch

    import paper_2602_00290_amd as tt
    from paper_2602_00290_amd.serve import Server, make_requests

    probs = _mix()
    arrivals = [0.0, 0.0, 0.002, 0.004, 0.004, 0.01]
    reqs = make_requests(probs, arrivals)
    nbytes = [tt.workspace_bytes(p) + 256 for p in probs]
    # a budget that holds about two requests at a time forces queueing on memory
    srv = Server(budget_bytes=int(2.2 * max(nbytes)), max_active=3, n_streams=2, chunk=2, keep_results=True)
    out = srv.run(reqs)
    assert out["requests"] == len(probs)
    assert out["max_active"] <= 3
    assert out["peak_workspace_bytes"] <= srv.budget
    assert np.isfinite(out["p99_ms"]) and out["p50_ms"] > 0
    for i, p in enumerate(probs):
        s = tt.Solver(p)
        s.solve(p.n_steps)
        Z, Th, Ph = s.get_cores()
        Zs, Ths, Phs = srv.results[i]
        assert Z.shape == Zs.shape and Th.shape == Ths.shape, f"request {i}: ranks differ"
        assert np.array_equal(Z, Zs) and np.array_equal(Th, Ths) and np.array_equal(Ph, Phs), f"request {i}"
        s.destroy()
    torch.cuda.synchronize()
