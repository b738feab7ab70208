"""tt_transport_create_noalloc: a solver on the library's static per-device
workspace (for callers that cannot allocate device memory), through the C
ABI, against tt_transport_create on a caller-allocated workspace.

Both run the same kernels on the same inputs, so the results must be bitwise
equal (the FP64 parity bar is 1e-10 against the oracle; equality here is
stronger).  Two calls in a row, the second with a smaller problem, show that
the array's previous contents do not leak into the next solve; a second
handle while the first holds the array is refused, and a problem above the
static size is rejected."""
import numpy as np
import pytest

import tt_inputs as ti

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_00290_amd as tt
    return tt


def _solve(tt, prob, steps, noalloc):
    s = tt.Solver(prob, noalloc=noalloc)
    st = s.solve(steps)
    cores = s.get_cores()
    s.destroy()
    return st, cores


def test_noalloc_equals_create_twice_with_a_smaller_second_problem(tt):
    big = ti.slab1d(n_cells=64, n_groups=8, n_theta=16, tol=1e-8, rank_cap=8)
    small = ti.slab1d(n_cells=24, n_groups=5, n_theta=8, tol=1e-7, rank_cap=6, T=0.2)
    for prob, steps in ((big, 40), (small, 25)):
        print(f"noalloc M={prob.M} steps={steps}", flush=True)
        st_a, ref = _solve(tt, prob, steps, noalloc=False)
        st_b, got = _solve(tt, prob, steps, noalloc=True)
        assert (st_b["r1"], st_b["r2"]) == (st_a["r1"], st_a["r2"])
        for a, b in zip(got, ref):
            np.testing.assert_array_equal(a, b)
        assert st_b["nan_flag"] == 0


def test_noalloc_refuses_a_second_holder_and_oversized_problems(tt):
    prob = ti.slab1d(n_cells=32, n_groups=4, n_theta=8)
    a = tt.Solver(prob, noalloc=True)
    with pytest.raises(tt.TTError) as e:
        tt.Solver(prob, noalloc=True)
    assert e.value.status == tt.TT_ERR_STATE
    a.solve(3)
    a.destroy()
    b = tt.Solver(prob, noalloc=True)     # free again after destroy
    b.destroy()
    with pytest.raises(tt.TTError) as e:
        tt.Solver(ti.plane2d(), noalloc=True)   # ~240 MiB of workspace
    assert e.value.status == tt.TT_ERR_INVALID_ARG
