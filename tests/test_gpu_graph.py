"""hipGraph replay of the step sequence (tt_transport_set_graph): solves with
graphs on give bitwise the results of launching every kernel, on every
replay, with the program's own launched work and synchronisations between
the replays (a graph is replayed many times after its capture), for the
fused FP32 path, the FP64 Gram and QR routes, the paper's step order, the
coupled medium temperature and randomized rounding; batched solves with
graphs equal the same solves alone."""
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


def _plane(prec, **kw):
    p = ti.plane2d(n=11, n_groups=4, n_theta=4, n_phi=6, tol=1e-6, rank_cap=12, precision=prec, seed=3)
    p.n_cells = (11, 9, 1)
    p.kappa0 = ti.lognormal_kappa0(p.n_cells, p.extent, 2, seed=3)
    p.T_cell = np.full(99, 0.1)
    return p.copy(**kw)


def _case(name):
    if name == "fp32_fused":
        return _plane(ti.PREC_FP32), None
    if name == "fp64_gram":
        return _plane(ti.PREC_FP64), 1
    if name == "fp64_qr_3d":
        p = ti.clumps3d(n=5, n_groups=3, n_theta=4, n_phi=4, tol=1e-7, rank_cap=16, precision=ti.PREC_FP64)
        p.n_cells = (5, 4, 3)
        p.kappa0 = ti.lognormal_kappa0(p.n_cells, p.extent, 3, seed=1)
        p.T_cell = np.full(60, 0.1)
        return p, 0
    if name == "paper_order":
        return _plane(ti.PREC_FP64, step_order=1), 0
    if name == "coupled":
        p = ti.slab1d(n_cells=30, n_groups=4, n_theta=8, tol=1e-8, rank_cap=8)
        return p.copy(heat_capacity=0.5, T_cell=np.full(30, 0.4)), None
    if name == "randomized":
        return _plane(ti.PREC_FP32, round_method=ti.ROUND_RAND, rand_oversample=4, rand_seed=9), None
    raise ValueError(name)


@pytest.mark.parametrize("name", ["fp32_fused", "fp64_gram", "fp64_qr_3d", "paper_order", "coupled", "randomized"])
def test_graph_replay_equals_launched_kernels(tt, name):
    import torch
    p, method = _case(name)
    stream = torch.cuda.Stream()
    print(f"graph {name}", flush=True)
    eager = tt.Solver(p, stream=stream, round_method=method)
    graph = tt.Solver(p, stream=stream, round_method=method)
    graph.set_graph(True)
    other = tt.Solver(_plane(ti.PREC_FP32), stream=stream)
    K = 9                                   # four graph replays and one launched step
    for rep in range(3):
        eager.reset()
        graph.reset()
        eager.solve(K)
        other.solve(3)                      # launched work between the replays
        torch.cuda.synchronize()
        graph.solve(K)
        for a, b in zip(graph.get_cores(), eager.get_cores()):
            np.testing.assert_array_equal(a, b)
    for s in (eager, graph, other):
        s.destroy()


def test_batched_graphs_equal_solves_alone(tt):
    import torch
    probs = [_plane(ti.PREC_FP32), _plane(ti.PREC_FP64), _case("fp64_qr_3d")[0]]
    alone = []
    for p in probs:
        s = tt.Solver(p)
        s.solve(10)
        alone.append(s.get_cores())
        s.destroy()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    solvers = [tt.Solver(p) for p in probs]
    for s in solvers:
        s.set_graph(True)
    for rep in range(2):
        for s in solvers:
            s.reset()
        tt.solve_batch(solvers, 10, streams)
        for s, ref in zip(solvers, alone):
            for a, b in zip(s.get_cores(), ref):
                np.testing.assert_array_equal(a, b)
