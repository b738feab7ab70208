"""Launch-shape tuning (tt_transport_tune, set_launch, get_launch) through the
C ABI against the oracle's rounding step (Section 3.1: the first-core steps
of the TT rounding).  The grids of the persistent contraction kernels and the
row split of the Gram change only the order of the Gram's partial sums, so
every shape must give the oracle's result at the path's own tolerance:

* FP64 Gram route with the 3D workload's angular shape (8 x 16 directions,
  cap 64, so k1 = 128): FP64 MFMA projection and output, the 128-column Gram
  over row ranges.  One step at explicit grids from a single block, through
  counts that are not multiples of the 8 XCDs, to the maximum: 1e-8, equal
  ranks.
* FP64 Gram route with at most 64 columns (the Gram partials fused into the
  projection, one per projection block), 2D: 1e-8, equal ranks.
* FP32 fused projection + Gram and fused output, the 2D workload at full
  size: 2e-6 (the FP32 state's bound), equal ranks.
* tune() on each: the chosen grids are within the maxima, the state is
  unchanged (the next step equals the oracle's step from the same cores), and
  later handles of the same problem (one at the same state, one in its
  initial state) take the grids from the cache file without timing.
* Invalid grids are refused.
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


def _case(name):
    if name == "fp64_k1_128":
        p = ti.clumps3d(n=24, n_groups=16, n_theta=8, n_phi=16, tol=1e-5, rank_cap=64, precision=ti.PREC_FP64)
        cores = ti.random_tt(p.M, 8, 16, 64, 16, seed=21, decay=0.9)
        return p, "gram", cores, 1e-8
    if name == "fp64_fused_gram":
        p = ti.plane2d(n=128, n_groups=32, n_theta=4, n_phi=6, tol=1e-6, rank_cap=24, precision=ti.PREC_FP64)
        cores = ti.random_tt(p.M, 4, 6, 16, 4, seed=23, decay=0.8)
        return p, "gram", cores, 1e-8
    p = ti.plane2d()                       # FP32, fused Gram path
    cores = ti.random_tt(p.M, 8, 8, 32, 8, seed=3, decay=0.8)
    return p, "auto", cores, 2e-6


_ORACLE = {}


def _oracle(name, p, cores):
    if name not in _ORACLE:
        _ORACLE[name] = ott.step(p, *cores)
    return _ORACLE[name]


def _solver(tt, p, method):
    return tt.Solver(p, round_method=tt.TT_ROUND_GRAM if method == "gram" else tt.TT_ROUND_AUTO)


CASES = ["fp64_k1_128", "fp64_fused_gram", "fp32_fused_2d"]


@pytest.mark.parametrize("name", CASES)
def test_every_grid_matches_the_oracle(tt, name):
    p, method, cores, bound = _case(name)
    Zo, To, Po, info = _oracle(name, p, cores)
    ref = full(Zo, To, Po)
    s = _solver(tt, p, method)
    cur, mx = s.get_launch()
    s.destroy()
    assert mx["project_blocks"] > 0 and mx["output_blocks"] > 0
    assert (mx["gram_blocks"] > 0) == (name == "fp64_k1_128")
    assert all(0 < cur[k] <= mx[k] for k in cur if mx[k] > 0)
    shapes = [(1, 1, 1), (7, 13, 37), (cur["project_blocks"], cur["output_blocks"], cur["gram_blocks"]),
              (mx["project_blocks"], mx["output_blocks"], mx["gram_blocks"])]
    for pb, ob, gb in shapes:
        gb = gb if mx["gram_blocks"] > 0 else 0
        print(f"tune: {name} M={p.M} grids project {pb} output {ob} gram {gb}", flush=True)
        s = _solver(tt, p, method)
        s.set_launch(project_blocks=pb, output_blocks=ob, gram_blocks=gb)
        got, _ = s.get_launch()
        assert got["project_blocks"] == pb and got["output_blocks"] == ob
        assert got["gram_blocks"] <= gb
        s.set_cores(*cores)
        s.solve(1)
        assert s.get_ranks() == (info["r1"], info["r2"])
        assert rel(full(*s.get_cores()), ref) < bound
        s.destroy()


@pytest.mark.parametrize("name", CASES)
def test_tune_keeps_the_state_and_caches(tt, name, tmp_path):
    p, method, cores, bound = _case(name)
    Zo, To, Po, info = _oracle(name, p, cores)
    cache = str(tmp_path / "tune.txt")
    print(f"tune: {name} M={p.M} tune()", flush=True)
    s = _solver(tt, p, method)
    s.set_cores(*cores)
    res = s.tune(cache)
    _, mx = s.get_launch()
    assert res["from_cache"] == 0
    for k in ("project", "output", "gram"):
        if mx[k + "_blocks"] == 0:
            assert res[k + "_blocks"] == 0
            continue
        assert 0 < res[k + "_blocks"] <= mx[k + "_blocks"]
        assert res[k + "_ms"] > 0 and res[k + "_ms_default"] > 0
        assert res[k + "_ms"] <= res[k + "_ms_default"]
    s.solve(1)
    assert s.get_ranks() == (info["r1"], info["r2"])
    assert rel(full(*s.get_cores()), full(Zo, To, Po)) < bound
    s.destroy()
    # a second handle of the same shape: the grids come from the cache
    s2 = _solver(tt, p, method)
    s2.set_cores(*cores)
    res2 = s2.tune(cache)
    assert res2["from_cache"] == 1
    assert all(res2[k] == res[k] for k in ("project_blocks", "output_blocks", "gram_blocks"))
    s2.solve(1)
    assert rel(full(*s2.get_cores()), full(Zo, To, Po)) < bound
    s2.destroy()
    # the key is the problem's shape, not the current ranks: a new handle in
    # its rank-1 initial state finds the same entry
    s3 = _solver(tt, p, method)
    res3 = s3.tune(cache)
    assert res3["from_cache"] == 1
    assert all(res3[k] == res[k] for k in ("project_blocks", "output_blocks", "gram_blocks"))
    s3.destroy()
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and lines[0].split()[1:] == [str(res[k]) for k in
                                                         ("project_blocks", "output_blocks", "gram_blocks")]


def test_invalid_grids_are_refused(tt):
    p = ti.plane2d(n=16, n_groups=4, n_theta=4, n_phi=4, tol=1e-6, rank_cap=8, precision=ti.PREC_FP64)
    s = tt.Solver(p, round_method=tt.TT_ROUND_QR)        # FP64 MFMA contractions, TSQR: no Gram grid
    _, mx = s.get_launch()
    assert mx["gram_blocks"] == 0 and mx["project_blocks"] > 0
    for kw in ({"project_blocks": mx["project_blocks"] + 1}, {"output_blocks": -1}, {"gram_blocks": 4}):
        with pytest.raises(tt.TTError) as e:
            s.set_launch(**kw)
        assert e.value.status == tt.TT_ERR_INVALID_ARG
    s.destroy()
