"""GPU checks of the diagnostics, the numeric-error path, checkpoint and
resume, the TSQR tree levels and the full-size shapes, through the C ABI
against the CPU oracle.

* Statistics (Section 3.2): the norm before truncation, the discarded tail,
  the compression and the storage factor k_s of the last rounding equal the
  oracle's for an FP64 QR step (1e-12 relative; ranks and counts exactly).
* A NaN in the state (host input through set_cores) is reported as
  TT_ERR_NUMERIC by solve; the kernels finish normally and the handle is
  usable again after reset.
* Checkpoint / resume: solve(K) equals solve(k), get_cores, set_cores on a
  fresh handle, solve(K - k) (1e-12 FP64; the warm-started Jacobi of the
  first step after a restore starts cold, which changes only rounding noise).
* The Householder TSQR tree: QR-route cores of 16 columns with several
  leaf blocks and one tree level, of 64 columns with three tree levels, and of
  128 columns whose last leaf block ends inside a row chunk, against the
  oracle at the FP64 bounds (1e-12 per step, 1e-10 per solve); and at tol
  1e-14 a 2D solve with TSQR rounding equals the dense march to 1e-10 (Gram
  rounding to 1e-5).
* Full sizes: the 128 x 128 x 32-group workload in FP64 (five TSQR levels),
  and the 3D workload's angular shape (8 x 16 directions, rank 64, so the
  sum has R1 = 450 and the projected core k1 = 128) on 24^3 cells x 16
  groups in FP64, FP32 and split BF16 at their bounds (1e-12, 2e-6, 5e-5 per
  step), plus a 24-step solve from the same seeded state at cap 64.
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
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _plane(n=(11, 9), G=4, nt=4, nphi=6, prec=ti.PREC_FP64, tol=1e-6, cap=16, seed=0):
    p = ti.plane2d(n=n[0], n_groups=G, n_theta=nt, n_phi=nphi, tol=tol, rank_cap=cap, precision=prec, seed=seed)
    p.n_cells = (n[0], n[1], 1)
    p.kappa0 = ti.lognormal_kappa0(p.n_cells, p.extent, 2, seed=seed)
    p.T_cell = np.full(n[0] * n[1], 0.1)
    return p


@pytest.mark.parametrize("dim", [1, 2])
def test_stats_match_oracle_info(tt, dim):
    # caps that bind, so that both the norm and a non-empty discarded tail are compared
    if dim == 1:
        p = ti.slab1d(n_cells=37, n_groups=5, n_theta=8, tol=1e-4, rank_cap=4)
        p.kappa0 = ti.lognormal_kappa0(p.n_cells, p.extent, 1, seed=3)
    else:
        p = _plane(tol=1e-4)
    print(f"stats dim={dim}", flush=True)
    s = tt.Solver(p, round_method=tt.TT_ROUND_QR)
    Z, Th, Ph = ti.random_tt(p.M, p.n_theta, p.n_phi, 4, min(3, p.n_phi), seed=9, decay=0.5)
    s.set_cores(Z, Th, Ph)
    st = s.solve(1)
    Zo, To, Po, info = ott.step(p, Z, Th, Ph)
    assert (st["r1"], st["r2"]) == (info["r1"], info["r2"])
    assert (st["max_R1"], st["max_R2"]) == (info["R1"], info["R2"])
    assert info["discarded"] > 1e-8 * info["norm"]     # the truncation is not empty
    assert st["norm"] == pytest.approx(info["norm"], rel=1e-12)
    assert st["discarded_rel"] == pytest.approx(info["discarded"] / info["norm"], rel=1e-9)
    assert st["compression"] == pytest.approx(ott.compression(p, info["r1"], info["r2"]), rel=1e-14)
    assert st["k_s"] == pytest.approx(info["k_s"], rel=1e-14)
    assert st["k_s_impl"] > 1.0
    assert st["energy"] == pytest.approx(ott.tt_energy(p, Zo, To, Po), rel=1e-11)
    assert st["nan_flag"] == 0
    s.destroy()


@pytest.mark.parametrize("prec", [ti.PREC_FP64, ti.PREC_FP32])
def test_nan_in_the_state_is_reported(tt, prec):
    p = _plane(prec=prec, tol=1e-6, cap=12)
    print(f"nan prec={prec}", flush=True)
    s = tt.Solver(p)
    Z, Th, Ph = ti.random_tt(p.M, p.n_theta, p.n_phi, 4, 3, seed=2, decay=0.6)
    Z[17, 2] = np.nan
    s.set_cores(Z, Th, Ph)
    with pytest.raises(tt.TTError) as e:
        s.solve(2)
    assert e.value.status == tt.TT_ERR_NUMERIC
    assert s.get_stats()["nan_flag"] == 1
    # the handle recovers from a clean state
    s.reset()
    st = s.solve(2)
    assert st["nan_flag"] == 0
    s.destroy()


@pytest.mark.parametrize("prec,method,bound", [(ti.PREC_FP64, "qr", 1e-12), (ti.PREC_FP32, "auto", 1e-6)])
def test_checkpoint_resume(tt, prec, method, bound):
    p = _plane(prec=prec, tol=1e-7, cap=16)
    rm = tt.TT_ROUND_QR if method == "qr" else tt.TT_ROUND_AUTO
    K, k = 20, 8
    print(f"checkpoint prec={prec}", flush=True)
    a = tt.Solver(p, round_method=rm)
    st_a = a.solve(K)
    ref = full(*a.get_cores())
    b = tt.Solver(p, round_method=rm)
    b.solve(k)
    cores = b.get_cores()
    b.destroy()
    c = tt.Solver(p, round_method=rm)
    c.set_cores(*cores)
    st_c = c.solve(K - k)
    assert (st_c["r1"], st_c["r2"]) == (st_a["r1"], st_a["r2"])
    assert rel(full(*c.get_cores()), ref) < bound
    a.destroy()
    c.destroy()


def test_tsqr_16_column_cores_with_a_tree_level(tt):
    # 1D, 256 cells x 16 groups, 16 Gauss-Legendre mu: k1 <= 16, M = 4096 rows
    # in eight 512-row leaf blocks, so one tree level of the 16-column TSQR runs
    p = ti.slab1d(n_cells=256, n_groups=16, n_theta=16, tol=1e-8, rank_cap=16)
    p.kappa0 = ti.lognormal_kappa0(p.n_cells, p.extent, 1, seed=4)
    print("tsqr 16-column tree", flush=True)
    s = tt.Solver(p, round_method=tt.TT_ROUND_QR)
    Z, Th, Ph = ti.random_tt(p.M, 16, 1, 6, 1, seed=3, decay=0.5)
    s.set_cores(Z, Th, Ph)
    s.solve(1)
    Zo, To, Po, info = ott.step(p, Z, Th, Ph)
    assert info["R1"] >= 16 and s.get_ranks() == (info["r1"], info["r2"])
    assert rel(full(*s.get_cores()), full(Zo, To, Po)) < 1e-12
    st = s.solve(10)
    (Zs, Ts, Ps), infos = ott.solve(p, 10, cores=(Zo, To, Po))
    assert (st["r1"], st["r2"]) == (infos[-1]["r1"], infos[-1]["r2"])
    assert rel(full(*s.get_cores()), full(Zs, Ts, Ps)) < 1e-10
    s.destroy()


def test_tsqr_64_column_cores_with_three_tree_levels(tt):
    # 2D, 50 x 50 cells x 8 groups, 8 x 8 directions: k1 = 64, M = 20000 rows
    # in 27 leaf blocks of four 192-row chunks (the last holds 32 rows), then
    # tree levels of 320-row blocks: six (the last with 128 rows), two (the
    # last with 64 rows) and one
    p = _plane(n=(50, 50), G=8, nt=8, nphi=8, tol=1e-7, cap=32, seed=5)
    print("tsqr 64-column three tree levels", flush=True)
    s = tt.Solver(p, round_method=tt.TT_ROUND_QR)
    Z, Th, Ph = ti.random_tt(p.M, 8, 8, 20, 8, seed=8, decay=0.75)
    s.set_cores(Z, Th, Ph)
    s.solve(1)
    Zo, To, Po, info = ott.step(p, Z, Th, Ph)
    assert info["R1"] >= 64 and s.get_ranks() == (info["r1"], info["r2"])
    assert rel(full(*s.get_cores()), full(Zo, To, Po)) < 1e-12
    st = s.solve(6)
    (Zs, Ts, Ps), infos = ott.solve(p, 6, cores=(Zo, To, Po))
    assert (st["r1"], st["r2"]) == (infos[-1]["r1"], infos[-1]["r2"])
    assert rel(full(*s.get_cores()), full(Zs, Ts, Ps)) < 1e-10
    s.destroy()


def test_tsqr_128_column_cores_with_a_ragged_leaf(tt):
    # 3D, 7 x 6 x 5 cells x 8 groups, 8 x 16 directions, from a rank-(64, 16)
    # state: k1 = 128, M = 1680 rows in five leaf blocks of four 96-row
    # chunks, the last holding 144 rows (one and a half chunks), then tree
    # levels of three blocks (the last with 128 rows), two and one
    rng = np.random.default_rng(6)
    p = ti.clumps3d(n=8, n_groups=8, n_theta=8, n_phi=16, tol=1e-9, rank_cap=64, precision=ti.PREC_FP64, T=0.3)
    p.n_cells = (7, 6, 5)
    p.kappa0 = rng.uniform(0.3, 3.0, 210)
    p.T_cell = np.full(210, 0.3)
    print(f"tsqr 128-column ragged leaf M={p.M}", flush=True)
    s = tt.Solver(p, round_method=tt.TT_ROUND_QR)
    Z, Th, Ph = ti.random_tt(p.M, 8, 16, 64, 16, seed=21, decay=0.9)
    s.set_cores(Z, Th, Ph)
    st = s.solve(1)
    Zo, To, Po, info = ott.step(p, Z, Th, Ph)
    assert (info["R1"], st["max_R1"]) == (450, 450)
    assert s.get_ranks() == (info["r1"], info["r2"])
    assert rel(full(*s.get_cores()), full(Zo, To, Po)) < 1e-12
    st = s.solve(4)
    (Zs, Ts, Ps), infos = ott.solve(p, 4, cores=(Zo, To, Po))
    assert (st["r1"], st["r2"]) == (infos[-1]["r1"], infos[-1]["r2"])
    assert rel(full(*s.get_cores()), full(Zs, Ts, Ps)) < 1e-10
    s.destroy()


def test_tsqr_rounding_at_tol_1e14_matches_the_dense_march(tt):
    # 2D, 12 x 10 cells x 4 groups, 8 x 8 directions, tol 1e-14 and a cap above
    # the solution's rank: with Householder TSQR rounding (64-column tile, four
    # leaf blocks and one tree level) the TT solve equals the dense FP64 march
    # to 1e-10 after 24 steps; Gram rounding, which resolves singular values
    # only down to ~1e-8 of the norm, stays within 1e-5
    p = _plane(n=(12, 10), G=4, nt=8, nphi=8, tol=1e-14, cap=64, seed=2)
    print(f"tol 1e-14 against the dense march M={p.M}", flush=True)
    ref = dense.march(p, dense.initial_dense(p), 24)
    errs = {}
    for name, method in (("qr", tt.TT_ROUND_QR), ("gram", tt.TT_ROUND_GRAM)):
        s = tt.Solver(p, round_method=method)
        s.solve(24)
        errs[name] = rel(full(*s.get_cores()), ref)
        s.destroy()
    print(f"rel-L2 against the dense march: {errs}", flush=True)
    assert errs["qr"] < 1e-10
    assert errs["gram"] < 1e-5


def test_plane2d_full_size_one_step_fp64(tt):
    # the 2D workload at full size in FP64 (Householder TSQR over 524288 rows:
    # 456 leaf blocks and four tree levels), one step from a rank-(32, 8) state
    p = ti.plane2d(precision=ti.PREC_FP64)
    print("plane2d full size fp64", flush=True)
    s = tt.Solver(p, round_method=tt.TT_ROUND_QR)
    Z, Th, Ph = ti.random_tt(p.M, 8, 8, 32, 8, seed=3, decay=0.8)
    s.set_cores(Z, Th, Ph)
    s.solve(1)
    Zo, To, Po, info = ott.step(p, Z, Th, Ph)
    assert s.get_ranks() == (info["r1"], info["r2"])
    assert rel(full(*s.get_cores()), full(Zo, To, Po)) < 1e-12
    s.destroy()


def _c3_shaped(n, G, prec, seed=0):
    # the 3D workload's generator and angular shape (8 x 16 directions,
    # 2 clumps x100 in a lognormal field, cap 64) on n^3 cells x G groups
    return ti.clumps3d(n=n, n_groups=G, n_theta=8, n_phi=16, tol=1e-5, rank_cap=64, precision=prec, seed=seed)


@pytest.mark.parametrize("prec,bound", [(ti.PREC_FP64, 1e-12), (ti.PREC_FP32, 2e-6), (ti.PREC_BF16X, 5e-5)])
def test_c3_shaped_one_step(tt, prec, bound):
    p = _c3_shaped(24, 16, prec)
    print(f"c3-shaped one step prec={prec} M={p.M}", flush=True)
    s = tt.Solver(p)
    Z, Th, Ph = ti.random_tt(p.M, 8, 16, 64, 16, seed=12, decay=0.9)
    s.set_cores(Z, Th, Ph)
    st = s.solve(1)
    Zo, To, Po, info = ott.step(p, Z, Th, Ph)
    assert (info["R1"], st["max_R1"]) == (450, 450)
    r1, r2 = s.get_ranks()
    if prec == ti.PREC_FP64:
        assert (r1, r2) == (info["r1"], info["r2"])
    else:
        assert abs(r1 - info["r1"]) <= 1 and abs(r2 - info["r2"]) <= 1
    slack = 2 * p.tol * ((r1, r2) != (info["r1"], info["r2"]))
    assert rel(full(*s.get_cores()), full(Zo, To, Po)) < bound + slack
    s.destroy()


@pytest.mark.parametrize("prec,bound", [(ti.PREC_FP64, 1e-10), (ti.PREC_FP32, 1e-4), (ti.PREC_BF16X, 1e-4)])
def test_c3_shaped_solve(tt, prec, bound):
    p = _c3_shaped(10, 8, prec, seed=1)
    K = 24
    print(f"c3-shaped solve prec={prec} M={p.M}", flush=True)
    s = tt.Solver(p)
    Z, Th, Ph = ti.random_tt(p.M, 8, 16, 64, 16, seed=13, decay=0.9)
    s.set_cores(Z, Th, Ph)
    st = s.solve(K)
    (Zo, To, Po), infos = ott.solve(p, K, cores=(Z, Th, Ph))
    assert max(i["R1"] for i in infos) == 450
    if prec == ti.PREC_FP64:
        assert (st["r1"], st["r2"]) == (infos[-1]["r1"], infos[-1]["r2"])
    assert rel(full(*s.get_cores()), full(Zo, To, Po)) < bound
    s.destroy()
