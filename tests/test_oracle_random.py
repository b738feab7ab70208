"""Pins of the oracle's randomized rounding (Section 3.1 footnote: sketch
ranks = solution ranks + a constant, then the SVD truncation at the same
tolerance; the compression is randomize-then-orthogonalize) and of its
counter-based generator (Philox-4x32-10, published known answers)."""
import os

import numpy as np
import pytest

import tt_inputs as ti
from oracle import dense, philox, tt as ott

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_philox_known_answers():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert philox.philox4x32_10(v[0:4], v[4:6]) == tuple(v[6:10])


def test_sketch_entries_are_the_generator_words_mapped_to_minus_one_one():
    e = philox.sketch_entries(0x1234567890, 1, 7, 6)
    for i in range(6):
        w = philox.philox4x32_10((i, 1, 7, 0), (0x34567890, 0x12))
        x = (w[0] << 21) | (w[1] >> 11)
        assert e[i] == x / 2.0 ** 52 - 1.0
    big = philox.sketch_entries(3, 0, 0, 200000)
    assert big.min() >= -1.0 and big.max() < 1.0
    # uniform on [-1, 1): mean 0 and variance 1/3 within sampling error (5 sigma)
    assert abs(big.mean()) < 5 * np.sqrt(1 / 3 / big.size)
    assert abs(big.var() - 1 / 3) < 5 * np.sqrt(4 / 45 / big.size)
    # cores, rounding passes and keys draw different numbers
    a = philox.sketch_entries(3, 0, 0, 8)
    for other in (philox.sketch_entries(3, 1, 0, 8), philox.sketch_entries(3, 0, 1, 8),
                  philox.sketch_entries(4, 0, 0, 8)):
        assert not np.any(a == other)


def _sum_case(r=3, seed=0):
    p = ti.plane2d(n=7, n_groups=3, n_theta=4, n_phi=6, T=0.3)
    p.n_cells = (7, 5, 1)
    p.kappa0 = np.random.default_rng(seed).uniform(0.3, 3.0, 35)
    p.T_cell = np.full(35, 0.3)
    Z, Th, Ph = ti.random_tt(p.M, 4, 6, r, r, seed=seed + 1, decay=0.7)
    return p, (Z, Th, Ph), ott.apply_step(p, Z, Th, Ph)


def test_precondition_equals_the_dense_randomized_range_projection():
    # brute force on the full tensor X (M, N_theta, N_phi): the random TT's
    # right part for bond 1 is T1[a, l, p] = sum_b G2[a, l, b] G3[b, p]; then
    # Q1 = basis(X_(1) T1^T), X1 = Q1^T X_(1), Q2 = basis(X1_(2) G3^T) and the
    # compressed tensor is Q1 Q2 Q2^T X1.  The core-wise contractions must give
    # the same tensor while the projection is far from the identity.
    p, _, (Z, Th, Ph) = _sum_case()
    R1, nt, R2 = Th.shape
    X = ott.full(Z, Th, Ph)
    l1, l2 = 5, 4
    G2, G3 = ott.sketch_cores(11, 2, l1, nt, l2, 6)
    T1 = np.einsum("alb,bp->alp", G2, G3).reshape(l1, nt * 6)
    Q1 = ott.range_basis(X.reshape(p.M, -1) @ T1.T)
    X1 = (Q1.T @ X.reshape(p.M, -1)).reshape(-1, 6)
    Q2 = ott.range_basis(X1 @ G3.T)
    Xt = (Q1 @ (Q2 @ (Q2.T @ X1)).reshape(Q1.shape[1], -1)).reshape(X.shape)
    Ct = ott.randomized_precondition(Z, Th, Ph, G2, G3)
    assert Ct[0].shape[1] == l1 and Ct[2].shape[0] == l2
    np.testing.assert_allclose(ott.full(*Ct), Xt, rtol=0, atol=1e-12 * np.abs(X).max())
    assert _rel(Xt, X) > 1e-3
    # the compressed TT is left-orthonormal
    np.testing.assert_allclose(Ct[0].T @ Ct[0], np.eye(l1), atol=1e-13)
    Q2c = Ct[1].reshape(-1, l2)
    np.testing.assert_allclose(Q2c.T @ Q2c, np.eye(l2), atol=1e-13)


def test_full_sketch_ranks_give_the_svd_rounding():
    # sketch ranks equal to the orthogonalised ranks of the sum span it, so the
    # compression is exact and the truncation is that of TT-SVD rounding
    # (unique for distinct singular values, Eckart-Young)
    p, (Z0, _, Ph0), (Z, Th, Ph) = _sum_case()
    R1, nt, R2 = Th.shape
    k2 = min(R2, 6)
    k1 = min(R1, nt * k2)
    a = ott.round_tt(Z, Th, Ph, 1e-4, 50)
    b = ott.randomized_round(Z, Th, Ph, 1e-4, 50, (Z0.shape[1], Ph0.shape[0]), 100, 5, 0)
    assert (b[3]["l1"], b[3]["l2"]) == (k1, k2)
    assert (a[3]["r1"], a[3]["r2"]) == (b[3]["r1"], b[3]["r2"])
    assert _rel(ott.full(*b[:3]), ott.full(*a[:3])) < 1e-12


def test_sketch_of_a_sum_with_lower_true_rank_is_exact():
    # three copies of a rank-(2, 2) TT: the sum has ranks (6, 6) but the tensor
    # has ranks (2, 2); sketch ranks (3, 3) capture it exactly
    Z, Th, Ph = ti.random_tt(60, 4, 6, 2, 2, seed=4)
    Zs, Ths, Phs = ott._assemble([Z, 2 * Z, -Z], [Th, Th, Th], [Ph, Ph, Ph], 4)
    X = ott.full(Z, Th, Ph) * 2.0
    G2, G3 = ott.sketch_cores(1, 0, 3, 4, 3, 6)
    Ct = ott.randomized_precondition(Zs, Ths, Phs, G2, G3)
    assert Ct[0].shape[1] == 2 and Ct[2].shape[0] == 2     # the null sketch direction is dropped
    assert _rel(ott.full(*Ct), X) < 1e-13


def test_randomized_solve_with_spanning_sketch_equals_the_dense_march():
    p = ti.slab1d(n_cells=13, n_groups=3, n_theta=6, T=0.3, tol=1e-14, rank_cap=60)
    p = p.copy(round_method=ti.ROUND_RAND, rand_oversample=60)
    steps = 6
    (Z, Th, Ph), _ = ott.solve(p, steps)
    ref = dense.march(p, dense.initial_dense(p), steps)
    assert _rel(ott.full(Z, Th, Ph), ref) < 1e-11


def test_randomized_solve_tracks_the_svd_solve_within_the_tolerance():
    # oversampling 4 as in the paper's k_s comparison: each pass discards at
    # most delta per bond after a compression that keeps the incoming ranks
    # plus 4; over K steps the two solutions stay within a few K tol
    p = ti.plane2d(n=8, n_groups=3, n_theta=4, n_phi=6, tol=1e-6, rank_cap=12)
    K = 10
    a, ia = ott.solve(p, K)
    b, ib = ott.solve(p.copy(round_method=ti.ROUND_RAND), K)
    assert _rel(ott.full(*b), ott.full(*a)) < 2 * K * p.tol
    assert all(i["l1"] <= i["R1"] for i in ib)
    # a different key draws different cores: the same bound, not the same tensor
    c, _ = ott.solve(p.copy(round_method=ti.ROUND_RAND, rand_seed=9), K)
    assert 0 < _rel(ott.full(*c), ott.full(*b)) < 2 * K * p.tol


def test_paper_step_order_numbers_both_rounding_passes():
    p = ti.slab1d(n_cells=11, n_groups=3, n_theta=6, T=0.3, tol=1e-6, rank_cap=8)
    p = p.copy(round_method=ti.ROUND_RAND, step_order=1)
    Z, Th, Ph = ott.initial_tt(p)
    one = ott.step(p, Z, Th, Ph, round_index=4)
    Zt, Tt, Pt, _ = ott._round(p, *ott.apply_transport(p, Z, Th, Ph), p.tol, p.rank_cap, (1, 1), 4)
    two = ott._round(p, *ott.apply_source(p, Zt, Tt, Pt), p.tol, p.rank_cap, (Zt.shape[1], Pt.shape[0]), 5)
    assert np.array_equal(ott.full(*one[:3]), ott.full(*two[:3]))
