"""The Gram route's tridiagonal eigensolver (projected first cores wider than
64 columns: Householder tridiagonalisation, Sturm multisection, twisted
eigenvectors, back-transformation; Jacobi when the vectors fail their
checks) through the C ABI against the oracle's SVD rounding (Section 3.1
footnote: the Gram matrix route of the rounding).

* One step of the 3D workload's angular shape (8 x 16 directions, cap 64, so
  k1 = 128) in FP64 with Gram rounding: equal ranks, 1e-8 (the Gram's
  resolution).
* A 12-step FP64 Gram solve with k1 = 96 (8 x 12 directions) from a seeded
  state: equal ranks, 1e-7.
* Plain rounding of constructed states with a known first-bond spectrum
  (Z = U diag(s), Theta with orthonormal rows, Phi = I): a spectrum graded
  over 12 decades, and one whose kept singular values come in exactly equal
  pairs (double eigenvalues, whose eigenvectors independent solves need not
  separate; whichever route the checks take, the result must hold), both
  truncated by the cap between pairs:
  equal ranks, 1e-8; the kept singular values equal the constructed ones
  to 1e-8 of the largest.
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


def test_gram_fp64_k1_128_one_step(tt):
    p = ti.clumps3d(n=24, n_groups=16, n_theta=8, n_phi=16, tol=1e-5, rank_cap=64, precision=ti.PREC_FP64)
    print(f"eig: k1=128 one step M={p.M}", flush=True)
    s = tt.Solver(p, round_method=tt.TT_ROUND_GRAM)
    Z, Th, Ph = ti.random_tt(p.M, 8, 16, 64, 16, seed=21, decay=0.9)
    s.set_cores(Z, Th, Ph)
    st = s.solve(1)
    Zo, To, Po, info = ott.step(p, Z, Th, Ph)
    assert st["max_R1"] == 450
    assert s.get_ranks() == (info["r1"], info["r2"])
    assert rel(full(*s.get_cores()), full(Zo, To, Po)) < 1e-8
    s.destroy()


def test_gram_fp64_k1_96_solve(tt):
    p = ti.clumps3d(n=8, n_groups=8, n_theta=8, n_phi=12, tol=1e-6, rank_cap=48, precision=ti.PREC_FP64, seed=2)
    K = 12
    print(f"eig: k1=96 solve M={p.M}", flush=True)
    s = tt.Solver(p, round_method=tt.TT_ROUND_GRAM)
    Z, Th, Ph = ti.random_tt(p.M, 8, 12, 48, 12, seed=22, decay=0.9)
    s.set_cores(Z, Th, Ph)
    st = s.solve(K)
    (Zo, To, Po), infos = ott.solve(p, K, cores=(Z, Th, Ph))
    assert (st["r1"], st["r2"]) == (infos[-1]["r1"], infos[-1]["r2"])
    assert rel(full(*s.get_cores()), full(Zo, To, Po)) < 1e-7
    s.destroy()


def _constructed(p, sv, seed):
    # X_(1) = Z Theta_(1) with Theta_(1) (r x 128) orthonormal rows, Phi = I:
    # the first bond's singular values are sv
    rng = np.random.default_rng(seed)
    r = len(sv)
    U, _ = np.linalg.qr(rng.standard_normal((p.M, r)))
    Z = U * sv
    Q, _ = np.linalg.qr(rng.standard_normal((p.n_theta * p.n_phi, p.n_theta * p.n_phi)))
    Th = Q[:r].reshape(r, p.n_theta, p.n_phi)
    Ph = np.eye(p.n_phi)
    return Z, Th, Ph


@pytest.mark.parametrize("kind", ["graded", "pairs"])
def test_plain_rounding_of_a_constructed_spectrum(tt, kind):
    p = ti.clumps3d(n=6, n_groups=8, n_theta=8, n_phi=16, tol=1e-14, rank_cap=96, precision=ti.PREC_FP64)
    if kind == "graded":
        sv = 10.0 ** (-12.0 * np.arange(80) / 80.0)
    else:
        sv = np.repeat(2.0 ** -np.arange(40), 2)          # s_{2k} = s_{2k+1}
    cap = 40                                              # between two pairs
    Z, Th, Ph = _constructed(p, sv, seed=5 if kind == "graded" else 6)
    print(f"eig: constructed {kind} M={p.M}", flush=True)
    s = tt.Solver(p, round_method=tt.TT_ROUND_GRAM)
    s.set_cores(Z, Th, Ph)
    s.round(p.tol, cap)
    Zo, To, Po, info = ott.round_tt(Z, Th, Ph, p.tol, cap)
    assert s.get_ranks() == (info["r1"], info["r2"]) == (cap, p.n_phi)
    got = full(*s.get_cores())
    assert rel(got, full(Zo, To, Po)) < 1e-8
    # the kept singular values of the first bond are the constructed ones, to
    # the Gram's resolution (eigenvalues to eps of the largest)
    s1 = np.linalg.svd(got.reshape(p.M, -1), compute_uv=False)[:cap]
    np.testing.assert_allclose(s1, sv[:cap], rtol=0, atol=1e-8 * sv[0])
    s.destroy()
