"""Pins of the internal-rank diagnostic of the oracle (the discussion of the
internal structure of the combined core).  CPU only."""
import numpy as np
import pytest

import tt_inputs as ti
from oracle import tt as ott


def _full(Z, Th, Ph):
    return np.einsum("ka,alb,bp->klp", Z, Th, Ph)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_spectra_equal_unfoldings_of_the_dense_tensor(seed):
    # with Theta', Phi' right-orthonormal, reshape(Z') has the singular values
    # of the dense tensor unfolded with nu (resp. x) as the row mode
    n_x, G, nt, npn = 7, 5, 4, 3
    Z, Th, Ph = ti.random_tt(n_x * G, nt, npn, 6, 3, seed=seed, decay=0.7)
    X = _full(Z, Th, Ph).reshape(n_x, G, nt, npn)
    out = ott.internal_ranks(n_x, G, Z, Th, Ph, 1e-8)
    s_nu = np.linalg.svd(X.transpose(1, 0, 2, 3).reshape(G, -1), compute_uv=False)
    s_x = np.linalg.svd(X.reshape(n_x, -1), compute_uv=False)
    np.testing.assert_allclose(out["s_nu"], s_nu[: len(out["s_nu"])], rtol=1e-10, atol=1e-13 * s_nu[0])
    np.testing.assert_allclose(out["s_x"], s_x[: len(out["s_x"])], rtol=1e-10, atol=1e-13 * s_x[0])


def test_separable_core_has_internal_rank_one():
    # Z[x, g, a] = f(g) h(x, a): rank 1 with nu as the row mode
    rng = np.random.default_rng(4)
    n_x, G, nt, npn, r1, r2 = 9, 6, 4, 2, 3, 2
    f = rng.uniform(0.5, 2.0, G)
    h = rng.standard_normal((n_x, r1))
    Z = np.einsum("g,xa->xga", f, h).reshape(n_x * G, r1)
    Th = rng.standard_normal((r1, nt, r2))
    Ph = rng.standard_normal((r2, npn))
    out = ott.internal_ranks(n_x, G, Z, Th, Ph, 1e-10)
    assert out["r_nux"] == 1
    assert out["r_xnu"] == min(n_x, G * r1, r1)
    n_tt = n_x * G * r1 + nt * r1 * r2 + npn * r2
    assert out["C_rel_nu"] == pytest.approx(n_tt / (G + n_x * r1 + nt * r1 * r2 + npn * r2))


def test_delta_rank_rule():
    s = np.array([3.0, 2.0, 1.0, 0.1])
    tot = np.sqrt(np.sum(s * s))
    assert ott.delta_rank_rel(s, 0.0) == 4
    assert ott.delta_rank_rel(s, 0.1 / tot * 1.0000001) == 3
    assert ott.delta_rank_rel(s, np.sqrt(1.01) / tot * 1.0000001) == 2
    assert ott.delta_rank_rel(s, 1.0) == 1


def _exact_rank(A, rel=1e-10):
    s = np.linalg.svd(A, compute_uv=False)
    return int(np.sum(s > rel * s[0])) if s.size and s[0] > 0 else 0


def _split_topology(X, row_mode, delta):
    """The split-core TT of the dense tensor X[x, g, l, p] built explicitly:
    the row mode (0: space x, 1: frequency g) is cut off first by a
    delta-truncated SVD (relative Frobenius tail <= delta), then the rest is
    split into (other mode x bond, theta) and (phi) cores by exact SVDs.
    Returns (kept rank, entries of the four cores, relative error of the
    four-core tensor, relative error with one rank fewer, exact ranks of the
    two angular bonds)."""
    n = X.shape
    other = 1 - row_mode
    Xr = np.moveaxis(X, row_mode, 0)                        # [row, other, l, p]
    A = Xr.reshape(n[row_mode], -1)
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    tot = np.linalg.norm(s)
    r = next(k for k in range(1, len(s) + 1) if np.linalg.norm(s[k:]) <= delta * tot)

    def approx(k):
        return (U[:, :k] * s[:k]) @ Vt[:k]

    W = (s[:r, None] * Vt[:r]).reshape(r * n[other], n[2] * n[3])
    r1 = _exact_rank(W)
    # then (bond x other mode) | (theta, phi), and (bond' x theta) | phi
    U1, s1, Vt1 = np.linalg.svd(W, full_matrices=False)
    B = (s1[:r1, None] * Vt1[:r1]).reshape(r1 * n[2], n[3])
    r2 = _exact_rank(B)
    entries = n[row_mode] * r + r * n[other] * r1 + r1 * n[2] * r2 + r2 * n[3]
    err = np.linalg.norm(approx(r) - A) / tot
    err_less = np.linalg.norm(approx(r - 1) - A) / tot if r > 1 else np.inf
    return r, entries, err, err_less, (r1, r2)


@pytest.mark.parametrize("seed,delta", [(0, 1e-2), (1, 1e-3), (2, 3e-2)])
def test_relative_compression_equals_entry_count_of_the_explicit_split_topologies(seed, delta):
    # C_rel (eqs. rel_compression_nu / rel_compression_x) is the TT entry count
    # over the entries of the topology with Z split in two: build each topology
    # from the dense tensor by a delta-truncated SVD of the cut-off mode, count
    # its entries, and check that it meets the error bound with the oracle's
    # internal rank and misses it with one fewer
    n_x, G, nt, npn, r1, r2 = 9, 6, 4, 3, 6, 3
    rng = np.random.default_rng(seed)
    # a core with structure across frequency: Z[x, g, a] = sum_j f_j(g) h_j(x, a) + noise
    f = rng.standard_normal((G, 3)) * np.array([1.0, 0.3, 0.05])
    h = rng.standard_normal((3, n_x, r1))
    Z = (np.einsum("gj,jxa->xga", f, h) + 1e-3 * rng.standard_normal((n_x, G, r1))).reshape(n_x * G, r1)
    Th = rng.standard_normal((r1, nt, r2))
    Ph = rng.standard_normal((r2, npn))
    X = _full(Z, Th, Ph).reshape(n_x, G, nt, npn)
    out = ott.internal_ranks(n_x, G, Z, Th, Ph, delta)
    n_tt = Z.size + Th.size + Ph.size
    for row_mode, rkey, ckey in ((1, "r_nux", "C_rel_nu"), (0, "r_xnu", "C_rel_x")):
        r, entries, err, err_less, bonds = _split_topology(X, row_mode, delta)
        assert bonds == (r1, r2)
        assert out[rkey] == r
        assert err <= delta * (1 + 1e-12) and err_less > delta
        assert out[ckey] == pytest.approx(n_tt / entries, rel=1e-14)
