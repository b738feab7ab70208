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
