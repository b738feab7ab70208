"""GPU parity of the internal delta-ranks of the combined core (the discussion
of the internal structure of Z and its relative compression equations) through
the C ABI against the oracle's SVDs of the two unfoldings of Z' = Z L_Theta.

The library forms the FP64 Gram of the N_X x (N_nu ld) unfolding on the device
and takes eigenvalues on the host, so a singular value carries an absolute
error of about sqrt(n eps) s_max (n = N_nu r1 <= 2048): the tests compare
singular values to 1e-6 s_max, the leading ones (above 1e-3 s_max) to 1e-8
relative, the ranks exactly wherever no tail norm lies within 1e-5 of the
threshold (else to one), and C_rel to 1e-12 whenever the ranks agree (it is a
ratio of integers)."""
import numpy as np
import pytest

import tt_inputs as ti
from oracle import tt as ott

pytestmark = pytest.mark.gpu

DELTAS = (1e-1, 1e-2, 1e-3, 1e-4, 1e-5)


@pytest.fixture(scope="module")
def tt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_00290_amd as tt
    return tt


def _ambiguous(s, delta, rel=1e-5):
    """True if a tail norm of s lies within rel of delta ||s||."""
    s = np.asarray(s, float)
    tot = np.sqrt(np.sum(s * s))
    tails = np.sqrt(np.maximum(np.concatenate([np.cumsum((s * s)[::-1])[::-1], [0.0]]), 0.0))
    return bool(np.any(np.abs(tails - delta * tot) <= rel * delta * tot + 1e-6 * s[0]))


def _compare(dev, ref, delta):
    for key, skey, rkey in (("nu", "s_nu", "r_nux"), ("x", "s_x", "r_xnu")):
        s_d, s_r = dev[skey], ref[skey]
        assert len(s_d) == len(s_r), key
        smax = s_r[0]
        np.testing.assert_allclose(s_d, s_r, rtol=0, atol=1e-6 * smax)
        lead = s_r > 1e-3 * smax
        np.testing.assert_allclose(s_d[lead], s_r[lead], rtol=1e-8)
        if _ambiguous(s_r, delta):
            assert abs(dev[rkey] - ref[rkey]) <= 1, (key, delta)
        else:
            assert dev[rkey] == ref[rkey], (key, delta, dev[rkey], ref[rkey])
    if dev["r_nux"] == ref["r_nux"]:
        assert dev["C_rel_nu"] == pytest.approx(ref["C_rel_nu"], rel=1e-12)
    if dev["r_xnu"] == ref["r_xnu"]:
        assert dev["C_rel_x"] == pytest.approx(ref["C_rel_x"], rel=1e-12)


def _problems():
    yield "slab1d_fp64", ti.slab1d(n_cells=48, n_groups=8, n_theta=8, tol=1e-10, rank_cap=16), 20
    # fused FP32 path; 7 x 5 cells and 6 groups leave ragged Gram tiles and cell chunks
    p = ti.plane2d(n=7, n_groups=6, n_theta=4, n_phi=8, tol=1e-6, rank_cap=24, precision=ti.PREC_FP32)
    p.n_cells = (7, 5, 1)
    p.kappa0 = ti.lognormal_kappa0(p.n_cells, p.extent, 2, seed=3)
    p.T_cell = np.full(p.n_x, 0.1)
    yield "plane2d_fp32", p, 12
    q = ti.plane2d(n=12, n_groups=10, n_theta=4, n_phi=8, tol=1e-5, rank_cap=32, precision=ti.PREC_BF16X)
    yield "plane2d_bf16x", q, 8


@pytest.mark.parametrize("case", [c[0] for c in _problems()])
def test_internal_ranks_match_oracle(tt, case):
    name, p, steps = next(c for c in _problems() if c[0] == case)
    print(f"internal ranks: {name} steps={steps}", flush=True)
    s = tt.Solver(p)
    s.solve(steps)
    Z, Th, Ph = s.get_cores()
    for delta in DELTAS:
        dev = s.internal_ranks(delta)
        ref = ott.internal_ranks(p.n_x, p.n_groups, Z, Th, Ph, delta)
        _compare(dev, ref, delta)
    s.destroy()


def test_gray_opacity_cold_medium_is_rank_one_in_frequency(tt):
    # Gray opacity, no emission and a Planck inflow: every group is the same
    # transport problem scaled by its inflow value, so the solution is
    # k_g f(x, theta, phi) and r_nux = 1 (the hohlraum case of the discussion).
    p = ti.slab1d(n_cells=40, n_groups=7, n_theta=8, tol=1e-10, rank_cap=16, T=1e-4)
    p = p.copy(kappa_scale=np.ones(7))
    s = tt.Solver(p)
    s.solve(25)
    r1, r2 = s.get_ranks()
    dev = s.internal_ranks(1e-5)
    assert dev["r_nux"] == 1
    assert dev["s_nu"][1] <= 1e-6 * dev["s_nu"][0]
    n_tt = p.n_x * p.n_groups * r1 + p.n_theta * r1 * r2 + p.n_phi * r2
    assert dev["C_rel_nu"] == pytest.approx(
        n_tt / (p.n_groups + p.n_x * r1 + p.n_theta * r1 * r2 + p.n_phi * r2), rel=1e-14)
    s.destroy()


def test_separable_core_set_by_hand(tt):
    # Z[(x, g), a] = u_g V[x, a]: internal rank one in frequency, and r_xnu =
    # rank(V) = r1 with distinct singular values known in closed form.
    p = ti.slab1d(n_cells=30, n_groups=9, n_theta=6, tol=1e-10, rank_cap=12)
    rng = np.random.default_rng(5)
    r1, r2 = 5, 3
    u = rng.uniform(0.5, 2.0, p.n_groups)
    V = np.linalg.qr(rng.standard_normal((p.n_x, r1)))[0] * np.array([5.0, 3.0, 1.0, 0.1, 0.01])
    Z = np.einsum("g,xa->xga", u, V).reshape(p.n_x * p.n_groups, r1)
    Ph = np.linalg.qr(rng.standard_normal((p.n_phi, r2)))[0].T if p.n_phi >= r2 else None
    if Ph is None:  # 1D: a single azimuth, so r2 = 1
        r2 = 1
        Ph = np.ones((1, p.n_phi)) / np.sqrt(p.n_phi)
    Th = np.linalg.qr(rng.standard_normal((p.n_theta * r2, r1)))[0].T.reshape(r1, p.n_theta, r2)
    s = tt.Solver(p)
    s.set_cores(Z, Th, Ph)
    sig = np.array([5.0, 3.0, 1.0, 0.1, 0.01])
    dev = s.internal_ranks(1e-4)
    assert dev["r_nux"] == 1
    # Theta and Phi are already right-orthonormal, so Z' = Z up to signs of its
    # columns: the x-unfolding is V (x) u^T with singular values ||u|| sig, the
    # frequency unfolding has rows u_g vec(V), a single singular value ||Z||_F.
    np.testing.assert_allclose(dev["s_x"][:r1], np.linalg.norm(u) * sig, rtol=1e-9)
    assert np.all(dev["s_x"][r1:] <= 1e-6 * dev["s_x"][0])
    assert dev["s_nu"][0] == pytest.approx(np.linalg.norm(Z), rel=1e-12)
    # relative tails of sig: after 4 values 0.01 / ||sig|| = 1.7e-3, after 3 values 1.7e-2
    assert dev["r_xnu"] == 5
    assert s.internal_ranks(1e-2)["r_xnu"] == 4
    assert s.internal_ranks(2e-2)["r_xnu"] == 3
    s.destroy()


def test_error_paths(tt):
    p = ti.slab1d(n_cells=16, n_groups=4, n_theta=4, tol=1e-10, rank_cap=8)
    s = tt.Solver(p)
    with pytest.raises(tt.TTError) as e:
        s.internal_ranks(-1.0)
    assert e.value.status == tt.TT_ERR_INVALID_ARG
    s.apply_op()
    with pytest.raises(tt.TTError) as e:
        s.internal_ranks(1e-3)
    assert e.value.status == tt.TT_ERR_STATE
    s.destroy()
    # N_nu * ld(r1) above the supported size
    q = ti.plane2d(n=4, n_groups=72, n_theta=4, n_phi=8, tol=1e-6, rank_cap=32)
    s = tt.Solver(q)
    rng = np.random.default_rng(0)
    r1, r2 = 32, 8
    s.set_cores(rng.standard_normal((q.n_x * q.n_groups, r1)), rng.standard_normal((r1, 4, r2)),
                rng.standard_normal((r2, 8)))
    with pytest.raises(tt.TTError) as e:
        s.internal_ranks(1e-3)
    assert e.value.status == tt.TT_ERR_INVALID_ARG
    s.destroy()


def test_gaussian_diffusion_internal_rank_one_when_gray(tt):
    # equal scattering opacities in every group make the multigroup diffusion a
    # gray problem scaled per group: r_nux = 1; a spread of opacities makes the
    # groups diffuse at different rates and r_nux > 1 (the Gaussian diffusion
    # discussion of the internal ranks)
    base = ti.gaussian_diffusion(n_cells=96, n_groups=4, n_theta=8, tol=1e-10, rank_cap=12)
    J0 = ti.gaussian_profile(base, 0.0).reshape(-1)
    out = {}
    for name, ks_max in (("gray", 1000.0), ("spread", 5000.0)):
        p = ti.gaussian_diffusion(n_cells=96, n_groups=4, n_theta=8, tol=1e-10, rank_cap=12,
                                  ks_min=1000.0, ks_max=ks_max)
        s = tt.Solver(p)
        s.set_cores(J0[:, None], np.ones((1, p.n_theta, 1)), np.ones((1, 1)))
        s.solve(400)
        out[name] = s.internal_ranks(1e-5)
        s.destroy()
    assert out["gray"]["r_nux"] == 1
    assert out["spread"]["r_nux"] > 1
