"""The C-ABI library: loads, exports every symbol the header declares, and its
host-only entry points behave (no GPU needed)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import tt_inputs as ti
from oracle import planck

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tt_transport.h")


@pytest.fixture(scope="module")
def tt():
    import paper_2602_00290_amd as tt
    return tt


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(tt_transport_\w+)\s*\(", text)))


def test_header_symbols_exported(tt):
    syms = declared_symbols()
    assert len(syms) >= 14
    for s in syms:
        assert hasattr(tt.lib, s), f"{s} not exported"
    assert set(syms) == set(tt.EXPORTED)


def _field_names(text, name):
    body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (name, name), text, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        # drop the type: everything up to the first declarator
        parts = decl.split(",")
        first = re.match(r".*?([\w]+)\s*(\[\d+\])?$", parts[0].strip()).group(1)
        names.append(first)
        for extra in parts[1:]:
            names.append(re.match(r"\s*\**\s*(\w+)", extra).group(1))
    return names


def test_struct_layout_matches_header(tt):
    # the binding's ctypes structs must have the header's field order
    text = open(HEADER).read()
    assert _field_names(text, "tt_problem") == [f for f, _ in tt.TTProblem._fields_]
    assert _field_names(text, "tt_stats") == [f for f, _ in tt.TTStats._fields_]
    assert _field_names(text, "tt_internal_ranks") == [f for f, _ in tt.TTInternalRanks._fields_]
    assert _field_names(text, "tt_tuning") == [f for f, _ in tt.TTTuning._fields_]


@pytest.mark.parametrize("T", [0.0, 0.03, 0.1, 1.0, 2.7696])
def test_library_planck_matches_oracle_quadrature(tt, T):
    for edges in (ti.log_group_edges(8, 0.01, 10.0), ti.log_group_edges(64, 0.01, 10.0),
                  np.array([0.0, 1.5, 1.6, np.inf]), np.array([0.0, np.inf])):
        lib = tt.group_emission(edges, T)
        ref = planck.group_emission(edges, T)
        np.testing.assert_allclose(lib, ref, rtol=2e-13, atol=1e-300)
        if T > 0:
            assert lib.sum() == pytest.approx(planck.gray_emission(T), rel=1e-13)


def test_workspace_bytes_and_validation(tt):
    p = ti.slab1d(n_cells=16, n_groups=4, n_theta=8)
    assert tt.workspace_bytes(p) > 16 * 4 * 8
    for bad in (p.copy(dim=4), p.copy(rank_cap=0), p.copy(cfl=-1.0), p.copy(tol=-1.0),
                p.copy(bc=(2, 0, 0, 0, 0, 0)), p.copy(precision=7)):
        with pytest.raises(tt.TTError) as e:
            tt.workspace_bytes(bad)
        assert e.value.status == tt.TT_ERR_INVALID_ARG
    p2 = ti.plane2d(n=16, n_groups=8, n_theta=4, n_phi=4)
    assert tt.workspace_bytes(p2) > tt.workspace_bytes(p2.copy(rank_cap=4))


def test_create_rejects_small_or_null_workspace_without_gpu(tt):
    p = ti.slab1d(n_cells=16, n_groups=4, n_theta=8)
    ps = tt.ProblemStruct(p)
    h = ctypes.c_void_p()
    st = tt.lib.tt_transport_create(ctypes.byref(ps.s), None, 1 << 20, None, ctypes.byref(h))
    assert st == tt.TT_ERR_INVALID_ARG
    fake = ctypes.c_void_p(1 << 30)   # never dereferenced: the size check fails first
    st = tt.lib.tt_transport_create(ctypes.byref(ps.s), fake, 64, None, ctypes.byref(h))
    assert st == tt.TT_ERR_OOM
    assert b"workspace too small" in tt.lib.tt_transport_last_error()


def test_coupled_temperature_validation(tt):
    p = ti.thermal_relax(n_cells=4)
    fixed = p.copy(heat_capacity=0.0, T_rad0=None)
    # the coupled problem carries T, its initial copy, J* per row, edges and weights
    assert tt.workspace_bytes(p) > tt.workspace_bytes(fixed)
    for bad in (p.copy(heat_capacity=-1.0), p.copy(heat_capacity=float("inf"))):
        with pytest.raises(tt.TTError) as e:
            tt.workspace_bytes(bad)
        assert e.value.status == tt.TT_ERR_INVALID_ARG
    # both step orders are accepted, with or without the coupling
    assert tt.workspace_bytes(fixed.copy(step_order=1)) > 0
    assert tt.workspace_bytes(p.copy(step_order=1)) == tt.workspace_bytes(p)


def test_kappa_full_validation(tt):
    p = ti.slab1d(n_cells=16, n_groups=4, n_theta=4)
    K = np.outer(p.kappa0, p.kappa_scale)
    q = p.copy(kappa_full=K, kappa0=None, kappa_scale=None)
    # the full field takes N_X N_nu doubles of workspace more
    assert tt.workspace_bytes(q) >= tt.workspace_bytes(p) + 16 * 4 * 8
    with pytest.raises(tt.TTError) as e:
        tt.workspace_bytes(p.copy(kappa0=None))
    assert e.value.status == tt.TT_ERR_INVALID_ARG


def test_flux_and_scattering_validation(tt):
    p = ti.slab1d(n_cells=16, n_groups=4, n_theta=4)
    ks = np.ones((16, 4))
    base = tt.workspace_bytes(p)
    # scattering: the opacity, J^{m+1} and the pre-pass rows (3 N_X N_nu doubles)
    assert tt.workspace_bytes(p.copy(kappa_s_full=ks)) >= base + 3 * 16 * 4 * 8
    assert tt.workspace_bytes(p.copy(flux=ti.FLUX_RUSANOV, rusanov_s=0.0)) > 0
    assert tt.workspace_bytes(p.copy(kappa_s_full=ks, step_order=1)) == tt.workspace_bytes(p.copy(kappa_s_full=ks))
    # randomized rounding: sketch buffers, and its oversampling is checked
    assert tt.workspace_bytes(p.copy(round_method=ti.ROUND_RAND)) > tt.workspace_bytes(p.copy(round_method=ti.ROUND_GRAM))
    for bad in (p.copy(round_method=4), p.copy(round_method=ti.ROUND_RAND, rand_oversample=0),
                p.copy(round_method=ti.ROUND_RAND, rand_oversample=129)):
        with pytest.raises(tt.TTError) as e:
            tt.workspace_bytes(bad)
        assert e.value.status == tt.TT_ERR_INVALID_ARG
    assert tt.workspace_bytes(p.copy(round_method=ti.ROUND_GRAM, rand_oversample=0)) > 0
    # HLL: FP64 data without scattering or a coupled temperature, beta > 0
    assert tt.workspace_bytes(p.copy(flux=ti.FLUX_HLL, precision=ti.PREC_FP64)) > 0
    for bad in (p.copy(flux=3), p.copy(flux=ti.FLUX_RUSANOV, rusanov_s=1.5),
                p.copy(flux=ti.FLUX_RUSANOV, rusanov_s=float("nan")),
                p.copy(flux=ti.FLUX_HLL, precision=ti.PREC_FP32),
                p.copy(flux=ti.FLUX_HLL, precision=ti.PREC_FP64, kappa_s_full=ks),
                p.copy(flux=ti.FLUX_HLL, precision=ti.PREC_FP64, hll_beta=0.0),
                p.copy(flux=ti.FLUX_HLL, precision=ti.PREC_FP64, hll_beta=float("inf"))):
        with pytest.raises(tt.TTError) as e:
            tt.workspace_bytes(bad)
        assert e.value.status == tt.TT_ERR_INVALID_ARG
