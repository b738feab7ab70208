"""Python side of the dense FP64 oracle (ctypes wrapper around dense.c).

TEST INFRASTRUCTURE ONLY: only tests, the smoke check and the benchmark's CPU
baseline leg use this module.  It shares no code with the GPU library.

The discretisation (Section 2.1 "Numerics"; operator form in Appendix A):
forward-Euler upwind streaming, then the backward-Euler operator-split source
update with zero scattering, density 1 and fixed temperature,
I^{m+1} = (I* + c dt kappa eps) / (1 + c dt kappa).

With a heat capacity C_v = rho c_v > 0 the medium temperature is coupled
(Section 2.1, the coupled source stage): per cell, the stage temperature T+
is the root of the scalar equation the paper writes for it,
    T^m - T+ - sum_g (4 pi dt kappa_g / C_v) (eps_g(T+) - J_g^{m+1}(T+)) = 0,
with J^{m+1} = (J* / (c dt) + kappa eps(T+)) / (1 / (c dt) + kappa) the
angle-mean of the implicitly updated intensity (J* that of the intensity
after streaming); the intensity is updated with eps(T+), and the new medium
temperature follows from total-energy conservation,
    C_v (T^{m+1} - T^m) = (4 pi / c) sum_g (J*_g - J_g^{m+1}),
J = (1 / 4 pi) sum_lp w_l w_p I (the quadrature weights sum to 4 pi).

Isotropic elastic scattering (the kappa_s term of the transport equation and
of its backward-Euler source update, Section 2.1) with a = c dt kappa_a,
b = c dt kappa_s: the angle mean of the update gives
J^{m+1} = (J* + a eps) / (1 + a) (scattering drops out), and then
I^{m+1} = (I* + a eps + b J^{m+1}) / (1 + a + b).

The Rusanov flux (the second of the three stencils Section 2.1 names) is
taken in the transport half: see dense.c.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import sys

import numpy as np

from scipy import optimize

from . import planck

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "_dense.so")
SRC = os.path.join(HERE, "dense.c")

FACE_VACUUM, FACE_INFLOW_PLANCK, FACE_PERIODIC, FACE_INFLOW_VALUES = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile dense.c with gcc + OpenMP into oracle/_dense.so."""
    if force or not os.path.exists(SO) or os.path.getmtime(SO) < os.path.getmtime(SRC):
        cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", SRC, "-o", SO + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(SO + ".tmp", SO)
    return SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(SO):
            build()
        L = ctypes.CDLL(SO)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.oracle_dense_march.argtypes = [
            ctypes.c_int, ip, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, ip, dp,
            ctypes.c_double, ctypes.c_double, dp, dp, ctypes.c_int, ctypes.c_int]
        L.oracle_dense_march.restype = ctypes.c_int
        L.oracle_dense_transport.argtypes = [
            ctypes.c_int, ip, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, ip, dp,
            ctypes.c_double, ctypes.c_double, dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_double]
        L.oracle_dense_transport.restype = ctypes.c_int
        L.oracle_dense_transport_hll.argtypes = [
            ctypes.c_int, ip, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, ip, dp,
            ctypes.c_double, ctypes.c_double, dp, dp, ctypes.c_int, dp, ctypes.c_double]
        L.oracle_dense_transport_hll.restype = ctypes.c_int
        L.oracle_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


# ---------------------------------------------------------------------------
# problem-derived quantities (independent of the GPU library's own setup)
# ---------------------------------------------------------------------------

def time_step(prob) -> float:
    """dt = CFL / (c * sum_d 1/dx_d) over the active axes."""
    inv = 0.0
    for d in range(prob.dim):
        inv += prob.n_cells[d] / prob.extent[d]
    return prob.cfl / (prob.c * inv)


def kappa_field(prob) -> np.ndarray:
    """(N_X, N_nu) opacity kappa_{a,g}(x) of the transport equation (Section 2):
    the full field when given, else kappa0(x) * scale(g)."""
    kf = getattr(prob, "kappa_full", None)
    if kf is not None:
        return np.asarray(kf, float).reshape(prob.n_x, prob.n_groups)
    return np.outer(np.asarray(prob.kappa0, float), np.asarray(prob.kappa_scale, float))


def kappa_s_field(prob) -> np.ndarray:
    """(N_X, N_nu) scattering opacity kappa_{s,g}(x) (zero when not given)."""
    ks = getattr(prob, "kappa_s_full", None)
    if ks is None:
        return np.zeros((prob.n_x, prob.n_groups))
    return np.asarray(ks, float).reshape(prob.n_x, prob.n_groups)


def flux_params(prob):
    """(flux, s): 0 for the upwind flux, 1 for Rusanov with s = S+ / c, 2 for
    HLL (s unused)."""
    flux = int(getattr(prob, "flux", 0))
    return flux, float(getattr(prob, "rusanov_s", 1.0)) if flux == 1 else 0.0


def kappa_total(prob) -> np.ndarray:
    """(N_X, N_nu) absorption plus scattering opacity: the optical depth of the
    HLL flux (tau_{c,f}, per cell and group)."""
    return kappa_field(prob) + kappa_s_field(prob)


def _plain(prob) -> bool:
    return flux_params(prob)[0] == 0 and getattr(prob, "kappa_s_full", None) is None


def emission(prob) -> np.ndarray:
    return planck.emission_field(prob.edges, prob.T_cell)


def ghost_values(prob) -> np.ndarray:
    """(6, N_nu) isotropic ghost intensities of each face (zero where unused)."""
    G = prob.n_groups
    out = np.zeros((6, G))
    for f in range(6):
        kind = prob.bc[f]
        if kind == FACE_INFLOW_PLANCK:
            out[f] = planck.group_emission(prob.edges, float(prob.bc_T[f]))
        elif kind == FACE_INFLOW_VALUES:
            out[f] = np.asarray(prob.bc_values)[f]
    return out


def initial_dense(prob) -> np.ndarray:
    """Isotropic Planck state, shape (N_X*N_nu, N_theta, N_phi): at the initial
    radiation temperature when the problem gives one, else at the medium
    temperature."""
    T_rad = getattr(prob, "T_rad0", None)
    eps = (emission(prob) if T_rad is None else planck.emission_field(prob.edges, T_rad)).reshape(-1)
    return np.broadcast_to(eps[:, None, None], (prob.M, prob.n_theta, prob.n_phi)).copy()


def march(prob, I0: np.ndarray, n_steps: int, n_threads: int = 0, dt: float = None) -> np.ndarray:
    """n_steps full steps (transport + source) of the dense FP64 scheme."""
    if not _plain(prob):
        I = np.ascontiguousarray(I0, dtype=np.float64).copy()
        for _ in range(n_steps):
            I = source(prob, transport(prob, I, n_threads, dt=dt), dt=dt)
        return I
    I = np.ascontiguousarray(I0, dtype=np.float64).copy()
    work = np.empty_like(I)
    nc = np.ascontiguousarray(np.asarray(prob.n_cells, dtype=np.int32))
    ext = np.ascontiguousarray(np.asarray(prob.extent, dtype=np.float64))
    bc = np.ascontiguousarray(np.asarray(prob.bc, dtype=np.int32))
    ghost = np.ascontiguousarray(ghost_values(prob))
    kap = np.ascontiguousarray(kappa_field(prob))
    eps = np.ascontiguousarray(emission(prob))
    mu = np.ascontiguousarray(np.asarray(prob.mu, float))
    phi = np.ascontiguousarray(np.asarray(prob.phi, float))
    if dt is None:
        dt = time_step(prob)
    rc = lib().oracle_dense_march(prob.dim, _ip(nc), _dp(ext), prob.n_groups, prob.n_theta,
                                  prob.n_phi, _dp(mu), _dp(phi), _dp(kap), _dp(eps), _ip(bc),
                                  _dp(ghost), float(prob.c), float(dt), _dp(I), _dp(work),
                                  int(n_steps), int(n_threads))
    if rc != 0:
        raise RuntimeError("oracle_dense_march failed")
    return I


def transport(prob, I: np.ndarray, n_threads: int = 0, dt: float = None) -> np.ndarray:
    """Transport half-step only (no source update): upwind, Rusanov or HLL flux."""
    I = np.ascontiguousarray(I, dtype=np.float64)
    out = np.empty_like(I)
    nc = np.ascontiguousarray(np.asarray(prob.n_cells, dtype=np.int32))
    ext = np.ascontiguousarray(np.asarray(prob.extent, dtype=np.float64))
    bc = np.ascontiguousarray(np.asarray(prob.bc, dtype=np.int32))
    ghost = np.ascontiguousarray(ghost_values(prob))
    mu = np.ascontiguousarray(np.asarray(prob.mu, float))
    phi = np.ascontiguousarray(np.asarray(prob.phi, float))
    flux, s_rus = flux_params(prob)
    if flux == 2:
        kap = np.ascontiguousarray(kappa_total(prob).reshape(-1))
        rc = lib().oracle_dense_transport_hll(
            prob.dim, _ip(nc), _dp(ext), prob.n_groups, prob.n_theta, prob.n_phi, _dp(mu), _dp(phi),
            _ip(bc), _dp(ghost), float(prob.c), float(time_step(prob) if dt is None else dt), _dp(I), _dp(out),
            int(n_threads), _dp(kap), float(getattr(prob, "hll_beta", 20.0)))
        if rc != 0:
            raise RuntimeError("oracle_dense_transport_hll failed")
        return out
    rc = lib().oracle_dense_transport(
        prob.dim, _ip(nc), _dp(ext), prob.n_groups, prob.n_theta, prob.n_phi, _dp(mu), _dp(phi),
        _ip(bc), _dp(ghost), float(prob.c), float(time_step(prob) if dt is None else dt), _dp(I), _dp(out),
        int(n_threads), flux, s_rus)
    if rc != 0:
        raise RuntimeError("oracle_dense_transport failed")
    return out


def source(prob, I: np.ndarray, dt: float = None) -> np.ndarray:
    """Implicit absorption/emission and isotropic scattering update at fixed T
    (rho = 1)."""
    dt = time_step(prob) if dt is None else dt
    kap = kappa_field(prob).reshape(-1)
    eps = emission(prob).reshape(-1)
    a = prob.c * dt * kap
    if getattr(prob, "kappa_s_full", None) is None:
        return (I + (a * eps)[:, None, None]) / (1.0 + a)[:, None, None]
    b = prob.c * dt * kappa_s_field(prob).reshape(-1)
    J_new = (mean_intensity(prob, I).reshape(-1) + a * eps) / (1.0 + a)
    return (I + (a * eps + b * J_new)[:, None, None]) / (1.0 + a + b)[:, None, None]


def energy(prob, I: np.ndarray) -> float:
    """Quadrature-weighted radiation content sum_cells dV sum_g sum_lp w_l w_p I."""
    dV = float(np.prod([prob.extent[d] / prob.n_cells[d] for d in range(prob.dim)]))
    w = np.outer(prob.w_theta, prob.w_phi)
    return dV * float(np.einsum("klp,lp->", I, w))


def num_threads() -> int:
    return int(lib().oracle_num_threads())


# ---------------------------------------------------------------------------
# coupled medium temperature (Section 2.1, coupled source stage)
# ---------------------------------------------------------------------------

def mean_intensity(prob, I: np.ndarray) -> np.ndarray:
    """(N_X, N_nu) angle means J = (1 / 4 pi) sum_lp w_l w_p I."""
    w = np.outer(prob.w_theta, prob.w_phi)
    J = np.einsum("klp,lp->k", I, w) / (4.0 * np.pi)
    return J.reshape(prob.n_x, prob.n_groups)


def stage_temperature(prob, T_m: float, J_star: np.ndarray, kappa: np.ndarray, dt: float) -> float:
    """Root T+ of the paper's scalar equation for one cell (written with
    J^{m+1}(T+) spelled out), by Brent's method on a sign-changing bracket.
    The left side falls strictly with T+ (eps_g rises with T); at T+ = 0 it
    is T^m + sum_g (4 pi dt kappa_g / C_v) J*_g d_g >= 0, and at
    T_hi = that value it is <= 0."""
    C = float(prob.heat_capacity)
    cdt = prob.c * dt

    def f(T):
        eps = planck.group_emission_quad(prob.edges, T)
        J_new = (J_star / cdt + kappa * eps) / (1.0 / cdt + kappa)
        return T_m - T - float(np.sum(4.0 * np.pi * dt * kappa / C * (eps - J_new)))

    hi = T_m + float(np.sum(4.0 * np.pi * dt * kappa / C * J_star / (1.0 + cdt * kappa)))
    hi = max(hi, T_m, 1e-300)
    f_hi = f(hi)
    while f_hi > 0.0:   # the bracket end rounded below the root (tiny coupling terms)
        hi = 2.0 * hi
        f_hi = f(hi)
    if f_hi == 0.0:
        return hi
    f_lo = f(0.0)
    if f_lo <= 0.0:
        return 0.0
    return optimize.brentq(f, 0.0, hi, xtol=1e-300, rtol=8.9e-16, maxiter=500)


def coupled_source(prob, I_star: np.ndarray, T: np.ndarray):
    """Coupled source stage on the dense intensity after streaming: returns
    (I^{m+1}, T^{m+1})."""
    dt = time_step(prob)
    kap = kappa_field(prob)                      # (N_X, N_nu)
    J_star = mean_intensity(prob, I_star)
    T = np.asarray(T, dtype=float)
    eps = np.zeros_like(kap)
    for x in range(prob.n_x):
        Tp = stage_temperature(prob, float(T[x]), J_star[x], kap[x], dt)
        eps[x] = planck.group_emission_quad(prob.edges, Tp)
    a = (prob.c * dt * kap).reshape(-1)
    b = (prob.c * dt * kappa_s_field(prob)).reshape(-1)
    # J^{m+1} of the implicit update (independent of the scattering opacity)
    Jn = (J_star.reshape(-1) + a * eps.reshape(-1)) / (1.0 + a)
    I_new = (I_star + (a * eps.reshape(-1) + b * Jn)[:, None, None]) / (1.0 + a + b)[:, None, None]
    J_new = mean_intensity(prob, I_new)
    T_new = T + 4.0 * np.pi / (prob.c * float(prob.heat_capacity)) * np.sum(J_star - J_new, axis=1)
    return I_new, T_new


def march_coupled(prob, I0: np.ndarray, T0, n_steps: int, n_threads: int = 0):
    """n_steps of streaming + coupled source; returns (I, T)."""
    I = np.ascontiguousarray(I0, dtype=np.float64).copy()
    T = np.asarray(T0, dtype=float).copy()
    for _ in range(n_steps):
        I, T = coupled_source(prob, transport(prob, I, n_threads), T)
    return I, T


def total_energy(prob, I: np.ndarray, T) -> float:
    """Radiation plus medium energy: dV (sum_k (1 / c) sum_lp w I + C_v sum_x T)."""
    dV = float(np.prod([prob.extent[d] / prob.n_cells[d] for d in range(prob.dim)]))
    return energy(prob, I) / prob.c + dV * float(prob.heat_capacity) * float(np.sum(T))
