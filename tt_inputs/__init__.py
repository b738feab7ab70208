"""Seeded synthetic problem generators for multigroup TT radiation transport.

This module only builds the *inputs* of a transport solve: mesh sizes, group
edges, angular quadrature nodes and weights, opacity fields, boundary
settings and solver knobs.  It contains none of the method's arithmetic (no
transport step, no Planck integral, no tensor-train algebra), so both the
GPU library and the independent CPU oracle can consume the same arrays.

Conventions (the paper's problem statement, Section 2 and Section 4):

* The frequency axis is split into ``n_groups`` bins with edges
  ``nu_0 = 0 < nu_1 < ... < nu_{N-1} < nu_N = inf``; the interior edges are
  logarithmically spaced (Section 4, introduction of the test problems).
* Angles use a latitude/longitude product set uniform in ``cos(theta)`` and
  ``phi`` (Section 4); one-dimensional slabs use Gauss-Legendre ``mu`` with a
  single azimuthal node.
* Cells are numbered with x fastest: ``cell = ix + Nx*(iy + Ny*iz)``; the
  merged spatio-spectral row index is ``k = cell*N_nu + g`` (Section 3.1, the
  merged Z core).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

# Boundary kinds for each of the six faces x-, x+, y-, y+, z-, z+.
BC_VACUUM = 0          # ghost intensity 0
BC_INFLOW_PLANCK = 1   # isotropic ghost intensity eps_g(T_b)
BC_PERIODIC = 2        # wrap-around (both faces of the axis must be periodic)
BC_INFLOW_VALUES = 3   # isotropic ghost intensity given per group

# Contraction precision of the GPU path (rounding is always FP64).
PREC_FP64 = 0
PREC_FP32 = 1
PREC_BF16X = 2
ROUND_QR, ROUND_GRAM, ROUND_AUTO, ROUND_RAND = 0, 1, 2, 3


@dataclasses.dataclass
class Problem:
    """All inputs of one transport solve (plain arrays and scalars)."""

    name: str
    dim: int
    n_cells: tuple
    extent: tuple
    edges: np.ndarray            # (N_nu + 1,), edges[0] = 0, edges[-1] = inf
    kappa0: np.ndarray           # (N_X,) spatial opacity factor
    kappa_scale: np.ndarray      # (N_nu,) group opacity factor
    T_cell: np.ndarray           # (N_X,) fixed medium temperature
    mu: np.ndarray               # (N_theta,) cos(theta) nodes
    w_theta: np.ndarray          # (N_theta,)
    phi: np.ndarray              # (N_phi,)
    w_phi: np.ndarray            # (N_phi,)
    bc: tuple = (BC_INFLOW_PLANCK, 0, 0, 0, 0, 0)
    bc_T: tuple = (1.0, 0.0, 0.0, 0.0, 0.0, 0.0)
    bc_values: Optional[np.ndarray] = None   # (6, N_nu) for BC_INFLOW_VALUES
    c: float = 1.0
    cfl: float = 0.5
    tol: float = 1e-8
    rank_cap: int = 8
    precision: int = PREC_FP64
    step_order: int = 0          # 0: one rounding per step; 1: round after transport and after source
    round_method: int = 2        # 0: Householder QR, 1: Gram, 2: QR for FP64 data, Gram otherwise, 3: randomized
    n_steps: int = 1
    seed: int = 0
    heat_capacity: float = 0.0   # rho c_v per volume; 0: fixed medium temperature, > 0: coupled temperature
    T_rad0: Optional[np.ndarray] = None   # (N_X,) initial radiation temperature (None: T_cell)
    kappa_full: Optional[np.ndarray] = None   # (N_X, N_nu) opacity per cell and group (None: kappa0 x kappa_scale)
    kappa_s_full: Optional[np.ndarray] = None  # (N_X, N_nu) isotropic scattering opacity (None: no scattering)
    flux: int = 0                # streaming flux: 0 upwind, 1 Rusanov
    rusanov_s: float = 1.0       # Rusanov wave speed S+ / c (1: S+ = c, 0: central differences)
    hll_beta: float = 20.0       # HLL: optical-depth factor of the interface wave-speed reduction
    rand_oversample: int = 4     # randomized rounding: sketch ranks = current ranks + this
    rand_seed: int = 0           # randomized rounding: key of the counter-based generator

    # ----- derived sizes (pure bookkeeping) -----
    @property
    def n_groups(self) -> int:
        return len(self.edges) - 1

    @property
    def n_x(self) -> int:
        return int(np.prod(self.n_cells))

    @property
    def M(self) -> int:
        return self.n_x * self.n_groups

    @property
    def n_theta(self) -> int:
        return len(self.mu)

    @property
    def n_phi(self) -> int:
        return len(self.phi)

    @property
    def dense_entries(self) -> int:
        return self.M * self.n_theta * self.n_phi

    def copy(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


# ---------------------------------------------------------------------------
# group edges and group opacity scale
# ---------------------------------------------------------------------------

def log_group_edges(n_groups: int, nu_lo: float, nu_hi: float) -> np.ndarray:
    """Edges 0, nu_1..nu_{N-1} log-spaced over [nu_lo, nu_hi], inf."""
    if n_groups < 1:
        raise ValueError("n_groups must be >= 1")
    if n_groups == 1:
        return np.array([0.0, np.inf])
    interior = np.geomspace(nu_lo, nu_hi, n_groups - 1)
    return np.concatenate([[0.0], interior, [np.inf]])


def group_centers(edges: np.ndarray) -> np.ndarray:
    """Representative frequency of each group.

    Interior groups use the geometric mean of their edges; the two open groups
    [0, nu_1) and [nu_{N-1}, inf) extend the logarithmic spacing by half a step.
    """
    n = len(edges) - 1
    if n == 1:
        return np.array([1.0])
    fin = edges[1:-1]
    ratio = fin[1] / fin[0] if len(fin) > 1 else 10.0
    cen = np.empty(n)
    cen[0] = fin[0] / math.sqrt(ratio)
    cen[-1] = fin[-1] * math.sqrt(ratio)
    for g in range(1, n - 1):
        cen[g] = math.sqrt(edges[g] * edges[g + 1])
    return cen


def nu_power_scale(edges: np.ndarray, power: float = -3.0) -> np.ndarray:
    """kappa_g = kappa0 * nu_g**power, the configs' group opacity law."""
    return group_centers(edges) ** power


# ---------------------------------------------------------------------------
# angular quadratures
# ---------------------------------------------------------------------------

def gauss_legendre_mu(n: int):
    mu, w = np.polynomial.legendre.leggauss(n)
    return mu, w


def midpoint_mu(n: int):
    mu = -1.0 + (np.arange(n) + 0.5) * (2.0 / n)
    return mu, np.full(n, 2.0 / n)


def midpoint_phi(n: int):
    phi = (np.arange(n) + 0.5) * (2.0 * math.pi / n)
    return phi, np.full(n, 2.0 * math.pi / n)


# ---------------------------------------------------------------------------
# opacity fields
# ---------------------------------------------------------------------------

def gaussian_field(shape_xyz: Sequence[int], spacing: Sequence[float], corr_len: float,
                   rng: np.random.Generator) -> np.ndarray:
    """Zero-mean, unit-sample-variance Gaussian field with squared-exponential
    covariance exp(-r^2 / (2 l^2)), synthesised by FFT filtering of white noise
    on the cell-centre grid (periodic embedding).  Returned flat, x fastest."""
    shape = tuple(int(s) for s in reversed(shape_xyz))      # (Nz, Ny, Nx)
    sp = tuple(float(h) for h in reversed(spacing))
    white = rng.standard_normal(shape)
    k2 = np.zeros(shape)
    for ax, (n, h) in enumerate(zip(shape, sp)):
        if n == 1:
            continue
        k = 2.0 * math.pi * np.fft.fftfreq(n, d=h)
        sh = [1] * len(shape)
        sh[ax] = n
        k2 = k2 + (k ** 2).reshape(sh)
    amp = np.exp(-k2 * corr_len ** 2 / 4.0)
    f = np.fft.ifftn(np.fft.fftn(white) * amp).real
    f = f - f.mean()
    sd = f.std()
    if sd > 0:
        f = f / sd
    return f.ravel()


def cell_centres(n_cells, extent) -> np.ndarray:
    """(N_X, 3) cell-centre coordinates, x fastest."""
    axes = [(np.arange(n) + 0.5) * (L / n) for n, L in zip(n_cells, extent)]
    zz, yy, xx = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)


def lognormal_kappa0(n_cells, extent, dim, sigma=1.0, corr_len=0.1, seed=0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    spacing = [L / n for n, L in zip(n_cells, extent)]
    g = gaussian_field(n_cells, spacing, corr_len, rng)
    return np.exp(sigma * g)


def add_clumps(kappa0, n_cells, extent, clumps, factor=100.0) -> np.ndarray:
    x = cell_centres(n_cells, extent)
    out = kappa0.copy()
    for centre, radius in clumps:
        d2 = ((x - np.asarray(centre)) ** 2).sum(axis=1)
        out[d2 <= radius ** 2] *= factor
    return out


def multi_material_kappa(n_cells, extent, edges, n_materials, seed=0, power_range=(1.0, 3.0),
                         jitter=0.5) -> np.ndarray:
    """(N_X, N_nu) opacity of n_materials materials on a seeded Voronoi
    partition of the domain: material m has kappa_m(nu_g) = a_m nu_g^-p_m
    exp(jitter z_{m,g}), a_m lognormal, p_m uniform in power_range, z standard
    normal, so the opacity matrix has rank min(n_materials, N_nu) when every
    material holds a cell (the multi-material setting whose rank equals the
    number of materials)."""
    rng = np.random.default_rng(seed)
    x = cell_centres(n_cells, extent)
    dim = x.shape[1]
    seeds = rng.uniform(0.0, 1.0, (n_materials, dim)) * np.asarray(extent[:dim], float)
    mat = np.argmin(((x[:, None, :] - seeds[None, :, :]) ** 2).sum(axis=2), axis=1)
    # make every material own at least its nearest cell
    for m in range(n_materials):
        mat[np.argmin(((x - seeds[m]) ** 2).sum(axis=1))] = m
    nu = group_centers(edges)
    a = np.exp(rng.standard_normal(n_materials))
    p = rng.uniform(*power_range, n_materials)
    K = a[:, None] * nu[None, :] ** (-p[:, None]) * np.exp(jitter * rng.standard_normal((n_materials, len(nu))))
    return K[mat]


# ---------------------------------------------------------------------------
# the five workload shapes
# ---------------------------------------------------------------------------

def _angles(dim, n_theta, n_phi, gl=False):
    if dim == 1:
        mu, wt = gauss_legendre_mu(n_theta) if gl else midpoint_mu(n_theta)
        return mu, wt, np.zeros(1), np.full(1, 2.0 * math.pi)
    mu, wt = midpoint_mu(n_theta)
    phi, wp = midpoint_phi(n_phi)
    return mu, wt, phi, wp


def slab1d(n_cells=64, n_groups=8, n_theta=16, kappa0=1.0, T=0.1, T_b=1.0, tol=1e-8,
           rank_cap=8, precision=PREC_FP64, n_steps=128, cfl=0.5, seed=0, nu=(0.01, 10.0)):
    """1D slab x in [0,1], Gauss-Legendre mu, left Planck inflow, uniform medium."""
    edges = log_group_edges(n_groups, *nu)
    mu, wt, phi, wp = _angles(1, n_theta, 1, gl=True)
    return Problem(
        name="slab1d", dim=1, n_cells=(n_cells, 1, 1), extent=(1.0, 1.0, 1.0), edges=edges,
        kappa0=np.full(n_cells, float(kappa0)), kappa_scale=nu_power_scale(edges),
        T_cell=np.full(n_cells, float(T)), mu=mu, w_theta=wt, phi=phi, w_phi=wp,
        bc=(BC_INFLOW_PLANCK, 0, 0, 0, 0, 0), bc_T=(T_b, 0, 0, 0, 0, 0),
        cfl=cfl, tol=tol, rank_cap=rank_cap, precision=precision, n_steps=n_steps, seed=seed)


def plane2d(n=128, n_groups=32, n_theta=8, n_phi=8, T=0.1, T_b=1.0, tol=1e-6, rank_cap=32,
            precision=PREC_FP32, n_steps=512, cfl=0.5, seed=0, sigma=1.0, corr_len=0.1,
            nu=(0.01, 10.0)):
    """2D square [0,1]^2, seeded lognormal kappa0, left Planck inflow."""
    nc = (n, n, 1)
    ext = (1.0, 1.0, 1.0)
    edges = log_group_edges(n_groups, *nu)
    mu, wt, phi, wp = _angles(2, n_theta, n_phi)
    k0 = lognormal_kappa0(nc, ext, 2, sigma=sigma, corr_len=corr_len, seed=seed)
    return Problem(
        name="plane2d", dim=2, n_cells=nc, extent=ext, edges=edges, kappa0=k0,
        kappa_scale=nu_power_scale(edges), T_cell=np.full(n * n, float(T)), mu=mu, w_theta=wt,
        phi=phi, w_phi=wp, bc=(BC_INFLOW_PLANCK, 0, 0, 0, 0, 0), bc_T=(T_b, 0, 0, 0, 0, 0),
        cfl=cfl, tol=tol, rank_cap=rank_cap, precision=precision, n_steps=n_steps, seed=seed)


# Planck and Boltzmann constants (cgs) to express frequency edges given in Hz
# as h nu / k_B in temperature units, and the radiation constant of the
# emission units (h = k = 1): (4 pi / c) sum_g eps_g(T) = a T^4, a = 8 pi^5 / (15 c).
H_CGS = 6.62607015e-27
KB_CGS = 1.380649e-16


def radiation_constant(c: float = 1.0) -> float:
    return 8.0 * math.pi ** 5 / (15.0 * c)


FLUX_UPWIND, FLUX_RUSANOV, FLUX_HLL = 0, 1, 2


def gaussian_diffusion(n_cells=128, n_groups=4, n_theta=16, ks_min=1000.0, ks_max=2000.0, width=0.25,
                       cfl=1.0, tol=1e-8, rank_cap=16, precision=PREC_FP64, seed=0, n_steps=2400):
    """1D Gaussian pulse diffusing through a purely scattering slab on
    [-5, 5] (stored as [0, 10], x - 5 the physical coordinate): kappa_a = 0,
    kappa_{s,g} ~ U[ks_min, ks_max] per group (seeded), the Rusanov flux with
    S+ = 0, vacuum faces, c = 1.  The initial state (gaussian_initial) is the
    isotropic field J_g(0, x) with 4 D_g t_{0,g} = width for every group, so all
    groups start equal.  D_g = c / (3 kappa_{s,g})."""
    rng = np.random.default_rng(seed)
    ks = np.sort(rng.uniform(ks_min, ks_max, n_groups))
    edges = log_group_edges(n_groups, 0.01, 10.0)
    mu, wt, phi, wp = _angles(1, n_theta, 1, gl=True)
    return Problem(
        name="gaussian_diffusion", dim=1, n_cells=(n_cells, 1, 1), extent=(10.0, 1.0, 1.0), edges=edges,
        kappa0=np.zeros(n_cells), kappa_scale=np.ones(n_groups), T_cell=np.zeros(n_cells), mu=mu, w_theta=wt,
        phi=phi, w_phi=wp, bc=(BC_VACUUM, BC_VACUUM, 0, 0, 0, 0), bc_T=(0.0,) * 6, cfl=cfl, tol=tol,
        rank_cap=rank_cap, precision=precision, n_steps=n_steps, seed=seed,
        kappa_s_full=np.tile(ks, (n_cells, 1)), flux=FLUX_RUSANOV, rusanov_s=0.0)


def gaussian_profile(prob, t: float, width: float = 0.25, A: float = 1.0) -> np.ndarray:
    """(N_X, N_nu) closed-form mean intensity of the diffusing pulse at time t:
    A / sqrt(4 pi D (t0 + t)) exp(-x^2 / (4 D (t0 + t))), with 4 D t0 = width."""
    x = cell_centres(prob.n_cells, prob.extent)[:, 0] - 0.5 * prob.extent[0]
    ks = np.asarray(prob.kappa_s_full, float).reshape(prob.n_x, prob.n_groups)[0]
    D = prob.c / (3.0 * ks)
    w = width + 4.0 * D * t              # 4 D (t0 + t)
    return A / np.sqrt(np.pi * w)[None, :] * np.exp(-x[:, None] ** 2 / w[None, :])


def thermal_relax(n_cells=1, n_theta=2, c_v=8.0, T=10.0, T_r=1.0, kappas=(10.0, 1.0, 0.1), k_hz=1.5e11,
                  cfl=0.1, t_final=40.0, tol=1e-12, rank_cap=8, precision=PREC_FP64):
    """Thermal relaxation with three groups (Section 4): periodic homogeneous
    slab of unit cells, rho = 1, c_v = 8 in units where a = c = 1 (so the
    heat capacity here is 8 a), medium at T = 10, radiation initially Planck
    at T_r = 1, group edges nu_1 = k and nu_2 = 2 k (k = 1.5e11 Hz) and group
    opacities 10, 1, 0.1."""
    nu1 = H_CGS * k_hz / KB_CGS
    edges = np.array([0.0, nu1, 2.0 * nu1, np.inf])
    mu, wt, phi, wp = _angles(1, n_theta, 1, gl=True)
    dt = cfl   # unit cells and c = 1
    return Problem(
        name="thermal_relax", dim=1, n_cells=(n_cells, 1, 1), extent=(float(n_cells), 1.0, 1.0), edges=edges,
        kappa0=np.ones(n_cells), kappa_scale=np.asarray(kappas, float), T_cell=np.full(n_cells, float(T)),
        mu=mu, w_theta=wt, phi=phi, w_phi=wp, bc=(BC_PERIODIC, BC_PERIODIC, 0, 0, 0, 0),
        bc_T=(0, 0, 0, 0, 0, 0), c=1.0, cfl=cfl, tol=tol, rank_cap=rank_cap, precision=precision,
        n_steps=int(round(t_final / dt)), heat_capacity=c_v * radiation_constant(1.0),
        T_rad0=np.full(n_cells, float(T_r)))


C3_CLUMPS = (((0.35, 0.5, 0.5), 0.1), ((0.65, 0.4, 0.6), 0.08))


def clumps3d(n=64, n_groups=64, n_theta=8, n_phi=16, T=0.1, T_b=1.0, tol=1e-5, rank_cap=64,
             precision=PREC_BF16X, n_steps=384, cfl=0.5, seed=0, nu=(0.01, 10.0)):
    """3D cube [0,1]^3, lognormal kappa0 with two dense spherical clumps (x100)."""
    nc = (n, n, n)
    ext = (1.0, 1.0, 1.0)
    edges = log_group_edges(n_groups, *nu)
    mu, wt, phi, wp = _angles(3, n_theta, n_phi)
    k0 = lognormal_kappa0(nc, ext, 3, seed=seed)
    k0 = add_clumps(k0, nc, ext, C3_CLUMPS, 100.0)
    return Problem(
        name="clumps3d", dim=3, n_cells=nc, extent=ext, edges=edges, kappa0=k0,
        kappa_scale=nu_power_scale(edges), T_cell=np.full(n ** 3, float(T)), mu=mu, w_theta=wt,
        phi=phi, w_phi=wp, bc=(BC_INFLOW_PLANCK, 0, 0, 0, 0, 0), bc_T=(T_b, 0, 0, 0, 0, 0),
        cfl=cfl, tol=tol, rank_cap=rank_cap, precision=precision, n_steps=n_steps, seed=seed)


def clumps3d_slab(n=64, nz=4, slab=0, **kw):
    """One z-slab (n x n x nz cells) of the clumps3d cube with the cube's
    opacity field (same seed) cut to the slab and the cube's cell spacing, so
    a step costs nz / n of the cube's.  Used to time the dense CPU reference on
    a bounded part of the 64^3 workload."""
    cube = clumps3d(n=n, **kw)
    k0 = np.asarray(cube.kappa0).reshape(n, n, n)[slab * nz:(slab + 1) * nz].ravel().copy()
    return cube.copy(name="clumps3d_slab", n_cells=(n, n, nz), extent=(1.0, 1.0, nz / n), kappa0=k0,
                     T_cell=np.asarray(cube.T_cell).reshape(n, n, n)[slab * nz:(slab + 1) * nz].ravel().copy())


def spikes3d(n=256, n_groups=128, n_theta=16, n_phi=16, T=0.1, T_b=1.0, tol=1e-5, rank_cap=128,
             precision=PREC_BF16X, n_steps=8, cfl=0.5, seed=0, nu=(0.01, 10.0)):
    """3D cube, lognormal kappa0, 8 random groups with kappa x50 (line-like spikes)."""
    nc = (n, n, n)
    ext = (1.0, 1.0, 1.0)
    edges = log_group_edges(n_groups, *nu)
    mu, wt, phi, wp = _angles(3, n_theta, n_phi)
    k0 = lognormal_kappa0(nc, ext, 3, seed=seed)
    rng = np.random.default_rng(seed + 1000)
    scale = nu_power_scale(edges)
    spikes = rng.choice(n_groups, size=min(8, n_groups), replace=False)
    scale[spikes] *= 50.0
    return Problem(
        name="spikes3d", dim=3, n_cells=nc, extent=ext, edges=edges, kappa0=k0, kappa_scale=scale,
        T_cell=np.full(n ** 3, float(T)), mu=mu, w_theta=wt, phi=phi, w_phi=wp,
        bc=(BC_INFLOW_PLANCK, 0, 0, 0, 0, 0), bc_T=(T_b, 0, 0, 0, 0, 0), cfl=cfl, tol=tol,
        rank_cap=rank_cap, precision=precision, n_steps=n_steps, seed=seed)


def spikes3d_slab(n=256, nz=32, slab=0, n_groups=128, n_theta=16, n_phi=16, T=0.1, T_b=1.0, tol=1e-5,
                  rank_cap=18, precision=PREC_BF16X, n_steps=8, cfl=0.5, seed=0, nu=(0.01, 10.0)):
    """One z-slab (n x n x nz cells) of the spikes3d cube: the share of one GPU
    when the cube is split into n / nz slabs along z.  The opacity field is the
    cube's (same seed), cut to the slab; the slab's z faces are vacuum (in a
    split run they would be exchanged halos).  Cells keep the cube's spacing."""
    cube = spikes3d(n=n, n_groups=n_groups, n_theta=n_theta, n_phi=n_phi, T=T, T_b=T_b, tol=tol,
                    rank_cap=rank_cap, precision=precision, n_steps=n_steps, cfl=cfl, seed=seed, nu=nu)
    k0 = np.asarray(cube.kappa0).reshape(n, n, n)[slab * nz:(slab + 1) * nz].ravel().copy()
    return cube.copy(name="spikes3d_slab", n_cells=(n, n, nz), extent=(1.0, 1.0, nz / n), kappa0=k0,
                     T_cell=np.full(n * n * nz, float(T)))


def served_requests(n_requests=256, seed=0, steps=64):
    """Request mix of the served batch: half 1D (16 GL mu), half 2D (8x8); cells per
    dimension ~ U{64..256}; groups ~ U{16..64}; rank caps ~ U{4..48}; seeded kappa0."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_requests):
        is2d = bool(rng.integers(0, 2))
        ncell = int(rng.integers(64, 257))
        ng = int(rng.integers(16, 65))
        cap = int(rng.integers(4, 49))
        prec = PREC_FP32 if rng.integers(0, 2) else PREC_FP64
        s = int(rng.integers(0, 2 ** 31 - 1))
        if is2d:
            p = plane2d(n=ncell, n_groups=ng, rank_cap=cap, precision=prec, n_steps=steps, seed=s)
        else:
            p = slab1d(n_cells=ncell, n_groups=ng, rank_cap=cap, precision=prec, n_steps=steps,
                       seed=s, kappa0=1.0)
            p = p.copy(kappa0=lognormal_kappa0(p.n_cells, p.extent, 1, seed=s))
        p.name = f"req{i}"
        out.append(p)
    return out


def poisson_arrivals(n, rate, seed=0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def random_tt(M, n_theta, n_phi, r1, r2, seed=0, decay=0.5):
    """Random TT cores (Z: M x r1, Theta: r1 x N_theta x r2, Phi: r2 x N_phi) with
    geometrically decaying scales, used as seeded test states."""
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((M, r1)) * (decay ** np.arange(r1))
    Th = rng.standard_normal((r1, n_theta, r2))
    Ph = rng.standard_normal((r2, n_phi)) * (decay ** np.arange(r2))[:, None]
    return Z, Th, Ph


CONFIGS = {
    "slab1d": slab1d,
    "plane2d": plane2d,
    "clumps3d": clumps3d,
    "spikes3d": spikes3d,
}
