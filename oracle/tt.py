"""Tensor-train (TT) algebra of the multigroup transport step, in plain numpy FP64.

TEST INFRASTRUCTURE ONLY: the oracle the GPU path is compared with.  It shares
no code with the GPU library.

Format (Section 3.1, the merged spatio-spectral decomposition):
    I[k, l, p] = sum_{a,b} Z[k, a] Theta[a, l, b] Phi[b, p],
with k = cell*N_nu + g, Z of shape (N_X N_nu, r1), Theta (r1, N_theta, r2),
Phi (r2, N_phi).

Transport operator (Appendix A, "Value of n"): the upwind update is the
identity plus n = 2 d_X rank-1 TT operators, one per (axis, sign of n_d).  The
operator for (d, +) acts on Z as -lambda_d (I - O_{d-}) and multiplies the
angular cores by the positive part of n_d; (d, -) acts as -lambda_d (O_{d+} - I)
with the negative part.  Boundary ghost values enter as a rank-1 Dirichlet TT
(the blue TT of the Appendix A figure), one per inflow face.  The source update
(Section 2.1, backward Euler at fixed T, no scattering) is a Hadamard product
with the rank-1 field d = 1/(1 + c dt kappa) plus the rank-1 emission term
c dt kappa eps d (Section 3.1: rank-1 TT lift of spatio-spectral fields).

The Rusanov flux (Section 2.1 names it among the three stencils; Appendix A,
"Value of n", shows it is also two rank-1 operators per axis) gives, per axis
d, with lambda = lambda_d and s = S+ / c: one term with the full direction
component n_d acting on Z as -(lambda / 2)(O_{d+} - O_{d-}), and one without
angular factor acting as (lambda s / 2)(O_{d+} - 2 I + O_{d-}).  In every
case a ghost value enters the rank-1 Dirichlet term of a face through the
coefficient its term puts on the shift that leaves the domain there.

The HLL flux (Section 2.1: the asymptotic-preserving stencil, the only one
whose multigroup form changes, through a per-group optical depth; Appendix
A: still the upwind structure, two rank-1 operators per axis, with spatially
varying coefficients): per axis the n_d^+ and n_d^- terms of the upwind flux
with the spatial parts built from the interface factors eps (hll_eps) of the
row's own group opacity, so the coefficients vary per (cell, group) row.

Isotropic scattering (kappa_s, Section 2.1 source update): with
a = c dt kappa_a, b = c dt kappa_s and J* the angle mean of the transported
TT, the source becomes d I* plus the rank-1 isotropic column
d (a eps + b J^{m+1}), d = 1 / (1 + a + b), J^{m+1} = (J* + a eps) / (1 + a).

The sum is formed explicitly: Z_new is the block row [Z, S_1 Z, ..., S_n Z,
bc..., emission], Theta_new is block diagonal and Phi_new is stacked, so the
ranks after the update are (n+1) r + n_bc + 1 (Appendix A, ranks of the
green TT plus the source's rank growth).

Rounding: TT-SVD rounding of Oseledets (2011), which the paper cites for its
SVD rounding method: right-to-left orthogonalisation by QR, then a
left-to-right sweep of truncated SVDs, each bond truncated at
delta = tol * ||X||_F / sqrt(d - 1) with d = 3 cores.
"""
from __future__ import annotations

import math

import numpy as np

from . import dense, philox


# ---------------------------------------------------------------------------
# the operator terms
# ---------------------------------------------------------------------------

def direction_factors(prob):
    """For each (axis, sign) term a pair (g[N_theta], h[N_phi]) with
    g(l) h(p) = n_d^{+/-}(l, p), the positive / negative part of the direction
    component.  Returned as a list of (axis, sign, g, h)."""
    mu = np.asarray(prob.mu, float)
    phi = np.asarray(prob.phi, float)
    terms = []
    if prob.dim == 1:
        one = np.ones(prob.n_phi)
        terms.append((0, +1, np.maximum(mu, 0.0), one))
        terms.append((0, -1, np.minimum(mu, 0.0), one))
        return terms
    st = np.sqrt(np.maximum(0.0, 1.0 - mu * mu))
    cp, sp = np.cos(phi), np.sin(phi)
    terms.append((0, +1, st, np.maximum(cp, 0.0)))
    terms.append((0, -1, st, np.minimum(cp, 0.0)))
    terms.append((1, +1, st, np.maximum(sp, 0.0)))
    terms.append((1, -1, st, np.minimum(sp, 0.0)))
    if prob.dim == 3:
        one = np.ones(prob.n_phi)
        terms.append((2, +1, np.maximum(mu, 0.0), one))
        terms.append((2, -1, np.minimum(mu, 0.0), one))
    return terms


def hll_eps(prob, axis):
    """Interface factors of the HLL flux along `axis` for every row k = cell
    N_nu + g: eps = (1 - exp(-tau)) / tau with tau = beta dx (kappa_k + kappa
    of the neighbour row) / 2 (kappa: absorption plus scattering; the row's own
    opacity on a non-periodic boundary face).  Returns (eps_low, eps_high),
    each of shape (M,), for the faces towards cell - e_d and cell + e_d."""
    kap = dense.kappa_total(prob)                      # (N_X, N_nu)
    beta = float(getattr(prob, "hll_beta", 20.0))
    dx = prob.extent[axis] / prob.n_cells[axis]
    idx, N = _cell_index(prob)
    periodic = prob.bc[2 * axis] == dense.FACE_PERIODIC
    out = []
    for s in (-1, +1):
        j = idx.copy()
        j[:, axis] += s
        inside = (j[:, axis] >= 0) & (j[:, axis] < N[axis])
        if periodic:
            j[:, axis] %= N[axis]
            inside[:] = True
        src = np.where(inside, j[:, 0] + N[0] * (j[:, 1] + N[1] * j[:, 2]), np.arange(len(idx)))
        tau = beta * dx * 0.5 * (kap + kap[src])
        safe = np.where(tau > 0.0, tau, 1.0)
        out.append(np.where(tau > 0.0, -np.expm1(-safe) / safe, 1.0).reshape(-1))
    return out[0], out[1]


def transport_terms(prob):
    """The streaming operator's rank-1 terms as (axis, g, h, c0, cm, cp): the
    angular factors g[N_theta], h[N_phi] and the spatial part
    c0 I + cm O_{d-} + cp O_{d+} ((O_{d-/+} Z)[cell] = Z[cell -/+ e_d]).
    The coefficients are scalars, or per-row arrays (M,) for the HLL flux,
    whose interface factors depend on the row's group opacity."""
    dt = dense.time_step(prob)
    flux, s_rus = dense.flux_params(prob)
    out = []
    if flux == 2:
        # HLL (Appendix A: the upwind-structured form with spatially varying
        # coefficients): for n_d >= 0 the flux through the faces is
        # c n_d [(1 + eps)/2 I_L + (1 - eps)/2 I_R], for n_d < 0
        # c n_d [(1 - eps)/2 I_L + (1 + eps)/2 I_R]
        for axis, sgn, g, h in direction_factors(prob):
            lam = prob.c * dt / (prob.extent[axis] / prob.n_cells[axis])
            eL, eR = hll_eps(prob, axis)
            if sgn > 0:
                out.append((axis, g, h, -lam * 0.5 * (eL + eR), lam * 0.5 * (1.0 + eL), -lam * 0.5 * (1.0 - eR)))
            else:
                out.append((axis, g, h, lam * 0.5 * (eL + eR), lam * 0.5 * (1.0 - eL), -lam * 0.5 * (1.0 + eR)))
        return out
    if flux == 0:
        for axis, sgn, g, h in direction_factors(prob):
            lam = prob.c * dt / (prob.extent[axis] / prob.n_cells[axis])
            if sgn > 0:   # -lambda n^+ (I - O_{d-})
                out.append((axis, g, h, -lam, lam, 0.0))
            else:         # -lambda n^- (O_{d+} - I)
                out.append((axis, g, h, lam, 0.0, -lam))
        return out
    mu = np.asarray(prob.mu, float)
    phi = np.asarray(prob.phi, float)
    st = np.sqrt(np.maximum(0.0, 1.0 - mu * mu))
    for axis in range(prob.dim):
        lam = prob.c * dt / (prob.extent[axis] / prob.n_cells[axis])
        if prob.dim == 1 or axis == 2:
            g, h = mu.copy(), np.ones(prob.n_phi)
        else:
            g, h = st.copy(), (np.cos(phi) if axis == 0 else np.sin(phi))
        out.append((axis, g, h, 0.0, 0.5 * lam, -0.5 * lam))
        if s_rus != 0.0:
            out.append((axis, np.ones(prob.n_theta), np.ones(prob.n_phi), -lam * s_rus, 0.5 * lam * s_rus,
                        0.5 * lam * s_rus))
    return out


def _cell_index(prob):
    nx = int(prob.n_cells[0])
    ny = int(prob.n_cells[1]) if prob.dim > 1 else 1
    nz = int(prob.n_cells[2]) if prob.dim > 2 else 1
    cell = np.arange(nx * ny * nz)
    return np.stack([cell % nx, (cell // nx) % ny, cell // (nx * ny)], axis=1), (nx, ny, nz)


def shift(prob, Z: np.ndarray, axis: int, s: int) -> np.ndarray:
    """(O Z)[cell] = Z[cell + s e_axis]; zero outside the domain unless the axis is
    periodic, in which case the index wraps."""
    G = prob.n_groups
    idx, N = _cell_index(prob)
    r = Z.shape[1]
    Zc = Z.reshape(-1, G, r)
    j = idx.copy()
    j[:, axis] += s
    periodic = prob.bc[2 * axis] == dense.FACE_PERIODIC
    inside = (j[:, axis] >= 0) & (j[:, axis] < N[axis])
    if periodic:
        j[:, axis] %= N[axis]
        inside[:] = True
    src = j[:, 0] + N[0] * (j[:, 1] + N[1] * j[:, 2])
    out = np.zeros_like(Zc)
    out[inside] = Zc[src[inside]]
    return out.reshape(-1, r)


def bc_columns(prob):
    """Rank-1 Dirichlet terms: list of (z[M], g[N_theta], h[N_phi]).  On the
    first cell layer of an inflow face at the low end of axis d, each term of
    that axis contributes cm * ghost_g with its angular factors (its O_{d-}
    shift reads the ghost there); at the high end cp * ghost_g on the last
    layer.  Upwind: +lambda ghost with n_d^+ (low), -lambda ghost with n_d^-
    (high)."""
    ghost = dense.ghost_values(prob)
    idx, N = _cell_index(prob)
    cols = []
    for face in range(2 * prob.dim):
        kind = prob.bc[face]
        if kind not in (dense.FACE_INFLOW_PLANCK, dense.FACE_INFLOW_VALUES):
            continue
        axis, high = face // 2, face % 2
        layer = (idx[:, axis] == (N[axis] - 1 if high else 0)).astype(float)
        for ax, g, h, c0, cm, cp in transport_terms(prob):
            coef = cp if high else cm
            if ax != axis or np.all(np.asarray(coef) == 0.0):
                continue
            coef = np.asarray(coef, float).reshape(-1, prob.n_groups) if np.ndim(coef) else coef
            z = (coef * layer[:, None] * ghost[face][None, :]).reshape(-1)
            cols.append((z, g, h))
    return cols


def n_bc(prob) -> int:
    return len(bc_columns(prob))


def _assemble(blocksZ, blocksTh, blocksPh, n_theta):
    """Explicit TT sum: Z concatenated, Theta block diagonal, Phi stacked."""
    Z = np.concatenate(blocksZ, axis=1)
    R1 = sum(t.shape[0] for t in blocksTh)
    R2 = sum(t.shape[2] for t in blocksTh)
    Th = np.zeros((R1, n_theta, R2))
    a = b = 0
    for t in blocksTh:
        Th[a:a + t.shape[0], :, b:b + t.shape[2]] = t
        a += t.shape[0]
        b += t.shape[2]
    Ph = np.concatenate(blocksPh, axis=0)
    return Z, Th, Ph


def apply_transport(prob, Z, Th, Ph):
    """I* = (identity + sum of the n rank-1 upwind operators) I + Dirichlet terms."""
    bZ, bT, bP = [Z], [Th], [Ph]

    def scaled(c, X):   # scalar or per-row coefficient times the rows of X
        return c * X if np.ndim(c) == 0 else np.asarray(c)[:, None] * X

    for axis, g, h, c0, cm, cp in transport_terms(prob):
        SZ = scaled(c0, Z)
        if np.any(np.asarray(cm) != 0.0):
            SZ = SZ + scaled(cm, shift(prob, Z, axis, -1))
        if np.any(np.asarray(cp) != 0.0):
            SZ = SZ + scaled(cp, shift(prob, Z, axis, +1))
        bZ.append(SZ)
        bT.append(Th * g[None, :, None])
        bP.append(Ph * h[None, :])
    for z, g, h in bc_columns(prob):
        bZ.append(z[:, None])
        bT.append(g[None, :, None].copy())
        bP.append(h[None, :].copy())
    return _assemble(bZ, bT, bP, prob.n_theta)


def apply_source(prob, Z, Th, Ph):
    """Backward-Euler absorption/emission (and isotropic scattering) at fixed
    T: d * I + d (c dt kappa eps + c dt kappa_s J^{m+1})."""
    dt = dense.time_step(prob)
    kap = dense.kappa_field(prob).reshape(-1)
    eps = dense.emission(prob).reshape(-1)
    a = prob.c * dt * kap
    if getattr(prob, "kappa_s_full", None) is None:
        d = 1.0 / (1.0 + a)
        col = a * eps * d
    else:
        b = prob.c * dt * dense.kappa_s_field(prob).reshape(-1)
        d = 1.0 / (1.0 + a + b)
        # angle mean of the TT: J*[k] = (1 / 4 pi) sum_a Z[k, a] sum_{l,b,p} w_l Theta[a,l,b] Phi[b,p] w_p
        e = np.einsum("alb,l,bp,p->a", Th, np.asarray(prob.w_theta, float), Ph, np.asarray(prob.w_phi, float))
        J_star = Z @ e / (4.0 * np.pi)
        J_new = (J_star + a * eps) / (1.0 + a)
        col = (a * eps + b * J_new) * d
    bZ = [Z * d[:, None], col[:, None]]
    bT = [Th, np.ones((1, prob.n_theta, 1))]
    bP = [Ph, np.ones((1, prob.n_phi))]
    return _assemble(bZ, bT, bP, prob.n_theta)


def apply_step(prob, Z, Th, Ph):
    """Transport followed by the source update, as one explicit TT sum."""
    return apply_source(prob, *apply_transport(prob, Z, Th, Ph))


def full(Z, Th, Ph) -> np.ndarray:
    return np.einsum("ka,alb,bp->klp", Z, Th, Ph, optimize=True)


def initial_tt(prob):
    """Rank-1 isotropic Planck state at the medium temperature."""
    eps = dense.emission(prob).reshape(-1)
    return eps[:, None].copy(), np.ones((1, prob.n_theta, 1)), np.ones((1, prob.n_phi))


# ---------------------------------------------------------------------------
# TT-SVD rounding
# ---------------------------------------------------------------------------

def delta_rank(s: np.ndarray, delta: float, cap: int) -> int:
    """Smallest r >= 1 with ||s[r:]||_2 <= delta, then capped."""
    n = len(s)
    tail = np.sqrt(np.cumsum((s[::-1] ** 2))[::-1])    # tail[i] = ||s[i:]||
    r = n
    for i in range(1, n):
        if tail[i] <= delta:
            r = i
            break
    return max(1, min(r, cap, n))


def round_tt(Z, Th, Ph, tol: float, cap: int):
    """TT-SVD rounding (Oseledets 2011): orthogonalise right-to-left with QR of
    the row-unfolded cores, then truncate left-to-right with delta-truncated
    SVDs.  Returns (Z, Theta, Phi, info); cores are in Oseledets' gauge
    (Z and Theta left-orthonormal, the norm carried by Phi)."""
    R1, nt, R2 = Th.shape
    # right-to-left orthogonalisation
    q, r = np.linalg.qr(Ph.T)                 # Ph = r^T q^T
    Ph_o = q.T
    Th1 = np.einsum("alb,bc->alc", Th, r.T)   # absorb the triangular factor
    k2 = Th1.shape[2]
    q, r = np.linalg.qr(Th1.reshape(R1, nt * k2).T)
    Th_o = q.T.reshape(-1, nt, k2)
    Z1 = Z @ r.T
    # left-to-right compression
    U, s, Vt = np.linalg.svd(Z1, full_matrices=False)
    norm = float(np.sqrt(np.sum(s ** 2)))
    delta = tol * norm / math.sqrt(2.0)
    r1 = delta_rank(s, delta, cap)
    Zo = U[:, :r1]
    C2 = np.einsum("ja,alb->jlb", s[:r1, None] * Vt[:r1], Th_o)
    U2, s2, Vt2 = np.linalg.svd(C2.reshape(r1 * nt, k2), full_matrices=False)
    r2 = delta_rank(s2, delta, cap)
    Tho = U2[:, :r2].reshape(r1, nt, r2)
    Pho = (s2[:r2, None] * Vt2[:r2]) @ Ph_o
    info = dict(norm=norm, r1=r1, r2=r2, sv1=s, sv2=s2,
                discarded=float(math.sqrt(np.sum(s[r1:] ** 2) + np.sum(s2[r2:] ** 2))),
                R1=R1, R2=R2, k_s=storage_factor((Z, Th, Ph), (Zo, Tho, Pho)))
    return Zo, Tho, Pho, info


def storage_factor(before, after) -> float:
    """k_s of one rounding (Section 3.2 and the appendix on compression): the
    entries of the TT as it stands before rounding (the explicit sum the SVD
    method forms) over the entries of the rounded TT, counted on the arrays."""
    return float(sum(a.size for a in before)) / float(sum(a.size for a in after))


# Randomized rounding (Section 3.1 footnote: the solver's third rounding
# method).  Each pass first compresses the TT sum to sketch ranks equal to the
# incoming solution ranks plus a constant (the "randomized preconditioning"),
# then truncates the result with the same delta-truncated TT-SVD rounding as
# the SVD method.  The compression is the randomize-then-orthogonalize scheme
# of the cited randomized rounding work (Al Daas et al. 2023): contract the
# sum from the right with a random TT of the sketch ranks, take an orthonormal
# basis of the sketch of the first core, project the sum onto it, and repeat
# for the middle core.  The random cores are counter-based (oracle.philox),
# uniform on [-1, 1).

RAND_KEEP = 1e-7     # a sketch direction is kept when its singular value exceeds RAND_KEEP times the largest
ROUND_RAND = 3


def sketch_ranks(R1: int, R2: int, n_theta: int, n_phi: int, r_in, p: int):
    """Sketch ranks (l1, l2): the incoming ranks plus p, at most the ranks the
    sum has after right-to-left orthogonalisation, k2 = min(R2, N_phi) and
    k1 = min(R1, N_theta k2)."""
    k2 = min(R2, n_phi)
    k1 = min(R1, n_theta * k2)
    return min(r_in[0] + p, k1), min(r_in[1] + p, k2)


def sketch_cores(seed: int, round_index: int, l1: int, n_theta: int, l2: int, n_phi: int):
    """The random TT's second core (l1, N_theta, l2) and third core (l2, N_phi)."""
    G2 = philox.sketch_entries(seed, 0, round_index, l1 * n_theta * l2).reshape(l1, n_theta, l2)
    G3 = philox.sketch_entries(seed, 1, round_index, l2 * n_phi).reshape(l2, n_phi)
    return G2, G3


def range_basis(Y: np.ndarray, sv_out=None) -> np.ndarray:
    """Orthonormal basis of the numerical range of Y: the left singular vectors
    whose singular values exceed RAND_KEEP times the largest (at least one).
    The singular values relative to the largest are appended to sv_out."""
    U, s, _ = np.linalg.svd(Y, full_matrices=False)
    keep = max(1, int(np.sum(s > RAND_KEEP * s[0]))) if s.size and s[0] > 0 else 1
    if sv_out is not None:
        sv_out.append(s / s[0] if s.size and s[0] > 0 else s)
    return U[:, :keep]


def randomized_precondition(Z, Th, Ph, G2, G3, sv_out=None):
    """Randomize-then-orthogonalize compression of the TT (Z, Theta, Phi) with
    the random cores G2 (l1, N_theta, l2) and G3 (l2, N_phi).  Returns the
    left-orthonormal TT (Q1, Q2, Phi') of ranks at most (l1, l2); the two
    sketches' relative singular values are appended to sv_out."""
    R1, nt, R2 = Th.shape
    W3 = Ph @ G3.T                                   # R2 x l2: right contraction of the last core
    W2 = np.einsum("alb,glh,bh->ag", Th, G2, W3)     # R1 x l1: and of the last two
    Q1 = range_basis(Z @ W2, sv_out)                 # M x l1'
    Th1 = np.einsum("ja,alb->jlb", Q1.T @ Z, Th)     # (Q1^T Z) x_1 Theta: l1' x N_theta x R2
    Th1m = Th1.reshape(-1, R2)
    Q2 = range_basis(Th1m @ W3, sv_out)              # (l1' N_theta) x l2'
    Ph1 = (Q2.T @ Th1m) @ Ph                         # l2' x N_phi
    return Q1, Q2.reshape(Q1.shape[1], nt, Q2.shape[1]), Ph1


def randomized_round(Z, Th, Ph, tol: float, cap: int, r_in, p: int, seed: int, round_index: int):
    """Randomized rounding of the TT sum (Z, Theta, Phi) whose incoming
    solution had ranks r_in: compression to the sketch ranks, then round_tt."""
    R1, nt, R2 = Th.shape
    l1, l2 = sketch_ranks(R1, R2, nt, Ph.shape[1], r_in, p)
    G2, G3 = sketch_cores(seed, round_index, l1, nt, l2, Ph.shape[1])
    svs = []
    Zo, Tho, Pho, info = round_tt(*randomized_precondition(Z, Th, Ph, G2, G3, svs), tol, cap)
    info.update(R1=R1, R2=R2, l1=l1, l2=l2, sketch_sv=svs)
    return Zo, Tho, Pho, info


def _round(prob, Z, Th, Ph, tol, cap, r_in, round_index):
    if getattr(prob, "round_method", 2) == ROUND_RAND:
        return randomized_round(Z, Th, Ph, tol, cap, r_in, prob.rand_oversample, prob.rand_seed, round_index)
    return round_tt(Z, Th, Ph, tol, cap)


def step(prob, Z, Th, Ph, tol=None, cap=None, round_index=0):
    """One step then truncate.  step_order 0: one rounding after transport and
    source; step_order 1: round after the transport and again after the source
    (the paper's order, Section 3.1 closing paragraph).  round_index numbers
    the rounding passes (it keys the randomized method's sketch)."""
    tol = prob.tol if tol is None else tol
    cap = prob.rank_cap if cap is None else cap
    r_in = (Z.shape[1], Ph.shape[0])
    if prob.step_order == 1:
        Z, Th, Ph, _ = _round(prob, *apply_transport(prob, Z, Th, Ph), tol, cap, r_in, round_index)
        return _round(prob, *apply_source(prob, Z, Th, Ph), tol, cap, (Z.shape[1], Ph.shape[0]), round_index + 1)
    return _round(prob, *apply_step(prob, Z, Th, Ph), tol, cap, r_in, round_index)


def solve(prob, n_steps=None, cores=None, tol=None, cap=None):
    Z, Th, Ph = initial_tt(prob) if cores is None else cores
    n_steps = prob.n_steps if n_steps is None else n_steps
    per = 2 if prob.step_order == 1 else 1
    infos = []
    for m in range(n_steps):
        Z, Th, Ph, info = step(prob, Z, Th, Ph, tol, cap, round_index=m * per)
        infos.append(info)
    return (Z, Th, Ph), infos


def compression(prob, r1: int, r2: int) -> float:
    """Section 3.2: dense entries over TT entries."""
    n_tt = prob.M * r1 + prob.n_theta * r1 * r2 + prob.n_phi * r2
    return prob.dense_entries / n_tt


def tt_energy(prob, Z, Th, Ph) -> float:
    """Quadrature-weighted content computed on the cores (TT integration)."""
    dV = float(np.prod([prob.extent[d] / prob.n_cells[d] for d in range(prob.dim)]))
    a = np.einsum("alb,l,bp,p->a", Th, np.asarray(prob.w_theta), Ph, np.asarray(prob.w_phi))
    return dV * float(Z.sum(axis=0) @ a)


# ---------------------------------------------------------------------------
# internal ranks of the combined core (the discussion of the internal
# structure of Z: internal delta-ranks and relative compression ratios)
# ---------------------------------------------------------------------------

def right_orthonormal_gauge(Z, Th, Ph):
    """Z' such that (Z', Theta', Phi') is the same tensor with Theta' and Phi'
    right-orthonormal: Phi = L_Phi Q_Phi, then the row unfolding of
    Theta x_3 L_Phi = L_Theta Q_Theta (QRs of the transposes), Z' = Z L_Theta."""
    r1, nt, r2 = Th.shape
    qp, rp = np.linalg.qr(Ph.T)                    # Phi^T = Q R, Phi = R^T Q^T
    Thp = np.einsum("alb,bc->alc", Th, rp.T)       # Theta x_3 L_Phi
    qt, rt = np.linalg.qr(Thp.reshape(r1, -1).T)   # unfolding^T = Q R
    return Z @ rt.T


def delta_rank_rel(s: np.ndarray, delta: float) -> int:
    """Smallest k with ||s[k:]||_2 <= delta ||s||_2 (s sorted descending), at least 1."""
    s = np.asarray(s, float)
    tot = float(np.sum(s * s))
    tail = np.concatenate([np.cumsum((s * s)[::-1])[::-1], [0.0]])
    for k in range(1, len(s) + 1):
        if math.sqrt(max(tail[k], 0.0)) <= delta * math.sqrt(tot):
            return k
    return len(s)


def internal_ranks(n_x: int, n_groups: int, Z, Th, Ph, delta: float) -> dict:
    """Internal delta-ranks of the combined core: r_nux from the SVD of
    reshape(Z', [N_nu, N_X r1]) and r_xnu from reshape(Z', [N_X, N_nu r1]), Z'
    in the right-orthonormal gauge (so the local error is the global one),
    with the relative compression ratios C_rel^nu and C_rel^x (the TT entry
    count over the entries of the split-core topologies)."""
    r1, nt, r2 = Th.shape
    npn = Ph.shape[1]
    Zp = right_orthonormal_gauge(Z, Th, Ph).reshape(n_x, n_groups, r1)   # [x, g, a]
    s_nu = np.linalg.svd(Zp.transpose(1, 0, 2).reshape(n_groups, n_x * r1), compute_uv=False)
    s_x = np.linalg.svd(Zp.reshape(n_x, n_groups * r1), compute_uv=False)
    r_nux = delta_rank_rel(s_nu, delta)
    r_xnu = delta_rank_rel(s_x, delta)
    n_tt = n_x * n_groups * r1 + nt * r1 * r2 + npn * r2
    c_nu = n_tt / (n_groups * r_nux + n_x * r_nux * r1 + nt * r1 * r2 + npn * r2)
    c_x = n_tt / (n_x * r_xnu + n_groups * r_xnu * r1 + nt * r1 * r2 + npn * r2)
    return {"r_nux": r_nux, "r_xnu": r_xnu, "C_rel_nu": c_nu, "C_rel_x": c_x, "s_nu": s_nu, "s_x": s_x}
