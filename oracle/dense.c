/*
 * Dense FP64 full-grid march for the multigroup discrete-ordinates upwind
 * finite-volume scheme with implicit absorption/emission at fixed medium
 * temperature.  TEST INFRASTRUCTURE ONLY: the oracle that the tensor-train
 * GPU path is checked against.  It shares no code with that path.
 *
 * One step (Section 2.1 "Numerics": forward-Euler transport with the upwind
 * flux, then the backward-Euler operator-split source update with the
 * scattering opacity set to zero, density 1 and T held fixed):
 *
 *   I*      = I - sum_d lambda_d [ n_d^+ (I_c - I_{c-e_d}) + n_d^- (I_{c+e_d} - I_c) ]
 *   I^{m+1} = (I* + c dt kappa eps) / (1 + c dt kappa)
 *
 * with lambda_d = c dt / dx_d, n^+ = max(n, 0), n^- = min(n, 0).  Ghost
 * intensities: the given isotropic value on inflow faces, 0 on vacuum faces,
 * wrap-around on periodic axes.
 *
 * The transport half alone (oracle_dense_transport) also takes the Rusanov flux
 * (Section 2.1 names upwind, Rusanov and HLL; the Rusanov interface flux for
 * the flux function c n_d I is (c n_d / 2)(I_L + I_R) - (S+ / 2)(I_R - I_L)):
 *
 *   I* = I - sum_d [ (lambda_d / 2) n_d (I_{c+e_d} - I_{c-e_d})
 *                    - (lambda_d s / 2) (I_{c+e_d} - 2 I_c + I_{c-e_d}) ],
 *
 * s = S+ / c.  Ghost intensities enter both neighbours for every direction.
 *
 * The HLL flux (oracle_dense_transport_hll; Section 2.1 names it as the
 * asymptotic-preserving stencil whose only multigroup change is a per-group
 * optical depth tau_{c,f}): at each interface the flux of c n_d I with wave
 * speeds +-c |n_d| eps, reduced by the interface's optical depth,
 *
 *   F = (c n_d / 2)(I_L + I_R) - (c |n_d| eps / 2)(I_R - I_L),
 *   eps = (1 - exp(-tau)) / tau,  tau = beta dx_d (kappa_L + kappa_R) / 2,
 *
 * kappa the total (absorption + scattering) opacity of the two cells in the
 * group (the inside cell's on a boundary face); eps -> 1 in thin cells (the
 * upwind flux) and -> 1 / tau in thick ones (central differences, so the
 * numerical diffusion stays below the physical one in the diffusion limit).
 *
 * Direction vector: in 1D n_x = mu; in 2D/3D n = (sin t cos p, sin t sin p, mu)
 * with sin t = sqrt(1 - mu^2).
 *
 * Layout of the dense intensity: I[((cell * G + g) * NT + l) * NP + p],
 * cell = ix + Nx * (iy + Ny * iz).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { FACE_VACUUM = 0, FACE_INFLOW_PLANCK = 1, FACE_PERIODIC = 2, FACE_INFLOW_VALUES = 3 };

static void direction(int dim, double mu, double ph, double n[3]) {
    if (dim == 1) {
        n[0] = mu; n[1] = 0.0; n[2] = 0.0;
        return;
    }
    double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    n[0] = st * cos(ph);
    n[1] = st * sin(ph);
    n[2] = (dim == 3) ? mu : 0.0;
}

/* Value of the neighbour of cell (ix,iy,iz) one step along axis d in
   direction s (+1/-1), for group g and angle index a; returns ghost values
   outside the domain. */
static double neighbour(const double* I, const int N[3], int d, int s, const int idx[3],
                        int g, int G, int A, int a, const int* bc, const double* ghost) {
    int j[3] = { idx[0], idx[1], idx[2] };
    j[d] += s;
    if (j[d] < 0 || j[d] >= N[d]) {
        int face = 2 * d + (s > 0 ? 1 : 0);
        if (bc[face] == FACE_PERIODIC) {
            j[d] = (j[d] + N[d]) % N[d];
        } else if (bc[face] == FACE_VACUUM) {
            return 0.0;
        } else {
            return ghost[face * G + g];
        }
    }
    long cell = j[0] + (long)N[0] * (j[1] + (long)N[1] * j[2]);
    return I[(cell * G + g) * (long)A + a];
}

int oracle_dense_march(int dim, const int* n_cells, const double* extent, int G, int NT, int NP,
                       const double* mu, const double* phi, const double* kappa, const double* eps,
                       const int* bc, const double* ghost, double c, double dt, double* I,
                       double* work, int n_steps, int n_threads) {
    int N[3] = { n_cells[0], dim > 1 ? n_cells[1] : 1, dim > 2 ? n_cells[2] : 1 };
    long NX = (long)N[0] * N[1] * N[2];
    int A = NT * NP;
    double lam[3];
    for (int d = 0; d < 3; ++d) lam[d] = (d < dim) ? c * dt / (extent[d] / N[d]) : 0.0;
    double* nd = (double*)malloc(sizeof(double) * 3 * A);
    if (!nd) return -1;
    for (int l = 0; l < NT; ++l)
        for (int p = 0; p < NP; ++p) direction(dim, mu[l], phi[p], nd + 3 * (l * NP + p));
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
    double* src = I;
    double* dst = work;
    for (int step = 0; step < n_steps; ++step) {
#pragma omp parallel for schedule(static)
        for (long cell = 0; cell < NX; ++cell) {
            int idx[3];
            idx[0] = (int)(cell % N[0]);
            idx[1] = (int)((cell / N[0]) % N[1]);
            idx[2] = (int)(cell / ((long)N[0] * N[1]));
            for (int g = 0; g < G; ++g) {
                double kap = kappa[cell * G + g];
                double em = eps[cell * G + g];
                double denom = 1.0 + c * dt * kap;
                for (int a = 0; a < A; ++a) {
                    double v = src[(cell * G + g) * (long)A + a];
                    double acc = v;
                    for (int d = 0; d < dim; ++d) {
                        double n = nd[3 * a + d];
                        if (n > 0.0) {
                            double up = neighbour(src, N, d, -1, idx, g, G, A, a, bc, ghost);
                            acc -= lam[d] * n * (v - up);
                        } else if (n < 0.0) {
                            double dn = neighbour(src, N, d, +1, idx, g, G, A, a, bc, ghost);
                            acc -= lam[d] * n * (dn - v);
                        }
                    }
                    dst[(cell * G + g) * (long)A + a] = (acc + c * dt * kap * em) / denom;
                }
            }
        }
        double* t = src; src = dst; dst = t;
    }
    if (src != I) memcpy(I, src, sizeof(double) * NX * G * A);
    free(nd);
    return 0;
}

/* Transport half only (no source), one step: used for the paper's step order
   where rounding happens between the transport and the source update, and
   for the Rusanov flux (flux = 1, s = S+ / c); flux = 0 is the upwind flux. */
int oracle_dense_transport(int dim, const int* n_cells, const double* extent, int G, int NT, int NP,
                           const double* mu, const double* phi, const int* bc, const double* ghost,
                           double c, double dt, const double* I, double* out, int n_threads, int flux,
                           double s_rus) {
    int N[3] = { n_cells[0], dim > 1 ? n_cells[1] : 1, dim > 2 ? n_cells[2] : 1 };
    long NX = (long)N[0] * N[1] * N[2];
    int A = NT * NP;
    double lam[3];
    for (int d = 0; d < 3; ++d) lam[d] = (d < dim) ? c * dt / (extent[d] / N[d]) : 0.0;
    double* nd = (double*)malloc(sizeof(double) * 3 * A);
    if (!nd) return -1;
    for (int l = 0; l < NT; ++l)
        for (int p = 0; p < NP; ++p) direction(dim, mu[l], phi[p], nd + 3 * (l * NP + p));
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel for schedule(static)
    for (long cell = 0; cell < NX; ++cell) {
        int idx[3];
        idx[0] = (int)(cell % N[0]);
        idx[1] = (int)((cell / N[0]) % N[1]);
        idx[2] = (int)(cell / ((long)N[0] * N[1]));
        for (int g = 0; g < G; ++g) {
            for (int a = 0; a < A; ++a) {
                double v = I[(cell * G + g) * (long)A + a];
                double acc = v;
                for (int d = 0; d < dim; ++d) {
                    double n = nd[3 * a + d];
                    if (flux == 1) {
                        double lo = neighbour(I, N, d, -1, idx, g, G, A, a, bc, ghost);
                        double hi = neighbour(I, N, d, +1, idx, g, G, A, a, bc, ghost);
                        acc -= 0.5 * lam[d] * n * (hi - lo);
                        acc += 0.5 * lam[d] * s_rus * (hi - 2.0 * v + lo);
                    } else if (n > 0.0) {
                        double up = neighbour(I, N, d, -1, idx, g, G, A, a, bc, ghost);
                        acc -= lam[d] * n * (v - up);
                    } else if (n < 0.0) {
                        double dn = neighbour(I, N, d, +1, idx, g, G, A, a, bc, ghost);
                        acc -= lam[d] * n * (dn - v);
                    }
                }
                out[(cell * G + g) * (long)A + a] = acc;
            }
        }
    }
    free(nd);
    return 0;
}

/* Total opacity of the neighbour of `cell` along axis d in direction s for
   group g, or the cell's own on a non-periodic boundary face. */
static double kappa_across(const double* kap, const int N[3], int d, int s, const int idx[3], long cell, int g,
                           int G, const int* bc) {
    int j[3] = { idx[0], idx[1], idx[2] };
    j[d] += s;
    if (j[d] < 0 || j[d] >= N[d]) {
        int face = 2 * d + (s > 0 ? 1 : 0);
        if (bc[face] != FACE_PERIODIC) return kap[cell * G + g];
        j[d] = (j[d] + N[d]) % N[d];
    }
    long nc = j[0] + (long)N[0] * (j[1] + (long)N[1] * j[2]);
    return kap[nc * G + g];
}

/* eps(tau) = (1 - exp(-tau)) / tau, 1 at tau = 0 */
static double hll_eps(double tau) { return tau > 0.0 ? -expm1(-tau) / tau : 1.0; }

/* Transport half with the HLL flux, one step (no source).  kap: total
   opacity per (cell, group) row; beta: the optical-depth factor. */
int oracle_dense_transport_hll(int dim, const int* n_cells, const double* extent, int G, int NT, int NP,
                               const double* mu, const double* phi, const int* bc, const double* ghost, double c,
                               double dt, const double* I, double* out, int n_threads, const double* kap,
                               double beta) {
    int N[3] = { n_cells[0], dim > 1 ? n_cells[1] : 1, dim > 2 ? n_cells[2] : 1 };
    long NX = (long)N[0] * N[1] * N[2];
    int A = NT * NP;
    double lam[3], dx[3];
    for (int d = 0; d < 3; ++d) {
        dx[d] = (d < dim) ? extent[d] / N[d] : 1.0;
        lam[d] = (d < dim) ? c * dt / dx[d] : 0.0;
    }
    double* nd = (double*)malloc(sizeof(double) * 3 * A);
    if (!nd) return -1;
    for (int l = 0; l < NT; ++l)
        for (int p = 0; p < NP; ++p) direction(dim, mu[l], phi[p], nd + 3 * (l * NP + p));
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel for schedule(static)
    for (long cell = 0; cell < NX; ++cell) {
        int idx[3];
        idx[0] = (int)(cell % N[0]);
        idx[1] = (int)((cell / N[0]) % N[1]);
        idx[2] = (int)(cell / ((long)N[0] * N[1]));
        for (int g = 0; g < G; ++g) {
            double epsL[3], epsR[3];
            const double k0 = kap[cell * G + g];
            for (int d = 0; d < dim; ++d) {
                epsL[d] = hll_eps(beta * dx[d] * 0.5 * (k0 + kappa_across(kap, N, d, -1, idx, cell, g, G, bc)));
                epsR[d] = hll_eps(beta * dx[d] * 0.5 * (k0 + kappa_across(kap, N, d, +1, idx, cell, g, G, bc)));
            }
            for (int a = 0; a < A; ++a) {
                double v = I[(cell * G + g) * (long)A + a];
                double acc = v;
                for (int d = 0; d < dim; ++d) {
                    const double n = nd[3 * a + d], an = fabs(n);
                    const double lo = neighbour(I, N, d, -1, idx, g, G, A, a, bc, ghost);
                    const double hi = neighbour(I, N, d, +1, idx, g, G, A, a, bc, ghost);
                    /* lambda (F_{+1/2} - F_{-1/2}) / c */
                    const double fr = 0.5 * n * (v + hi) - 0.5 * an * epsR[d] * (hi - v);
                    const double fl = 0.5 * n * (lo + v) - 0.5 * an * epsL[d] * (v - lo);
                    acc -= lam[d] * (fr - fl);
                }
                out[(cell * G + g) * (long)A + a] = acc;
            }
        }
    }
    free(nd);
    return 0;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
