// Host runtime and C ABI of the TT multigroup transport library (gfx950).
//
// One rounding pass (a "round") over the pending operator runs these kernels
// on the caller's stream, with every rank decided on the device:
//   k_prep         right-to-left QR of the small cores of the TT sum; builds
//                  the gather operand G = fold(L_Theta)            (1 block)
//   k_gather_gemm  B = Z_new L_Theta without forming Z_new           (project)
//   k_tsqr x L     Householder TSQR of B -> R_B   (or k_gram + k_sum_parts)
//   k_svd_chain    SVD of R_B, truncation of both bonds, new Theta/Phi (1 block)
//   k_gather_gemm  Z_out = B V_r                                     (output)
//   k_commit       new ranks become current
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <type_traits>
#include <string>
#include <vector>

#include "../../include/tt_transport.h"
#include "k_bf16x.hpp"
#include "k_big.hpp"
#include "k_fused.hpp"
#include "k_f64.hpp"
#include "k_batch.hpp"
#include "k_gram.hpp"
#include "k_mfma.hpp"
#include "k_couple.hpp"
#include "k_diag.hpp"
#include "k_small.hpp"
#include "k_rand.hpp"
#include "planck.hpp"
#include "tt_common.hpp"

using namespace ttrt;

namespace {

thread_local std::string g_err;

tt_status fail(tt_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) return fail(TT_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

enum KClass {
    KC_PREP = 0, KC_PROJECT = 1, KC_FACTOR = 2, KC_TREE = 3, KC_SVD = 4, KC_OUTPUT = 5, KC_DIAG = 6, KC_COUPLE = 7,
    KC_ANGLE = 8, KC_STENCIL = 9, KC_COUNT = 10
};

// Largest grid the launch-shape tuner tries for the persistent contraction
// kernels (four blocks per CU); the partial buffers are sized for it.
constexpr int kTuneMaxBlocks = 1024;

// Rows per thread in the 128-column TSQR leaf (chunks of 4 x this many rows):
// longer chunks mean fewer column steps per block over the tall first core,
// and 24 still fits two blocks per CU (122 VGPRs; 32 takes 154, one block).
constexpr int kTsqrBrLeaf128 = 24;
// and in the 64-column leaf (chunks of 8 x this many rows)
constexpr int kTsqrBrLeaf64 = 24;
// Rows per thread in the 64-column tree levels (1024 threads, blocks of 16 x
// this many rows): 320-row blocks reduce five R factors each, so plane2d
// takes four tree levels of 73 us instead of five of 66 us with 16 rows (24
// rows: four of 80 us)
constexpr int kTsqrBrTree64 = 20;
// Tree levels of the 64- and 128-column tiles have few blocks, each one chain
// of column steps: they take 1024 threads (16 and 8 row groups) of 20 and 16
// rows, so a column step is short (plane2d: 83 -> 66 us per level against 512
// threads of 32 rows); the 16-column tile takes 512 threads of 16 rows.
// Leaf blocks of the TSQR at most: two resident blocks per CU on 256 CUs,
// so the whole first core is one wave of blocks and the tree starts from as
// few R factors as that allows.
constexpr int kTsqrMaxLeaves = 512;

struct Plan {
    int dim = 1, nx = 1, ny = 1, nz = 1;
    long long NX = 0, M = 0;
    int G = 0, nt = 0, np = 0;
    int n_terms = 0, n_bc = 0, cap = 1;
    int r1cap = 1, r2cap = 1, R1cap = 1, R2cap = 1, k1cap = 1, k2cap = 1, ldzcap = 8, ldbcap = 8;
    int n_gather_max = 1, n_r1_max = 1;
    int KP = 64, chunk = 128;      // rows per chunk of a TSQR leaf block
    int chunk_t = 128;              // and of a tree-level block
    int KPt = 64;                   // column tile of the TSQR (16 for QR-route cores of k1cap <= 16)
    std::vector<int> levP;          // blocks per TSQR level
    std::vector<long long> levRows; // rows per block per level
    std::vector<long long> levN;    // rows of the level input
    int Pg = 1;                     // blocks (row ranges, one partial each) of the first core's Gram
    long long rowsg = 0;            // rows per Gram block
    int Pg_max = 1;
    bool svd_fast = false;          // all SVD-chain matrices fit the LDS layout
    size_t elem = 8;                // bytes per stored element of Z / B
    // fused FP32 Gram path: projection + FP64 Gram in one kernel, output
    // contraction from Z with V_r folded into the operand (B never stored)
    bool fused = false;
    int nct_p = 4, nct_o = 2;       // 16-column MFMA tiles of B / of Z_out
    int fused_T = 1;                // K groups of 16 at the rank caps
    int fused_blocks = 1;           // blocks of the projection + Gram kernel (one partial each)
    int fused_blocks_o = 1;         // blocks of the output kernel
    int fused_blocks_max = 1;       // largest grid of either (the partial buffer's size)
    long long fused_tiles = 0;      // 32-row tiles
    size_t lds_p = 0, lds_o = 0;
    size_t B_bytes = 0;
    // workspace layout (byte offsets)
    size_t o_Gsw = 0, o_Gfold = 0, o_GP = 0, o_aux = 0, o_R1 = 0, o_R2 = 0, o_zero = 0, o_nbr = 0;
    // split-BF16 operands (precision TT_PREC_BF16X): chunked, column-major hi / lo
    bool bf16x = false;
    int nct_b = 4, nct_bo = 2, kc_g = 1, kc_v = 1;
    size_t o_Gh = 0, o_Gl = 0, o_Vh = 0, o_Vl = 0;
    int rw1 = 0, rw2 = 0;           // widths of the rank-1 row blocks (transport / source operators)
    bool fused_overflow = false;
    // randomized rounding (TT_ROUND_RAND): sketch buffers
    bool rand = false;
    size_t o_rG = 0, o_rQTh = 0, o_rQPh = 0, o_rP = 0, o_rVeff = 0, o_rw = 0;
    bool row_tables = false;        // per-row d, neighbour and rank-1 tables (fused and split-BF16 paths)
    // FP64 data: projection and output contractions on FP64 MFMA (k_mm_f64)
    bool f64mm = false;
    int nct_f = 1, nct_fo = 1;      // 16-column tiles of B / of Z_out
    int f64_blocks = 1;             // blocks of the persistent projection kernel (one Gram partial each when fused)
    int f64_blocks_o = 1;           // blocks of the persistent output kernel
    int f64_blocks_max = 1;         // largest grid of either
    // direction-space projection (Y = Z W, then the operator's stencil on Y)
    // for 128-column FP64 cores once both small-core factors are square
    bool stencil = false;
    bool stencil32 = false;         // ... on FP32 data (FP32 MFMA Y = Z W, FP32 Y and B)
    int st_blocks = 1;              // blocks of the stencil kernel
    size_t o_Y = 0, o_Wst = 0, o_Cst = 0, o_WstF = 0;
    size_t o_state, o_Z0, o_Z1, o_B, o_Th0, o_Th1, o_Ph0, o_Ph1, o_LTh, o_QTh, o_QPh, o_G, o_V, o_RA, o_RB, o_small,
        o_k0, o_ks, o_kfull = 0, o_eps, o_ghost, o_gtab, o_htab, o_ThN, o_PhN, o_sv, o_colsum;
    size_t small_bytes = 0, n_parts_max = 1;
    // coupled medium temperature (heat_capacity > 0)
    bool coupled = false;
    bool kfull = false;   // opacity given per (cell, group) row
    bool kscat = false;   // isotropic scattering opacity given
    bool prepass = false; // the source column depends on the state (coupled T or scattering)
    int flux = 0;         // 0 upwind, 1 Rusanov
    double rus_s = 1.0;   // Rusanov S+ / c
    size_t o_T = 0, o_T0 = 0, o_Js = 0, o_edges = 0, o_wth = 0, o_wph = 0, o_kscat = 0, o_jn = 0;
    size_t k1sq = 1;                // k1cap x (k1cap | 1): SVD-chain matrices outside LDS
    size_t o_desc = 0;
    // A2 scratch (doubles): the operand of the second-bond QR, the first-bond
    // matrix T outside LDS, or the second-bond Gram matrix
    size_t a2n() const {
        const size_t m2 = (size_t)nt * k2cap;
        return std::max(std::max(m2 * R1cap, k1sq), (size_t)k2cap * (size_t)(k2cap | 1));
    }
    size_t bytes = 0;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool is_inflow(int kind) { return kind == TT_BC_INFLOW_PLANCK || kind == TT_BC_INFLOW_VALUES; }

tt_status validate(const tt_problem* p) {
    if (!p) return fail(TT_ERR_INVALID_ARG, "problem is NULL");
    if (p->dim < 1 || p->dim > 3) return fail(TT_ERR_INVALID_ARG, "dim must be 1, 2 or 3");
    for (int d = 0; d < p->dim; ++d) {
        if (p->n_cells[d] < 1) return fail(TT_ERR_INVALID_ARG, "n_cells must be >= 1");
        if (!(p->extent[d] > 0.0)) return fail(TT_ERR_INVALID_ARG, "extent must be > 0");
    }
    if (p->n_groups < 1 || !p->group_edges) return fail(TT_ERR_INVALID_ARG, "need n_groups >= 1 and group_edges");
    if (!(p->group_edges[0] >= 0.0)) return fail(TT_ERR_INVALID_ARG, "group_edges[0] must be >= 0");
    for (int g = 0; g < p->n_groups; ++g)
        if (!(p->group_edges[g + 1] > p->group_edges[g])) return fail(TT_ERR_INVALID_ARG, "group edges must increase");
    if (!p->T_cell) return fail(TT_ERR_INVALID_ARG, "T_cell is required");
    if (!p->kappa_full && (!p->kappa0 || !p->kappa_group_scale))
        return fail(TT_ERR_INVALID_ARG, "kappa_full, or kappa0 and kappa_group_scale, are required");
    if (p->n_theta < 1 || !p->mu || !p->w_theta) return fail(TT_ERR_INVALID_ARG, "need n_theta >= 1, mu and w_theta");
    if (p->n_phi < 1 || !p->w_phi) return fail(TT_ERR_INVALID_ARG, "need n_phi >= 1 and w_phi");
    if (p->dim == 1 && p->n_phi != 1) return fail(TT_ERR_INVALID_ARG, "dim == 1 requires n_phi == 1");
    if (p->dim > 1 && !p->phi) return fail(TT_ERR_INVALID_ARG, "phi is required for dim > 1");
    for (int l = 0; l < p->n_theta; ++l)
        if (!(p->mu[l] >= -1.0 && p->mu[l] <= 1.0)) return fail(TT_ERR_INVALID_ARG, "mu must lie in [-1, 1]");
    for (int f = 0; f < 6; ++f) {
        if (p->bc[f] < 0 || p->bc[f] > 3) return fail(TT_ERR_INVALID_ARG, "unknown boundary kind");
        if (f < 2 * p->dim && p->bc[f] == TT_BC_INFLOW_VALUES && !p->bc_values)
            return fail(TT_ERR_INVALID_ARG, "TT_BC_INFLOW_VALUES needs bc_values");
        if (f < 2 * p->dim && p->bc[f] == TT_BC_INFLOW_PLANCK && !(p->bc_T[f] >= 0.0))
            return fail(TT_ERR_INVALID_ARG, "bc_T must be >= 0");
    }
    for (int d = 0; d < p->dim; ++d)
        if ((p->bc[2 * d] == TT_BC_PERIODIC) != (p->bc[2 * d + 1] == TT_BC_PERIODIC))
            return fail(TT_ERR_INVALID_ARG, "periodic boundaries must be set on both faces of an axis");
    if (!(p->c > 0.0) || !(p->cfl > 0.0)) return fail(TT_ERR_INVALID_ARG, "c and cfl must be > 0");
    if (!(p->tol >= 0.0)) return fail(TT_ERR_INVALID_ARG, "tol must be >= 0");
    if (p->rank_cap < 1) return fail(TT_ERR_INVALID_ARG, "rank_cap must be >= 1");
    if (p->precision < 0 || p->precision > 2) return fail(TT_ERR_INVALID_ARG, "unknown precision");
    if (p->round_method < 0 || p->round_method > 3) return fail(TT_ERR_INVALID_ARG, "unknown round_method");
    if (p->round_method == TT_ROUND_RAND && (p->rand_oversample < 1 || p->rand_oversample > 128))
        return fail(TT_ERR_INVALID_ARG, "rand_oversample must lie in [1, 128] for randomized rounding");
    if (p->paper_step_order < 0 || p->paper_step_order > 1) return fail(TT_ERR_INVALID_ARG, "paper_step_order must be 0 or 1");
    if (!(p->heat_capacity >= 0.0) || !std::isfinite(p->heat_capacity))
        return fail(TT_ERR_INVALID_ARG, "heat_capacity must be finite and >= 0");
    if (p->flux != TT_FLUX_UPWIND && p->flux != TT_FLUX_RUSANOV && p->flux != TT_FLUX_HLL)
        return fail(TT_ERR_INVALID_ARG, "unknown flux");
    if (p->flux == TT_FLUX_HLL) {
        if (!(p->hll_beta > 0.0) || !std::isfinite(p->hll_beta))
            return fail(TT_ERR_INVALID_ARG, "hll_beta must be finite and > 0");
        if (p->precision != TT_PREC_FP64)
            return fail(TT_ERR_INVALID_ARG, "the HLL flux needs FP64 data (TT_PREC_FP64)");
        if (p->kappa_s_full || p->heat_capacity > 0.0)
            return fail(TT_ERR_INVALID_ARG, "the HLL flux is provided without scattering or a coupled temperature");
    }
    if (p->flux == TT_FLUX_RUSANOV && !(p->rusanov_s >= 0.0 && p->rusanov_s <= 1.0))
        return fail(TT_ERR_INVALID_ARG, "rusanov_s must lie in [0, 1]");
    return TT_OK;
}

tt_status make_plan_impl(const tt_problem* p, Plan& P, bool allow_fused) {
    tt_status s = validate(p);
    if (s != TT_OK) return s;
    P.dim = p->dim;
    P.nx = p->n_cells[0];
    P.ny = p->dim > 1 ? p->n_cells[1] : 1;
    P.nz = p->dim > 2 ? p->n_cells[2] : 1;
    P.NX = (long long)P.nx * P.ny * P.nz;
    P.G = p->n_groups;
    P.M = P.NX * P.G;
    P.nt = p->n_theta;
    P.np = p->n_phi;
    P.n_terms = 2 * p->dim;
    P.flux = p->flux;
    P.rus_s = p->flux == TT_FLUX_RUSANOV ? p->rusanov_s : 0.0;
    // inflow columns: one per inflow face; the Rusanov dissipation adds a second
    const int per_face = ((P.flux == TT_FLUX_RUSANOV && P.rus_s != 0.0) || P.flux == TT_FLUX_HLL) ? 2 : 1;
    P.n_bc = 0;
    for (int f = 0; f < 2 * p->dim; ++f) P.n_bc += is_inflow(p->bc[f]) ? per_face : 0;
    P.cap = p->rank_cap;
    const long long full1 = std::min<long long>(P.M, (long long)P.nt * P.np);
    P.r1cap = (int)std::min<long long>(P.cap, full1);
    P.r2cap = std::min(P.cap, P.np);
    const int nrb = 1 + P.n_terms;
    P.n_r1_max = P.n_bc + 1;
    // HLL: one gather block per (term, shift): the centre and both neighbours
    P.n_gather_max = P.flux == TT_FLUX_HLL ? 1 + 3 * P.n_terms : 1 + P.n_terms;
    P.R1cap = nrb * P.r1cap + P.n_r1_max;
    P.R2cap = nrb * P.r2cap + P.n_r1_max;
    P.k2cap = std::min(P.R2cap, P.np);
    P.k1cap = std::min(P.R1cap, P.nt * P.k2cap);
    P.ldzcap = ld_for_rank(P.r1cap);
    P.ldbcap = ld_for_rank(P.k1cap);
    if (P.k1cap > 128) return fail(TT_ERR_INVALID_ARG, "projected first-core rank above 128 is not supported");
    P.KP = P.k1cap <= 64 ? 64 : 128;
    {
        // fixed LDS layout of the SVD chain: 64 x 64 matrices (ld 65) and a
        // bond-2 matrix of at most 256 rows x 16 columns
        const size_t reg0 = std::max<size_t>(64 * 65, 257 * 16);
        const size_t need = reg0 + 2 * 64 * 65 + 2 * 64 + (size_t)P.k2cap * P.k2cap + P.k2cap;
        // the fixed layout pays for 64 columns whatever k1 is: for k1 <= 32 the
        // Gram route's two-sided Jacobi is faster on the actual order (1D FP32,
        // k1 = 16: 11.1 -> 6.6 ms per 64 steps); the QR route's fixed one-sided
        // Jacobi stays faster there (30 against 41 ms for the 1D slab)
        const bool gram_route = p->round_method == TT_ROUND_GRAM || p->round_method == TT_ROUND_RAND ||
                                (p->round_method == TT_ROUND_AUTO && p->precision != TT_PREC_FP64);
        P.svd_fast = P.k1cap <= 64 && !(gram_route && P.k1cap <= 32) && (long long)P.r1cap * P.nt <= 256 &&
                     P.k2cap <= 16 && need * sizeof(double) <= (size_t)kSmallLdsBytes;
    }
    // TSQR tile: a QR-route core of at most 16 columns uses a 16-column tile
    // with 32 row groups (512-row chunks: the 1D slab's core is one chunk)
    {
        const int method_q = p->round_method == TT_ROUND_AUTO
                                 ? (p->precision == TT_PREC_FP64 ? TT_ROUND_QR : TT_ROUND_GRAM)
                                 : p->round_method;
        P.KPt = (method_q == TT_ROUND_QR && P.k1cap <= 16) ? 16 : P.KP;
    }
    P.chunk = P.KPt == 16 ? 32 * 16 : (P.KP == 64 ? 8 * kTsqrBrLeaf64 : 4 * kTsqrBrLeaf128);
    P.chunk_t = P.KPt == 16 ? 32 * 16 : (P.KP == 64 ? 16 * kTsqrBrTree64 : 8 * 16);
    P.elem = p->precision == TT_PREC_FP64 ? 8 : 4;
    {
        const int method = p->round_method == TT_ROUND_AUTO
                               ? (p->precision == TT_PREC_FP64 ? TT_ROUND_QR : TT_ROUND_GRAM)
                               : p->round_method;
        P.fused_T = (P.n_gather_max * P.ldzcap + P.n_r1_max + 15) / 16;
        P.nct_p = P.ldbcap <= 32 ? 2 : 4;
        P.nct_o = P.ldzcap <= 32 ? 2 : 4;
        P.lds_p = fused_lds_bytes(P.nct_p, true, P.fused_T);
        P.lds_o = fused_lds_bytes(P.nct_o, false, P.fused_T);
        P.rand = method == TT_ROUND_RAND;
        P.fused = allow_fused && p->precision == TT_PREC_FP32 && (method == TT_ROUND_GRAM || P.rand) && P.k1cap <= 64 &&
                  P.ldzcap <= 64 &&
                  (long long)(P.M + 64) * P.ldzcap < (1LL << 31) && std::max(P.lds_p, P.lds_o) <= 160 * 1024;
        P.fused_tiles = (P.M + 31) / 32;
        const long long want = (P.fused_tiles + kFusedWaves - 1) / kFusedWaves;
        P.fused_blocks = (int)std::max<long long>(1, std::min<long long>(256, want));
        if (P.fused_blocks > 8) P.fused_blocks = P.fused_blocks / 8 * 8;
        P.fused_blocks_o = (int)std::max<long long>(1, std::min<long long>(512, want));
        if (P.fused_blocks_o > 8) P.fused_blocks_o = P.fused_blocks_o / 8 * 8;
        P.fused_blocks_max = std::max(P.fused_blocks, P.fused_blocks_o);
    }
    // FP64 MFMA contractions: B up to 128 columns, Z_out up to 64
    {
        auto nct_for = [](int ld) { return ld <= 16 ? 1 : (ld <= 32 ? 2 : (ld <= 64 ? 4 : 8)); };
        P.f64mm = p->precision == TT_PREC_FP64 && P.ldbcap <= 128 && P.ldzcap <= 64 && P.M < (1LL << 31);
        P.nct_f = nct_for(P.ldbcap);
        P.nct_fo = nct_for(P.ldzcap);
        const long long nrb = (P.M + kF64Rows - 1) / kF64Rows;
        P.f64_blocks = (int)std::max<long long>(1, std::min<long long>(256, nrb));
        if (P.f64_blocks > 8) P.f64_blocks = P.f64_blocks / 8 * 8;
        P.f64_blocks_o = P.f64_blocks;
        P.stencil = P.f64mm && P.nct_f == 8;
        // FP32 data with a stored B of more than 64 columns: the same pass
        P.stencil32 = p->precision == TT_PREC_FP32 && !P.fused && P.ldbcap > 64 && P.ldbcap <= 128 &&
                      P.M < (1LL << 31);
        P.stencil = P.stencil || P.stencil32;
        P.st_blocks = (int)std::max<long long>(1, std::min<long long>(256, (P.M + kStRows - 1) / kStRows / kStWaves));
        if (P.st_blocks > 8) P.st_blocks = P.st_blocks / 8 * 8;
        // launch-shape tuning may take up to four blocks per CU
        P.f64_blocks_max = (int)std::max<long long>(1, std::min<long long>(kTuneMaxBlocks, nrb));
        if (P.f64_blocks_max > 8) P.f64_blocks_max = P.f64_blocks_max / 8 * 8;
    }
    // TSQR levels
    {
        long long n = P.M;
        // four chunks per leaf block, more once the blocks would exceed the
        // cap; a small core (fewer than four such blocks) gets one chunk per
        // block, and its tree stays short
        long long want = (n + 4 * P.chunk - 1) / (4 * P.chunk);
        if (want < 4) want = (n + P.chunk - 1) / P.chunk;
        int P1 = (int)std::min<long long>(kTsqrMaxLeaves, std::max<long long>(1, want));
        long long rows = (n + P1 - 1) / P1;
        rows = (rows + P.chunk - 1) / P.chunk * P.chunk;
        P1 = (int)((n + rows - 1) / rows);
        P.levP.push_back(P1); P.levRows.push_back(rows); P.levN.push_back(n);
        int prev = P1;
        while (prev > 1) {
            // only the first k1 <= k1cap rows of each R factor can be non-zero
            long long nn = (long long)prev * P.k1cap;
            // one chunk per block (at least two factors): the levels have
            // few blocks, so the chain of column steps per block is the time
            long long rr = std::max<long long>(P.chunk_t, 2LL * P.k1cap);
            rr = (rr + P.chunk_t - 1) / P.chunk_t * P.chunk_t;
            int Pn = (int)((nn + rr - 1) / rr);
            P.levP.push_back(Pn); P.levRows.push_back(rr); P.levN.push_back(nn);
            prev = Pn;
        }
        P.n_parts_max = (size_t)P.levP[0];
    }
    {
        long long rows = std::max<long long>(64, (P.M + 1023) / 1024);
        rows = (rows + 15) / 16 * 16;
        P.Pg = (int)((P.M + rows - 1) / rows);
        P.rowsg = rows;
        P.Pg_max = P.Pg;   // the most partials any Gram row split may take
        P.n_parts_max = std::max<size_t>(P.n_parts_max, (size_t)P.Pg);
        P.n_parts_max = std::max<size_t>(P.n_parts_max, (size_t)(P.f64mm ? P.f64_blocks_max : P.f64_blocks));
    }
    // layout
    size_t off = 0;
    auto take = [&](size_t b) { size_t o = off; off = align256(off + std::max<size_t>(b, 8)); return o; };
    const size_t d = sizeof(double);
    P.o_state = take(sizeof(DevState));
    P.o_Z0 = take((size_t)P.M * P.ldzcap * P.elem);
    P.o_Z1 = take((size_t)P.M * P.ldzcap * P.elem);
    P.B_bytes = (size_t)P.M * P.ldbcap * P.elem;
    if (P.fused)   // B is not stored; keep a staging buffer for explicit TT-sum reads
        P.B_bytes = std::min<size_t>(P.B_bytes, std::max<size_t>((size_t)16 << 20, (size_t)P.R1cap * sizeof(double)));
    P.o_B = take(P.B_bytes);
    if (P.stencil) {
        P.o_Y = take((size_t)P.M * (P.ldbcap + (P.stencil32 ? kYPadF : kYPad)) * P.elem);
        P.o_Wst = take((size_t)P.ldzcap * P.ldbcap * sizeof(double));
        P.o_Cst = take((size_t)(kStNG + kStZ) * P.ldbcap * sizeof(double));
        if (P.stencil32) P.o_WstF = take((size_t)P.ldzcap * P.ldbcap * sizeof(float));
    }
    P.bf16x = p->precision == TT_PREC_BF16X;
    if (P.bf16x && P.M >= (1LL << 31))
        return fail(TT_ERR_INVALID_ARG, "split-BF16 contractions need fewer than 2^31 rows of Z");
    if (P.bf16x) {
        P.nct_b = P.ldbcap <= 64 ? 4 : 8;
        P.nct_bo = P.ldzcap <= 32 ? 2 : 4;
        P.kc_g = (P.n_gather_max * P.ldzcap + P.n_r1_max + kBxKC - 1) / kBxKC;
        P.kc_v = (P.ldbcap + kBxKC - 1) / kBxKC;
        const size_t gb = (size_t)P.kc_g * 16 * P.nct_b * kBxKC * 2, vb = (size_t)P.kc_v * 16 * P.nct_bo * kBxKC * 2;
        P.o_Gh = take(gb);
        P.o_Gl = take(gb);
        P.o_Vh = take(vb);
        P.o_Vl = take(vb);
    }
    if (P.fused) {
        P.o_Gsw = take((size_t)P.fused_T * P.nct_p * 256 * sizeof(float));
        P.o_Gfold = take((size_t)P.fused_T * P.nct_o * 256 * sizeof(float));
        P.o_GP = take((size_t)P.fused_blocks_max * gram_blocks(P.nct_p) * 256 * d);
    }
    if (P.rand) {
        P.o_rG = take((size_t)P.KP * P.KP * d);
        P.o_rQTh = take((size_t)P.k1cap * P.nt * P.k2cap * d);
        P.o_rQPh = take((size_t)P.k2cap * P.np * d);
        P.o_rP = take((size_t)P.k1cap * P.k1cap * d);
        P.o_rVeff = take((size_t)P.k1cap * P.k1cap * d);
        P.o_rw = take(rand_work_doubles(P.k1cap, P.nt, P.np, P.k2cap) * d);
    }
    P.row_tables = P.fused || P.bf16x;
    if (P.row_tables) {
        P.o_aux = take((size_t)P.M * sizeof(float2));
        // rank-1 columns as dense row blocks: the full (or transport) operator, and
        // the source operator when the paper's step order is used
        const int nr1_t = p->paper_step_order ? P.n_bc : P.n_bc + 1;
        P.rw1 = nr1_t > 0 ? round_up(nr1_t, 4) : 0;
        P.rw2 = p->paper_step_order ? 4 : 0;
        P.o_R1 = take((size_t)P.M * std::max(P.rw1, 1) * sizeof(float));
        P.o_R2 = take((size_t)P.M * std::max(P.rw2, 1) * sizeof(float));
        P.o_zero = take(1024);   // zero region for loads with nothing to read
        P.o_nbr = take((size_t)P.M * P.n_terms * sizeof(int));
    }
    P.o_Th0 = take((size_t)P.r1cap * P.nt * P.r2cap * d);
    P.o_Th1 = take((size_t)P.r1cap * P.nt * P.r2cap * d);
    P.o_Ph0 = take((size_t)P.r2cap * P.np * d);
    P.o_Ph1 = take((size_t)P.r2cap * P.np * d);
    P.o_LTh = take((size_t)P.R1cap * P.k1cap * d);
    P.o_QTh = take((size_t)P.k1cap * P.nt * P.k2cap * d);
    P.o_QPh = take((size_t)P.k2cap * P.np * d);
    P.o_G = take((size_t)(P.n_gather_max * P.ldzcap + P.n_r1_max) * P.ldbcap * P.elem);
    P.o_V = take((size_t)P.ldbcap * P.ldzcap * P.elem);
    P.o_RA = take(P.n_parts_max * P.KP * P.KP * d);
    P.o_RB = take(P.n_parts_max * P.KP * P.KP * d);
    // small scratch: A1, Q1, A2, Q2, tau, J, Th2, C2, V2, sv, perm, flag
    const size_t m2 = (size_t)P.nt * P.k2cap;
    P.small_bytes = 0;
    P.small_bytes += align256((size_t)P.np * P.R2cap * d);
    P.small_bytes += align256(((size_t)P.np * P.np + (size_t)P.R2cap * P.k2cap) * d);
    // matrices of the SVD chain outside LDS use an odd leading dimension (k1 | 1)
    P.k1sq = (size_t)P.k1cap * (size_t)(P.k1cap | 1);
    P.small_bytes += align256(P.a2n() * d);
    P.small_bytes += align256(m2 * P.k1cap * d);
    P.small_bytes += align256((size_t)std::max(P.R1cap, P.R2cap) * d);
    P.small_bytes += align256(P.k1sq * d);
    P.small_bytes += align256((size_t)P.r1cap * m2 * d);
    P.small_bytes += align256((size_t)P.r1cap * P.nt * P.k2cap * d);
    P.small_bytes += align256((size_t)P.k2cap * P.k2cap * d);
    P.small_bytes += align256((size_t)(3 * P.k1cap + P.k2cap) * d);
    P.small_bytes += align256((size_t)(P.k1cap + P.k2cap) * sizeof(int));
    P.small_bytes += align256(sizeof(int));
    P.small_bytes += align256(P.k1sq * d);
    P.small_bytes += align256((size_t)P.k1cap * P.k1cap * d);
    P.o_small = take(P.small_bytes);
    P.o_k0 = take((size_t)P.NX * d);
    P.o_ks = take((size_t)P.G * d);
    P.kfull = p->kappa_full != nullptr;
    if (P.kfull) P.o_kfull = take((size_t)P.M * d);
    P.o_eps = take((size_t)P.M * d);
    P.o_ghost = take((size_t)6 * P.G * d);
    P.o_gtab = take((size_t)(1 + P.n_terms) * P.nt * d);
    P.o_htab = take((size_t)(1 + P.n_terms) * P.np * d);
    P.o_ThN = take((size_t)P.R1cap * P.nt * P.R2cap * d);
    P.o_PhN = take((size_t)P.R2cap * P.np * d);
    P.o_sv = take((size_t)(P.k1cap + P.k2cap) * d);
    P.o_colsum = take((size_t)256 * 128 * d);
    P.o_desc = take(sizeof(SmallSolve));   // descriptor of the persistent small-solve kernel
    P.coupled = p->heat_capacity > 0.0;
    P.kscat = p->kappa_s_full != nullptr;
    P.prepass = P.coupled || P.kscat;
    if (P.coupled) {
        // coupled medium temperature: T and its initial value
        P.o_T = take((size_t)P.NX * d);
        P.o_T0 = take((size_t)P.NX * d);
    }
    if (P.kscat) {
        // scattering opacity and J^{m+1} per row
        P.o_kscat = take((size_t)P.M * d);
        P.o_jn = take((size_t)P.M * d);
    }
    if (P.prepass) {
        // source pre-pass: J* per row, group edges and quadrature weights
        P.o_Js = take((size_t)P.M * d);
        P.o_edges = take((size_t)(P.G + 1) * d);
        P.o_wth = take((size_t)P.nt * d);
        P.o_wph = take((size_t)P.np * d);
    }
    P.bytes = off;
    if (P.flux == TT_FLUX_HLL && !P.f64mm)
        return fail(TT_ERR_INVALID_ARG, "the HLL flux needs the FP64 MFMA contractions (projected rank <= 128, rank cap <= 64)");
    // element offsets of the rank-1 blocks from Z must fit 32 bits
    // the fused kernels address Z, the rank-1 blocks and the zero region with
    // 32-bit byte offsets from the current Z
    P.fused_overflow = P.fused && (long long)(P.o_zero - P.o_Z0) + 1024 >= (1LL << 32);
    return TT_OK;
}

tt_status make_plan(const tt_problem* p, Plan& P) {
    tt_status s = make_plan_impl(p, P, true);
    if (s == TT_OK && P.fused_overflow) {
        P = Plan();
        s = make_plan_impl(p, P, false);
    }
    return s;
}

}  // namespace

struct tt_handle {
    Plan P;
    int noalloc_dev = -1;             // device whose static workspace this handle holds (-1: caller's workspace)
    Geom geom{};
    int precision = 0, round_method = 0, step_order = 0;
    int rand_p = 4;                   // randomized rounding: sketch ranks = ranks + rand_p
    unsigned long long rand_seed = 0; // and the key of its counter-based generator
    double tol = 0.0;
    double dt = 0.0;
    double dV = 1.0;
    char* ws = nullptr;
    hipStream_t create_stream = nullptr;
    int zcur = 0, ccur = 0;
    int pending = OP_NONE;
    OpDesc ops[4];
    std::vector<double> w_theta, w_phi;
    std::vector<double> eps_host;    // emission at the medium temperature (row order)
    std::vector<double> init_host;   // initial first core: emission at the initial radiation temperature
    std::vector<double> T_host;      // medium temperature as given (fixed unless coupled)
    double heat_capacity = 0.0, c = 1.0;
    int qe_full = -1, qe_source = -1;   // emission columns of the full and source operators
    // timing
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
    std::vector<int> ev_class;
    size_t ev_used = 0;
    double kernel_ms[KC_COUNT] = {0};
    long long kernel_launches[KC_COUNT] = {0};
    double flops[KC_COUNT] = {0};
    double last_seconds = 0.0;
    int last_steps = 0;
    // hipGraph replay of the step sequence (tt_transport_set_graph): two steps
    // per graph, so the ping-pong buffers are back at the captured parity; one
    // graph per parity of the current buffers
    bool use_graph = false;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t graph_exec[2] = {nullptr, nullptr};

    template <typename T>
    T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
    DevState* st() const { return at<DevState>(P.o_state); }
    void* Zc() const { return ws + (zcur ? P.o_Z1 : P.o_Z0); }
    void* Zn() const { return ws + (zcur ? P.o_Z0 : P.o_Z1); }
    double* Thc() const { return at<double>(ccur ? P.o_Th1 : P.o_Th0); }
    double* Thn() const { return at<double>(ccur ? P.o_Th0 : P.o_Th1); }
    double* Phc() const { return at<double>(ccur ? P.o_Ph1 : P.o_Ph0); }
    double* Phn() const { return at<double>(ccur ? P.o_Ph0 : P.o_Ph1); }
    RowData rowdata() const {
        return RowData{at<double>(P.o_k0), at<double>(P.o_ks), at<double>(P.o_eps), at<double>(P.o_ghost),
                       P.kfull ? at<double>(P.o_kfull) : nullptr, P.kscat ? at<double>(P.o_kscat) : nullptr,
                       P.kscat ? at<double>(P.o_jn) : nullptr};
    }
    RandBufs rand_bufs() {
        return RandBufs{at<double>(P.o_rG), at<double>(P.o_rQTh), at<double>(P.o_rQPh), at<double>(P.o_rP),
                        at<double>(P.o_rVeff), at<double>(P.o_rw)};
    }
    SmallScratch scratch() const {
        SmallScratch s;
        char* b = ws + P.o_small;
        const size_t d = sizeof(double);
        const size_t m2 = (size_t)P.nt * P.k2cap;
        s.A1 = (double*)b; b += align256((size_t)P.np * P.R2cap * d);
        s.Q1 = (double*)b; b += align256(((size_t)P.np * P.np + (size_t)P.R2cap * P.k2cap) * d);
        s.A2 = (double*)b; b += align256(P.a2n() * d);
        s.Q2 = (double*)b; b += align256(m2 * P.k1cap * d);
        s.tau = (double*)b; b += align256((size_t)std::max(P.R1cap, P.R2cap) * d);
        s.J = (double*)b; b += align256(P.k1sq * d);
        s.Th2 = (double*)b; b += align256((size_t)P.r1cap * m2 * d);
        s.C2 = (double*)b; b += align256((size_t)P.r1cap * P.nt * P.k2cap * d);
        s.V2 = (double*)b; b += align256((size_t)P.k2cap * P.k2cap * d);
        s.sv = (double*)b; b += align256((size_t)(3 * P.k1cap + P.k2cap) * d);
        s.perm = (int*)b; b += align256((size_t)(P.k1cap + P.k2cap) * sizeof(int));
        s.flag = (int*)b; b += align256(sizeof(int));
        s.W = (double*)b; b += align256(P.k1sq * d);
        s.Wkeep = (double*)b;
        return s;
    }

    // event timing around one launch
    size_t ev_begin(int cls, hipStream_t s) {
        if (!timing) return (size_t)-1;
        if (ev_used == ev_pool.size()) {
            hipEvent_t a, b;
            if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return (size_t)-1;
            ev_pool.push_back({a, b});
            ev_class.push_back(cls);
        }
        ev_class[ev_used] = cls;
        (void)hipEventRecord(ev_pool[ev_used].first, s);
        return ev_used++;
    }
    void ev_end(size_t i, hipStream_t s) {
        if (i == (size_t)-1) return;
        (void)hipEventRecord(ev_pool[i].second, s);
    }
    void ev_collect() {
        for (size_t i = 0; i < ev_used; ++i) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev_pool[i].first, ev_pool[i].second) == hipSuccess) {
                kernel_ms[ev_class[i]] += ms;
                kernel_launches[ev_class[i]] += 1;
            }
        }
        ev_used = 0;
    }
};

namespace {

void build_ops(tt_handle* h, const tt_problem* p) {
    const Plan& P = h->P;
    auto term_index = [&](int axis, int sign) { return 1 + 2 * axis + (sign > 0 ? 0 : 1); };
    for (int kind = 0; kind < 4; ++kind) {
        OpDesc& o = h->ops[kind];
        std::memset(&o, 0, sizeof(o));
        for (int i = 0; i < kMaxBlocks; ++i) o.rshift[i] = -1;
        o.n_rblk = 1;
        o.rfac[0] = 0;
        o.rcoef0[0] = 1.0;
        o.n_gather = 1;
        const bool stream = kind == OP_FULL || kind == OP_TRANSPORT;
        const bool source = kind == OP_FULL || kind == OP_SOURCE;
        for (int i = 0; i < kMaxBlocks; ++i) o.rshift2[i] = -1;
        if (stream && P.flux == TT_FLUX_HLL) {
            // HLL (Appendix A: the upwind structure with spatially varying
            // coefficients): per axis the n^+ and n^- terms, each with gather
            // blocks for the centre and both neighbours carrying per-row weights
            o.hll = 1;
            o.gterm[0] = 0;
            o.gwk[0] = 0;
            for (int axis = 0; axis < P.dim; ++axis) {
                for (int sign = 1; sign >= -1; sign -= 2) {
                    const int t = o.n_rblk++;
                    o.rfac[t] = term_index(axis, sign);
                    o.rcoef0[t] = 0.0;
                    for (int kind = 0; kind < 3; ++kind) {
                        const int j = o.n_gather++;
                        o.gaxis[j] = axis;
                        o.gdir[j] = kind == 0 ? 0 : (kind == 1 ? -1 : 1);
                        o.gterm[j] = t;
                        o.gwk[j] = 1 + (sign > 0 ? 0 : 3) + kind;
                    }
                }
            }
            // an inflow ghost enters both terms of its axis through the shift
            // that leaves the domain: (1 +- eps) / 2 of the face's factor
            for (int f = 0; f < 2 * P.dim; ++f) {
                if (!is_inflow(p->bc[f])) continue;
                const int axis = f / 2, high = f & 1;
                const double lam = h->geom.lam[axis];
                for (int sign = 1; sign >= -1; sign -= 2) {
                    const int q = o.n_r1++;
                    o.r1kind[q] = 2;
                    o.r1face[q] = f;
                    o.r1fac[q] = term_index(axis, sign);
                    o.r1coef[q] = high ? -lam : lam;
                    o.r1hll[q] = high ? (sign > 0 ? 2 : 1) : (sign > 0 ? 1 : 2);
                }
            }
        } else if (stream && P.flux == TT_FLUX_RUSANOV) {
            // per axis: (n_d) (-(lambda / 2)) (O_{d+} - O_{d-}) and, when S+ > 0,
            // (1) (lambda s / 2) (O_{d+} - 2 I + O_{d-}); gather blocks c - e_d, c + e_d
            const double sr = P.rus_s;
            for (int axis = 0; axis < P.dim; ++axis) {
                const double lam = h->geom.lam[axis];
                const int jm = o.n_gather++, jp = o.n_gather++;
                o.gaxis[jm] = axis;
                o.gdir[jm] = -1;
                o.gaxis[jp] = axis;
                o.gdir[jp] = +1;
                int t = o.n_rblk++;
                o.rfac[t] = 1 + 2 * axis;
                o.rcoef0[t] = 0.0;
                o.rshift[t] = jm;
                o.rcoef[t] = 0.5 * lam;
                o.rshift2[t] = jp;
                o.rcoef2[t] = -0.5 * lam;
                if (sr != 0.0) {
                    t = o.n_rblk++;
                    o.rfac[t] = 2 + 2 * axis;
                    o.rcoef0[t] = -lam * sr;
                    o.rshift[t] = jm;
                    o.rcoef[t] = 0.5 * lam * sr;
                    o.rshift2[t] = jp;
                    o.rcoef2[t] = 0.5 * lam * sr;
                }
            }
            // a ghost enters each term of the face's axis through the coefficient
            // of the shift that leaves the domain there
            for (int f = 0; f < 2 * P.dim; ++f) {
                if (!is_inflow(p->bc[f])) continue;
                const int axis = f / 2, high = f & 1;
                const double lam = h->geom.lam[axis];
                int q = o.n_r1++;
                o.r1kind[q] = 1;
                o.r1face[q] = f;
                o.r1fac[q] = 1 + 2 * axis;
                o.r1coef[q] = high ? -0.5 * lam : 0.5 * lam;
                if (sr != 0.0) {
                    q = o.n_r1++;
                    o.r1kind[q] = 1;
                    o.r1face[q] = f;
                    o.r1fac[q] = 2 + 2 * axis;
                    o.r1coef[q] = 0.5 * lam * sr;
                }
            }
        } else if (stream) {
            for (int axis = 0; axis < P.dim; ++axis) {
                for (int sign = 1; sign >= -1; sign -= 2) {
                    const int t = o.n_rblk++;
                    const double lam = h->geom.lam[axis];
                    o.rfac[t] = term_index(axis, sign);
                    const int j = o.n_gather++;
                    o.gaxis[j] = axis;
                    // the (d,+) term reads the upwind neighbour c - e_d; the (d,-) term c + e_d
                    o.gdir[j] = sign > 0 ? -1 : +1;
                    o.rshift[t] = j;
                    o.rcoef0[t] = sign > 0 ? -lam : lam;
                    o.rcoef[t] = sign > 0 ? lam : -lam;
                }
            }
            for (int f = 0; f < 2 * P.dim; ++f) {
                if (!is_inflow(p->bc[f])) continue;
                const int q = o.n_r1++;
                o.r1kind[q] = 1;
                o.r1face[q] = f;
                o.r1fac[q] = term_index(f / 2, (f & 1) ? -1 : +1);
                o.r1coef[q] = (f & 1) ? -h->geom.lam[f / 2] : h->geom.lam[f / 2];
            }
        }
        if (source) {
            const int q = o.n_r1++;
            o.r1kind[q] = 0;
            o.r1fac[q] = 0;
            o.scale_d = 1;
        }
    }
}

template <typename T>
tt_status upload(void* dst, const std::vector<T>& v, hipStream_t s) {
    if (v.empty()) return TT_OK;
    HIP_TRY(hipMemcpyAsync(dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return TT_OK;
}

tt_status read_state(tt_handle* h, DevState& out, hipStream_t s) {
    HIP_TRY(hipMemcpyAsync(&out, h->st(), sizeof(DevState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return TT_OK;
}

tt_status write_state(tt_handle* h, const DevState& in, hipStream_t s) {
    HIP_TRY(hipMemcpyAsync(h->st(), &in, sizeof(DevState), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return TT_OK;
}

template <typename T>
tt_status set_cores_impl(tt_handle* h, int r1, int r2, const double* Z, const double* Th, const double* Ph,
                         hipStream_t s) {
    const Plan& P = h->P;
    const int ldz = ld_for_rank(r1);
    std::vector<T> zb((size_t)P.M * ldz, (T)0);
    for (long long k = 0; k < P.M; ++k)
        for (int a = 0; a < r1; ++a) zb[(size_t)k * ldz + a] = (T)Z[(size_t)k * r1 + a];
    h->zcur = 0;
    h->ccur = 0;
    HIP_TRY(hipMemcpyAsync(h->Zc(), zb.data(), zb.size() * sizeof(T), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(h->Thc(), Th, (size_t)r1 * P.nt * r2 * sizeof(double), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(h->Phc(), Ph, (size_t)r2 * P.np * sizeof(double), hipMemcpyHostToDevice, s));
    DevState st;
    std::memset(&st, 0, sizeof(st));
    st.r1 = r1; st.r2 = r2; st.ldz = ldz;
    st.max_R1 = r1; st.max_R2 = r2;
    h->pending = OP_NONE;
    return write_state(h, st, s);
}

tt_status reset_impl(tt_handle* h, hipStream_t s) {
    const Plan& P = h->P;
    std::vector<double> th((size_t)P.nt, 1.0), ph((size_t)P.np, 1.0);
    if (P.coupled)
        HIP_TRY(hipMemcpyAsync(h->ws + P.o_T, h->ws + P.o_T0, (size_t)P.NX * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (h->precision == TT_PREC_FP64) return set_cores_impl<double>(h, 1, 1, h->init_host.data(), th.data(), ph.data(), s);
    return set_cores_impl<float>(h, 1, 1, h->init_host.data(), th.data(), ph.data(), s);
}

// Neighbour structure and rank-1 block of operator `opkind` for the fused
// kernels (offsets relative to the current Z buffer).
FusedNbr fused_nbr(const tt_handle* h, int opkind) {
    const Plan& P = h->P;
    const OpDesc& op = h->ops[opkind];
    FusedNbr f;
    std::memset(&f, 0, sizeof(f));
    f.n_gather = op.n_gather;
    f.ns = P.n_terms;
    f.scale_d = op.scale_d;
    const size_t zoff = h->zcur ? P.o_Z1 : P.o_Z0;
    if (op.n_r1 > 0) {
        const bool src = opkind == OP_SOURCE;
        f.rw = src ? P.rw2 : P.rw1;
        f.roff = ((long long)(src ? P.o_R2 : P.o_R1) - (long long)zoff) / (long long)sizeof(float);
    }
    f.zoff = ((long long)P.o_zero - (long long)zoff) / (long long)sizeof(float);
    return f;
}

// Fused FP32 Gram rounding pass (after k_prep): projection + FP64 Gram in one
// persistent MFMA kernel, fixed-order sum of the block partials, SVD chain
// (which also folds V_r into the gather operand), then Z_out straight from Z.
// The fused FP32 projection + Gram partials (P.fused_blocks partials in GP).
template <int NP>
void launch_fused_project(tt_handle* h, int opkind, hipStream_t s) {
    const Plan& P = h->P;
    hipLaunchKernelGGL((k_fused_f32<NP, true>), dim3(P.fused_blocks), dim3(kFusedThreads), P.lds_p, s, h->geom,
                       fused_nbr(h, opkind), (const DevState*)h->st(), (const float*)h->Zc(),
                       (const float*)h->at<float>(P.o_Gsw), (float*)nullptr, h->at<float2>(P.o_aux),
                       h->at<int>(P.o_nbr), h->at<double>(P.o_GP), P.fused_tiles);
}

// The fused FP32 output Z_out from Z with V_r folded into the operand.
template <int NO>
void launch_fused_output(tt_handle* h, int opkind, hipStream_t s) {
    const Plan& P = h->P;
    hipLaunchKernelGGL((k_fused_f32<NO, false>), dim3(P.fused_blocks_o), dim3(kFusedThreads), P.lds_o, s, h->geom,
                       fused_nbr(h, opkind), (const DevState*)h->st(), (const float*)h->Zc(),
                       (const float*)h->at<float>(P.o_Gfold), (float*)h->Zn(), h->at<float2>(P.o_aux),
                       h->at<int>(P.o_nbr), (double*)nullptr, P.fused_tiles);
}

template <int NP, int NO>
tt_status round_fused_t(tt_handle* h, int opkind, double tol, int cap, hipStream_t s) {
    const Plan& P = h->P;
    DevState* st = h->st();
    SmallScratch sc = h->scratch();
    float* Gop = h->at<float>(P.o_G);
    float* V = h->at<float>(P.o_V);
    double* GP = h->at<double>(P.o_GP);
    double* RB = h->at<double>(P.o_RB);
    size_t e = h->ev_begin(KC_PROJECT, s);
    launch_fused_project<NP>(h, opkind, s);
    h->ev_end(e, s);
    e = h->ev_begin(KC_TREE, s);
    hipLaunchKernelGGL((k_sum_gram<NP>), dim3((gram_blocks(NP) * 256 + 31) / 32), dim3(256), 0, s, (const double*)GP,
                       P.fused_blocks, RB, P.KP);
    h->ev_end(e, s);
    e = h->ev_begin(KC_SVD, s);
    const double* Gin = RB;
    const double* QThIn = h->at<double>(P.o_QTh);
    const double* QPhIn = h->at<double>(P.o_QPh);
    const double* Wk = sc.Wkeep;
    const RandBufs rb = h->rand_bufs();
    if (P.rand) {
        hipLaunchKernelGGL(k_rand_sketch, dim3(1), dim3(kSmallThreads), kSmallLdsBytes, s, h->geom, st, Gin, P.KP,
                           QThIn, QPhIn, h->rand_p, h->rand_seed, rb, P.KP);
        Gin = rb.G;
        QThIn = rb.QTh;
        QPhIn = rb.QPh;
        Wk = rb.Veff;
    }
    if (P.svd_fast)
        hipLaunchKernelGGL((k_svd_chain<float, true>), dim3(1), dim3(kSmallThreads), kSmallLdsBytes, s, h->geom, st,
                           Gin, P.KP, 1, QThIn, QPhIn, tol, std::min(cap, P.r1cap), std::min(cap, P.r2cap), sc,
                           h->Thn(), h->Phn(), V, h->at<double>(P.o_sv), (const float*)Gop, h->at<float>(P.o_Gfold),
                           NO);
    else
        hipLaunchKernelGGL((k_svd_chain<float, false>), dim3(1), dim3(kSmallThreads), kSmallLdsBytes, s, h->geom, st,
                           Gin, P.KP, 1, QThIn, QPhIn, tol, std::min(cap, P.r1cap), std::min(cap, P.r2cap), sc,
                           h->Thn(), h->Phn(), V, h->at<double>(P.o_sv), (const float*)Gop, h->at<float>(P.o_Gfold),
                           NO);
    if (P.rand)
        hipLaunchKernelGGL(k_rand_fold<float>, dim3(1), dim3(1024), 0, s, st, (const double*)rb.P,
                           (const double*)sc.Wkeep, rb.Veff, V);
    hipLaunchKernelGGL(k_fold<float>, dim3(64), dim3(256), 0, s, (const DevState*)st, (const float*)Gop, Wk,
                       h->at<float>(P.o_Gfold), NO);
    h->ev_end(e, s);
    e = h->ev_begin(KC_OUTPUT, s);
    launch_fused_output<NO>(h, opkind, s);
    h->ev_end(e, s);
    hipLaunchKernelGGL(k_commit, dim3(1), dim3(64), 0, s, st);
    HIP_TRY(hipGetLastError());
    h->zcur ^= 1;
    h->ccur ^= 1;
    return TT_OK;
}

tt_status round_fused(tt_handle* h, int opkind, double tol, int cap, hipStream_t s) {
    const Plan& P = h->P;
    if (P.nct_p == 4)
        return P.nct_o == 4 ? round_fused_t<4, 4>(h, opkind, tol, cap, s) : round_fused_t<4, 2>(h, opkind, tol, cap, s);
    return P.nct_o == 4 ? round_fused_t<2, 4>(h, opkind, tol, cap, s) : round_fused_t<2, 2>(h, opkind, tol, cap, s);
}

// FP64 MFMA contractions (k_mm_f64): the projection B = Z_new L_Theta, with
// the FP64 Gram partials of B fused in when `gram` (16 NCT <= 64 columns), and
// the output Z_out = B V_r.
template <int MODE, int NCT, bool GRAM>
void launch_mm_f64(tt_handle* h, const OpDesc& op, const double* A, const double* Gop, double* Out, double* parts,
                   hipStream_t s) {
    const Plan& P = h->P;
    // one row tile per wave where two would spill: 128 columns, or 64 with the fused Gram
    constexpr int RT = (NCT == 8 || (NCT == 4 && GRAM)) ? 1 : 2;
    const int nb = MODE == MODE_OUTPUT ? P.f64_blocks_o : P.f64_blocks;
    if (MODE == MODE_PROJECT && op.hll)
        hipLaunchKernelGGL((k_mm_f64<MODE, NCT, GRAM, RT, true>), dim3(nb), dim3(kF64Threads),
                           f64_lds_bytes(NCT, GRAM, RT, true), s, h->geom, op, (const DevState*)h->st(), A, Gop, Out,
                           h->rowdata(), parts);
    else
        hipLaunchKernelGGL((k_mm_f64<MODE, NCT, GRAM, RT>), dim3(nb), dim3(kF64Threads),
                           f64_lds_bytes(NCT, GRAM, RT, false, MODE == MODE_OUTPUT ? kF64OutChunks : 0), s, h->geom, op,
                           (const DevState*)h->st(), A, Gop, Out,
                           h->rowdata(), parts);
}

void project_f64(tt_handle* h, const OpDesc& op, bool gram, double* parts, hipStream_t s) {
    const Plan& P = h->P;
    const double* Z = (const double*)h->Zc();
    const double* G = h->at<double>(P.o_G);
    double* B = h->at<double>(P.o_B);
    switch (P.nct_f) {
        case 1: gram ? launch_mm_f64<MODE_PROJECT, 1, true>(h, op, Z, G, B, parts, s)
                     : launch_mm_f64<MODE_PROJECT, 1, false>(h, op, Z, G, B, parts, s); break;
        case 2: gram ? launch_mm_f64<MODE_PROJECT, 2, true>(h, op, Z, G, B, parts, s)
                     : launch_mm_f64<MODE_PROJECT, 2, false>(h, op, Z, G, B, parts, s); break;
        case 4: gram ? launch_mm_f64<MODE_PROJECT, 4, true>(h, op, Z, G, B, parts, s)
                     : launch_mm_f64<MODE_PROJECT, 4, false>(h, op, Z, G, B, parts, s); break;
        default: launch_mm_f64<MODE_PROJECT, 8, false>(h, op, Z, G, B, parts, s); break;
    }
}

void output_f64(tt_handle* h, const OpDesc& op, hipStream_t s) {
    const Plan& P = h->P;
    const double* B = h->at<double>(P.o_B);
    const double* V = h->at<double>(P.o_V);
    double* Zo = (double*)h->Zn();
    switch (P.nct_fo) {
        case 1: launch_mm_f64<MODE_OUTPUT, 1, false>(h, op, B, V, Zo, nullptr, s); break;
        case 2: launch_mm_f64<MODE_OUTPUT, 2, false>(h, op, B, V, Zo, nullptr, s); break;
        default: launch_mm_f64<MODE_OUTPUT, 4, false>(h, op, B, V, Zo, nullptr, s); break;
    }
}

// Small-core QR of Theta and Phi, L_Theta and the gather operand of
// operator `opkind` for the current state (k_prep).
// Whether operator `opkind`'s projection may run in direction space (the
// prep then decides per pass: only when both small-core factors are square).
bool stencil_op(const tt_handle* h, int opkind) {
    const OpDesc& op = h->ops[opkind];
    return h->P.stencil && !op.hll && op.n_gather <= kStNG && op.n_r1 <= kStZ;
}

template <typename T>
void launch_prep(tt_handle* h, int opkind, hipStream_t s) {
    const Plan& P = h->P;
    constexpr bool f32 = std::is_same<T, float>::value;
    const bool fused = f32 && P.fused;
    const bool sten = stencil_op(h, opkind);
    hipLaunchKernelGGL(k_prep<T>, dim3(1), dim3(kSmallThreads), kSmallLdsBytes, s, h->geom, h->ops[opkind], h->st(),
                       h->Thc(), h->Phc(), h->at<double>(P.o_gtab), h->at<double>(P.o_htab), h->scratch(),
                       h->at<double>(P.o_LTh), P.k1cap, h->at<double>(P.o_QTh), h->at<double>(P.o_QPh),
                       h->at<T>(P.o_G), fused ? h->at<T>(P.o_Gsw) : (T*)nullptr, P.nct_p,
                       sten ? h->at<double>(P.o_Wst) : (double*)nullptr, sten ? h->at<double>(P.o_Cst) : (double*)nullptr);
}

// The projection B = Z_new L_Theta into the stored first core (every path but
// the fused FP32 one); with FP64 MFMA contractions on the Gram route and at
// most 64 columns, the FP64 Gram partials of B come with it (in RA).
template <typename T>
tt_status launch_project(tt_handle* h, int opkind, hipStream_t s) {
    const Plan& P = h->P;
    const OpDesc& op = h->ops[opkind];
    DevState* st = h->st();
    T* Gop = h->at<T>(P.o_G);
    T* B = h->at<T>(P.o_B);
    constexpr bool f32 = std::is_same<T, float>::value;
    const unsigned gx = (unsigned)((P.M + 63) / 64);
    const unsigned gx128 = (unsigned)((P.M + 127) / 128);
    if constexpr (!f32) {
        if (P.f64mm && stencil_op(h, opkind)) {
            // direction space when the prep found both factors square (the
            // kernels read its flag; otherwise these two exit and the
            // gathered projection below runs)
            double* Yb = h->at<double>(P.o_Y);
            size_t e = h->ev_begin(KC_ANGLE, s);
            hipLaunchKernelGGL((k_mm_f64<MODE_ANGLE, 8, false, 1>), dim3(P.f64_blocks), dim3(kF64Threads),
                               f64_lds_bytes(8, false, 1, false, kF64AngChunks), s, h->geom, op, (const DevState*)st,
                               (const double*)h->Zc(), (const double*)h->at<double>(P.o_Wst), Yb, h->rowdata(),
                               (double*)nullptr);
            h->ev_end(e, s);
            e = h->ev_begin(KC_STENCIL, s);
            hipLaunchKernelGGL(k_stencil_f64, dim3(P.st_blocks), dim3(64 * kStWaves), 0, s, h->geom, op,
                               (const DevState*)st, (const double*)Yb, (const double*)h->at<double>(P.o_Cst),
                               (double*)B, h->rowdata());
            h->ev_end(e, s);
        }
    }
    if constexpr (f32) {
        if (P.stencil32 && stencil_op(h, opkind)) {
            // the same on FP32 data: W to FP32, Y = Z W on FP32 MFMA, the
            // stencil with FP64 sums into the FP32 B
            float* Yf = h->at<float>(P.o_Y);
            float* Wf = h->at<float>(P.o_WstF);
            size_t e = h->ev_begin(KC_ANGLE, s);
            const int nw = P.ldzcap * P.ldbcap;
            hipLaunchKernelGGL(k_f64_to_f32, dim3((nw + 255) / 256), dim3(256), 0, s,
                               (const double*)h->at<double>(P.o_Wst), Wf, nw);
            hipLaunchKernelGGL((k_gemm_f32_mfma<MODE_ANGLE, 128>), dim3(gx128, 1), dim3(256), 0, s,
                               h->geom, op, (const DevState*)st, (const float*)h->Zc(), (const float*)Wf, Yf,
                               h->rowdata());
            h->ev_end(e, s);
            e = h->ev_begin(KC_STENCIL, s);
            hipLaunchKernelGGL(k_stencil_f32, dim3(P.st_blocks), dim3(64 * kStWaves), 0, s, h->geom, op,
                               (const DevState*)st, (const float*)Yf, (const double*)h->at<double>(P.o_Cst),
                               (float*)B, h->rowdata());
            h->ev_end(e, s);
        }
    }
    const size_t e = h->ev_begin(KC_PROJECT, s);
    if constexpr (f32) {
        if (P.bf16x) {
            __bf16* gh = h->at<__bf16>(P.o_Gh);
            __bf16* gl = h->at<__bf16>(P.o_Gl);
            hipLaunchKernelGGL(k_split_bf16, dim3(64), dim3(256), 0, s, (const DevState*)st, 0, (const float*)Gop,
                               16 * P.nct_b, P.kc_g, gh, gl);
            // the operator's rank-1 block: the source operator's, or the full
            // (transport, with the paper's step order) operator's
            const bool srcop = opkind == OP_SOURCE;
            if ((srcop ? P.rw2 : P.rw1) < op.n_r1) return fail(TT_ERR_STATE, "no rank-1 row block for this operator");
            const BxRows rows{h->at<float2>(P.o_aux), h->at<int>(P.o_nbr), P.n_terms,
                              h->at<float>(srcop ? P.o_R2 : P.o_R1), srcop ? P.rw2 : P.rw1};
            if (P.nct_b == 8)
                hipLaunchKernelGGL((k_gemm_bf16x<MODE_PROJECT, 8>), dim3(gx128), dim3(256), 0, s, h->geom, op,
                                   (const DevState*)st, (const float*)h->Zc(), (const __bf16*)gh, (const __bf16*)gl,
                                   (float*)B, rows);
            else
                hipLaunchKernelGGL((k_gemm_bf16x<MODE_PROJECT, 4>), dim3(gx128), dim3(256), 0, s, h->geom, op,
                                   (const DevState*)st, (const float*)h->Zc(), (const __bf16*)gh, (const __bf16*)gl,
                                   (float*)B, rows);
        } else {
            hipLaunchKernelGGL((k_gemm_f32_mfma<MODE_PROJECT, 64>), dim3(gx128, (P.ldbcap + 63) / 64), dim3(256), 0, s,
                               h->geom, op, (const DevState*)st, (const float*)h->Zc(), (const float*)Gop, (float*)B,
                               h->rowdata());
        }
    } else if (P.f64mm) {
        project_f64(h, op, h->round_method != TT_ROUND_QR && P.nct_f <= 4, h->at<double>(P.o_RA), s);
    } else
        hipLaunchKernelGGL((k_gather_gemm<T, MODE_PROJECT>), dim3(gx, (P.ldbcap + 63) / 64), dim3(256), 0, s, h->geom,
                           op, st, (const T*)h->Zc(), (const T*)Gop, B, h->rowdata());
    h->ev_end(e, s);
    return TT_OK;
}

// FP64 Gram partials of the stored first core B, one per block of P.Pg (each
// over P.rowsg rows), into RA.  Not used where the projection forms them.
template <typename T>
void launch_gram_parts(tt_handle* h, hipStream_t s) {
    const Plan& P = h->P;
    const DevState* st = h->st();
    const T* B = h->at<T>(P.o_B);
    double* RA = h->at<double>(P.o_RA);
    if constexpr (std::is_same<T, double>::value) {
        if (P.f64mm) {   // 128 columns
            hipLaunchKernelGGL(k_gram_f64_mfma_w8d, dim3(P.Pg), dim3(256), 0, s, (const double*)B, st, P.M, P.rowsg,
                               RA);
            return;
        }
    } else {
        if (P.KP == 128) {
            hipLaunchKernelGGL(k_gram_f64_mfma_w8, dim3(P.Pg), dim3(256), 0, s, (const float*)B, st, P.M, P.rowsg, RA);
            return;
        }
        if (P.KP == 64) {
            hipLaunchKernelGGL(k_gram_f64_mfma, dim3(P.Pg), dim3(256), 0, s, (const float*)B, st, P.M, P.rowsg, RA);
            return;
        }
    }
    if (P.KP == 64)
        hipLaunchKernelGGL((k_gram<T, 64>), dim3(P.Pg), dim3(256), 0, s, B, st, P.M, P.rowsg, RA);
    else
        hipLaunchKernelGGL((k_gram<T, 128>), dim3(P.Pg), dim3(256), 0, s, B, st, P.M, P.rowsg, RA);
}

// One rounding pass applying operator `op` (OP_NONE: plain rounding).
template <typename T>
tt_status round_impl(tt_handle* h, int opkind, double tol, int cap, hipStream_t s) {
    const Plan& P = h->P;
    const OpDesc& op = h->ops[opkind];
    DevState* st = h->st();
    SmallScratch sc = h->scratch();
    T* Gop = h->at<T>(P.o_G);
    T* B = h->at<T>(P.o_B);
    T* V = h->at<T>(P.o_V);
    double* QTh = h->at<double>(P.o_QTh);
    double* QPh = h->at<double>(P.o_QPh);
    size_t e;

    constexpr bool f32 = std::is_same<T, float>::value;
    e = h->ev_begin(KC_PREP, s);
    launch_prep<T>(h, opkind, s);
    h->ev_end(e, s);
    if constexpr (f32) {
        if (P.fused) return round_fused(h, opkind, tol, cap, s);
    }

    const unsigned gx = (unsigned)((P.M + 63) / 64);
    const unsigned gx128 = (unsigned)((P.M + 127) / 128);
    {
        const tt_status r = launch_project<T>(h, opkind, s);   // timed per kernel inside
        if (r != TT_OK) return r;
    }

    const double* RB = nullptr;
    int ldr = P.KP;
    int gram = 0;
    double* RA = h->at<double>(P.o_RA);
    double* RBuf = h->at<double>(P.o_RB);
    if (h->round_method == TT_ROUND_QR) {
        const double* in = nullptr;
        double* out = RA;
        for (size_t L = 0; L < P.levP.size(); ++L) {
            e = h->ev_begin(L == 0 ? KC_FACTOR : KC_TREE, s);
            if (P.KPt == 16) {
                if (L == 0)
                    hipLaunchKernelGGL((k_tsqr<T, 16, 32, 16>), dim3(P.levP[L]), dim3(512), 0, s, (const T*)B, 0, 1, 0,
                                       P.levN[L], P.levRows[L], (const DevState*)st, out);
                else
                    hipLaunchKernelGGL((k_tsqr<double, 16, 32, 16>), dim3(P.levP[L]), dim3(512), 0, s, in, 16, 0, P.k1cap,
                                       P.levN[L], P.levRows[L], (const DevState*)st, out);
            } else if (P.KP == 64) {
                if (L == 0)
                    hipLaunchKernelGGL((k_tsqr<T, 64, 8, kTsqrBrLeaf64>), dim3(P.levP[L]), dim3(512), 0, s, (const T*)B, 0, 1, 0,
                                       P.levN[L], P.levRows[L], (const DevState*)st, out);
                else
                    hipLaunchKernelGGL((k_tsqr<double, 64, 16, kTsqrBrTree64>), dim3(P.levP[L]), dim3(1024), 0, s, in, 64, 0, P.k1cap,
                                       P.levN[L], P.levRows[L], (const DevState*)st, out);
            } else {
                if (L == 0)
                    hipLaunchKernelGGL((k_tsqr<T, 128, 4, kTsqrBrLeaf128>), dim3(P.levP[L]), dim3(512), 0, s, (const T*)B, 0, 1, 0,
                                       P.levN[L], P.levRows[L], (const DevState*)st, out);
                else
                    hipLaunchKernelGGL((k_tsqr<double, 128, 8, 16>), dim3(P.levP[L]), dim3(1024), 0, s, in, 128, 0, P.k1cap,
                                       P.levN[L], P.levRows[L], (const DevState*)st, out);
            }
            h->ev_end(e, s);
            in = out;
            out = (out == RA) ? RBuf : RA;
        }
        RB = in;
        ldr = P.KPt;
    } else if (!f32 && P.f64mm) {
        // FP64 Gram of the stored B: fused into the projection (partials in RA)
        // for up to 64 columns, else the 128-column FP64 MFMA Gram over B
        gram = 1;
        e = h->ev_begin(KC_FACTOR, s);
        if (P.nct_f == 8) launch_gram_parts<T>(h, s);
        h->ev_end(e, s);
        e = h->ev_begin(KC_TREE, s);
        switch (P.nct_f) {
            case 1: hipLaunchKernelGGL(k_sum_gram<1>, dim3((gram_blocks(1) * 256 + 31) / 32), dim3(256), 0, s,
                                       (const double*)RA, P.f64_blocks, RBuf, P.KP); break;
            case 2: hipLaunchKernelGGL(k_sum_gram<2>, dim3((gram_blocks(2) * 256 + 31) / 32), dim3(256), 0, s,
                                       (const double*)RA, P.f64_blocks, RBuf, P.KP); break;
            case 4: hipLaunchKernelGGL(k_sum_gram<4>, dim3((gram_blocks(4) * 256 + 31) / 32), dim3(256), 0, s,
                                       (const double*)RA, P.f64_blocks, RBuf, P.KP); break;
            default: hipLaunchKernelGGL(k_sum_gram<8>, dim3((gram_blocks(8) * 256 + 31) / 32), dim3(256), 0, s,
                                        (const double*)RA, P.Pg, RBuf, P.KP); break;
        }
        h->ev_end(e, s);
        RB = RBuf;
    } else {
        gram = 1;
        e = h->ev_begin(KC_FACTOR, s);
        launch_gram_parts<T>(h, s);
        h->ev_end(e, s);
        if (f32 && P.KP == 128) {
            e = h->ev_begin(KC_TREE, s);
            hipLaunchKernelGGL(k_sum_gram<8>, dim3((gram_blocks(8) * 256 + 31) / 32), dim3(256), 0, s,
                               (const double*)RA, P.Pg, RBuf, P.KP);
            h->ev_end(e, s);
        } else {
            e = h->ev_begin(KC_TREE, s);
            const int n = P.KP * P.KP;
            hipLaunchKernelGGL(k_sum_parts, dim3((n + 31) / 32), dim3(256), 0, s, (const double*)RA, P.Pg, n, RBuf);
            h->ev_end(e, s);
        }
        RB = RBuf;
    }

    e = h->ev_begin(KC_SVD, s);
    const double* QThIn = QTh;
    const double* QPhIn = QPh;
    const RandBufs rb = h->rand_bufs();
    if (P.rand) {
        hipLaunchKernelGGL(k_rand_sketch, dim3(1), dim3(kSmallThreads), kSmallLdsBytes, s, h->geom, st, RB, ldr, QThIn,
                           QPhIn, h->rand_p, h->rand_seed, rb, P.KP);
        RB = rb.G;
        ldr = P.KP;
        QThIn = rb.QTh;
        QPhIn = rb.QPh;
    }
    if (P.svd_fast)
        hipLaunchKernelGGL((k_svd_chain<T, true>), dim3(1), dim3(kSmallThreads), kSmallLdsBytes, s, h->geom, st, RB, ldr,
                           gram, QThIn, QPhIn, tol, std::min(cap, P.r1cap), std::min(cap, P.r2cap), sc, h->Thn(),
                           h->Phn(), V, h->at<double>(P.o_sv), (const T*)nullptr, (T*)nullptr, 0);
    else
        hipLaunchKernelGGL((k_svd_chain<T, false>), dim3(1), dim3(kSmallThreads), kSmallLdsBytes, s, h->geom, st, RB, ldr,
                           gram, QThIn, QPhIn, tol, std::min(cap, P.r1cap), std::min(cap, P.r2cap), sc, h->Thn(),
                           h->Phn(), V, h->at<double>(P.o_sv), (const T*)nullptr, (T*)nullptr, 0);
    if (P.rand)
        hipLaunchKernelGGL(k_rand_fold<T>, dim3(1), dim3(1024), 0, s, st, (const double*)rb.P, (const double*)sc.Wkeep,
                           rb.Veff, V);
    h->ev_end(e, s);

    e = h->ev_begin(KC_OUTPUT, s);
    if constexpr (f32) {
        if (P.bf16x) {
            __bf16* vh = h->at<__bf16>(P.o_Vh);
            __bf16* vl = h->at<__bf16>(P.o_Vl);
            hipLaunchKernelGGL(k_split_bf16, dim3(16), dim3(256), 0, s, (const DevState*)st, 1, (const float*)V,
                               16 * P.nct_bo, P.kc_v, vh, vl);
            if (P.nct_bo == 4)
                hipLaunchKernelGGL((k_gemm_bf16x<MODE_OUTPUT, 4>), dim3(gx128), dim3(256), 0, s, h->geom, op,
                                   (const DevState*)st, (const float*)B, (const __bf16*)vh, (const __bf16*)vl,
                                   (float*)h->Zn(), BxRows{});
            else
                hipLaunchKernelGGL((k_gemm_bf16x<MODE_OUTPUT, 2>), dim3(gx128), dim3(256), 0, s, h->geom, op,
                                   (const DevState*)st, (const float*)B, (const __bf16*)vh, (const __bf16*)vl,
                                   (float*)h->Zn(), BxRows{});
        } else if (P.ldzcap <= 32)
            hipLaunchKernelGGL((k_gemm_f32_mfma<MODE_OUTPUT, 32>), dim3(gx128, 1), dim3(256), 0, s, h->geom, op,
                               (const DevState*)st, (const float*)B, (const float*)V, (float*)h->Zn(), h->rowdata());
        else
            hipLaunchKernelGGL((k_gemm_f32_mfma<MODE_OUTPUT, 64>), dim3(gx128, (P.ldzcap + 63) / 64), dim3(256), 0, s,
                               h->geom, op, (const DevState*)st, (const float*)B, (const float*)V, (float*)h->Zn(),
                               h->rowdata());
    } else if (P.f64mm) {
        output_f64(h, op, s);
    } else {
        hipLaunchKernelGGL((k_gather_gemm<T, MODE_OUTPUT>), dim3(gx, (P.ldzcap + 63) / 64), dim3(256), 0, s, h->geom,
                           op, (const DevState*)st, (const T*)B, (const T*)V, (T*)h->Zn(), h->rowdata());
    }
    h->ev_end(e, s);
    hipLaunchKernelGGL(k_commit, dim3(1), dim3(64), 0, s, st);
    HIP_TRY(hipGetLastError());
    h->zcur ^= 1;
    h->ccur ^= 1;
    return TT_OK;
}

tt_status round_dispatch(tt_handle* h, int opkind, double tol, int cap, hipStream_t s) {
    if (h->precision == TT_PREC_FP64) return round_impl<double>(h, opkind, tol, cap, s);
    return round_impl<float>(h, opkind, tol, cap, s);
}

CoupleArgs couple_args(tt_handle* h) {
    const Plan& P = h->P;
    CoupleArgs a;
    a.edges = h->at<double>(P.o_edges);
    a.wth = h->at<double>(P.o_wth);
    a.wph = h->at<double>(P.o_wph);
    a.gtab = h->at<double>(P.o_gtab);
    a.htab = h->at<double>(P.o_htab);
    a.T = h->at<double>(P.o_T);
    a.Js = h->at<double>(P.o_Js);
    a.eps = h->at<double>(P.o_eps);
    a.R1 = (P.row_tables && P.rw1 > 0) ? h->at<float>(P.o_R1) : nullptr;
    a.rw1 = P.rw1;
    a.qe1 = h->qe_full;
    a.R2 = (P.row_tables && P.rw2 > 0) ? h->at<float>(P.o_R2) : nullptr;
    a.rw2 = P.rw2;
    a.qe2 = h->qe_source;
    a.nbr = P.row_tables ? h->at<int>(P.o_nbr) : nullptr;
    a.ns = P.n_terms;
    a.heat_capacity = h->heat_capacity;
    a.dt = h->dt;
    a.c = h->c;
    a.coupled = P.coupled ? 1 : 0;
    a.jn = P.kscat ? h->at<double>(P.o_jn) : nullptr;
    return a;
}

// Blocks of the coupling kernels: enough for one pass over the cells, at most
// `cap` (the pre-pass rebuilds its one-column operand per block, so it runs
// one resident round, 3 blocks per CU at its register count, and loops).
unsigned couple_grid(const Plan& P, long long cap) {
    const long long per_block = 4LL * (64 / couple_seg(P.G));   // cells per block and pass
    return (unsigned)std::max<long long>(1, std::min<long long>(cap, (P.NX + per_block - 1) / per_block));
}

// One step with the coupled medium temperature: the stage temperature and
// emission before the rounding pass of the full operator, the
// energy-conserving temperature update after it.
template <typename T>
tt_status coupled_step(tt_handle* h, hipStream_t s) {
    const Plan& P = h->P;
    const CoupleArgs a = couple_args(h);
    const size_t lds_pre = couple_lds_doubles(P.n_gather_max * P.ldzcap + P.n_r1_max, 1 + P.n_terms, P.r1cap, P.r2cap) *
                           sizeof(double);
    const bool paper = h->step_order == 1;
    tt_status r = TT_OK;
    if (paper) {
        // the paper's order (Sec. 3.1): transport and round, then the source
        // stage on the rounded state, whose angle means are J*
        r = round_dispatch(h, OP_TRANSPORT, h->tol, P.cap, s);
        if (r != TT_OK) return r;
    }
    size_t e = h->ev_begin(KC_COUPLE, s);
    hipLaunchKernelGGL(k_couple_pre<T>, dim3(couple_grid(P, 768)), dim3(kCoupleThreads), lds_pre, s, h->geom,
                       h->ops[paper ? OP_NONE : OP_TRANSPORT], h->rowdata(), (const DevState*)h->st(),
                       (const T*)h->Zc(), (const double*)h->Thc(), (const double*)h->Phc(), a);
    h->ev_end(e, s);
    HIP_TRY(hipGetLastError());
    r = round_dispatch(h, paper ? OP_SOURCE : OP_FULL, h->tol, P.cap, s);
    if (r != TT_OK) return r;
    if (!P.coupled) return TT_OK;
    const size_t lds_post = (size_t)(P.r1cap + P.r2cap + 8) * sizeof(double);
    e = h->ev_begin(KC_COUPLE, s);
    hipLaunchKernelGGL(k_couple_post<T>, dim3(couple_grid(P, 2048)), dim3(kCoupleThreads), lds_post, s, h->geom,
                       (const DevState*)h->st(), (const T*)h->Zc(), (const double*)h->Thc(), (const double*)h->Phc(), a);
    h->ev_end(e, s);
    HIP_TRY(hipGetLastError());
    return TT_OK;
}

tt_status step_impl(tt_handle* h, hipStream_t s) {
    tt_status r;
    if (h->P.prepass) {
        if (h->pending != OP_NONE) return fail(TT_ERR_STATE, "an unrounded operator is pending");
        return h->precision == TT_PREC_FP64 ? coupled_step<double>(h, s) : coupled_step<float>(h, s);
    }
    if (h->pending != OP_NONE) {
        r = round_dispatch(h, h->pending, h->tol, h->P.cap, s);
        h->pending = OP_NONE;
        if (r != TT_OK) return r;
        if (h->step_order == 1) return round_dispatch(h, OP_SOURCE, h->tol, h->P.cap, s);
        return TT_OK;
    }
    if (h->step_order == 1) {
        r = round_dispatch(h, OP_TRANSPORT, h->tol, h->P.cap, s);
        if (r != TT_OK) return r;
        return round_dispatch(h, OP_SOURCE, h->tol, h->P.cap, s);
    }
    return round_dispatch(h, OP_FULL, h->tol, h->P.cap, s);
}

template <typename T>
tt_status energy_impl(tt_handle* h, hipStream_t s, double* energy, int* nanflag) {
    const Plan& P = h->P;
    DevState st;
    tt_status r = read_state(h, st, s);
    if (r != TT_OK) return r;
    double* parts = h->at<double>(P.o_colsum);
    hipLaunchKernelGGL(k_colsum<T>, dim3(256), dim3(1024), 0, s, (const DevState*)h->st(), (const T*)h->Zc(), P.M, parts);
    HIP_TRY(hipGetLastError());
    std::vector<double> hp((size_t)256 * 128);
    std::vector<double> th((size_t)st.r1 * P.nt * st.r2), ph((size_t)st.r2 * P.np);
    HIP_TRY(hipMemcpyAsync(hp.data(), parts, hp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(th.data(), h->Thc(), th.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(ph.data(), h->Phc(), ph.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    double E = 0.0;
    bool bad = false;
    for (int a = 0; a < st.r1; ++a) {
        double cs = 0.0;
        for (int b = 0; b < 256; ++b) cs += hp[(size_t)b * 128 + a];
        if (!std::isfinite(cs)) bad = true;
        // e_a = sum_{l,q} Theta[a,l,q] w_l sum_p Phi[q,p] w_p
        double ea = 0.0;
        for (int l = 0; l < P.nt; ++l)
            for (int q = 0; q < st.r2; ++q) {
                double pw = 0.0;
                for (int p = 0; p < P.np; ++p) pw += ph[(size_t)q * P.np + p] * h->w_phi[p];
                ea += th[((size_t)a * P.nt + l) * st.r2 + q] * h->w_theta[l] * pw;
            }
        E += cs * ea;
    }
    *energy = E * h->dV;
    *nanflag = (bad || st.nan_flag) ? 1 : 0;
    return TT_OK;
}

tt_status fill_stats(tt_handle* h, tt_stats* out, hipStream_t s) {
    DevState st;
    tt_status r = read_state(h, st, s);
    if (r != TT_OK) return r;
    const Plan& P = h->P;
    std::memset(out, 0, sizeof(*out));
    out->steps = h->last_steps;
    out->r1 = st.r1;
    out->r2 = st.r2;
    out->max_R1 = st.max_R1;
    out->max_R2 = st.max_R2;
    if (h->P.rand) {
        out->sketch_r1 = st.l1s;
        out->sketch_r2 = st.l2s;
    }
    out->direction_space_rounds = st.stencil_rounds;
    out->norm = st.norm;
    out->discarded_rel = st.norm > 0 ? std::sqrt(std::max(st.disc2, 0.0)) / st.norm : 0.0;
    double E = 0.0;
    int bad = 0;
    r = (h->precision == TT_PREC_FP64) ? energy_impl<double>(h, s, &E, &bad) : energy_impl<float>(h, s, &E, &bad);
    if (r != TT_OK) return r;
    out->energy = E;
    out->nan_flag = bad;
    if (P.coupled) {
        std::vector<double> T((size_t)P.NX);
        HIP_TRY(hipMemcpyAsync(T.data(), h->ws + P.o_T, T.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        double sum = 0.0;
        for (double t : T) {
            if (!std::isfinite(t)) out->nan_flag = 1;
            sum += t;
        }
        out->medium_energy = h->dV * h->heat_capacity * sum;
    }
    const double dense = (double)P.M * P.nt * P.np;
    const double tt = (double)P.M * st.r1 + (double)P.nt * st.r1 * st.r2 + (double)P.np * st.r2;
    out->compression = dense / tt;
    // Storage factor k_s of the last rounding pass (Sec. 3.2 and the appendix
    // on compression): entries of the TT sum before rounding, as the SVD
    // rounding forms it explicitly (ranks R1, R2), over the rounded TT.
    // k_s_impl: this library's own peak of the pass, at the sizes it reached:
    // input Z, the stored projected core B (M x k1; none on the fused path),
    // output Z and the (R1, R2) middle core, over the rounded TT.
    if (st.rounds > 0 && st.R1 > 0 && st.R2 > 0) {
        const double sum = (double)P.M * st.R1 + (double)P.nt * st.R1 * st.R2 + (double)P.np * st.R2;
        out->k_s = sum / tt;
        // (plus Y = Z W, M x k1, when the pass projected in direction space)
        const double bst = P.fused ? 0.0 : (double)P.M * st.k1 * (st.stencil ? 2.0 : 1.0);
        const double impl = (double)P.M * (st.r1_in + st.r1) + bst + (double)P.nt * st.R1 * st.R2 +
                            (double)P.np * st.R2;
        out->k_s_impl = impl / tt;
    } else {
        out->k_s = 1.0;
        out->k_s_impl = 1.0;
    }
    out->seconds = h->last_seconds;
    for (int i = 0; i < KC_COUNT; ++i) {
        out->kernel_ms[i] = h->kernel_ms[i];
        out->kernel_launches[i] = h->kernel_launches[i];
    }
    out->flops[KC_PROJECT] = st.fl[0];
    out->flops[KC_ANGLE] = st.fl_dir[0];
    out->flops[KC_STENCIL] = st.fl_dir[1];
    out->flops[KC_FACTOR] = st.fl[1];
    out->flops[KC_OUTPUT] = st.fl[2];
    return TT_OK;
}

// ---------------------------------------------------------------------------
// host linear algebra for the internal-rank diagnostic (small matrices, FP64)
// ---------------------------------------------------------------------------

// R factor (min(m, n) x n, row-major, upper trapezoidal) of the Householder
// QR of the m x n row-major matrix A (overwritten).
std::vector<double> host_qr_r(std::vector<double> A, int m, int n) {
    const int q = std::min(m, n);
    for (int k = 0; k < q; ++k) {
        double nrm = 0.0;
        for (int i = k; i < m; ++i) nrm += A[(size_t)i * n + k] * A[(size_t)i * n + k];
        nrm = std::sqrt(nrm);
        if (nrm == 0.0) continue;
        const double alpha = A[(size_t)k * n + k] > 0 ? -nrm : nrm;
        std::vector<double> v((size_t)(m - k));
        for (int i = k; i < m; ++i) v[i - k] = A[(size_t)i * n + k];
        v[0] -= alpha;
        double vv = 0.0;
        for (double x : v) vv += x * x;
        if (vv == 0.0) continue;
        for (int j = k; j < n; ++j) {
            double dot = 0.0;
            for (int i = k; i < m; ++i) dot += v[i - k] * A[(size_t)i * n + j];
            const double f = 2.0 * dot / vv;
            for (int i = k; i < m; ++i) A[(size_t)i * n + j] -= f * v[i - k];
        }
    }
    std::vector<double> R((size_t)q * n, 0.0);
    for (int i = 0; i < q; ++i)
        for (int j = i; j < n; ++j) R[(size_t)i * n + j] = A[(size_t)i * n + j];
    return R;
}

// Eigenvalues (descending) of the symmetric n x n row-major matrix A:
// Householder reduction to tridiagonal form, then bisection on the Sturm
// sequence count of each eigenvalue.
std::vector<double> host_sym_eigenvalues(std::vector<double> A, int n) {
    std::vector<double> d((size_t)n), e((size_t)std::max(n - 1, 0));
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;   // trailing block starts at k + 1
        double nrm = 0.0;
        for (int i = k + 1; i < n; ++i) nrm += A[(size_t)i * n + k] * A[(size_t)i * n + k];
        nrm = std::sqrt(nrm);
        if (nrm == 0.0) continue;
        const double alpha = A[(size_t)(k + 1) * n + k] > 0 ? -nrm : nrm;
        std::vector<double> v((size_t)m), p((size_t)m);
        for (int i = 0; i < m; ++i) v[i] = A[(size_t)(k + 1 + i) * n + k];
        v[0] -= alpha;
        double vv = 0.0;
        for (double x : v) vv += x * x;
        if (vv == 0.0) continue;
        const double beta = 2.0 / vv;
        // p = beta A v, w = p - (beta / 2) (v^T p) v;  A <- A - v w^T - w v^T on the trailing block
        for (int i = 0; i < m; ++i) {
            double s = 0.0;
            for (int j = 0; j < m; ++j) s += A[(size_t)(k + 1 + i) * n + k + 1 + j] * v[j];
            p[i] = beta * s;
        }
        double vp = 0.0;
        for (int i = 0; i < m; ++i) vp += v[i] * p[i];
        for (int i = 0; i < m; ++i) p[i] -= 0.5 * beta * vp * v[i];
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) A[(size_t)(k + 1 + i) * n + k + 1 + j] -= v[i] * p[j] + p[i] * v[j];
        A[(size_t)(k + 1) * n + k] = alpha;
        A[(size_t)k * n + k + 1] = alpha;
        for (int i = k + 2; i < n; ++i) A[(size_t)i * n + k] = A[(size_t)k * n + i] = 0.0;
    }
    for (int i = 0; i < n; ++i) d[i] = A[(size_t)i * n + i];
    for (int i = 0; i + 1 < n; ++i) e[i] = A[(size_t)(i + 1) * n + i];
    // Gershgorin interval
    double lo = 0.0, hi = 0.0;
    for (int i = 0; i < n; ++i) {
        const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(e[i]) : 0.0);
        lo = std::min(lo, d[i] - r);
        hi = std::max(hi, d[i] + r);
    }
    const double scale = std::max(std::fabs(lo), std::fabs(hi));
    auto count_below = [&](double x) {   // number of eigenvalues < x
        int c = 0;
        double q = 1.0;
        for (int i = 0; i < n; ++i) {
            q = d[i] - x - (i > 0 ? e[i - 1] * e[i - 1] / q : 0.0);
            if (q == 0.0) q = -1e-300 * std::max(scale, 1e-300);
            if (q < 0.0) ++c;
        }
        return c;
    };
    std::vector<double> ev((size_t)n);
    for (int k = 0; k < n; ++k) {   // k-th smallest
        double a = lo, b = hi;
        for (int it = 0; it < 200 && b - a > 4e-16 * std::max(scale, 1e-300); ++it) {
            const double mid = 0.5 * (a + b);
            if (count_below(mid) > k) b = mid; else a = mid;
        }
        ev[(size_t)(n - 1 - k)] = 0.5 * (a + b);
    }
    return ev;
}

// Smallest k >= 1 with sqrt(sum_{j >= k} s_j^2) <= delta * sqrt(sum_j s_j^2), s descending
int delta_rank_host(const std::vector<double>& s, double delta) {
    double tot = 0.0;
    for (double x : s) tot += x * x;
    double tail = tot;
    for (size_t k = 1; k <= s.size(); ++k) {
        tail -= s[k - 1] * s[k - 1];
        if (std::sqrt(std::max(tail, 0.0)) <= delta * std::sqrt(tot)) return (int)k;
    }
    return (int)s.size();
}

}  // namespace

// ---------------------------------------------------------------------------
// Persistent ragged small-solve kernel (k_solve_small)
// ---------------------------------------------------------------------------

// Why a handle cannot run in k_solve_small ("" when it can).
std::string small_ineligible(const tt_handle* h) {
    const Plan& P = h->P;
    if (h->precision != TT_PREC_FP64) return "FP64 data only";
    if (h->round_method != TT_ROUND_QR) return "Householder QR rounding only";
    if (P.KPt != 16) return "a projected first core of at most 16 columns only";
    if (h->step_order != 0) return "one rounding per step only";
    if (P.prepass) return "no coupled temperature or scattering";
    if (P.flux == TT_FLUX_HLL) return "the upwind or Rusanov flux only";
    if (!P.svd_fast) return "the SVD chain's fixed LDS layout is needed";
    if (h->pending != OP_NONE) return "an unrounded operator is pending";
    if (h->timing) return "per-kernel timing is on";
    return "";
}

SmallSolve small_desc(tt_handle* h, int n_steps) {
    const Plan& P = h->P;
    SmallSolve q;
    std::memset(&q, 0, sizeof(q));
    q.g = h->geom;
    q.op = h->ops[OP_FULL];
    q.st = h->st();
    q.Z[0] = (double*)(h->ws + P.o_Z0);
    q.Z[1] = (double*)(h->ws + P.o_Z1);
    q.Th[0] = h->at<double>(P.o_Th0);
    q.Th[1] = h->at<double>(P.o_Th1);
    q.Ph[0] = h->at<double>(P.o_Ph0);
    q.Ph[1] = h->at<double>(P.o_Ph1);
    q.gtab = h->at<double>(P.o_gtab);
    q.htab = h->at<double>(P.o_htab);
    q.sc = h->scratch();
    q.LTh = h->at<double>(P.o_LTh);
    q.QTh = h->at<double>(P.o_QTh);
    q.QPh = h->at<double>(P.o_QPh);
    q.Gop = h->at<double>(P.o_G);
    q.B = h->at<double>(P.o_B);
    q.V = h->at<double>(P.o_V);
    q.R = h->at<double>(P.o_RA);
    q.sv = h->at<double>(P.o_sv);
    q.rd = h->rowdata();
    q.tol = h->tol;
    q.k1cap = P.k1cap;
    q.cap1 = std::min(P.cap, P.r1cap);
    q.cap2 = std::min(P.cap, P.r2cap);
    q.n_steps = n_steps;
    // Z and the small cores flip together; both start at the handle's current parity
    q.zcur0 = h->zcur;
    return q;
}

// ---------------------------------------------------------------------------
// Launch-shape tuning
// ---------------------------------------------------------------------------
//
// The persistent contraction kernels (FP64 MFMA projection and output, fused
// FP32 projection + Gram and output) and the Gram of a stored first core take
// their grid from the plan.  How many blocks run best depends on the shape
// (rows, columns, K) and on how many blocks of the kernel fit a CU at its
// register and LDS use, so the tuner times candidate grids on the handle's
// own state and keeps the fastest, and a cache file keyed by device and shape
// saves the timing next time.
namespace {

struct TuneUse {
    bool project, output, gram;
};

// Which tunable kernels the plan's rounding pass launches.
TuneUse tune_use(const tt_handle* h) {
    const Plan& P = h->P;
    TuneUse u{false, false, false};
    u.project = u.output = P.f64mm || P.fused;
    u.gram = h->round_method != TT_ROUND_QR && !P.fused && !(P.f64mm && P.nct_f <= 4);
    return u;
}

void launch_current(const tt_handle* h, tt_tuning* t) {
    const Plan& P = h->P;
    const TuneUse u = tune_use(h);
    *t = tt_tuning{};
    t->project_blocks = !u.project ? 0 : (P.f64mm ? P.f64_blocks : P.fused_blocks);
    t->output_blocks = !u.output ? 0 : (P.f64mm ? P.f64_blocks_o : P.fused_blocks_o);
    t->gram_blocks = u.gram ? P.Pg : 0;
}

void launch_maximum(const tt_handle* h, tt_tuning* t) {
    const Plan& P = h->P;
    const TuneUse u = tune_use(h);
    *t = tt_tuning{};
    t->project_blocks = !u.project ? 0 : (P.f64mm ? P.f64_blocks_max : P.fused_blocks_max);
    t->output_blocks = !u.output ? 0 : (P.f64mm ? P.f64_blocks_max : P.fused_blocks_max);
    t->gram_blocks = u.gram ? P.Pg_max : 0;
}

// Rows per Gram block for about `nb` blocks: a multiple of 16, at least 64.
long long gram_rows_for(const Plan& P, int nb) {
    long long rows = std::max<long long>(64, (P.M + nb - 1) / nb);
    return (rows + 15) / 16 * 16;
}

// Check the shapes of `t` (0: keep) against the plan; message on failure.
bool launch_valid(const tt_handle* h, const tt_tuning& t, std::string* why) {
    tt_tuning mx;
    launch_maximum(h, &mx);
    auto check = [&](int v, int m, const char* name) {
        if (v == 0) return true;
        if (m == 0) {
            *why = std::string("this plan launches no tunable ") + name + " kernel";
            return false;
        }
        if (v < 1 || v > m) {
            *why = std::string(name) + " blocks must be in [1, " + std::to_string(m) + "], got " + std::to_string(v);
            return false;
        }
        return true;
    };
    return check(t.project_blocks, mx.project_blocks, "projection") &&
           check(t.output_blocks, mx.output_blocks, "output") && check(t.gram_blocks, mx.gram_blocks, "Gram");
}

// Set the shapes of `t` (0: keep); `t` must be valid.
void launch_apply(tt_handle* h, const tt_tuning& t) {
    Plan& P = h->P;
    if (t.project_blocks > 0) (P.f64mm ? P.f64_blocks : P.fused_blocks) = t.project_blocks;
    if (t.output_blocks > 0) (P.f64mm ? P.f64_blocks_o : P.fused_blocks_o) = t.output_blocks;
    if (t.gram_blocks > 0) {
        P.rowsg = gram_rows_for(P, t.gram_blocks);
        P.Pg = (int)((P.M + P.rowsg - 1) / P.rowsg);
    }
}

// Cache key: the device and the problem's shape (the plan's caps, not the
// current ranks), so that a new handle of the same problem finds the grids
// tuned at another handle's steady state.
std::string tune_key(const tt_handle* h, int opkind) {
    const Plan& P = h->P;
    int dev = 0;
    hipDeviceProp_t prop{};
    std::string arch = "unknown";
    int cus = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        arch = prop.gcnArchName;
        cus = prop.multiProcessorCount;
    }
    for (char& c : arch)
        if (c == ' ' || c == '\t' || c == '\n') c = '_';
    char buf[512];
    snprintf(buf, sizeof buf, "%s/cu%d/prec%d/route%d/M%lld/G%d/dim%d/ang%dx%d/cap%d/R1cap%d/k1cap%d/fused%d/hll%d",
             arch.c_str(), cus, h->precision, h->round_method, P.M, P.G, P.dim, P.nt, P.np, P.cap, P.R1cap,
             P.k1cap, P.fused ? 1 : 0, h->ops[opkind].hll ? 1 : 0);
    return buf;
}

// The last entry for `key` in the cache file (lines "key project output gram").
bool cache_lookup(const char* path, const std::string& key, tt_tuning* out) {
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char line[1024], k[600];
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        int a = 0, b = 0, c = 0;
        if (sscanf(line, "%599s %d %d %d", k, &a, &b, &c) == 4 && key == k) {
            *out = tt_tuning{};
            out->project_blocks = a;
            out->output_blocks = b;
            out->gram_blocks = c;
            found = true;
        }
    }
    fclose(f);
    return found;
}

// Average duration (ms) of one launch of `launch` on `s`: one untimed launch,
// a timed one that sets the batch size (about 20 ms of launches, at most 20),
// then the best of two timed batches.
template <class F>
tt_status time_launch(F&& launch, hipStream_t s, hipEvent_t e0, hipEvent_t e1, double* out) {
    float ms = 0.f;
    launch();
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(e0, s));
    launch();
    HIP_TRY(hipEventRecord(e1, s));
    HIP_TRY(hipEventSynchronize(e1));
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    const int reps = std::max(1, std::min(20, (int)(20.0 / std::max(ms, 1e-3f))));
    double best = ms;
    for (int b = 0; b < 2; ++b) {
        HIP_TRY(hipEventRecord(e0, s));
        for (int i = 0; i < reps; ++i) launch();
        HIP_TRY(hipEventRecord(e1, s));
        HIP_TRY(hipEventSynchronize(e1));
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        best = std::min(best, (double)ms / reps);
    }
    HIP_TRY(hipGetLastError());
    *out = best;
    return TT_OK;
}

// Grid candidates up to `maxb`, the default first.
std::vector<int> grid_candidates(int def, int maxb) {
    static const int base[] = {64, 128, 192, 256, 384, 512, 768, 1024};
    std::vector<int> c{def};
    for (int b : base)
        if (b <= maxb && b != def) c.push_back(b);
    return c;
}

// Time every candidate of one kernel (`set` installs a shape, `run` launches
// the kernel) and keep the fastest, unless it is within 2 % of the default.
template <class Set, class Run>
tt_status tune_one(const std::vector<int>& cand, Set&& set, Run&& run, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                   int* best_out, double* best_ms, double* def_ms) {
    std::vector<double> t(cand.size(), 0.0);
    for (size_t i = 0; i < cand.size(); ++i) {
        set(cand[i]);
        const tt_status r = time_launch(run, s, e0, e1, &t[i]);
        if (r != TT_OK) return r;
    }
    size_t b = 0;
    for (size_t i = 1; i < cand.size(); ++i)
        if (t[i] < t[b]) b = i;
    if (b != 0 && t[b] > 0.98 * t[0]) b = 0;
    set(cand[b]);
    *best_out = cand[b];
    *best_ms = t[b];
    *def_ms = t[0];
    return TT_OK;
}

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

template <typename T>
tt_status tune_impl(tt_handle* h, const char* cache, tt_tuning* out, hipStream_t s) {
    Plan& P = h->P;
    const TuneUse u = tune_use(h);
    const int opkind = h->step_order == 1 ? OP_TRANSPORT : OP_FULL;
    const OpDesc& op = h->ops[opkind];
    const std::string key = tune_key(h, opkind);
    if (cache) {
        tt_tuning c;
        std::string why;
        if (cache_lookup(cache, key, &c) && launch_valid(h, c, &why)) {
            launch_apply(h, c);
            launch_current(h, out);
            out->from_cache = 1;
            return TT_OK;
        }
        FILE* f = fopen(cache, "a");
        if (!f) return fail(TT_ERR_INVALID_ARG, std::string("cannot write the tuning cache ") + cache);
        fclose(f);
    }
    // the gather operand and the pending sum's shapes for the current state
    // (the next rounding pass recomputes the same)
    launch_prep<T>(h, opkind, s);
    HIP_TRY(hipGetLastError());
    EventPair ev;
    HIP_TRY(hipEventCreate(&ev.a));
    HIP_TRY(hipEventCreate(&ev.b));
    tt_tuning res;
    launch_current(h, &res);
    tt_tuning mx;
    launch_maximum(h, &mx);
    tt_status r = TT_OK;
    if (u.project) {
        auto set = [&](int nb) { (P.f64mm ? P.f64_blocks : P.fused_blocks) = nb; };
        auto run = [&]() {
            if (P.f64mm)
                (void)launch_project<T>(h, opkind, s);
            else if (P.nct_p == 4)
                launch_fused_project<4>(h, opkind, s);
            else
                launch_fused_project<2>(h, opkind, s);
        };
        r = tune_one(grid_candidates(res.project_blocks, mx.project_blocks), set, run, s, ev.a, ev.b,
                     &res.project_blocks, &res.project_ms, &res.project_ms_default);
        if (r != TT_OK) return r;
    }
    if (u.gram) {
        r = launch_project<T>(h, opkind, s);   // B for the Gram
        if (r != TT_OK) return r;
        std::vector<int> cand{P.Pg};
        for (int nb : {256, 384, 512, 768, 1024}) {
            if (nb > mx.gram_blocks) continue;
            const long long rows = gram_rows_for(P, nb);
            const int pg = (int)((P.M + rows - 1) / rows);
            if (std::find(cand.begin(), cand.end(), pg) == cand.end()) cand.push_back(pg);
        }
        auto set = [&](int nb) {
            P.rowsg = gram_rows_for(P, nb);
            P.Pg = (int)((P.M + P.rowsg - 1) / P.rowsg);
        };
        auto run = [&]() { launch_gram_parts<T>(h, s); };
        r = tune_one(cand, set, run, s, ev.a, ev.b, &res.gram_blocks, &res.gram_ms, &res.gram_ms_default);
        if (r != TT_OK) return r;
    }
    if (u.output) {
        auto set = [&](int nb) { (P.f64mm ? P.f64_blocks_o : P.fused_blocks_o) = nb; };
        auto run = [&]() {
            if (P.f64mm)
                output_f64(h, op, s);
            else if (P.nct_o == 4)
                launch_fused_output<4>(h, opkind, s);
            else
                launch_fused_output<2>(h, opkind, s);
        };
        r = tune_one(grid_candidates(res.output_blocks, mx.output_blocks), set, run, s, ev.a, ev.b,
                     &res.output_blocks, &res.output_ms, &res.output_ms_default);
        if (r != TT_OK) return r;
    }
    launch_current(h, out);
    out->project_ms = res.project_ms;
    out->output_ms = res.output_ms;
    out->gram_ms = res.gram_ms;
    out->project_ms_default = res.project_ms_default;
    out->output_ms_default = res.output_ms_default;
    out->gram_ms_default = res.gram_ms_default;
    out->from_cache = 0;
    if (cache) {
        FILE* f = fopen(cache, "a");
        if (!f) return fail(TT_ERR_INVALID_ARG, std::string("cannot write the tuning cache ") + cache);
        fprintf(f, "%s %d %d %d\n", key.c_str(), out->project_blocks, out->output_blocks, out->gram_blocks);
        fclose(f);
    }
    return TT_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Static workspace for tt_transport_create_noalloc
// ---------------------------------------------------------------------------
//
// A file-scope device array: every GPU the library runs on holds its own copy
// from module load until the process ends.  Host code never passes its name
// to a kernel or a copy (in host code the name is a host-side stand-in):
// each device's address is taken once, with that device current, by
// hipGetSymbolAddress and kept here.  One handle at a time may hold a
// device's array; the array keeps the last handle's contents, and create
// initialises every part of the workspace a solve reads.
namespace {
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
tt_handle* g_scratch_owner[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
// Address of the current device's static workspace (taken on the first call
// on that device).  Call with g_scratch_mu held.
tt_status scratch_address(int dev, void** out) {
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(TT_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return TT_OK;
}
}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

size_t tt_transport_workspace_bytes(const tt_problem* p) {
    Plan P;
    if (make_plan(p, P) != TT_OK) return 0;
    return P.bytes;
}

tt_status tt_transport_group_emission(const double* edges, int n_groups, double T, double* out) {
    if (!edges || !out || n_groups < 1) return fail(TT_ERR_INVALID_ARG, "bad arguments");
    ttrt::group_emission(edges, n_groups, T, out);
    return TT_OK;
}

tt_status tt_transport_create(const tt_problem* p, void* dev_workspace, size_t bytes, void* stream, tt_handle** out) {
    if (!out) return fail(TT_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    Plan P;
    tt_status r = make_plan(p, P);
    if (r != TT_OK) return r;
    if (!dev_workspace) return fail(TT_ERR_INVALID_ARG, "workspace is NULL");
    if (bytes < P.bytes) return fail(TT_ERR_OOM, "workspace too small: need " + std::to_string(P.bytes) + " bytes");
    if (((uintptr_t)dev_workspace) & 255) return fail(TT_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    for (long long i = 0; i < P.NX; ++i)
        if (!(p->T_cell[i] >= 0.0) || !std::isfinite(p->T_cell[i]))
            return fail(TT_ERR_INVALID_ARG, "T_cell must be finite and >= 0");
    if (p->kappa_s_full)
        for (long long k = 0; k < P.M; ++k)
            if (!(p->kappa_s_full[k] >= 0.0) || !std::isfinite(p->kappa_s_full[k]))
                return fail(TT_ERR_INVALID_ARG, "kappa_s_full must be finite and >= 0");
    if (p->kappa_full) {
        for (long long k = 0; k < P.M; ++k)
            if (!(p->kappa_full[k] >= 0.0) || !std::isfinite(p->kappa_full[k]))
                return fail(TT_ERR_INVALID_ARG, "kappa_full must be finite and >= 0");
    } else {
        for (long long i = 0; i < P.NX; ++i)
            if (!(p->kappa0[i] >= 0.0) || !std::isfinite(p->kappa0[i]))
                return fail(TT_ERR_INVALID_ARG, "kappa0 must be finite and >= 0");
        for (int g = 0; g < P.G; ++g)
            if (!(p->kappa_group_scale[g] >= 0.0) || !std::isfinite(p->kappa_group_scale[g]))
                return fail(TT_ERR_INVALID_ARG, "kappa_group_scale must be finite and >= 0");
    }
    {
        static bool attrs_set = false;
        if (!attrs_set) {
            HIP_TRY(hipFuncSetAttribute((const void*)k_prep<double>, hipFuncAttributeMaxDynamicSharedMemorySize, kSmallLdsBytes));
            HIP_TRY(hipFuncSetAttribute((const void*)k_prep<float>, hipFuncAttributeMaxDynamicSharedMemorySize, kSmallLdsBytes));
            HIP_TRY(hipFuncSetAttribute((const void*)k_svd_chain<double, true>, hipFuncAttributeMaxDynamicSharedMemorySize, kSmallLdsBytes));
            HIP_TRY(hipFuncSetAttribute((const void*)k_svd_chain<float, true>, hipFuncAttributeMaxDynamicSharedMemorySize, kSmallLdsBytes));
            HIP_TRY(hipFuncSetAttribute((const void*)k_svd_chain<double, false>, hipFuncAttributeMaxDynamicSharedMemorySize, kSmallLdsBytes));
            HIP_TRY(hipFuncSetAttribute((const void*)k_svd_chain<float, false>, hipFuncAttributeMaxDynamicSharedMemorySize, kSmallLdsBytes));
            HIP_TRY(hipFuncSetAttribute((const void*)k_rand_sketch, hipFuncAttributeMaxDynamicSharedMemorySize, kSmallLdsBytes));
            HIP_TRY(hipFuncSetAttribute((const void*)k_fused_f32<2, true>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
            HIP_TRY(hipFuncSetAttribute((const void*)k_fused_f32<4, true>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
            HIP_TRY(hipFuncSetAttribute((const void*)k_fused_f32<2, false>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
            HIP_TRY(hipFuncSetAttribute((const void*)k_fused_f32<4, false>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
            // the FP64 MFMA kernels: their own dynamic LDS (they also hold a little static LDS)
            const std::pair<const void*, size_t> f64k[] = {
                {(const void*)k_mm_f64<MODE_PROJECT, 1, false, 2>, f64_lds_bytes(1, false, 2)},
                {(const void*)k_mm_f64<MODE_PROJECT, 1, true, 2>, f64_lds_bytes(1, true, 2)},
                {(const void*)k_mm_f64<MODE_PROJECT, 2, false, 2>, f64_lds_bytes(2, false, 2)},
                {(const void*)k_mm_f64<MODE_PROJECT, 2, true, 2>, f64_lds_bytes(2, true, 2)},
                {(const void*)k_mm_f64<MODE_PROJECT, 4, false, 2>, f64_lds_bytes(4, false, 2)},
                {(const void*)k_mm_f64<MODE_PROJECT, 4, true, 1>, f64_lds_bytes(4, true, 1)},
                {(const void*)k_mm_f64<MODE_PROJECT, 8, false, 1>, f64_lds_bytes(8, false, 1)},
                {(const void*)k_mm_f64<MODE_ANGLE, 8, false, 1>, f64_lds_bytes(8, false, 1, false, kF64AngChunks)},
                {(const void*)k_mm_f64<MODE_OUTPUT, 1, false, 2>, f64_lds_bytes(1, false, 2, false, kF64OutChunks)},
                {(const void*)k_mm_f64<MODE_OUTPUT, 2, false, 2>, f64_lds_bytes(2, false, 2, false, kF64OutChunks)},
                {(const void*)k_mm_f64<MODE_OUTPUT, 4, false, 2>, f64_lds_bytes(4, false, 2, false, kF64OutChunks)},
                {(const void*)k_mm_f64<MODE_PROJECT, 1, false, 2, true>, f64_lds_bytes(1, false, 2, true)},
                {(const void*)k_mm_f64<MODE_PROJECT, 1, true, 2, true>, f64_lds_bytes(1, true, 2, true)},
                {(const void*)k_mm_f64<MODE_PROJECT, 2, false, 2, true>, f64_lds_bytes(2, false, 2, true)},
                {(const void*)k_mm_f64<MODE_PROJECT, 2, true, 2, true>, f64_lds_bytes(2, true, 2, true)},
                {(const void*)k_mm_f64<MODE_PROJECT, 4, false, 2, true>, f64_lds_bytes(4, false, 2, true)},
                {(const void*)k_mm_f64<MODE_PROJECT, 4, true, 1, true>, f64_lds_bytes(4, true, 1, true)},
                {(const void*)k_mm_f64<MODE_PROJECT, 8, false, 1, true>, f64_lds_bytes(8, false, 1, true)}};
            for (const auto& fk : f64k)
                HIP_TRY(hipFuncSetAttribute(fk.first, hipFuncAttributeMaxDynamicSharedMemorySize, (int)fk.second));
            attrs_set = true;
        }
    }
    hipStream_t s = (hipStream_t)stream;
    tt_handle* h = new tt_handle();
    h->P = P;
    h->precision = p->precision;
    h->round_method = p->round_method == TT_ROUND_AUTO
                          ? (p->precision == TT_PREC_FP64 ? TT_ROUND_QR : TT_ROUND_GRAM)
                          : p->round_method;
    h->step_order = p->paper_step_order;
    h->rand_p = p->rand_oversample;
    h->rand_seed = p->rand_seed;
    h->tol = p->tol;
    h->ws = (char*)dev_workspace;
    h->create_stream = s;
    // geometry and time step: dt = cfl / (c sum_d 1/dx_d)
    Geom& g = h->geom;
    g.dim = P.dim; g.nx = P.nx; g.ny = P.ny; g.nz = P.nz; g.G = P.G; g.M = P.M; g.nt = P.nt; g.np = P.np;
    g.n_terms = P.n_terms; g.n_bc = P.n_bc;
    double inv = 0.0;
    h->dV = 1.0;
    for (int d = 0; d < P.dim; ++d) {
        const double dx = p->extent[d] / p->n_cells[d];
        inv += 1.0 / dx;
        h->dV *= dx;
    }
    h->dt = p->cfl / (p->c * inv);
    g.cdt = p->c * h->dt;
    for (int d = 0; d < 3; ++d) {
        g.periodic[d] = (d < P.dim && p->bc[2 * d] == TT_BC_PERIODIC) ? 1 : 0;
        g.lam[d] = d < P.dim ? p->c * h->dt / (p->extent[d] / p->n_cells[d]) : 0.0;
        g.dx[d] = d < P.dim ? p->extent[d] / p->n_cells[d] : 1.0;
    }
    g.hbeta = p->flux == TT_FLUX_HLL ? p->hll_beta : 0.0;
    {
        int q = 0;
        for (int f = 0; f < 2 * P.dim; ++f)
            if (is_inflow(p->bc[f])) g.bc_face[q++] = f;
    }
    build_ops(h, p);
    h->w_theta.assign(p->w_theta, p->w_theta + P.nt);
    h->w_phi.assign(p->w_phi, p->w_phi + P.np);
    // emission per merged row, from the distinct cell temperatures
    std::vector<double> eps((size_t)P.M);
    {
        std::map<double, std::vector<double>> cache;
        for (long long c = 0; c < P.NX; ++c) {
            auto it = cache.find(p->T_cell[c]);
            if (it == cache.end()) {
                std::vector<double> e((size_t)P.G);
                ttrt::group_emission(p->group_edges, P.G, p->T_cell[c], e.data());
                it = cache.emplace(p->T_cell[c], std::move(e)).first;
            }
            std::copy(it->second.begin(), it->second.end(), eps.begin() + c * P.G);
        }
    }
    h->eps_host = eps;
    h->T_host.assign(p->T_cell, p->T_cell + P.NX);
    h->heat_capacity = p->heat_capacity;
    h->c = p->c;
    // initial radiation: isotropic Planck at T_rad0 when given, else at the medium temperature
    h->init_host = eps;
    if (p->T_rad0) {
        std::vector<double> e((size_t)P.G);
        for (long long c = 0; c < P.NX; ++c) {
            ttrt::group_emission(p->group_edges, P.G, p->T_rad0[c], e.data());
            std::copy(e.begin(), e.end(), h->init_host.begin() + c * P.G);
        }
    }
    for (int q = 0; q < h->ops[OP_FULL].n_r1; ++q)
        if (h->ops[OP_FULL].r1kind[q] == 0) h->qe_full = q;
    for (int q = 0; q < h->ops[OP_SOURCE].n_r1; ++q)
        if (h->ops[OP_SOURCE].r1kind[q] == 0) h->qe_source = q;
    std::vector<double> ghost((size_t)6 * P.G, 0.0);
    for (int f = 0; f < 2 * P.dim; ++f) {
        if (p->bc[f] == TT_BC_INFLOW_PLANCK) ttrt::group_emission(p->group_edges, P.G, p->bc_T[f], &ghost[(size_t)f * P.G]);
        if (p->bc[f] == TT_BC_INFLOW_VALUES)
            for (int gg = 0; gg < P.G; ++gg) ghost[(size_t)f * P.G + gg] = p->bc_values[(size_t)f * P.G + gg];
    }
    // angular factors of each operator term: g(l) h(p) = positive / negative part
    // of n_d (upwind), or rows 1 + 2 d = n_d and 2 + 2 d = 1 (Rusanov)
    const int nf = 1 + P.n_terms;
    std::vector<double> gtab((size_t)nf * P.nt, 1.0), htab((size_t)nf * P.np, 1.0);
    for (int axis = 0; axis < P.dim; ++axis) {
        for (int si = 0; si < 2; ++si) {
            const int t = 1 + 2 * axis + si;
            const bool pos = si == 0;
            for (int l = 0; l < P.nt; ++l) {
                const double mu = p->mu[l];
                const double st = std::sqrt(std::max(0.0, 1.0 - mu * mu));
                double gv;
                if (P.flux == TT_FLUX_RUSANOV) gv = pos ? ((P.dim == 1 || axis == 2) ? mu : st) : 1.0;
                else if (P.dim == 1 || axis == 2) gv = pos ? std::max(mu, 0.0) : std::min(mu, 0.0);
                else gv = st;
                gtab[(size_t)t * P.nt + l] = gv;
            }
            for (int pp = 0; pp < P.np; ++pp) {
                double hv = 1.0;
                if (P.dim > 1 && axis < 2) {
                    const double v = axis == 0 ? std::cos(p->phi[pp]) : std::sin(p->phi[pp]);
                    if (P.flux == TT_FLUX_RUSANOV) hv = pos ? v : 1.0;
                    else hv = pos ? std::max(v, 0.0) : std::min(v, 0.0);
                }
                htab[(size_t)t * P.np + pp] = hv;
            }
        }
    }
    // with kappa_full the factored arrays are unused (zero-filled)
    std::vector<double> k0((size_t)P.NX, 0.0), ks((size_t)P.G, 0.0);
    if (!p->kappa_full) {
        k0.assign(p->kappa0, p->kappa0 + P.NX);
        ks.assign(p->kappa_group_scale, p->kappa_group_scale + P.G);
    }
    tt_status u;
    if (p->kappa_full) {
        std::vector<double> kf(p->kappa_full, p->kappa_full + P.M);
        if ((u = upload(h->at<double>(P.o_kfull), kf, s)) != TT_OK) { delete h; return u; }
    }
    if ((u = upload(h->at<double>(P.o_k0), k0, s)) != TT_OK) { delete h; return u; }
    if ((u = upload(h->at<double>(P.o_ks), ks, s)) != TT_OK) { delete h; return u; }
    if ((u = upload(h->at<double>(P.o_eps), eps, s)) != TT_OK) { delete h; return u; }
    if ((u = upload(h->at<double>(P.o_ghost), ghost, s)) != TT_OK) { delete h; return u; }
    if ((u = upload(h->at<double>(P.o_gtab), gtab, s)) != TT_OK) { delete h; return u; }
    if ((u = upload(h->at<double>(P.o_htab), htab, s)) != TT_OK) { delete h; return u; }
    if (P.kscat) {
        std::vector<double> ksv(p->kappa_s_full, p->kappa_s_full + P.M);
        if ((u = upload(h->at<double>(P.o_kscat), ksv, s)) != TT_OK) { delete h; return u; }
        if (hipMemsetAsync(h->ws + P.o_jn, 0, (size_t)P.M * sizeof(double), s) != hipSuccess) { delete h; return fail(TT_ERR_HIP, "memset"); }
    }
    if (P.coupled)
        if ((u = upload(h->at<double>(P.o_T0), h->T_host, s)) != TT_OK) { delete h; return u; }
    if (P.prepass) {
        std::vector<double> edges(p->group_edges, p->group_edges + P.G + 1);
        if ((u = upload(h->at<double>(P.o_edges), edges, s)) != TT_OK) { delete h; return u; }
        if ((u = upload(h->at<double>(P.o_wth), h->w_theta, s)) != TT_OK) { delete h; return u; }
        if ((u = upload(h->at<double>(P.o_wph), h->w_phi, s)) != TT_OK) { delete h; return u; }
    }
    if (hipMemsetAsync(h->ws + P.o_G, 0, P.o_V - P.o_G, s) != hipSuccess) { delete h; return fail(TT_ERR_HIP, "memset"); }
    if (P.row_tables) {
        if (hipMemsetAsync(h->ws + P.o_zero, 0, 1024, s) != hipSuccess) { delete h; return fail(TT_ERR_HIP, "memset"); }
        const dim3 gr((unsigned)((P.M + 255) / 256));
        hipLaunchKernelGGL(k_row_aux, gr, dim3(256), 0, s, h->geom, h->rowdata(), h->at<float2>(P.o_aux));
        hipLaunchKernelGGL(k_nbr_table, gr, dim3(256), 0, s, h->geom, h->ops[OP_FULL], P.n_terms, h->at<int>(P.o_nbr));
        if (P.rw1 > 0)
            hipLaunchKernelGGL(k_rank1_rows, gr, dim3(256), 0, s, h->geom, h->ops[h->step_order ? OP_TRANSPORT : OP_FULL],
                               h->rowdata(), P.rw1, h->at<float>(P.o_R1));
        if (P.rw2 > 0)
            hipLaunchKernelGGL(k_rank1_rows, gr, dim3(256), 0, s, h->geom, h->ops[OP_SOURCE], h->rowdata(), P.rw2,
                               h->at<float>(P.o_R2));
        if (hipGetLastError() != hipSuccess) { delete h; return fail(TT_ERR_HIP, "row table launch"); }
    }
    if ((u = reset_impl(h, s)) != TT_OK) { delete h; return u; }
    *out = h;
    return TT_OK;
}

tt_status tt_transport_create_noalloc(const tt_problem* p, void* stream, tt_handle** out) {
    if (!out) return fail(TT_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    Plan P;
    tt_status r = make_plan(p, P);
    if (r != TT_OK) return r;
    if (P.bytes > kNoAllocBytes)
        return fail(TT_ERR_INVALID_ARG, "the problem needs " + std::to_string(P.bytes) +
                                            " bytes of workspace, above the static workspace of " +
                                            std::to_string(kNoAllocBytes) + " bytes: use tt_transport_create");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(TT_ERR_INVALID_ARG, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_owner[dev])
        return fail(TT_ERR_STATE, "the static workspace of this device is held by another handle: destroy it first");
    void* ws = nullptr;
    r = scratch_address(dev, &ws);
    if (r != TT_OK) return r;
    r = tt_transport_create(p, ws, kNoAllocBytes, stream, out);
    if (r != TT_OK) return r;
    (*out)->noalloc_dev = dev;
    g_scratch_owner[dev] = *out;
    return TT_OK;
}

tt_status tt_transport_reset(tt_handle* h, void* stream) {
    if (!h) return fail(TT_ERR_INVALID_ARG, "handle is NULL");
    return reset_impl(h, (hipStream_t)stream);
}

tt_status tt_transport_apply_op(tt_handle* h, void* stream) {
    (void)stream;
    if (!h) return fail(TT_ERR_INVALID_ARG, "handle is NULL");
    if (h->pending != OP_NONE) return fail(TT_ERR_STATE, "an unrounded operator is already pending");
    if (h->P.prepass)
        return fail(TT_ERR_STATE, "a coupled-temperature or scattering problem advances only by whole steps (solve / step_batch)");
    h->pending = h->step_order == 1 ? OP_TRANSPORT : OP_FULL;
    return TT_OK;
}

tt_status tt_transport_round(tt_handle* h, double tol, int rank_cap, void* stream) {
    if (!h) return fail(TT_ERR_INVALID_ARG, "handle is NULL");
    if (!(tol >= 0.0) || rank_cap < 1) return fail(TT_ERR_INVALID_ARG, "need tol >= 0 and rank_cap >= 1");
    if (rank_cap > h->P.cap) rank_cap = h->P.cap;
    const int op = h->pending;
    h->pending = OP_NONE;
    return round_dispatch(h, op, tol, rank_cap, (hipStream_t)stream);
}

namespace {
// Capture two steps of h on stream s into the graph of the current parity.
tt_status capture_two_steps(tt_handle* h, hipStream_t s) {
    const int par = h->zcur;
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    tt_status r = step_impl(h, s);
    if (r == TT_OK) r = step_impl(h, s);
    hipGraph_t gph = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &gph);
    if (r != TT_OK) {
        if (gph) (void)hipGraphDestroy(gph);
        return r;
    }
    if (e != hipSuccess) return fail(TT_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    if (h->zcur != par) {
        (void)hipGraphDestroy(gph);
        return fail(TT_ERR_STATE, "two steps did not return to the captured buffer parity");
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t e2 = hipGraphInstantiate(&ex, gph, nullptr, nullptr, 0);
    if (e2 != hipSuccess) {
        (void)hipGraphDestroy(gph);
        return fail(TT_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
    }
    h->graph[par] = gph;
    h->graph_exec[par] = ex;
    return TT_OK;
}

void drop_graphs(tt_handle* h) {
    for (int i = 0; i < 2; ++i) {
        if (h->graph_exec[i]) (void)hipGraphExecDestroy(h->graph_exec[i]);
        if (h->graph[i]) (void)hipGraphDestroy(h->graph[i]);
        h->graph_exec[i] = nullptr;
        h->graph[i] = nullptr;
    }
}

// n_steps steps: graph replays of two steps while at least two remain (when
// graphs are on and the handle allows them), launched steps otherwise.
tt_status run_steps(tt_handle* h, int n_steps, hipStream_t s) {
    int i = 0;
    if (h->use_graph && !h->timing && h->pending == OP_NONE && s != nullptr) {
        for (; i + 2 <= n_steps; i += 2) {
            const int par = h->zcur;
            if (!h->graph_exec[par]) {
                tt_status r = capture_two_steps(h, s);
                if (r != TT_OK) return r;
            }
            HIP_TRY(hipGraphLaunch(h->graph_exec[par], s));
        }
    }
    for (; i < n_steps; ++i) {
        tt_status r = step_impl(h, s);
        if (r != TT_OK) return r;
        if (h->timing && h->ev_used > 4096) {
            HIP_TRY(hipStreamSynchronize(s));
            h->ev_collect();
        }
    }
    return TT_OK;
}
}  // namespace

tt_status tt_transport_tune(tt_handle* h, const char* cache_path, tt_tuning* out, void* stream) {
    if (!h || !out) return fail(TT_ERR_INVALID_ARG, "tune: NULL handle or out");
    if (h->pending != OP_NONE) return fail(TT_ERR_STATE, "tune: an unrounded operator is pending");
    hipStream_t s = (hipStream_t)stream;
    const tt_status r = h->precision == TT_PREC_FP64 ? tune_impl<double>(h, cache_path, out, s)
                                                     : tune_impl<float>(h, cache_path, out, s);
    drop_graphs(h);   // captured graphs hold the old grids
    return r;
}

tt_status tt_transport_set_launch(tt_handle* h, const tt_tuning* shapes) {
    if (!h || !shapes) return fail(TT_ERR_INVALID_ARG, "set_launch: NULL handle or shapes");
    std::string why;
    if (!launch_valid(h, *shapes, &why)) return fail(TT_ERR_INVALID_ARG, "set_launch: " + why);
    launch_apply(h, *shapes);
    drop_graphs(h);
    return TT_OK;
}

tt_status tt_transport_get_launch(tt_handle* h, tt_tuning* current, tt_tuning* maximum) {
    if (!h) return fail(TT_ERR_INVALID_ARG, "get_launch: NULL handle");
    if (current) launch_current(h, current);
    if (maximum) launch_maximum(h, maximum);
    return TT_OK;
}

tt_status tt_transport_set_graph(tt_handle* h, int on) {
    if (!h) return fail(TT_ERR_INVALID_ARG, "handle is NULL");
    h->use_graph = on != 0;
    if (!h->use_graph) drop_graphs(h);
    return TT_OK;
}

tt_status tt_transport_solve(tt_handle* h, int n_steps, tt_stats* out, void* stream) {
    if (!h) return fail(TT_ERR_INVALID_ARG, "handle is NULL");
    if (n_steps < 0) return fail(TT_ERR_INVALID_ARG, "n_steps must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    for (int i = 0; i < KC_COUNT; ++i) { h->kernel_ms[i] = 0; h->kernel_launches[i] = 0; h->flops[i] = 0; }
    {
        DevState st;
        tt_status r = read_state(h, st, s);
        if (r != TT_OK) return r;
        for (int i = 0; i < 4; ++i) st.fl[i] = 0.0;
        r = write_state(h, st, s);
        if (r != TT_OK) return r;
    }
    auto t0 = std::chrono::steady_clock::now();
    {
        tt_status r = run_steps(h, n_steps, s);
        if (r != TT_OK) return r;
    }
    HIP_TRY(hipStreamSynchronize(s));
    auto t1 = std::chrono::steady_clock::now();
    h->ev_collect();
    h->last_seconds = std::chrono::duration<double>(t1 - t0).count();
    h->last_steps = n_steps;
    if (out) {
        tt_status r = fill_stats(h, out, s);
        if (r != TT_OK) return r;
        if (out->nan_flag) return fail(TT_ERR_NUMERIC, "NaN or Inf in the TT state");
    }
    return TT_OK;
}

tt_status tt_transport_get_ranks(tt_handle* h, int* r1, int* r2) {
    if (!h) return fail(TT_ERR_INVALID_ARG, "handle is NULL");
    DevState st;
    tt_status r = read_state(h, st, h->create_stream);
    if (r != TT_OK) return r;
    if (r1) *r1 = st.r1;
    if (r2) *r2 = st.r2;
    return TT_OK;
}

tt_status tt_transport_get_cores(tt_handle* h, double* Z, double* Theta, double* Phi, void* stream) {
    if (!h) return fail(TT_ERR_INVALID_ARG, "handle is NULL");
    hipStream_t s = (hipStream_t)stream;
    const Plan& P = h->P;
    DevState st;
    tt_status r = read_state(h, st, s);
    if (r != TT_OK) return r;
    if (h->pending != OP_NONE) {
        // explicit TT sum: Z_new in row chunks through the B buffer, small cores directly
        const OpDesc& op = h->ops[h->pending];
        const int R1 = op.n_rblk * st.r1 + op.n_r1, R2 = op.n_rblk * st.r2 + op.n_r1;
        if (Z) {
            double* buf = h->at<double>(P.o_B);
            const long long cap_rows = std::max<long long>(1, (long long)(P.B_bytes / sizeof(double)) / R1);
            for (long long k0 = 0; k0 < P.M; k0 += cap_rows) {
                const long long nr = std::min(cap_rows, P.M - k0);
                if (h->precision == TT_PREC_FP64)
                    hipLaunchKernelGGL(k_materialize<double>, dim3(1024), dim3(256), 0, s, h->geom, op, (const DevState*)h->st(),
                                       (const double*)h->Zc(), h->rowdata(), k0, nr, buf);
                else
                    hipLaunchKernelGGL(k_materialize<float>, dim3(1024), dim3(256), 0, s, h->geom, op, (const DevState*)h->st(),
                                       (const float*)h->Zc(), h->rowdata(), k0, nr, buf);
                HIP_TRY(hipGetLastError());
                HIP_TRY(hipMemcpyAsync(Z + k0 * R1, buf, (size_t)nr * R1 * sizeof(double), hipMemcpyDeviceToHost, s));
                HIP_TRY(hipStreamSynchronize(s));
            }
        }
        hipLaunchKernelGGL(k_sum_small_cores, dim3(64), dim3(256), 0, s, h->geom, op, (const DevState*)h->st(),
                           (const double*)h->Thc(), (const double*)h->Phc(), (const double*)h->at<double>(P.o_gtab),
                           (const double*)h->at<double>(P.o_htab), h->at<double>(P.o_ThN), h->at<double>(P.o_PhN));
        HIP_TRY(hipGetLastError());
        if (Theta) HIP_TRY(hipMemcpyAsync(Theta, h->at<double>(P.o_ThN), (size_t)R1 * P.nt * R2 * sizeof(double), hipMemcpyDeviceToHost, s));
        if (Phi) HIP_TRY(hipMemcpyAsync(Phi, h->at<double>(P.o_PhN), (size_t)R2 * P.np * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        return TT_OK;
    }
    if (Z) {
        if (h->precision == TT_PREC_FP64) {
            std::vector<double> zb((size_t)P.M * st.ldz);
            HIP_TRY(hipMemcpyAsync(zb.data(), h->Zc(), zb.size() * sizeof(double), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            for (long long k = 0; k < P.M; ++k)
                for (int a = 0; a < st.r1; ++a) Z[(size_t)k * st.r1 + a] = zb[(size_t)k * st.ldz + a];
        } else {
            std::vector<float> zb((size_t)P.M * st.ldz);
            HIP_TRY(hipMemcpyAsync(zb.data(), h->Zc(), zb.size() * sizeof(float), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            for (long long k = 0; k < P.M; ++k)
                for (int a = 0; a < st.r1; ++a) Z[(size_t)k * st.r1 + a] = zb[(size_t)k * st.ldz + a];
        }
    }
    if (Theta) HIP_TRY(hipMemcpyAsync(Theta, h->Thc(), (size_t)st.r1 * P.nt * st.r2 * sizeof(double), hipMemcpyDeviceToHost, s));
    if (Phi) HIP_TRY(hipMemcpyAsync(Phi, h->Phc(), (size_t)st.r2 * P.np * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return TT_OK;
}

tt_status tt_transport_set_cores(tt_handle* h, int r1, int r2, const double* Z, const double* Theta, const double* Phi,
                                 void* stream) {
    if (!h) return fail(TT_ERR_INVALID_ARG, "handle is NULL");
    if (!Z || !Theta || !Phi) return fail(TT_ERR_INVALID_ARG, "cores must not be NULL");
    if (r1 < 1 || r2 < 1 || r1 > h->P.r1cap || r2 > h->P.r2cap)
        return fail(TT_ERR_INVALID_ARG, "ranks must be within [1, cap] (r1 <= " + std::to_string(h->P.r1cap) +
                                            ", r2 <= " + std::to_string(h->P.r2cap) + ")");
    hipStream_t s = (hipStream_t)stream;
    if (h->precision == TT_PREC_FP64) return set_cores_impl<double>(h, r1, r2, Z, Theta, Phi, s);
    return set_cores_impl<float>(h, r1, r2, Z, Theta, Phi, s);
}

tt_status tt_transport_internal_ranks(tt_handle* h, double delta, tt_internal_ranks* out, double* sv_nu, int n_sv_nu,
                                      double* sv_x, int n_sv_x, void* stream) {
    if (!h || !out) return fail(TT_ERR_INVALID_ARG, "handle and out must be non-NULL");
    if (!(delta >= 0.0)) return fail(TT_ERR_INVALID_ARG, "delta must be >= 0");
    const Plan& P = h->P;
    hipStream_t s = (hipStream_t)stream;
    DevState st;
    tt_status r = read_state(h, st, s);
    if (r != TT_OK) return r;
    if (h->pending != OP_NONE) return fail(TT_ERR_STATE, "an unrounded operator is pending");
    const int r1 = st.r1, r2 = st.r2, ldz = st.ldz, G = P.G, nt = P.nt, np = P.np;
    const long long NX = P.NX;
    const int n = G * ldz;
    if (n > 2048) return fail(TT_ERR_INVALID_ARG, "internal ranks: N_nu * ld(r1) above 2048 is not supported");
    // raw Gram of the N_X x (N_nu ldz) unfolding of Z on the device, in strips
    // of rows that fit the round scratch
    const int ntile = (n + 63) / 64;
    const int per = (int)std::min<size_t>((size_t)n, P.B_bytes / ((size_t)n * sizeof(double)));
    if (per < 1) return fail(TT_ERR_STATE, "internal ranks: round scratch below one row of the Gram");
    double* Gd = h->at<double>(P.o_B);
    std::vector<double> Gr((size_t)n * n), th((size_t)r1 * nt * r2), ph((size_t)r2 * np);
    for (int lo = 0; lo < n; lo += per) {
        const int hi = std::min(n, lo + per);
        const unsigned tiles_y = (unsigned)((hi - 1) / 64 - lo / 64 + 1);
        if (h->precision == TT_PREC_FP64)
            hipLaunchKernelGGL(k_unfold_gram<double>, dim3(ntile, tiles_y), dim3(256), 0, s, (const double*)h->Zc(),
                               NX, n, lo, hi, Gd);
        else
            hipLaunchKernelGGL(k_unfold_gram<float>, dim3(ntile, tiles_y), dim3(256), 0, s, (const float*)h->Zc(), NX,
                               n, lo, hi, Gd);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(Gr.data() + (size_t)lo * n, Gd, (size_t)(hi - lo) * n * sizeof(double),
                               hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipMemcpyAsync(th.data(), h->Thc(), th.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(ph.data(), h->Phc(), ph.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) Gr[(size_t)i * n + j] = Gr[(size_t)j * n + i];
    // right-orthonormal gauge: Phi = L_Phi Q_Phi, Theta x_3 L_Phi = L_Theta Q_Theta, Z' = Z L_Theta
    std::vector<double> pt((size_t)np * r2);
    for (int b = 0; b < r2; ++b)
        for (int p = 0; p < np; ++p) pt[(size_t)p * r2 + b] = ph[(size_t)b * np + p];
    const std::vector<double> Rp = host_qr_r(pt, np, r2);   // r2 x r2 (r2 <= N_phi)
    const int m2 = nt * r2;
    std::vector<double> tt((size_t)m2 * r1);                  // (Theta x_3 L_Phi) unfolding, transposed
    for (int a = 0; a < r1; ++a)
        for (int l = 0; l < nt; ++l)
            for (int c = 0; c < r2; ++c) {
                double v = 0.0;
                for (int b = c; b < r2; ++b) v += th[((size_t)a * nt + l) * r2 + b] * Rp[(size_t)c * r2 + b];
                tt[((size_t)l * r2 + c) * r1 + a] = v;
            }
    const int q = std::min(m2, r1);
    const std::vector<double> Rt = host_qr_r(tt, m2, r1);     // q x r1; L_Theta = Rt^T (r1 x q)
    // G_x = (L (x) I)^T G_raw (L (x) I) over (g, i) with i < q;  G_nu[g, g'] = sum_i G_x[(g,i),(g',i)]
    const int nx = G * q;
    std::vector<double> Gx((size_t)nx * nx), tmp((size_t)ldz * q);
    for (int g = 0; g < G; ++g)
        for (int g2 = 0; g2 < G; ++g2) {
            // block (g, g2) of G_raw is ldz x ldz; rows/cols a < r1 carry data
            for (int a = 0; a < r1; ++a)
                for (int j = 0; j < q; ++j) {
                    double v = 0.0;
                    for (int b = j; b < r1; ++b) v += Gr[(size_t)(g * ldz + a) * n + g2 * ldz + b] * Rt[(size_t)j * r1 + b];
                    tmp[(size_t)a * q + j] = v;
                }
            for (int i = 0; i < q; ++i)
                for (int j = 0; j < q; ++j) {
                    double v = 0.0;
                    for (int a = i; a < r1; ++a) v += Rt[(size_t)i * r1 + a] * tmp[(size_t)a * q + j];
                    Gx[(size_t)(g * q + i) * nx + g2 * q + j] = v;
                }
        }
    std::vector<double> Gn((size_t)G * G, 0.0);
    for (int g = 0; g < G; ++g)
        for (int g2 = 0; g2 < G; ++g2)
            for (int i = 0; i < q; ++i) Gn[(size_t)g * G + g2] += Gx[(size_t)(g * q + i) * nx + g2 * q + i];
    auto singular = [](std::vector<double> ev) {
        for (double& x : ev) x = std::sqrt(std::max(x, 0.0));
        return ev;
    };
    std::vector<double> s_nu = singular(host_sym_eigenvalues(Gn, G));
    std::vector<double> s_x = singular(host_sym_eigenvalues(Gx, nx));
    // a matrix with N_X rows has at most N_X nonzero singular values
    if ((long long)s_x.size() > NX) s_x.resize((size_t)NX);
    if ((long long)s_nu.size() > NX * q) s_nu.resize((size_t)(NX * q));
    const int r_nux = delta_rank_host(s_nu, delta), r_xnu = delta_rank_host(s_x, delta);
    const double n_tt = (double)NX * G * r1 + (double)nt * r1 * r2 + (double)np * r2;
    out->r_nux = r_nux;
    out->r_xnu = r_xnu;
    out->C_rel_nu = n_tt / ((double)G * r_nux + (double)NX * r_nux * r1 + (double)nt * r1 * r2 + (double)np * r2);
    out->C_rel_x = n_tt / ((double)NX * r_xnu + (double)G * r_xnu * r1 + (double)nt * r1 * r2 + (double)np * r2);
    out->n_sv_nu = (int)s_nu.size();
    out->n_sv_x = (int)s_x.size();
    if (sv_nu)
        for (int i = 0; i < std::min(n_sv_nu, (int)s_nu.size()); ++i) sv_nu[i] = s_nu[i];
    if (sv_x)
        for (int i = 0; i < std::min(n_sv_x, (int)s_x.size()); ++i) sv_x[i] = s_x[i];
    return TT_OK;
}

tt_status tt_transport_get_temperature(tt_handle* h, double* T, void* stream) {
    if (!h || !T) return fail(TT_ERR_INVALID_ARG, "handle and T must be non-NULL");
    const Plan& P = h->P;
    if (!P.coupled) {
        std::copy(h->T_host.begin(), h->T_host.end(), T);
        return TT_OK;
    }
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(T, h->ws + P.o_T, (size_t)P.NX * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return TT_OK;
}

tt_status tt_transport_get_stats(tt_handle* h, tt_stats* out) {
    if (!h || !out) return fail(TT_ERR_INVALID_ARG, "NULL argument");
    return fill_stats(h, out, h->create_stream);
}

tt_status tt_transport_set_timing(tt_handle* h, int on) {
    if (!h) return fail(TT_ERR_INVALID_ARG, "handle is NULL");
    h->timing = on != 0;
    return TT_OK;
}

tt_status tt_transport_step_batch(tt_handle** hs, int n, void** streams, int n_streams) {
    if (!hs || n < 0 || !streams || n_streams < 1) return fail(TT_ERR_INVALID_ARG, "bad arguments");
    for (int i = 0; i < n; ++i) {
        if (!hs[i]) return fail(TT_ERR_INVALID_ARG, "NULL handle");
        for (int j = i + 1; j < n; ++j)
            if (hs[i] == hs[j]) return fail(TT_ERR_INVALID_ARG, "handles must be distinct");
    }
    for (int i = 0; i < n; ++i) {
        tt_status r = step_impl(hs[i], (hipStream_t)streams[i % n_streams]);
        if (r != TT_OK) return r;
    }
    return TT_OK;
}

tt_status tt_transport_solve_batch(tt_handle** hs, int n, int n_steps, void** streams, int n_streams, tt_stats* out) {
    if (n_steps < 0) return fail(TT_ERR_INVALID_ARG, "n_steps must be >= 0");
    auto t0 = std::chrono::steady_clock::now();
    {
        tt_status r = tt_transport_step_batch(hs, 0, streams, n_streams);   // argument checks
        if (r != TT_OK) return r;
        for (int i = 0; i < n; ++i) {
            if (!hs[i]) return fail(TT_ERR_INVALID_ARG, "NULL handle");
            for (int j = i + 1; j < n; ++j)
                if (hs[i] == hs[j]) return fail(TT_ERR_INVALID_ARG, "handles must be distinct");
        }
    }
    // two steps of every handle at a time (one graph launch each for handles
    // with graphs on), interleaved across the streams
    int k = 0;
    for (; k + 2 <= n_steps; k += 2)
        for (int i = 0; i < n; ++i) {
            tt_status r = run_steps(hs[i], 2, (hipStream_t)streams[i % n_streams]);
            if (r != TT_OK) return r;
        }
    for (; k < n_steps; ++k) {
        tt_status r = tt_transport_step_batch(hs, n, streams, n_streams);
        if (r != TT_OK) return r;
    }
    for (int i = 0; i < n_streams; ++i) HIP_TRY(hipStreamSynchronize((hipStream_t)streams[i]));
    auto t1 = std::chrono::steady_clock::now();
    const double sec = std::chrono::duration<double>(t1 - t0).count();
    for (int i = 0; i < n; ++i) {
        hs[i]->last_seconds = sec;
        hs[i]->last_steps = n_steps;
        hs[i]->ev_collect();
        if (out) {
            tt_status r = fill_stats(hs[i], &out[i], (hipStream_t)streams[i % n_streams]);
            if (r != TT_OK) return r;
        }
    }
    return TT_OK;
}

tt_status tt_transport_solve_small_batch(tt_handle** hs, int n, const int* n_steps, void* stream, tt_stats* out) {
    if (!hs || n < 0 || (n > 0 && !n_steps)) return fail(TT_ERR_INVALID_ARG, "bad arguments");
    for (int i = 0; i < n; ++i) {
        if (!hs[i]) return fail(TT_ERR_INVALID_ARG, "NULL handle");
        if (n_steps[i] < 0) return fail(TT_ERR_INVALID_ARG, "n_steps must be >= 0");
        for (int j = i + 1; j < n; ++j)
            if (hs[i] == hs[j]) return fail(TT_ERR_INVALID_ARG, "handles must be distinct");
        const std::string why = small_ineligible(hs[i]);
        if (!why.empty()) return fail(TT_ERR_INVALID_ARG, "handle " + std::to_string(i) + ": " + why);
        if (hs[i]->zcur != hs[i]->ccur) return fail(TT_ERR_STATE, "handle " + std::to_string(i) + ": core parity");
    }
    hipStream_t s = (hipStream_t)stream;
    {
        static bool attr = false;
        if (!attr) {
            HIP_TRY(hipFuncSetAttribute((const void*)k_solve_small, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)kBatchLdsBytes));
            attr = true;
        }
    }
    auto t0 = std::chrono::steady_clock::now();
    for (int b0 = 0; b0 < n; b0 += kBatchMax) {
        const int nb = std::min(kBatchMax, n - b0);
        SmallBatch batch;
        std::memset(&batch, 0, sizeof(batch));
        for (int i = 0; i < nb; ++i) {
            tt_handle* h = hs[b0 + i];
            for (int c = 0; c < KC_COUNT; ++c) { h->kernel_ms[c] = 0; h->kernel_launches[c] = 0; h->flops[c] = 0; }
            DevState st;
            tt_status r = read_state(h, st, s);
            if (r != TT_OK) return r;
            for (int c = 0; c < 4; ++c) st.fl[c] = 0.0;
            r = write_state(h, st, s);
            if (r != TT_OK) return r;
            const SmallSolve q = small_desc(h, n_steps[b0 + i]);
            SmallSolve* dq = reinterpret_cast<SmallSolve*>(h->ws + h->P.o_desc);
            HIP_TRY(hipMemcpyAsync(dq, &q, sizeof(q), hipMemcpyHostToDevice, s));
            batch.req[i] = dq;
        }
        HIP_TRY(hipStreamSynchronize(s));   // the descriptors are in place (their host copies go out of scope)
        hipLaunchKernelGGL(k_solve_small, dim3(nb), dim3(kSmallThreads), kBatchLdsBytes, s, batch);
        HIP_TRY(hipGetLastError());
        for (int i = 0; i < nb; ++i) {
            tt_handle* h = hs[b0 + i];
            if (n_steps[b0 + i] & 1) {
                h->zcur ^= 1;
                h->ccur ^= 1;
            }
        }
    }
    HIP_TRY(hipStreamSynchronize(s));
    auto t1 = std::chrono::steady_clock::now();
    const double sec = std::chrono::duration<double>(t1 - t0).count();
    for (int i = 0; i < n; ++i) {
        hs[i]->last_seconds = sec;
        hs[i]->last_steps = n_steps[i];
        if (out) {
            tt_status r = fill_stats(hs[i], &out[i], s);
            if (r != TT_OK) return r;
        }
    }
    return TT_OK;
}

tt_status tt_transport_destroy(tt_handle* h) {
    if (!h) return TT_OK;
    drop_graphs(h);
    if (h->noalloc_dev >= 0) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (g_scratch_owner[h->noalloc_dev] == h) g_scratch_owner[h->noalloc_dev] = nullptr;
    }
    for (auto& pr : h->ev_pool) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    delete h;
    return TT_OK;
}

const char* tt_transport_last_error(void) { return g_err.c_str(); }

}  // extern "C"
