// FP64 contractions of the first core on gfx950 FP64 MFMA (v_mfma_f64_16x16x4f64).
//
//   MODE_PROJECT: B[k,:] = d_k ( sum_j Z[nbr_j(k),:] G_j + sum_q z_q(k) G_rank1[q] )
//                 (B = Z_new L_Theta of the pending TT sum, without Z_new)
//   MODE_OUTPUT:  Z_out = B V_r
//
// Each block runs 8 waves over row blocks of 16 RT rows per wave (RT = 2
// 16-row tiles; RT = 1 where two would spill registers: 128 columns, or 64
// with the fused Gram's 40 accumulator doubles) and loops over consecutive row
// blocks (a contiguous range per block, consecutive ranges on one XCD).  K runs in chunks of 32:
// each lane loads its A fragment straight into registers, four consecutive K
// values per row tile and 16-K group (a 4-aligned run of K never crosses a
// gather block: every leading dimension is a multiple of 8), and the operand
// chunk is staged in LDS, column-major, in two buffers (one barrier per
// chunk); the next chunk's loads are in flight while the current one
// computes.  The row data of a row block (d, neighbour rows, rank-1 values)
// is derived from the row indices and the problem arrays into LDS at its
// start, so no per-row tables are read.
//
// v_mfma_f64_16x16x4f64 lane layout (64 lanes, l = m + 16 q):
//   A[i][k] from lane i + 16 k, B[k][j] from lane j + 16 k,
//   D[i][j] in lane j + 16 (i % 4), register i / 4.
// In 16-K group t lane (m, q) supplies K = 16 t + 4 q + e to the e-th MFMA
// (A row m; B column 16 c + m), so one pair of 16-byte loads feeds four MFMAs.
// Consecutive MFMAs go to different accumulators (RT NCT independent chains).
// The accumulator of a row tile holds row 4 r + q, column 16 c + m in
// register r of lane (m, q): for a fixed r that is an A/B operand of a K = 4
// step over the rows 4 r .. 4 r + 3, which is how the fused FP64 Gram B^T B
// is accumulated from the accumulators (GRAM = true).  Each block writes the
// upper 16 x 16 blocks of its partial Gram matrix for k_sum_gram<NCT>.
#pragma once

#include "k_fused.hpp"

namespace ttrt {

constexpr int kF64Waves = 8;
constexpr int kF64Threads = 64 * kF64Waves;
constexpr int kF64Rows = 32 * kF64Waves;   // rows per row block (two row tiles per wave)
constexpr int kF64KC = 32;                 // K per staged chunk
constexpr int kF64LdK = kF64KC + 2;        // LDS column stride (doubles) of the staged operand
constexpr int kF64Z = kMaxBC + 4;          // rank-1 value rows (read four at a time)

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Gather blocks whose rows the row data holds: the identity and the shifted
// copies (upwind, Rusanov), or up to kMaxBlocks with the HLL flux's
// per-(term, shift) blocks.
__host__ __device__ constexpr int f64_nbr_rows(bool hll) { return hll ? kMaxBlocks : kMaxTerms + 1; }

// Chunks of the resident operand of the output (V_r, K = ldb <= 128) and of
// Y = Z W (W, K = ldz <= 64).
constexpr int kF64OutChunks = 128 / kF64KC;
constexpr int kF64AngChunks = 64 / kF64KC;

// Dynamic LDS bytes of k_mm_f64<MODE, NCT, GRAM, RT, HLL>: the projection's
// two operand buffers and the row data of 128 RT rows (the Gram reduction at
// the end reuses the space); the output's whole operand.
__host__ __device__ inline size_t f64_lds_bytes(int nct, bool gram, int rt, bool hll = false, int out_chunks = 0) {
    if (out_chunks > 0) return (size_t)out_chunks * 16 * nct * kF64LdK * sizeof(double);
    const size_t nrow = (size_t)16 * rt * kF64Waves;
    const size_t op = (size_t)2 * 16 * nct * kF64LdK * sizeof(double);
    const size_t rows = nrow * (sizeof(double) + f64_nbr_rows(hll) * sizeof(int)) +
                        (size_t)kF64Z * nrow * sizeof(double) + (hll ? (size_t)kMaxBlocks * nrow * sizeof(double) : 0);
    const size_t main = op + rows;
    const size_t red = gram ? (size_t)(kF64Waves / 2) * gram_blocks(nct) * 256 * sizeof(double) : 0;
    return main > red ? main : red;
}

// x / d and x % d for 0 <= x < 2^31 and 1 <= d: the FP64 product with the
// reciprocal is within one of the quotient, which the remainder corrects.
__device__ __forceinline__ int divmod_d(int x, int d, double rcp, int& rem) {
    int q = (int)((double)x * rcp);
    int r = x - q * d;
    if (r < 0) { --q; r += d; }
    if (r >= d) { ++q; r -= d; }
    rem = r;
    return q;
}

template <int MODE, int NCT, bool GRAM, int RT, bool HLL = false>
__global__ __launch_bounds__(kF64Threads) void k_mm_f64(Geom g, OpDesc op, const DevState* __restrict__ st,
                                                         const double* __restrict__ A,
                                                         const double* __restrict__ Gop, double* __restrict__ Out,
                                                         RowData rd, double* __restrict__ Gpart) {
    constexpr int NP = 16 * NCT;
    constexpr int NB = gram_blocks(NCT);
    constexpr int ROWS = 16 * RT * kF64Waves;   // rows per row block
    extern __shared__ __align__(16) unsigned char f64_lds[];
    // the operator's per-block tables (dynamically indexed: kept out of SGPRs)
    __shared__ int s_gax[kMaxBlocks], s_gdir[kMaxBlocks], s_r1kind[kMaxBlocks], s_r1face[kMaxBlocks];
    __shared__ int s_gwk[kMaxBlocks], s_r1hll[kMaxBlocks];
    __shared__ double s_r1coef[kMaxBlocks];
    double* Bs0 = reinterpret_cast<double*>(f64_lds);                         // 2 x [NP][kF64LdK]
    double* rowd = Bs0 + (size_t)2 * NP * kF64LdK;                             // [rows]
    double* rowz = rowd + ROWS;                                            // [kF64Z][rows]
    double* rowc = rowz + (size_t)kF64Z * ROWS;                            // HLL: [blocks][rows] weights
    int* nbr = reinterpret_cast<int*>(rowc + (HLL ? (size_t)kMaxBlocks * ROWS : 0));   // [blocks][rows]

    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const int m = l & 15, q = l >> 4;
    if (tid < kMaxBlocks) {
        s_gax[tid] = op.gaxis[tid];
        s_gdir[tid] = op.gdir[tid];
        s_r1kind[tid] = op.r1kind[tid];
        s_r1face[tid] = op.r1face[tid];
        s_r1coef[tid] = op.r1coef[tid];
        s_gwk[tid] = op.gwk[tid];
        s_r1hll[tid] = op.r1hll[tid];
    }
    // the gathered projection stands aside for the direction-space one, and
    // Y = Z W is formed only for it (uniform exits)
    if (MODE == MODE_PROJECT && st->stencil) return;
    if (MODE == MODE_ANGLE && !st->stencil) return;
    int lda, K, KG, ldo, nblk, kper, ldg;
    if (MODE == MODE_PROJECT) {
        lda = st->ldz; kper = st->ldz; nblk = op.n_gather; KG = nblk * kper; K = st->kall; ldo = st->ldb;
        ldg = st->ldb;
    } else if (MODE == MODE_ANGLE) {
        lda = st->ldz; kper = st->ldz; nblk = 1; KG = kper; K = kper; ldo = st->ldb + kYPad; ldg = st->ldb;
    } else {
        lda = st->ldb; kper = st->ldb; nblk = 1; KG = kper; K = kper; ldo = st->ldzn; ldg = st->ldzn;
    }
    const int n_kc = (K + kF64KC - 1) / kF64KC;
    const FastDiv dkp(kper);
    const double rG = 1.0 / g.G, rnx = 1.0 / g.nx, rny = 1.0 / g.ny;

    // contiguous row-block ranges per block; consecutive ranges on one XCD
    // (blocks are dealt to the 8 XCDs round robin)
    const long long nrb = (g.M + ROWS - 1) / ROWS;
    const int nbk = gridDim.x, b = blockIdx.x;
    const int lb = (nbk % 8 == 0) ? (b % 8) * (nbk / 8) + b / 8 : b;
    const long long rb_begin = (long long)lb * nrb / nbk, rb_end = (long long)(lb + 1) * nrb / nbk;

    f64x4 gacc[GRAM ? NB : 1];
#pragma unroll
    for (int i = 0; i < (GRAM ? NB : 1); ++i) gacc[i] = (f64x4){0.0, 0.0, 0.0, 0.0};

    // operand chunk kc (K rows k0 .. k0 + 31, NP columns, zero beyond K and
    // ldg) into registers: slot s holds column n = s % NP of the K rows
    // 2 (s / NP) and 2 (s / NP) + 1, so that consecutive lanes read
    // consecutive columns (coalesced) and write 16 bytes along K into the
    // [n][k] layout, lanes n .. n + 15 starting 4 banks apart
    constexpr int OPP = kF64KC * NP / 2;                 // slots per chunk
    constexpr int OPN = (OPP + kF64Threads - 1) / kF64Threads;
    f64x2 opr[OPN];
    auto fetch_op = [&](int kc) __attribute__((always_inline)) {
        const double* gk = Gop + (size_t)kc * kF64KC * ldg;   // uniform chunk base, 32-bit offsets
        const int kr = K - kc * kF64KC;                       // K rows left from the chunk start
#pragma unroll
        for (int v = 0; v < OPN; ++v) {
            const int idx = tid + kF64Threads * v;
            const int n = idx % NP, kk = 2 * (idx / NP);
            f64x2 x = (f64x2){0.0, 0.0};
            if (idx < OPP && n < ldg) {
                const int o = kk * ldg + n;
                if (kk < kr) x[0] = gk[o];
                if (kk + 1 < kr) x[1] = gk[o + ldg];
            }
            opr[v] = x;
        }
    };
    auto store_op = [&](double* Bs) __attribute__((always_inline)) {
#pragma unroll
        for (int v = 0; v < OPN; ++v) {
            const int idx = tid + kF64Threads * v;
            if (idx < OPP)
                *reinterpret_cast<f64x2*>(Bs + (size_t)(idx % NP) * kF64LdK + 2 * (idx / NP)) = opr[v];
        }
    };
    // this lane's A fragments of one 16-K group (flat index t = 2 kc + gi):
    // RT row tiles, four consecutive K values each; loaded one group ahead
    f64x2 ra[RT][2];
    double rw[RT];   // HLL: the per-row weight of the fragment's gather block
    auto fetch_a = [&](int t) __attribute__((always_inline)) {
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const int r = 16 * RT * w + 16 * rt + m;
            const int k = 16 * t + 4 * q;
            f64x2 v0 = (f64x2){0.0, 0.0}, v1 = v0;
            if constexpr (HLL) rw[rt] = 1.0;
            if (k < KG) {
                const int j = dkp.q(k), cc = k - j * kper;
                const int src = nbr[j * ROWS + r];
                if constexpr (HLL) rw[rt] = rowc[j * ROWS + r];
                if (src >= 0) {
                    const double* ap = A + (long long)src * lda + cc;
                    v0 = *reinterpret_cast<const f64x2*>(ap);
                    v1 = *reinterpret_cast<const f64x2*>(ap + 2);
                }
            } else if (MODE == MODE_PROJECT && k < K) {
                const int qq = k - KG;
                v0 = (f64x2){rowz[qq * ROWS + r], rowz[(qq + 1) * ROWS + r]};
                v1 = (f64x2){rowz[(qq + 2) * ROWS + r], rowz[(qq + 3) * ROWS + r]};
            }
            ra[rt][0] = v0;
            ra[rt][1] = v1;
        }
    };
    const int n_grp = (K + 15) >> 4;   // 16-K groups with data (the last chunk may hold one)

    if constexpr (MODE != MODE_PROJECT) {
        // Z_out = B V_r (or Y = Z W).  V_r (K = ldb <= 128 rows) stays in LDS for the whole
        // kernel, chunk after chunk as staged, so the row-block loop has no
        // barrier: each lane streams its A fragments (four consecutive K of
        // one row of B) straight from memory two 16-K groups ahead, across
        // row-block boundaries, and the waves run independently.
        for (int kc = 0; kc < n_kc; ++kc) {
            fetch_op(kc);
            store_op(Bs0 + (size_t)kc * NP * kF64LdK);
        }
        __syncthreads();
        // groups per row block, even (the staged chunks hold two each; groups
        // past K read zeros), so that the two prefetch slots alternate with
        // the group's parity
        const int ng = 2 * n_kc;
        f64x2 rq[2][RT][2];
        auto fetch_o = [&](long long rb, int t, f64x2 (&dst)[RT][2]) __attribute__((always_inline)) {
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                const long long row = rb * ROWS + 16 * RT * w + 16 * rt + m;
                const int k = 16 * t + 4 * q;
                f64x2 v0 = (f64x2){0.0, 0.0}, v1 = v0;
                if (rb < rb_end && row < g.M && k < K) {
                    // Y = Z W walks Y's group-major rows, reading Z's row of
                    // the same (cell, grp)
                    long long arow = row;
                    if (MODE == MODE_ANGLE) {
                        const int NXc = (int)(g.M / g.G);
                        int cell = 0;
                        const int grp = divmod_d((int)row, NXc, 1.0 / NXc, cell);
                        arow = (long long)cell * g.G + grp;
                    }
                    const double* ap = A + arow * lda + k;
                    v0 = *reinterpret_cast<const f64x2*>(ap);
                    v1 = *reinterpret_cast<const f64x2*>(ap + 2);
                }
                dst[rt][0] = v0;
                dst[rt][1] = v1;
            }
        };
        // group t of row block rb with this slot's fragments, then the slot
        // takes the group two ahead (into the next row block past the end)
        auto group = [&](long long rb, int t, f64x2 (&slot)[RT][2], f64x4 (&acc)[RT][NCT])
                         __attribute__((always_inline)) {
            f64x2 a[RT][2];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                a[rt][0] = slot[rt][0];
                a[rt][1] = slot[rt][1];
            }
            if (t + 2 < ng)
                fetch_o(rb, t + 2, slot);
            else
                fetch_o(rb + 1, t + 2 - ng, slot);
            const double* Bs = Bs0 + (size_t)(t >> 1) * NP * kF64LdK + 16 * (t & 1);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                double bv[NCT];
#pragma unroll
                for (int c = 0; c < NCT; ++c) bv[c] = Bs[(size_t)(16 * c + m) * kF64LdK + 4 * q + e];
#pragma unroll
                for (int c = 0; c < NCT; ++c)
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt)
                        acc[rt][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rt][e >> 1][e & 1], bv[c], acc[rt][c],
                                                                          0, 0, 0);
            }
        };
        if (ng > 0) {
            fetch_o(rb_begin, 0, rq[0]);
            fetch_o(rb_begin, 1, rq[1]);
        }
        for (long long rb = rb_begin; rb < rb_end; ++rb) {
            f64x4 acc[RT][NCT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int c = 0; c < NCT; ++c) acc[rt][c] = (f64x4){0.0, 0.0, 0.0, 0.0};
            for (int t = 0; t < ng; t += 2) {
                group(rb, t, rq[0], acc);
                group(rb, t + 1, rq[1], acc);
            }
            const long long row0 = rb * ROWS;
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const long long row = row0 + 16 * RT * w + 16 * rt + 4 * r + q;
                    // Y is stored group-major (row grp N_X + cell), where the
                    // stencil's neighbours are 1, n_x and n_x n_y rows apart
                    long long orow = row;
                    // a direction-space pass leaves B group-major too: the
                    // output reads it in that order and writes Z_out in the
                    // state's (cell G + grp)
                    if (MODE == MODE_OUTPUT && st->stencil && row < g.M) {
                        const int NXc = (int)(g.M / g.G);
                        int cell = 0;
                        const int grp = divmod_d((int)row, NXc, 1.0 / NXc, cell);
                        orow = (long long)cell * g.G + grp;
                    }
#pragma unroll
                    for (int c = 0; c < NCT; ++c) {
                        const int col = 16 * c + m;
                        if (row < g.M && col < ldo) Out[orow * ldo + col] = acc[rt][c][r];
                    }
                }
        }
        return;
    }

    for (long long rb = rb_begin; rb < rb_end; ++rb) {
        const long long row0 = rb * ROWS;
        __syncthreads();   // the previous row block's readers of the row data are done
        if (tid < ROWS) {
            // one row per thread: cell, group and cell coordinates once, then the
            // neighbour rows of the gather blocks, d and the rank-1 values
            const long long k = row0 + tid;
            const bool ok = k < g.M;
            int grp = 0, ix = 0, iy = 0, iz = 0;
            const int cell = ok ? divmod_d((int)k, g.G, rG, grp) : 0;
            iy = divmod_d(cell, g.nx, rnx, ix);
            iz = divmod_d(iy, g.ny, rny, iy);
            const int idx3[3] = {ix, iy, iz}, n3[3] = {g.nx, g.ny, g.nz};
            const int st3[3] = {g.G, g.G * g.nx, g.G * g.nx * g.ny};
            // HLL: the row's face factors along each axis (towards cell -/+ e_d)
            double eL[3] = {1.0, 1.0, 1.0}, eR[3] = {1.0, 1.0, 1.0};
            if constexpr (HLL) {
                if (ok)
                    for (int ax = 0; ax < g.dim; ++ax) {
                        eL[ax] = hll_face_eps(g, rd, k, ax, -1);
                        eR[ax] = hll_face_eps(g, rd, k, ax, 1);
                    }
            }
            for (int j = 0; j < nblk; ++j) {
                int src = ok ? (int)k : -1;
                if (MODE == MODE_PROJECT && j > 0 && ok) {
                    const int ax = s_gax[j], dir = s_gdir[j];
                    int jj = idx3[ax] + dir;
                    const bool out = jj < 0 || jj >= n3[ax];
                    if (out && !g.periodic[ax]) src = -1;
                    else {
                        jj = out ? (jj + n3[ax]) % n3[ax] : jj;
                        src = (int)k + (jj - idx3[ax]) * st3[ax];
                    }
                }
                nbr[j * ROWS + tid] = src;
                if constexpr (HLL) {
                    const int ax = s_gax[j];
                    rowc[j * ROWS + tid] = s_gwk[j] == 0 ? 1.0 : hll_weight(s_gwk[j], eL[ax], eR[ax], g.lam[ax]);
                }
            }
            if (MODE == MODE_PROJECT) {
                double kap = 0.0;
                if (ok) kap = rd.kfull ? rd.kfull[k] : rd.kappa0[cell] * rd.kscale[grp];
                const double ktot = (ok && rd.kscat) ? kap + rd.kscat[k] : kap;
                rowd[tid] = (ok && op.scale_d) ? 1.0 / (1.0 + g.cdt * ktot) : 1.0;
                for (int qq = 0; qq < kF64Z; ++qq) {
                    double v = 0.0;
                    if (ok && qq < op.n_r1) {
                        if (s_r1kind[qq] == 0) {
                            v = g.cdt * kap * rd.eps[k];
                            if (rd.kscat) v += g.cdt * rd.kscat[k] * rd.jn[k];
                        } else {
                            const int face = s_r1face[qq], ax = face >> 1;
                            const int edge = (face & 1) ? n3[ax] - 1 : 0;
                            double coef = s_r1coef[qq];
                            if (s_r1kind[qq] == 2) {   // HLL inflow column: the face's factor
                                const double e = (face & 1) ? eR[ax] : eL[ax];
                                coef *= s_r1hll[qq] == 1 ? 0.5 * (1.0 + e) : 0.5 * (1.0 - e);
                            }
                            if (idx3[ax] == edge) v = coef * rd.ghost[face * g.G + grp];
                        }
                    }
                    rowz[qq * ROWS + tid] = v;
                }
            }
        }
        f64x4 acc[RT][NCT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int c = 0; c < NCT; ++c) acc[rt][c] = (f64x4){0.0, 0.0, 0.0, 0.0};
        __syncthreads();
        if (n_kc > 0) {
            fetch_op(0);
            fetch_a(0);
            store_op(Bs0);
        }
        for (int kc = 0; kc < n_kc; ++kc) {
            __syncthreads();   // chunk kc is in buffer kc & 1; the other buffer's readers are done
            const double* Bs = Bs0 + (size_t)(kc & 1) * NP * kF64LdK;
            const bool more = kc + 1 < n_kc;
            if (more) fetch_op(kc + 1);   // in flight while this chunk computes
#pragma unroll
            for (int gi = 0; gi < 2; ++gi) {
                const int t = 2 * kc + gi;
                if (t >= n_grp) break;    // an all-zero padding group (uniform)
                f64x2 a[RT][2];
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    if constexpr (HLL) {
                        a[rt][0] = ra[rt][0] * rw[rt];
                        a[rt][1] = ra[rt][1] * rw[rt];
                    } else {
                        a[rt][0] = ra[rt][0];
                        a[rt][1] = ra[rt][1];
                    }
                }
                if (t + 1 < n_grp) fetch_a(t + 1);   // the next group, across the chunk boundary
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    double bv[NCT];
#pragma unroll
                    for (int c = 0; c < NCT; ++c) bv[c] = Bs[(size_t)(16 * c + m) * kF64LdK + 16 * gi + 4 * q + e];
#pragma unroll
                    for (int c = 0; c < NCT; ++c)
#pragma unroll
                        for (int rt = 0; rt < RT; ++rt)
                            acc[rt][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rt][e >> 1][e & 1], bv[c],
                                                                              acc[rt][c], 0, 0, 0);
                }
            }
            if (more) store_op(Bs0 + (size_t)((kc + 1) & 1) * NP * kF64LdK);
        }
        // row factor d on the rows (row 4 r + q of the tile in register r) and store
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 16 * RT * w + 16 * rt + 4 * r + q;
                const long long row = row0 + i;
                const double d = MODE == MODE_PROJECT ? rowd[i] : 1.0;
#pragma unroll
                for (int c = 0; c < NCT; ++c) {
                    acc[rt][c][r] *= d;
                    const int col = 16 * c + m;
                    if (row < g.M && col < ldo) Out[row * ldo + col] = acc[rt][c][r];
                }
            }
        if constexpr (GRAM) {
            // B^T B over this wave's rows (rows past M are zero)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    int bi = 0;
#pragma unroll
                    for (int ga = 0; ga < NCT; ++ga)
#pragma unroll
                        for (int gb = ga; gb < NCT; ++gb) {
                            gacc[bi] = __builtin_amdgcn_mfma_f64_16x16x4f64(acc[rt][ga][r], acc[rt][gb][r], gacc[bi],
                                                                            0, 0, 0);
                            ++bi;
                        }
                }
        }
    }

    if constexpr (GRAM) {
        // fixed-order reduction of the 8 waves' partial Gram blocks through LDS
        double* red = reinterpret_cast<double*>(f64_lds);
        constexpr int PER = NB * 256;   // doubles per wave
        __syncthreads();
        for (int half = kF64Waves / 2; half >= 1; half >>= 1) {
            if (w >= half && w < 2 * half) {
#pragma unroll
                for (int bi = 0; bi < NB; ++bi)
#pragma unroll
                    for (int r = 0; r < 4; ++r) red[(size_t)(w - half) * PER + (bi * 4 + r) * 64 + l] = gacc[bi][r];
            }
            __syncthreads();
            if (w < half) {
#pragma unroll
                for (int bi = 0; bi < NB; ++bi)
#pragma unroll
                    for (int r = 0; r < 4; ++r) gacc[bi][r] += red[(size_t)w * PER + (bi * 4 + r) * 64 + l];
            }
            __syncthreads();
        }
        if (w == 0) {
            double* outp = Gpart + (size_t)b * PER;
#pragma unroll
            for (int bi = 0; bi < NB; ++bi)
#pragma unroll
                for (int r = 0; r < 4; ++r) outp[(bi * 4 + r) * 64 + l] = gacc[bi][r];
        }
    }
}

// ---------------------------------------------------------------------------
// Projection in direction space
// ---------------------------------------------------------------------------
//
// When both small-core factors are square (k2 = N_phi and k1 = N_theta N_phi,
// the steady state once the sum's ranks exceed the angle counts), the columns
// of L_Theta are the directions (theta, phi), and block t of the pending
// sum's angular core is the state's angular matrix W = Theta x_3 Phi
// (r1 x N_theta N_phi) scaled per direction by the term's factors
// g_t(theta) h_t(phi).  So B = Z_new L_Theta is
//   B[k, i] = d_k (sum_j C_j[i] Y[nbr_j(k), i] + sum_q z_q(k) R_q[i]),
// Y = Z W: one contraction over r1 (k_mm_f64<MODE_ANGLE>) instead of over
// the n_gather r1 + n_r1 gathered columns, then this kernel: C_j is gather
// block j's direction factor (the sum of its terms' coefficients times
// g_t h_t), R_q the direction row of rank-1 block q and z_q(k) its value on
// row k, d_k the implicit absorption factor, as in the gathered projection.

constexpr int kStWaves = 16;   // waves per block
constexpr int kStRows = 64;    // rows per wave batch: the lanes set up one row each
constexpr int kStZ = 8;        // rank-1 blocks at most on this path
constexpr int kStNG = kMaxTerms + 1;   // gather blocks at most (the row and its shifts)

__global__ __launch_bounds__(64 * kStWaves) void k_stencil_f64(Geom g, OpDesc op, const DevState* __restrict__ st,
                                                              const double* __restrict__ Y,
                                                              const double* __restrict__ Cst, double* __restrict__ B,
                                                              RowData rd) {
    if (!st->stencil) return;
    __shared__ double s_R[kStZ * 128];                       // rank-1 direction rows
    __shared__ double s_cf[kStNG * 128];                     // gather blocks' direction factors
    __shared__ int s_nbr[kStWaves][kStNG][kStRows];          // gather rows (-1: none)
    __shared__ double s_d[kStWaves][kStRows];                // absorption factor
    __shared__ double s_z[kStWaves][kStZ][kStRows];          // rank-1 values
    const int ldb = st->ldb, ng = op.n_gather, nq = op.n_r1;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    for (int i = tid; i < nq * ldb; i += 64 * kStWaves) {
        const int q = i / ldb, c = i - q * ldb;
        s_R[q * 128 + c] = Cst[(size_t)(ng + q) * ldb + c];
    }
    // tap slots: the centre 0, then (when the operator has both) x- in 1 and
    // x+ in 2, the other gather blocks after them in order; gather block
    // jslot[s] sits in slot s
    int jxm = -1, jxp = -1;
    for (int j = 1; j < ng; ++j)
        if (op.gaxis[j] == 0) {
            if (op.gdir[j] < 0) jxm = j;
            else jxp = j;
        }
    const bool xwin = jxm > 0 && jxp > 0;
    int jslot[kStNG], slotj[kStNG];
#pragma unroll
    for (int t = 0; t < kStNG; ++t) jslot[t] = t;
    if (xwin) {
        jslot[1] = jxm;
        jslot[2] = jxp;
        int t = 3;
        for (int j = 1; j < ng; ++j)
            if (j != jxm && j != jxp) jslot[t++] = j;
    }
#pragma unroll
    for (int t = 0; t < kStNG; ++t) slotj[jslot[t]] = t;
    for (int i = tid; i < kStNG * 128; i += 64 * kStWaves) {
        const int t = i >> 7, c = i & 127, j = jslot[t];
        s_cf[i] = (t < ng && c < ldb) ? Cst[(size_t)j * ldb + c] : 0.0;
    }
    const int c0 = 2 * l;
    const bool colok = c0 < ldb;   // ldb is a multiple of 8, so c0 + 1 < ldb too
    __syncthreads();

    // Rows are taken in Y's group-major order (grp N_X + cell), in batches of
    // 64.  When an x-y plane is a whole number of batches, a block's task is
    // one batch position pb of the plane in kStWaves consecutive planes of one
    // group: wave w takes plane iz0 + w, so most z-neighbours of a wave's
    // rows are the rows its neighbouring waves load at the same time (the
    // block's waves keep step by a barrier per task), and consecutive tasks,
    // dealt to the XCD's blocks in turn, are the next batch positions of the
    // plane (the y-neighbours when n_x = 64).  Each XCD sweeps a contiguous
    // region of tasks.  Otherwise the waves take consecutive batches in
    // turn.  B is written group-major like Y, in whole contiguous rows: the
    // Gram and the Householder QR of B do not depend on the row order, and
    // the output contraction maps the rows back to the state's order
    // (cell G + grp).
    const int nb = gridDim.x, b = blockIdx.x;
    const long long nbat = (g.M + kStRows - 1) / kStRows;
    const int NXc = g.nx * g.ny * g.nz;
    const int plane = g.nx * g.ny;
    const int PB = (plane % kStRows == 0) ? plane / kStRows : 0;   // batches per plane (0: no tiling)
    const int nzb = (g.nz + kStWaves - 1) / kStWaves;                // plane blocks per group
    const long long ntask = PB ? (long long)g.G * nzb * PB : (nbat + kStWaves - 1) / kStWaves;
    int nbx = nb, bx = b;            // blocks of this XCD, this block's index there
    long long reg0 = 0, reg1 = ntask;
    if (nb % 8 == 0) {
        const int xcd = b % 8;
        nbx = nb / 8;
        bx = b / 8;
        reg0 = xcd * ntask / 8;
        reg1 = (xcd + 1) * ntask / 8;
    }
    const double rNX = 1.0 / NXc, rnx = 1.0 / g.nx, rny = 1.0 / g.ny;
    for (long long task = reg0 + bx; task < reg1; task += nbx) {
        long long bt;
        bool have;
        if (PB) {
            const int pb = (int)(task % PB);
            const long long t2 = task / PB;
            const int zb = (int)(t2 % nzb), grp0 = (int)(t2 / nzb);
            const int iz = zb * kStWaves + w;
            have = iz < g.nz;
            bt = ((long long)grp0 * g.nz + iz) * PB + pb;
        } else {
            bt = task * kStWaves + w;
            have = bt < nbat;
        }
        const long long row0 = bt * kStRows;   // group-major
        if (have) {
            {
                // lane l: row data of group-major row row0 + l (row k of Z and B)
                const long long kg = row0 + l;
                const bool ok = kg < g.M;
                int cell = 0, ix = 0, iy = 0, iz = 0;
                const int grp = ok ? divmod_d((int)kg, NXc, rNX, cell) : 0;
                const long long k = (long long)cell * g.G + grp;
                iy = divmod_d(cell, g.nx, rnx, ix);
                iz = divmod_d(iy, g.ny, rny, iy);
                const int idx3[3] = {ix, iy, iz}, n3[3] = {g.nx, g.ny, g.nz};
                const int st3[3] = {1, g.nx, g.nx * g.ny};
                for (int j = 0; j < ng; ++j) {
                    int src = ok ? (int)kg : -1;
                    if (j > 0 && ok) {
                        const int ax = op.gaxis[j], dir = op.gdir[j];
                        int jj = idx3[ax] + dir;
                        const bool out = jj < 0 || jj >= n3[ax];
                        if (out && !g.periodic[ax]) src = -1;
                        else {
                            jj = out ? (jj + n3[ax]) % n3[ax] : jj;
                            src = (int)kg + (jj - idx3[ax]) * st3[ax];
                        }
                    }
                    s_nbr[w][slotj[j]][l] = src;
                }
                double kap = 0.0;
                if (ok) kap = rd.kfull ? rd.kfull[k] : rd.kappa0[cell] * rd.kscale[grp];
                const double ktot = (ok && rd.kscat) ? kap + rd.kscat[k] : kap;
                s_d[w][l] = (ok && op.scale_d) ? 1.0 / (1.0 + g.cdt * ktot) : 1.0;
                for (int qq = 0; qq < nq; ++qq) {
                    double v = 0.0;
                    if (ok) {
                        if (op.r1kind[qq] == 0) {
                            v = g.cdt * kap * rd.eps[k];
                            if (rd.kscat) v += g.cdt * rd.kscat[k] * rd.jn[k];
                        } else {
                            const int face = op.r1face[qq], ax = face >> 1;
                            const int edge = (face & 1) ? n3[ax] - 1 : 0;
                            if (idx3[ax] == edge) v = op.r1coef[qq] * rd.ghost[face * g.G + grp];
                        }
                    }
                    s_z[w][qq][l] = v;
                }
            }
            // the row data is read by the other lanes of this wave: LDS
            // operations of a wave complete in order, and the compiler keeps
            // them in program order across this barrier
            __builtin_amdgcn_wave_barrier();
            const int nrow = (int)((g.M - row0) < kStRows ? (g.M - row0) : kStRows);
            // the previous row's centre and x+ taps, and their rows (uniform):
            // along an x-line the centre of row i is row i - 1's x+ tap and
            // its x- tap is row i - 1's centre, so two of the loads are reused
            f64x2 pc = (f64x2){0.0, 0.0}, pxp = pc;
            int pc_row = -1, pxp_row = -1;
            for (int i = 0; i < nrow; ++i) {
                f64x2 y[kStNG];
                const int s0 = __builtin_amdgcn_readfirstlane(s_nbr[w][0][i]);
                const int s1 = __builtin_amdgcn_readfirstlane(s_nbr[w][1][i]);
                if (xwin && s0 >= 0 && s0 == pxp_row && s1 >= 0 && s1 == pc_row) {
                    y[0] = pxp;
                    y[1] = pc;
#pragma unroll
                    for (int j = 2; j < kStNG; ++j) {
                        y[j] = (f64x2){0.0, 0.0};
                        if (j < ng) {
                            const int src = s_nbr[w][j][i];
                            if (src >= 0 && colok)
                                y[j] = *reinterpret_cast<const f64x2*>(Y + (size_t)src * (ldb + kYPad) + c0);
                        }
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < kStNG; ++j) {
                        y[j] = (f64x2){0.0, 0.0};
                        if (j < ng) {
                            const int src = s_nbr[w][j][i];
                            if (src >= 0 && colok)
                                y[j] = *reinterpret_cast<const f64x2*>(Y + (size_t)src * (ldb + kYPad) + c0);
                        }
                    }
                }
                pc = y[0];
                pc_row = s0;
                pxp = y[2];
                pxp_row = xwin ? __builtin_amdgcn_readfirstlane(s_nbr[w][2][i]) : -1;
                f64x2 acc = (f64x2){0.0, 0.0};
#pragma unroll
                for (int j = 0; j < kStNG; ++j) acc += *reinterpret_cast<const f64x2*>(s_cf + j * 128 + c0) * y[j];
                for (int qq = 0; qq < nq; ++qq) {
                    const double z = s_z[w][qq][i];
                    acc += z * *reinterpret_cast<const f64x2*>(s_R + qq * 128 + c0);
                }
                if (colok) *reinterpret_cast<f64x2*>(B + (size_t)(row0 + i) * ldb + c0) = acc * s_d[w][i];
            }
            __builtin_amdgcn_wave_barrier();   // this batch's row data is read before the next overwrites it
        }
        __syncthreads();   // the block's waves start each task together
    }
}

// The same stencil for FP32 data (FP32 Y and B, rows of Y ldb + kYPadF
// floats apart), with FP32 sums as the gathered FP32 contraction forms B.
__global__ __launch_bounds__(64 * kStWaves) void k_stencil_f32(Geom g, OpDesc op, const DevState* __restrict__ st,
                                                              const float* __restrict__ Y,
                                                              const double* __restrict__ Cst, float* __restrict__ B,
                                                              RowData rd) {
    if (!st->stencil) return;
    __shared__ double s_R[kStZ * 128];                       // rank-1 direction rows
    __shared__ double s_cf[kStNG * 128];                     // gather blocks' direction factors
    __shared__ int s_nbr[kStWaves][kStNG][kStRows];          // gather rows (-1: none)
    __shared__ double s_d[kStWaves][kStRows];                // absorption factor
    __shared__ double s_z[kStWaves][kStZ][kStRows];          // rank-1 values
    const int ldb = st->ldb, ng = op.n_gather, nq = op.n_r1;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    for (int i = tid; i < nq * ldb; i += 64 * kStWaves) {
        const int q = i / ldb, c = i - q * ldb;
        s_R[q * 128 + c] = Cst[(size_t)(ng + q) * ldb + c];
    }
    for (int i = tid; i < kStNG * 128; i += 64 * kStWaves) {
        const int j = i >> 7, c = i & 127;
        s_cf[i] = (j < ng && c < ldb) ? Cst[(size_t)j * ldb + c] : 0.0;
    }
    // four columns per lane: the two half-waves take two rows at a time
    const int c0 = 4 * (l & 31), half = l >> 5;
    const bool colok = c0 < ldb;   // ldb is a multiple of 8, so c0 + 3 < ldb too
    __syncthreads();
    f32x4 cf32[kStNG];   // this lane's direction factors
#pragma unroll
    for (int j = 0; j < kStNG; ++j)
        cf32[j] = (f32x4){(float)s_cf[j * 128 + c0], (float)s_cf[j * 128 + c0 + 1], (float)s_cf[j * 128 + c0 + 2],
                          (float)s_cf[j * 128 + c0 + 3]};

    // Rows are taken in Y's group-major order (grp N_X + cell), in batches of
    // 64.  When an x-y plane is a whole number of batches, a block's task is
    // one batch position pb of the plane in kStWaves consecutive planes of one
    // group: wave w takes plane iz0 + w, so most z-neighbours of a wave's
    // rows are the rows its neighbouring waves load at the same time (the
    // block's waves keep step by a barrier per task), and consecutive tasks,
    // dealt to the XCD's blocks in turn, are the next batch positions of the
    // plane (the y-neighbours when n_x = 64).  Each XCD sweeps a contiguous
    // region of tasks.  Otherwise the waves take consecutive batches in
    // turn.  B is written group-major like Y, in whole contiguous rows: the
    // Gram and the Householder QR of B do not depend on the row order, and
    // the output contraction maps the rows back to the state's order
    // (cell G + grp).
    const int nb = gridDim.x, b = blockIdx.x;
    const long long nbat = (g.M + kStRows - 1) / kStRows;
    const int NXc = g.nx * g.ny * g.nz;
    const int plane = g.nx * g.ny;
    const int PB = (plane % kStRows == 0) ? plane / kStRows : 0;   // batches per plane (0: no tiling)
    const int nzb = (g.nz + kStWaves - 1) / kStWaves;                // plane blocks per group
    const long long ntask = PB ? (long long)g.G * nzb * PB : (nbat + kStWaves - 1) / kStWaves;
    int nbx = nb, bx = b;            // blocks of this XCD, this block's index there
    long long reg0 = 0, reg1 = ntask;
    if (nb % 8 == 0) {
        const int xcd = b % 8;
        nbx = nb / 8;
        bx = b / 8;
        reg0 = xcd * ntask / 8;
        reg1 = (xcd + 1) * ntask / 8;
    }
    const double rNX = 1.0 / NXc, rnx = 1.0 / g.nx, rny = 1.0 / g.ny;
    for (long long task = reg0 + bx; task < reg1; task += nbx) {
        long long bt;
        bool have;
        if (PB) {
            const int pb = (int)(task % PB);
            const long long t2 = task / PB;
            const int zb = (int)(t2 % nzb), grp0 = (int)(t2 / nzb);
            const int iz = zb * kStWaves + w;
            have = iz < g.nz;
            bt = ((long long)grp0 * g.nz + iz) * PB + pb;
        } else {
            bt = task * kStWaves + w;
            have = bt < nbat;
        }
        const long long row0 = bt * kStRows;   // group-major
        if (have) {
            {
                // lane l: row data of group-major row row0 + l (row k of Z and B)
                const long long kg = row0 + l;
                const bool ok = kg < g.M;
                int cell = 0, ix = 0, iy = 0, iz = 0;
                const int grp = ok ? divmod_d((int)kg, NXc, rNX, cell) : 0;
                const long long k = (long long)cell * g.G + grp;
                iy = divmod_d(cell, g.nx, rnx, ix);
                iz = divmod_d(iy, g.ny, rny, iy);
                const int idx3[3] = {ix, iy, iz}, n3[3] = {g.nx, g.ny, g.nz};
                const int st3[3] = {1, g.nx, g.nx * g.ny};
                for (int j = 0; j < ng; ++j) {
                    int src = ok ? (int)kg : -1;
                    if (j > 0 && ok) {
                        const int ax = op.gaxis[j], dir = op.gdir[j];
                        int jj = idx3[ax] + dir;
                        const bool out = jj < 0 || jj >= n3[ax];
                        if (out && !g.periodic[ax]) src = -1;
                        else {
                            jj = out ? (jj + n3[ax]) % n3[ax] : jj;
                            src = (int)kg + (jj - idx3[ax]) * st3[ax];
                        }
                    }
                    s_nbr[w][j][l] = src;
                }
                double kap = 0.0;
                if (ok) kap = rd.kfull ? rd.kfull[k] : rd.kappa0[cell] * rd.kscale[grp];
                const double ktot = (ok && rd.kscat) ? kap + rd.kscat[k] : kap;
                s_d[w][l] = (ok && op.scale_d) ? 1.0 / (1.0 + g.cdt * ktot) : 1.0;
                for (int qq = 0; qq < nq; ++qq) {
                    double v = 0.0;
                    if (ok) {
                        if (op.r1kind[qq] == 0) {
                            v = g.cdt * kap * rd.eps[k];
                            if (rd.kscat) v += g.cdt * rd.kscat[k] * rd.jn[k];
                        } else {
                            const int face = op.r1face[qq], ax = face >> 1;
                            const int edge = (face & 1) ? n3[ax] - 1 : 0;
                            if (idx3[ax] == edge) v = op.r1coef[qq] * rd.ghost[face * g.G + grp];
                        }
                    }
                    s_z[w][qq][l] = v;
                }
            }
            // the row data is read by the other lanes of this wave: LDS
            // operations of a wave complete in order, and the compiler keeps
            // them in program order across this barrier
            __builtin_amdgcn_wave_barrier();
            const int nrow = (int)((g.M - row0) < kStRows ? (g.M - row0) : kStRows);
            {
                for (int i0 = 0; i0 < nrow; i0 += 2) {
                    const int i = i0 + half;
                    const bool rok = i < nrow && colok;
                    // all taps' loads first, then the sums
                    f32x4 y[kStNG];
#pragma unroll
                    for (int j = 0; j < kStNG; ++j) {
                        y[j] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
                        if (j < ng && rok) {
                            const int src = s_nbr[w][j][i];
                            if (src >= 0) y[j] = *reinterpret_cast<const f32x4*>(Y + (size_t)src * (ldb + kYPadF) + c0);
                        }
                    }
                    f32x4 acc = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                    for (int j = 0; j < kStNG; ++j) acc += cf32[j] * y[j];
                    if (rok) {
                        for (int qq = 0; qq < nq; ++qq) {
                            const float z = (float)s_z[w][qq][i];
                            acc += z * (f32x4){(float)s_R[qq * 128 + c0], (float)s_R[qq * 128 + c0 + 1],
                                               (float)s_R[qq * 128 + c0 + 2], (float)s_R[qq * 128 + c0 + 3]};
                        }
                        *reinterpret_cast<f32x4*>(B + (size_t)(row0 + i) * ldb + c0) = acc * (float)s_d[w][i];
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();   // this batch's row data is read before the next overwrites it
        }
        __syncthreads();   // the block's waves start each task together
    }
}



}  // namespace ttrt
