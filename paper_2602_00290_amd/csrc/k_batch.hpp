// Persistent ragged small-solve kernel: one workgroup runs every step of one
// small request (the whole apply + round path of each step, all its steps) in
// a single launch, many requests side by side, each with its own grid, group
// count, ranks and step count.
//
// Small requests (FP64 data, Householder QR rounding, a projected first core
// of at most 16 columns, so that the TSQR of the whole first core is one
// block's job) spend most of a launched step on launch gaps: six small
// kernels per step.  Here a step is, inside one 1024-thread block:
//   prep_body          small-core QR and the gather operand G    (k_prep)
//   project_small      B = d (sum_j (O_j Z) G_j + rank-1 terms)  (VALU, FP64)
//   tsqr_body          R of B, one block over all rows (64 row groups)
//   svd_chain_body     SVD of R, truncation, new Theta / Phi, V_r (k_svd_chain)
//   output_small       Z_out = B V_r                             (VALU, FP64)
//   commit             the new ranks become current
// with block barriers between the phases.  The arithmetic of each phase is
// the launched path's (the same bodies for prep, TSQR and the SVD chain), so
// a request gives the same result alone or in any batch.
#pragma once

#include "k_f64.hpp"

namespace ttrt {

constexpr int kBatchMax = 256;                      // requests per launch (one block each)
constexpr size_t kBatchLdsBytes = 110 * 1024;       // dynamic LDS of the batch kernel

// Everything one request's steps need (written to the request's workspace).
struct SmallSolve {
    Geom g;
    OpDesc op;
    DevState* st;
    double* Z[2];           // ping-pong first cores (FP64)
    double* Th[2];
    double* Ph[2];
    const double* gtab;
    const double* htab;
    SmallScratch sc;
    double* LTh;
    double* QTh;
    double* QPh;
    double* Gop;
    double* B;
    double* V;
    double* R;
    double* sv;
    RowData rd;
    double tol;
    int k1cap, cap1, cap2, n_steps, zcur0;
};

struct SmallBatch {
    SmallSolve* req[kBatchMax];
};

// B = d (sum_j (O_j Z) G_j + sum_q z_q G_rank1[q]): one row per thread, the
// row's neighbours and rank-1 values once, then every column of B.
__device__ __forceinline__ void project_small(const SmallSolve& q, const double* __restrict__ Z) {
    const Geom& g = q.g;
    const OpDesc& op = q.op;
    const int ldz = q.st->ldz, ldb = q.st->ldb, nbl = op.n_gather, nr1 = op.n_r1;
    for (long long k = threadIdx.x; k < g.M; k += blockDim.x) {
        const double* rows[kMaxTerms + 1];
        for (int j = 0; j < nbl; ++j) {
            const long long r = j == 0 ? k : neighbour_row(g, k, op.gaxis[j], op.gdir[j]);
            rows[j] = r >= 0 ? Z + r * ldz : nullptr;
        }
        double z1[kMaxBC + 1];
        for (int qq = 0; qq < nr1; ++qq) z1[qq] = rank1_value(g, op, q.rd, k, qq);
        const double d = row_scale(g, op, q.rd, k);
        for (int c = 0; c < ldb; ++c) {
            double v = 0.0;
            for (int j = 0; j < nbl; ++j) {
                if (!rows[j]) continue;
                const double* G = q.Gop + (size_t)j * ldz * ldb + c;
                for (int a = 0; a < ldz; ++a) v += rows[j][a] * G[(size_t)a * ldb];
            }
            const double* G1 = q.Gop + (size_t)nbl * ldz * ldb + c;
            for (int qq = 0; qq < nr1; ++qq) v += z1[qq] * G1[(size_t)qq * ldb];
            q.B[k * ldb + c] = v * d;
        }
    }
}

// Z_out = B V_r over the new leading dimension (V_r is zero past the new rank).
__device__ __forceinline__ void output_small(const SmallSolve& q, double* __restrict__ Zo) {
    const int ldb = q.st->ldb, ldo = q.st->ldzn;
    for (long long k = threadIdx.x; k < q.g.M; k += blockDim.x) {
        const double* b = q.B + k * ldb;
        for (int c = 0; c < ldo; ++c) {
            double v = 0.0;
            for (int a = 0; a < ldb; ++a) v += b[a] * q.V[(size_t)a * ldo + c];
            Zo[k * ldo + c] = v;
        }
    }
}

// The phases as separate functions: each gets its own register allocation
// instead of the whole loop's (inlined, the descriptor fields held across
// the phases spill registers).
__device__ __noinline__ void phase_prep(const SmallSolve& q, int zc, double* lds, size_t cap) {
    prep_body<double>(q.g, q.op, q.st, q.Th[zc], q.Ph[zc], q.gtab, q.htab, q.sc, q.LTh, q.k1cap, q.QTh, q.QPh, q.Gop,
                      (double*)nullptr, 0, lds, cap);
}
__device__ __noinline__ void phase_project(const SmallSolve& q, int zc) { project_small(q, q.Z[zc]); }
__device__ __noinline__ void phase_tsqr(const SmallSolve& q) {
    tsqr_body<double, 16, 64, 16>(q.B, 0, 1, 0, q.g.M, q.g.M, q.st, q.R, 0);
}
__device__ __noinline__ void phase_chain(const SmallSolve& q, int zn, double* lds, size_t cap) {
    svd_chain_body<double, true>(q.g, q.st, q.R, 16, 0, q.QTh, q.QPh, q.tol, q.cap1, q.cap2, q.sc, q.Th[zn], q.Ph[zn],
                                 q.V, q.sv, (const double*)nullptr, (double*)nullptr, 0, lds, cap);
}
__device__ __noinline__ void phase_output(const SmallSolve& q, int zn) { output_small(q, q.Z[zn]); }

__global__ __launch_bounds__(kSmallThreads) void k_solve_small(SmallBatch batch) {
    extern __shared__ double lds[];
    __shared__ SmallSolve q;
    if (threadIdx.x == 0) q = *batch.req[blockIdx.x];
    __syncthreads();
    const size_t cap = kBatchLdsBytes / sizeof(double);
    for (int step = 0; step < q.n_steps; ++step) {
        const int zc = (q.zcur0 + step) & 1, zn = zc ^ 1;
        phase_prep(q, zc, lds, cap);
        __syncthreads();
        phase_project(q, zc);
        __syncthreads();
        phase_tsqr(q);
        __syncthreads();
        phase_chain(q, zn, lds, cap);
        __syncthreads();
        phase_output(q, zn);
        __syncthreads();
        if (threadIdx.x == 0) {
            DevState* st = q.st;
            st->r1_in = st->r1;
            st->r1 = st->r1n;
            st->r2 = st->r2n;
            st->ldz = st->ldzn;
        }
        __syncthreads();
    }
}

}  // namespace ttrt
