// Shared device-side definitions of the TT transport library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ttrt {

constexpr int kMaxTerms = 6;     // n = 2 d_X streaming terms
constexpr int kMaxBC = 12;       // inflow columns: one per inflow face (upwind), two with the Rusanov dissipation
constexpr int kMaxBlocks = 1 + kMaxTerms + kMaxBC + 1;

// Which operator a rounding pass applies to the stored TT before truncating.
enum OpKind : int {
    OP_NONE = 0,       // round the stored TT as it is (no operator)
    OP_FULL = 1,       // streaming + boundary terms, then absorption/emission
    OP_TRANSPORT = 2,  // streaming + boundary terms only
    OP_SOURCE = 3      // absorption/emission only
};

// Sizes that change from step to step live on the device so that a whole
// solve runs without host synchronisation.  Kernels read them at run time;
// grids are sized for the caps.
// Y's rows (direction-space projection) are ldb + kYPad elements apart (two
// extra 128-byte lines per row for FP64 data),
// so that the stencil's taps, whole rows 1, n_x and n_x n_y rows apart, do
// not all start at the same offset of a power-of-two address stride: over
// twelve allocations the 3D stencil took 11.0 ms on average against 12.1
// unpadded (11.3 with four lines)
constexpr int kYPad = 32;
// the same for FP32 data, in floats
constexpr int kYPadF = 32;
template <typename T> constexpr int y_pad() { return sizeof(T) == 8 ? kYPad : kYPadF; }

struct DevState {
    int r1, r2;        // ranks of the stored cores
    int ldz;           // leading dimension (columns) of the stored Z
    int R1, R2;        // ranks of the pending TT sum
    int k1, k2;        // ranks after right-to-left orthogonalisation
    int ldb;           // leading dimension of the projected core B (M x k1)
    int r1n, r2n;      // ranks after truncation
    int ldzn;          // leading dimension of the new Z
    int nan_flag;
    int max_R1, max_R2;
    int rounds;
    int canon, canon_prev;  // projection used the canonical angular basis (this / previous round)
    int k1_prev;            // k1 of the previous round (warm start validity)
    double norm;       // ||X||_F before truncation
    double disc2;      // squared discarded singular values (both bonds)
    double energy;
    double pad1;
    double fl[4];      // algorithmic flops accumulated: project, factor, output, small cores
    int sweeps[2];     // Jacobi sweeps of the last round (bond 1, bond 2)
    long long tph[8];  // wall_clock64 stamps at phase boundaries of the last SVD chain
    int kall;          // rows of the gather operand: n_gather * ldz + n_r1
    int k1b;           // columns of the projected core B (k1 until a randomized pass compresses the sum)
    int l1s, l2s;      // ranks of the last randomized compression (after dropping null sketch directions)
    int r1_in;         // first rank of the state the last rounding pass started from
    int stencil;       // 0, or this pass projects in direction space (Y = Z W, then the operator's
                       // stencil on Y) with this many direction rows (gather plus rank-1 blocks)
    int stencil_rounds; // rounding passes so far that projected in direction space
    double fl_dir[2];  // executed flops of the direction-space passes: Y = Z W, the stencil
};

// Static description of the problem shared by all kernels (passed by value).
struct Geom {
    int dim;
    int nx, ny, nz;
    int G;             // groups
    long long M;       // N_X * G rows of Z
    int nt, np;        // angular nodes
    int n_terms;       // 2 * dim
    int n_bc;          // inflow faces
    int periodic[3];   // per axis
    double lam[3];     // c dt / dx_d
    double cdt;        // c * dt
    double dx[3];      // cell widths
    double hbeta;      // HLL flux: optical-depth factor of the interface wave-speed reduction
    int bc_face[kMaxBC];   // face index of each inflow column
};

__host__ __device__ inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// Leading dimension used for Z and B rows (columns padded with zeros).
__host__ __device__ inline int ld_for_rank(int r) { return round_up(r < 1 ? 1 : r, 8); }

// Neighbour row of merged row k along axis d in direction s (+1 / -1); -1
// outside a non-periodic domain.
__device__ inline long long neighbour_row(const Geom& g, long long k, int d, int s) {
    long long cell = k / g.G;
    int grp = (int)(k - cell * g.G);
    int ix = (int)(cell % g.nx);
    long long rest = cell / g.nx;
    int iy = (int)(rest % g.ny);
    int iz = (int)(rest / g.ny);
    int idx = d == 0 ? ix : (d == 1 ? iy : iz);
    int n = d == 0 ? g.nx : (d == 1 ? g.ny : g.nz);
    long long stride = d == 0 ? 1 : (d == 1 ? (long long)g.nx : (long long)g.nx * g.ny);
    int j = idx + s;
    if (j < 0 || j >= n) {
        if (!g.periodic[d]) return -1;
        j = (j + n) % n;
    }
    long long ncell = cell + (long long)(j - idx) * stride;
    return ncell * g.G + grp;
}

// Cell index along axis d of merged row k.
__device__ inline int axis_index(const Geom& g, long long k, int d) {
    long long cell = k / g.G;
    if (d == 0) return (int)(cell % g.nx);
    long long rest = cell / g.nx;
    if (d == 1) return (int)(rest % g.ny);
    return (int)(rest / g.ny);
}

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace ttrt
