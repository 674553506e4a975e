// Device work-list records and kernel launchers of the DMRG library.
//
// Everything heavy (blocking + transformation, the normal->complementary
// transform, the integral-weighted operator sums and H_eff psi) is expressed
// as one kind of work: an output tile C (up to 96 rows x 96 columns of a
// sector block) accumulated as
//
//     C = sum_groups [ x_coef * X_g . U_g + xid_coef * U_g ],
//     U_g = sum_{c in g} alpha_c * A_c . B_c
//
// where every operand is a dense sector block in one of eight device
// buffers, optionally transposed or an identity.  For H_eff psi, A_c is a
// psi sub-block, B_c a right operator block (transposed) and X_g a left
// operator block: the two products of one term run back to back with the
// intermediate U_g held in registers (never written to memory).  For the
// transformation U^T O U, X_g = U^T, A_c = O (each component of the
// blocked operator), B_c = U.  A plain GEMM is the case X = identity with a
// single contribution.  Tiles are owned by exactly one workgroup and
// contributions are summed in list order, so results are deterministic.
#pragma once
#include <cstdint>

namespace dmrgk {

// Rows of an output tile and of U (inner dimension of X . U) for the
// one-wave-per-slice kernels: at most six MFMA row tiles.  Tiles whose rows
// all fit five row tiles (kShortRows) run a kernel compiled for five: a wave's
// FP32 accumulators, U and one chunk's fragments then fit 128 registers (four
// waves per SIMD) instead of 168 (three).
#ifndef DMRG_MAX_ROWS
#define DMRG_MAX_ROWS 96
#endif
constexpr int kMaxRows = DMRG_MAX_ROWS;
constexpr int kShortRows = 80;
// Tiles with more than kMaxRows rows (or U rows), up to kTallRows, run the
// tall kernel: one workgroup per 16-column slice, U formed once for all its
// rows and shared through LDS, so no row tile recomputes it.  Blocks taller
// than kTallRows are split exactly.
constexpr int kTallRows = 320;
constexpr int kMaxCols = 96;     // columns of an output tile
constexpr int kMaxBuf = 9;       // buffer 8: partial tiles of split tasks

// flag bits
enum : int32_t {
    F_TRANS_A = 1 << 6, F_TRANS_B = 1 << 7, F_ID_A = 1 << 8, F_ID_B = 1 << 9,
    G_TRANS_X = 1 << 3, G_HAS_X = 1 << 4,
};

struct Task {          // one output tile: rows 0..m-1, columns col0..col0+ncol-1 of a block
    int64_t c_off;     // element offset of the block (of the partial slot, if tile-local) in buffer cbuf
    int32_t ldc, m, n; // row stride, rows, columns of the whole block
    int32_t col0, ncol;
    int32_t g0, g1;    // group range
    int32_t cbuf;      // buffer id of C (bits 0-3) | accumulate << 8 | tile-local columns << 9
    int32_t pad;
};

struct Group {
    int64_t x_off;
    double x_coef, xid_coef;
    int32_t ldx, mu;   // mu = rows of U = inner dimension of X . U
    int32_t flags;     // xbuf (bits 0-2) | G_TRANS_X | G_HAS_X
    int32_t c0, c1;    // contribution range
    int32_t pad;
};

struct Contrib {
    int64_t a_off, b_off;
    double alpha;
    int32_t lda, ldb, k;
    int32_t flags;     // abuf (0-2) | bbuf (3-5) | F_TRANS_A | F_TRANS_B | F_ID_A | F_ID_B
};

template <typename T>
struct Bases {
    T* p[kMaxBuf];
    int64_t vstride[kMaxBuf];   // per-vector stride (batched vectors, grid.y)
};

// Task classes.  Tile classes c < kNumTileClass: tiles of 16n+1 .. 16n+16
// columns (n = c % kColClasses), computed as n+1 independent 16-column slices
// (one wave each), with rows (and U rows) up to kShortRows (c < kColClasses)
// or kMaxRows.  Wave classes kNumTileClass + (RT-1)*2 + (CT-1): tiles whose
// rows and U rows fit 16*RT and whose columns fit 16*CT (RT, CT <= 2), one
// wave each.  Tall classes kTallClass0 + n: tiles of 16n+1 .. 16n+16 columns
// with rows (or U rows) in (kMaxRows, kTallRows], one workgroup per slice.
constexpr int kColClasses = kMaxCols / 16;
constexpr int kNumTileClass = 2 * kColClasses;
constexpr int kTallClass0 = kNumTileClass + 4;
constexpr int kNumClass = kTallClass0 + kColClasses;
inline int col_class(int ncol) { return (ncol + 15) / 16 - 1; }
// rows: max of the tile rows and of every group's mu; tiles of tall_min rows
// or more run on the tall kernel (always above kMaxRows)
inline int task_class(int rows, int ncol, int tall_min = kMaxRows + 1) {
    if (rows > kMaxRows || (rows >= tall_min && rows > 32)) return kTallClass0 + col_class(ncol);
    if (rows <= 32 && ncol <= 32) return kNumTileClass + ((rows + 15) / 16 - 1) * 2 + (ncol + 15) / 16 - 1;
    return col_class(ncol) + (rows > kShortRows ? kColClasses : 0);
}
inline int class_rows(int cls) {
    if (cls >= kTallClass0) return kTallRows;
    return cls < kNumTileClass ? (cls >= kColClasses ? kMaxRows : kShortRows) : 16 * ((cls - kNumTileClass) / 2 + 1);
}
inline int class_cols(int cls) {
    if (cls >= kTallClass0) return 16 * (cls - kTallClass0 + 1);
    return cls < kNumTileClass ? 16 * (cls % kColClasses + 1) : 16 * ((cls - kNumTileClass) % 2 + 1);
}

// Records per task that fit the LDS staging of the kernels: a work list
// whose every task has at most kRecG groups, whose contributions (at most
// kRecC) are contiguous, runs with lds_records = true.
constexpr int kRecG = 48;
constexpr int kRecC = 128;

// A kernel launch as data (function, grid, block), for eager launches and for
// the nodes of a captured product graph.  func == nullptr: nothing to launch.
struct KernelDesc {
    const void* func = nullptr;
    unsigned gx = 0, gy = 0, bx = 0;
};
// Argument blocks of the chain kernels (Bases, tasks, ntask, groups,
// contributions, nvec) and of the reduction (reductions, Bases); ptrs[] is
// the kernel-parameter array of hipLaunchKernel / a graph kernel node.
template <typename T>
struct ChainArgs {
    Bases<T> b;
    const Task* t;
    int ntask;
    const Group* g;
    const Contrib* c;
    int nvec;
    void* ptrs[6];
    ChainArgs(const Bases<T>& b_, const Task* t_, int n_, const Group* g_, const Contrib* c_, int v_)
        : b(b_), t(t_), ntask(n_), g(g_), c(c_), nvec(v_), ptrs{&b, &t, &ntask, &g, &c, &nvec} {}
    ChainArgs(const ChainArgs&) = delete;
};
struct Reduce;
template <typename T>
struct ReduceArgs {
    const Reduce* r;
    Bases<T> b;
    void* ptrs[2];
    ReduceArgs(const Reduce* r_, const Bases<T>& b_) : r(r_), b(b_), ptrs{&r, &b} {}
    ReduceArgs(const ReduceArgs&) = delete;
};
KernelDesc chain_desc_f64(int cls, bool lds_records, int ntask, int nvec);
KernelDesc chain_desc_f32(int cls, bool lds_records, int ntask, int nvec);
KernelDesc reduce_desc_f64(int nred, int nvec);
KernelDesc reduce_desc_f32(int nred, int nvec);

// launchers (return hipError_t as int)
int launch_chain_f64(int cls, bool lds_records, const Task* t, int ntask, const Group* g, const Contrib* c,
                     const Bases<double>& b, int nvec, void* stream);
int launch_chain_f32(int cls, bool lds_records, const Task* t, int ntask, const Group* g, const Contrib* c,
                     const Bases<float>& b, int nvec, void* stream);

// A task whose group range is split writes each chunk's tile to its own slot
// of the partial buffer (tile-local: m x ncol, row stride ncol); the slots
// are then summed in slot order, so the result does not depend on scheduling:
//   C[r][col0 + j] (+)= sum_{s < nslot} P[poff + s*m*ncol + r*ncol + j]
constexpr int kPartialBuf = 8;
struct Reduce {
    int64_t c_off, poff;
    int32_t ldc, m, col0, ncol, nslot;
    int32_t cbuf;      // buffer id of C | accumulate << 8
};
int launch_reduce_f64(const Reduce* r, int nred, const Bases<double>& b, int nvec, void* stream);
int launch_reduce_f32(const Reduce* r, int nred, const Bases<float>& b, int nvec, void* stream);

int launch_cast_d2f(const double* in, float* out, int64_t n, void* stream);
int launch_cast_f2d(const float* in, double* out, int64_t n, void* stream);

// H_eff diagonal: for each psi sub-block o, diag[o](i,j) = sum over its
// contributions (x_off, y_off, coef): coef * X[i,i] * Y[j,j] (X or Y < 0 => 1)
struct DiagBlock { int64_t off; int32_t ma, mb; int32_t c0, c1; };
struct DiagTerm { int64_t x_off, y_off; double coef; int32_t ldx, ldy; int32_t xbuf, ybuf; };
int launch_diag(const DiagBlock* blocks, int nblock, const DiagTerm* terms, Bases<double> b,
                double* diag, void* stream);

// Davidson helpers (FP64)
// G[i*ldg + j] = <V_i, W_j>, i < nv, j < nw; vectors of length n at strides
int launch_gram(const double* V, int nv, const double* W, int nw, int64_t n,
                double* G, int ldg, double* scratch, void* stream);
// Y_j = sum_i C[i*ldc + j] V_i (+ beta Y_j) for j < ny
int launch_combine(const double* V, int nv, const double* C, int ldc, double* Y, int ny,
                   int64_t n, double beta, void* stream);
// t = r / (theta - d) with |theta - d| >= clamp; clamp < 0: t = r
int launch_precond(const double* r, const double* d, double theta, double clamp, double* t, int64_t n,
                   void* stream);
// symmetric eigen-decomposition of an n x n matrix (n <= 64), one workgroup,
// cyclic Jacobi; A row-major in, eigenvalues ascending in w, eigenvectors as
// columns of Z (row-major n x n)
int launch_jacobi(const double* A, int n, double* w, double* Z, void* stream);
// count of non-finite entries -> *flag (int)
int launch_nonfinite(const double* x, int64_t n, int* flag, void* stream);

// Decimation.  Gather of wavefunction sub-blocks into the dense per-sector
// matrices Psi_q (side-major): for vector v, element (i, j) of sub-block b
//   out[b.dst + part * b.pcol + v * b.vcol + (b.trans ? j * b.ld + i : i * b.ld + j)]
//     = scale * psi[v * dim + b.src + i * b.mb + j]
// (part 1 places a second set of vectors, the perturbation, after the first).
// Grid: one workgroup per (sub-block, vector).
struct GatherBlock { int64_t src, dst, vcol, pcol; int32_t ma, mb, ld, trans; };
int launch_psi_gather(const GatherBlock* blocks, int nblock, int nvec, const double* psi, int part, int64_t dim,
                      double scale, double* out, void* stream);
// kept eigenvectors, descending weight: iso[b.dst + i * b.k + c] =
// evec[b.src + i + (b.d - 1 - c) * b.d] (column-major ascending eigenvectors
// of a d x d matrix -> row-major d x k isometry)
struct EvecBlock { int64_t src, dst; int32_t d, k; };
int launch_evec_gather(const EvecBlock* blocks, int nblock, const double* evec, double* iso, void* stream);

}  // namespace dmrgk
