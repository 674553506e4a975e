// HIP kernels (gfx950) of the DMRG library.
//
// slice_kernel: the grouped, output-stationary sector-GEMM engine described
// in kernels.hpp, for output tiles of up to 96 rows x 16*NCT columns.  Every
// wave computes one 16-column slice of a tile on its own: per group, U
// (mu x 16) is accumulated in MFMA registers over the contributions and used
// directly as the B operand of X . U, so U never leaves the registers; the
// MFMA fragments of A_c, B_c and X come straight from global memory.
// wave_kernel: the same for tiles of at most 32 x 32.  MFMA 16x16x4 in f64
// or f32.
#include <hip/hip_runtime.h>
#include <cmath>
#include "kernels.hpp"

namespace dmrgk {

template <typename T> struct Mfma;
// Operand fragments of both 16x16x4 instructions: lane l holds A[l%16][l/16]
// and B[l/16][l%16].  Accumulator element v of lane l is column l%16 and row
// row(l/16, v), which differs between the two instructions (measured on
// gfx950): f64 rows are 4v + l/16, f32 rows are 4(l/16) + v.
template <> struct Mfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    __device__ static inline v4 mma(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static constexpr int row(int lk, int v) { return 4 * v + lk; }
};
template <> struct Mfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    __device__ static inline v4 mma(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static constexpr int row(int lk, int v) { return 4 * lk + v; }
};


// Four consecutive elements at a 32-bit element offset of a uniform base
// (element alignment only: the loads are 16-byte vector loads, which gfx950
// performs at any 4-byte alignment).
typedef float F4u __attribute__((ext_vector_type(4), aligned(4)));
typedef double D2u __attribute__((ext_vector_type(2), aligned(8)));
__device__ inline void ld4_at(const float* p, uint32_t off, float (&r)[4]) {
    const F4u v = *reinterpret_cast<const F4u*>(reinterpret_cast<const char*>(p) + off * 4u);
    r[0] = v.x; r[1] = v.y; r[2] = v.z; r[3] = v.w;
}
__device__ inline void ld4_at(const double* p, uint32_t off, double (&r)[4]) {
    const char* b = reinterpret_cast<const char*>(p) + off * 8u;
    const D2u v = *reinterpret_cast<const D2u*>(b);
    const D2u w = *reinterpret_cast<const D2u*>(b + 16);
    r[0] = v.x; r[1] = v.y; r[2] = w.x; r[3] = w.y;
}

__device__ inline bool is_identity(int flags) { return (flags & (F_ID_A | F_ID_B)) != 0; }

// Element (32-bit offset) of a uniform base pointer: the byte offset stays
// 32-bit so the load takes the scalar-base + vector-offset form.
template <typename T>
__device__ inline T ld_at(const T* p, uint32_t off) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + off * (uint32_t)sizeof(T));
}

// Group / contribution records of a task.  LR = false: straight from global
// memory (scalar loads).  LR = true: the task's records were copied to LDS
// once at its start (one coalesced load), so the per-chunk descriptor reads
// are LDS reads; values are made wave-uniform with readfirstlane.
template <typename R>
__device__ inline R lds_uniform(const R* p) {
    static_assert(sizeof(R) % 4 == 0, "record size");
    R r;
    const int* s = reinterpret_cast<const int*>(p);
    int* d = reinterpret_cast<int*>(&r);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(R) / 4); ++i) d[i] = __builtin_amdgcn_readfirstlane(s[i]);
    return r;
}

template <bool LR> struct Recs;
template <> struct Recs<false> {
    const Group* __restrict__ G;
    const Contrib* __restrict__ C;
    __device__ Group group(int g) const { return G[g]; }
    __device__ Contrib contrib(int c) const { return C[c]; }
};
template <> struct Recs<true> {
    const Group* sg;
    const Contrib* sc;
    int g0, cb;
    __device__ Group group(int g) const { return lds_uniform(sg + (g - g0)); }
    __device__ Contrib contrib(int c) const { return lds_uniform(sc + (c - cb)); }
};

// copies the records of groups g0..g1-1 and of their (contiguous)
// contributions to LDS with threads tid = 0..nt-1; returns the first
// contribution index
__device__ inline int stage_records(const Group* __restrict__ groups, const Contrib* __restrict__ contribs, int g0,
                                    int g1, Group* sg, Contrib* sc, int tid, int nt) {
    if (g1 <= g0) return 0;
    const int cb = groups[g0].c0;
    const int nc = groups[g1 - 1].c1 - cb;
    const int* gs = reinterpret_cast<const int*>(groups + g0);
    int* gd = reinterpret_cast<int*>(sg);
    for (int i = tid; i < (g1 - g0) * (int)(sizeof(Group) / 4); i += nt) gd[i] = gs[i];
    const int* cs = reinterpret_cast<const int*>(contribs + cb);
    int* cd = reinterpret_cast<int*>(sc);
    for (int i = tid; i < nc * (int)(sizeof(Contrib) / 4); i += nt) cd[i] = cs[i];
    return cb;
}

// The buffer table is read through the kernel-argument segment so that an
// index known only at run time becomes a scalar load rather than a select
// over registers; the table is the kernel's first argument (offset 0).
template <typename T>
__device__ inline const T* base_ptr(int buf, int vec) {
    typedef const __attribute__((address_space(4))) Bases<T>* KPtr;
    const KPtr b = (KPtr)__builtin_amdgcn_kernarg_segment_ptr();
    return b->p[buf] + (int64_t)vec * b->vstride[buf];
}

// Workgroup -> (unit, vector) of a launch over nvec vectors.  Workgroups are
// dealt to the eight XCDs in turn (linear id mod 8), so the nvec vectors of one
// unit are made consecutive workgroups of one XCD: the operator blocks they
// all read are then fetched into that XCD's L2 once and reused, instead of
// once per vector.  Units are spread over the XCDs as before (unit mod 8); the
// grid holds ceil(units / 8) * 8 * nvec workgroups and units past the end exit.
__device__ inline void unit_vec(int nvec, int& unit, int& vec) {
    const int L = blockIdx.x;
    if (nvec == 1) {
        unit = L;
        vec = 0;
        return;
    }
    const int local = L >> 3;
    vec = local % nvec;
    unit = (local / nvec) * 8 + (L & 7);
}
inline unsigned grid_units(int units, int nvec) {
    return nvec == 1 ? (unsigned)units : (unsigned)((units + 7) / 8 * 8 * nvec);
}
// Tall tasks: the nct column slices (and the nvec vectors) of one task, and
// runs of kTallRun consecutive tasks, run on workgroups of one XCD.  Column
// tiles of one output block are consecutive in the list (equal cost, stable
// order) and read the same psi rows and left-operator blocks, so those are
// fetched into that XCD's L2 once rather than once per slice or tile.
// Workgroup L (the XCD is L % 8) takes, with local = L / 8, m = nct*nvec and
// r = local / m: task ((r / kTallRun)*8 + L%8)*kTallRun + r % kTallRun, and
// sub-unit local % m = vec*nct + slice.  Runs go to the XCDs in turn, in list
// order.
constexpr int kTallRun = 4;
__device__ inline void tall_unit(int nct, int nvec, int& task, int& slice, int& vec) {
    const int L = blockIdx.x;
    const int m = nct * nvec;
    const int local = L >> 3;
    const int sub = local % m;
    const int r = local / m;
    task = ((r / kTallRun) * 8 + (L & 7)) * kTallRun + r % kTallRun;
    slice = sub % nct;
    vec = sub / nct;
}
inline unsigned grid_tall(int ntask, int nct, int nvec) {
    return (unsigned)((ntask + 8 * kTallRun - 1) / (8 * kTallRun) * 8 * kTallRun * nct * nvec);
}

// ---------------------------------------------------------------------------
// slice_kernel: output tiles of <= 96 rows x 16*NCT columns.  Every wave
// computes one 16-column slice of a tile on its own, four slices per
// workgroup (consecutive slices of one task share a workgroup, and so the
// CU's L1 for the A and X rows they all read).  MFMA fragments are loaded
// straight from global memory into operand registers -- one 16-byte vector
// load per lane and row tile where the operand's layout puts the lane's four
// k next to each other -- so the chunk loop has no LDS staging and no barrier.
// Small workgroups of independent waves matter: workgroups of five or six
// waves reached fewer than two per CU.
//
// Per group: U = sum_c alpha_c A_c B_c over 16-k chunks; then U's rows past
// mu (products of clamped A rows) are zeroed, the identity term xid * U is
// added, U is scaled by x_coef and C += X . U runs over U's row tiles.
// ---------------------------------------------------------------------------
// Waves per SIMD the slice kernel is compiled for: FP32 4 for tiles of five
// row tiles (128 registers), 3 for six (152 registers, no spills); FP64 2.
template <typename T, int RT> struct SliceOcc {
    static constexpr int waves = sizeof(T) == 4 ? (RT <= 5 ? 4 : 3) : 2;
};


template <typename T, int NCT, int RT, bool LR>
__global__ __launch_bounds__(256, (SliceOcc<T, RT>::waves)) void slice_kernel(Bases<T> Bargs,
                                                                        const Task* __restrict__ tasks,
                                                                        int ntask,
                                                                        const Group* __restrict__ groups,
                                                                        const Contrib* __restrict__ contribs,
                                                                        int nvec) {
    using V4 = typename Mfma<T>::v4;
    __shared__ Group sG[LR ? 4 : 1][LR ? kRecG : 1];
    __shared__ Contrib sC[LR ? 4 : 1][LR ? kRecC : 1];
    (void)Bargs;

    // four slices per workgroup: wave wv takes unit u = 4 wg + wv,
    // column slice u % NCT of task u / NCT
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;
    int wg, vec;
    unit_vec(nvec, wg, vec);
    const int u = wg * 4 + wv;
    if (u >= ntask * NCT) return;
    const int w = u % NCT;
    const int lr0 = lane & 15;
    const int lk0 = lane >> 4;
    const Task tk = tasks[u / NCT];
    const int ncv = min(tk.ncol, tk.n - tk.col0);   // valid columns of the tile
    const int nrm = (tk.m + 15) >> 4;                // output row tiles
    Recs<LR> R;
    if constexpr (LR) {   // each wave stages its own task's records; in-order LDS within a wave
        const int cb = stage_records(groups, contribs, tk.g0, tk.g1, sG[wv], sC[wv], lane, 64);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        R = Recs<true>{sG[wv], sC[wv], tk.g0, cb};
    } else {
        R = Recs<false>{groups, contribs};
    }

    V4 acc[RT];
#pragma unroll
    for (int i = 0; i < RT; ++i) acc[i] = V4{0, 0, 0, 0};
    // The lane coordinates are passed through an empty asm inside each loop,
    // so that the compiler recomputes the cheap per-lane bounds there instead
    // of hoisting dozens of lane masks out of the loops (which spilled).
    auto opaque = [](int x) { asm volatile("" : "+v"(x)); return x; };

    for (int g = tk.g0; g < tk.g1; ++g) {
        const Group gr = R.group(g);
        const int mu = gr.mu;
        const int nru = (mu + 15) >> 4;   // row tiles of U
        V4 U[RT];
#pragma unroll
        for (int i = 0; i < RT; ++i) U[i] = V4{0, 0, 0, 0};
        for (int c = gr.c0; c < gr.c1; ++c) {
            const Contrib ct = R.contrib(c);
            const T alpha = (T)ct.alpha;
            if (is_identity(ct.flags)) {
                // U rows row(g, v) of tile i += alpha * operand (or alpha * shifted I), this lane's column
                const int lr = opaque(lr0), lk = opaque(lk0);
                const int gcol = tk.col0 + 16 * w + lr;
                const bool colok = 16 * w + lr < ncv;
                const bool ida = (ct.flags & F_ID_A) != 0, idb = (ct.flags & F_ID_B) != 0;
                const T* P = ida ? base_ptr<T>((ct.flags >> 3) & 7, vec) + ct.b_off
                                 : base_ptr<T>(ct.flags & 7, vec) + ct.a_off;
                const bool tp = ida ? (ct.flags & F_TRANS_B) != 0 : (ct.flags & F_TRANS_A) != 0;
                const int ld = ida ? ct.ldb : ct.lda;
#pragma unroll
                for (int i = 0; i < RT; ++i) {
                    if (i >= nru) continue;
                    T x[4];
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = 16 * i + Mfma<T>::row(lk, v);
                        const bool ok = row < mu && colok;
                        if (ida && idb)   // a_off: diagonal offset of the identity (within the block)
                            x[v] = (row + (int)ct.a_off == gcol) ? T(1) : T(0);
                        else
                            x[v] = ld_at(P, ok ? (tp ? (uint32_t)(gcol * ld + row) : (uint32_t)(row * ld + gcol)) : 0u);
                    }
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = 16 * i + Mfma<T>::row(lk, v);
                        U[i][v] += (row < mu && colok) ? alpha * x[v] : T(0);
                    }
                }
                continue;
            }
            const T* Ap = base_ptr<T>(ct.flags & 7, vec) + ct.a_off;
            const T* Bp = base_ptr<T>((ct.flags >> 3) & 7, vec) + ct.b_off;
            const bool ta = (ct.flags & F_TRANS_A) != 0, tb = (ct.flags & F_TRANS_B) != 0;
            const int K = ct.k, lda = ct.lda, ldb = ct.ldb;
            // The chunk at k0: lane (r, g) covers k = k0 + 4g .. k0 + 4g + 3.  In
            // FP32 tiles of at most five row tiles, with K >= 4, it reads the four
            // k at kb = min(k0 + 4g, K - 4) instead, which always lie inside the
            // row, so a partial last chunk uses the same vector loads as a full
            // one; k below k0 + 4g (covered by the previous lane group) are then
            // dropped by zeroing B.  Otherwise the k past K read offset 0 of the
            // block (FP64 and six-row-tile tiles measured slower with the sliding
            // window).  Rows of A past mu read row 0 (they only reach U rows past
            // mu, zeroed below).
            const bool slide = sizeof(T) == 4 && RT <= 5 && K >= 4;
            auto fetch = [&](int k0, T (&fa)[RT][4], T (&fb)[4]) {
                const int lr = opaque(lr0), lk = opaque(lk0);
                const int gcol = tk.col0 + 16 * w + lr;
                const bool colok = 16 * w + lr < ncv;
                const int kk = k0 + 4 * lk;
                const int kb = slide ? min(kk, K - 4) : kk;
                const bool vec4 = slide || k0 + 16 <= K;   // the four k lie inside the row
#pragma unroll
                for (int i = 0; i < RT; ++i) {
                    if (i >= nru) continue;
                    const int row = 16 * i + lr;
                    const bool rok = row < mu;
                    if (!ta && vec4) {
                        ld4_at(Ap, rok ? (uint32_t)(row * lda + kb) : 0u, fa[i]);
                    } else {
#pragma unroll
                        for (int s = 0; s < 4; ++s) {
                            const int k = kb + s;
                            const bool ok = rok && k < K;
                            fa[i][s] = ld_at(Ap, ok ? (ta ? (uint32_t)(k * lda + row) : (uint32_t)(row * lda + k)) : 0u);
                        }
                    }
                }
                if (tb && vec4) {
                    ld4_at(Bp, colok ? (uint32_t)(gcol * ldb + kb) : 0u, fb);
                } else {
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        const int k = kb + s;
                        const bool ok = colok && k < K;
                        fb[s] = ld_at(Bp, ok ? (tb ? (uint32_t)(gcol * ldb + k) : (uint32_t)(k * ldb + gcol)) : 0u);
                    }
                }
            };
            // U += alpha * A . B of the chunk at k0.  B is zeroed at the k this
            // lane group does not own (below k0 + 4g or past K) and at columns
            // past the tile.
            auto mmas = [&](int k0, T (&fa)[RT][4], T (&fb)[4]) {
                const int lr = opaque(lr0), lk = opaque(lk0);
                const bool colok = 16 * w + lr < ncv;
                const int kk = k0 + 4 * lk;
                const int kb = slide ? min(kk, K - 4) : kk;
#pragma unroll
                for (int s = 0; s < 4; ++s) fb[s] = (colok && kb + s >= kk && kb + s < K) ? alpha * fb[s] : T(0);
#pragma unroll
                for (int i = 0; i < RT; ++i) {
                    if (i >= nru) continue;
#pragma unroll
                    for (int s = 0; s < 4; ++s) U[i] = Mfma<T>::mma(fa[i][s], fb[s], U[i]);
                }
            };
            for (int k0 = 0; k0 < K; k0 += 16) {
                T fa[RT][4], fb[4];
                fetch(k0, fa, fb);
                mmas(k0, fa, fb);
            }
        }
        {
            const int lk = opaque(lk0);
#pragma unroll
            for (int i = 0; i < RT; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (16 * i + Mfma<T>::row(lk, v) >= mu) U[i][v] = T(0);
        }
        if (gr.xid_coef != 0.0) {
            const T xi = (T)gr.xid_coef;
#pragma unroll
            for (int i = 0; i < RT; ++i) acc[i] += xi * U[i];
        }
        if (gr.flags & G_HAS_X) {
            const T* Xp = base_ptr<T>(gr.flags & 7, vec) + gr.x_off;
            const bool tx = (gr.flags & G_TRANS_X) != 0;
            const T xc = (T)gr.x_coef;
            const int ldx = gr.ldx;
#pragma unroll
            for (int i = 0; i < RT; ++i) U[i] *= xc;
            // X . U over U's row tiles q: lane (r, g) takes X rows 16i + r,
            // k = 16q + row(g, s), the rows U's accumulator holds in the lane
#pragma unroll
            for (int q = 0; q < RT; ++q) {
                if (q >= nru) continue;
                const int lr = opaque(lr0), lk = opaque(lk0);
                const bool full = 16 * q + 16 <= mu;
                T xf[RT][4];
#pragma unroll
                for (int i = 0; i < RT; ++i) {
                    if (i >= nrm) continue;
                    const int row = 16 * i + lr;
                    const bool rok = row < tk.m;
                    if (Mfma<T>::row(1, 0) == 4 && !tx && full) {
                        ld4_at(Xp, rok ? (uint32_t)(row * ldx + 16 * q + 4 * lk) : 0u, xf[i]);
                    } else {
#pragma unroll
                        for (int s = 0; s < 4; ++s) {
                            const int k = 16 * q + Mfma<T>::row(lk, s);
                            const bool ok = rok && k < mu;
                            xf[i][s] = ld_at(Xp, ok ? (tx ? (uint32_t)(k * ldx + row) : (uint32_t)(row * ldx + k)) : 0u);
                        }
                    }
                }
#pragma unroll
                for (int i = 0; i < RT; ++i) {
                    if (i >= nrm) continue;
#pragma unroll
                    for (int s = 0; s < 4; ++s) acc[i] = Mfma<T>::mma(xf[i][s], U[q][s], acc[i]);
                }
                __builtin_amdgcn_sched_barrier(0);   // one row tile of U at a time
            }
        }
    }

    const int cbuf = tk.cbuf & 15;
    const bool accum = (tk.cbuf >> 8) & 1;
    const bool local = (tk.cbuf >> 9) & 1;   // partial slot: columns from 0
    T* Cp = const_cast<T*>(base_ptr<T>(cbuf, vec)) + tk.c_off + (local ? 0 : tk.col0);
    const int lk = lk0;
    const int mycol = 16 * w + lr0;   // tile-local column of this lane
    if (mycol < ncv) {
#pragma unroll
        for (int i = 0; i < RT; ++i) {
            if (i >= nrm) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 16 * i + Mfma<T>::row(lk, v);
                if (row < tk.m) {
                    T* d = Cp + (uint32_t)(row * tk.ldc + mycol);
                    *d = accum ? *d + acc[i][v] : acc[i][v];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// tall_kernel: output tiles with more than kMaxRows rows (or U rows), up to
// kTallRows, one workgroup of four waves per 16-column slice.  Row tile j of
// U and of the output belongs to wave j % 4 (five per wave at most).  Per
// group, each wave forms its row tiles of U = sum_c alpha_c A_c B_c in MFMA
// registers (A_c rows are its own, B_c is read by all four waves through the
// CU's cache), adds the identity term to its own output rows, and writes
// x_coef * U^T to LDS; after one barrier every wave runs X . U for its output
// rows over all of U's rows, with U's fragments read from LDS.  U is thus
// formed once per slice however tall the block, where the one-wave kernels
// would recompute it for every 96-row tile.
//
// LDS holds U^T (16 columns x kTallRows rows, row stride LD): a lane's four
// consecutive k of one column are one 16-byte (FP32) or two 16-byte (FP64)
// reads, and LD is chosen so the sixteen columns of one read land in
// distinct banks.  FP32 double-buffers U (one barrier per group: the buffer a
// wave writes was last read before the previous barrier); FP64 keeps one
// buffer and a second barrier, which leaves LDS for three workgroups per CU.
// ---------------------------------------------------------------------------
// Straight-line chunk loops of the tall kernel's common cases, for a wave
// that owns NT row tiles (a compile-time count, so the loop has no per-tile
// branch and the memory-count waits can be partial: the products of the
// first tiles start while later tiles' fragments are still in flight).
// U formation with A row-major and B transposed (a psi block times a right
// operator block), over the full 16-k chunks; lanes outside the operand read
// its element 0 and a zero factor (B) or the later row mask (A) clears them.
template <typename T, int RW, int NT>
__device__ __forceinline__ void tall_u_fast(typename Mfma<T>::v4 (&U)[RW], const T* Ap, const T* Bp, int lda,
                                            int ldb, int kfull, int wv, int mu, int lr, int lk, int gcol,
                                            bool colok, T alpha) {
    const T acol = colok ? alpha : T(0);
    uint32_t boff = colok ? (uint32_t)(gcol * ldb + 4 * lk) : 0u;
    const uint32_t bstep = colok ? 16u : 0u;
    uint32_t aoff[NT], astep[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int row = 16 * (wv + 4 * t) + lr;
        const bool rok = row < mu;
        aoff[t] = rok ? (uint32_t)(row * lda + 4 * lk) : 0u;
        astep[t] = rok ? 16u : 0u;
    }
    // FP32 is software-pipelined: the next chunk's fragments are requested
    // before this chunk's products, so each wave keeps two chunks of loads in
    // flight (FP64 has no registers for a second set)
    constexpr bool pipe = sizeof(T) == 4 && NT <= 4;
    T fb[4], fa[NT][4];
    if constexpr (pipe) {
        ld4_at(Bp, boff, fb);
#pragma unroll
        for (int t = 0; t < NT; ++t) ld4_at(Ap, aoff[t], fa[t]);
    }
    for (int k0 = 0; k0 < kfull; k0 += 16) {
        if constexpr (!pipe) {
            ld4_at(Bp, boff, fb);
#pragma unroll
            for (int t = 0; t < NT; ++t) ld4_at(Ap, aoff[t], fa[t]);
        }
        T nb[4], na[NT][4];
        const bool more = pipe && k0 + 16 < kfull;
        boff += bstep;
#pragma unroll
        for (int t = 0; t < NT; ++t) aoff[t] += astep[t];
        if (more) {
            ld4_at(Bp, boff, nb);
#pragma unroll
            for (int t = 0; t < NT; ++t) ld4_at(Ap, aoff[t], na[t]);
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) fb[s] *= acol;
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int s = 0; s < 4; ++s) U[t] = Mfma<T>::mma(fa[t][s], fb[s], U[t]);
        if (more) {
#pragma unroll
            for (int s = 0; s < 4; ++s) fb[s] = nb[s];
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int s = 0; s < 4; ++s) fa[t][s] = na[t][s];
        }
    }
}

// X . U with X row-major over the full 16-row chunks of U (U^T in LDS at su,
// row stride LD); output rows at or beyond m accumulate values never stored.
template <typename T, int RW, int NT, int LD>
__device__ __forceinline__ void tall_x_fast(typename Mfma<T>::v4 (&acc)[RW], const T* Xp, int ldx, int qfull,
                                            const T* su, int wv, int m, int lr, int lk) {
    uint32_t xoff[NT], xstep[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int row = 16 * (wv + 4 * t) + lr;
        const bool rok = row < m;
        xoff[t] = rok ? (uint32_t)(row * ldx + 4 * lk) : 0u;
        xstep[t] = rok ? 16u : 0u;
    }
    const T* p = su + lr * LD + 4 * lk;
    for (int q = 0; q < qfull; ++q) {
        T ub[4], xf[NT][4];
        if constexpr (sizeof(T) == 4) {
            const float4 v = *reinterpret_cast<const float4*>(p + 16 * q);
            ub[0] = v.x; ub[1] = v.y; ub[2] = v.z; ub[3] = v.w;
        } else {
            const double2 a = *reinterpret_cast<const double2*>(p + 16 * q);
            const double2 b = *reinterpret_cast<const double2*>(p + 16 * q + 2);
            ub[0] = a.x; ub[1] = a.y; ub[2] = b.x; ub[3] = b.y;
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) ld4_at(Xp, xoff[t], xf[t]);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
#pragma unroll
            for (int s = 0; s < 4; ++s) acc[t] = Mfma<T>::mma(xf[t][s], ub[s], acc[t]);
            xoff[t] += xstep[t];
        }
    }
}

// The partial last chunks of both loops, as vector loads: lane group g takes
// the four k at kb = min(k0 + 4g, K - 4), which lie inside the operand, and a
// zero B (or U) factor drops the k below k0 + 4g that the previous group
// covers.  Needs K >= 4.
template <typename T, int RW, int NT>
__device__ __forceinline__ void tall_u_tail(typename Mfma<T>::v4 (&U)[RW], const T* Ap, const T* Bp, int lda,
                                            int ldb, int k0, int K, int wv, int mu, int lr, int lk, int gcol,
                                            bool colok, T alpha) {
    const int kk = k0 + 4 * lk;
    const int kb = min(kk, K - 4);
    T fb[4], fa[NT][4];
    ld4_at(Bp, colok ? (uint32_t)(gcol * ldb + kb) : 0u, fb);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int row = 16 * (wv + 4 * t) + lr;
        ld4_at(Ap, row < mu ? (uint32_t)(row * lda + kb) : 0u, fa[t]);
    }
    const T acol = colok ? alpha : T(0);
#pragma unroll
    for (int s = 0; s < 4; ++s) fb[s] = kb + s >= kk ? acol * fb[s] : T(0);
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int s = 0; s < 4; ++s) U[t] = Mfma<T>::mma(fa[t][s], fb[s], U[t]);
}

template <typename T, int RW, int NT, int LD>
__device__ __forceinline__ void tall_x_tail(typename Mfma<T>::v4 (&acc)[RW], const T* Xp, int ldx, int k0, int mu,
                                            const T* su, int wv, int m, int lr, int lk) {
    const int kk = k0 + 4 * lk;
    const int kb = min(kk, mu - 4);
    T ub[4], xf[NT][4];
    const T* p = su + lr * LD + kb;
#pragma unroll
    for (int s = 0; s < 4; ++s) ub[s] = kb + s >= kk ? p[s] : T(0);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int row = 16 * (wv + 4 * t) + lr;
        ld4_at(Xp, row < m ? (uint32_t)(row * ldx + kb) : 0u, xf[t]);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int s = 0; s < 4; ++s) acc[t] = Mfma<T>::mma(xf[t][s], ub[s], acc[t]);
}

// U formation with A row-major and B row-major (a psi block times a right
// operator used as its transpose): a lane's four k of B are a column of B,
// four separate loads per lane.  Instead each chunk of B (16 k x 16 columns)
// is read row-wise with one 16-byte load per lane, transposed through the
// wave's own LDS scratch (16 x 16 elements, an array of its own: no other
// wave touches it) and read back as one 16-byte (FP64: two) LDS read per
// lane.  K >= 16; the last partial chunk restarts at K - 16
// with the rows already summed zeroed in B.  Lanes outside the operand load
// nothing (B) or element 0 (A, cleared by the later row mask).
template <typename T, int RW, int NT>
__device__ __forceinline__ void tall_u_rowB(typename Mfma<T>::v4 (&U)[RW], const T* Ap, const T* Bp, int lda,
                                            int ldb, int K, int wv, int mu, int lr, int lk, int bcol0, int ncolv,
                                            T alpha, T* scr) {
    constexpr int SL = 16;                      // scratch row stride (16-byte aligned rows)
    const int lane = lr + 16 * lk;
    const int kr = lane >> 2, c4 = 4 * (lane & 3);
    uint32_t abase[NT];
    bool rok[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int row = 16 * (wv + 4 * t) + lr;
        rok[t] = row < mu;
        abase[t] = rok[t] ? (uint32_t)(row * lda) : 0u;
    }
    const int kfull = K & ~15;
    const int nch = kfull / 16 + (kfull < K ? 1 : 0);
    for (int c = 0; c < nch; ++c) {
        const bool last = c * 16 >= kfull;           // the partial chunk, restarted at K - 16
        const int k0 = last ? K - 16 : c * 16;
        const int kskip = last ? kfull - k0 : 0;     // rows already summed
        // B rows k0 + kr, columns c4..c4+3 of the slice
        T bq[4] = {T(0), T(0), T(0), T(0)};
        if (kr >= kskip) {
            const uint32_t o = (uint32_t)((k0 + kr) * ldb + bcol0 + c4);
            if (c4 + 4 <= ncolv) {
                ld4_at(Bp, o, bq);
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (c4 + j < ncolv) bq[j] = ld_at(Bp, o + (uint32_t)j);
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) scr[(c4 + j) * SL + kr] = alpha * bq[j];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        T fb[4];
        if constexpr (sizeof(T) == 4) {
            const float4 v = *reinterpret_cast<const float4*>(scr + lr * SL + 4 * lk);
            fb[0] = v.x; fb[1] = v.y; fb[2] = v.z; fb[3] = v.w;
        } else {
            const double2 v = *reinterpret_cast<const double2*>(scr + lr * SL + 4 * lk);
            const double2 u = *reinterpret_cast<const double2*>(scr + lr * SL + 4 * lk + 2);
            fb[0] = v.x; fb[1] = v.y; fb[2] = u.x; fb[3] = u.y;
        }
        T fa[NT][4];
#pragma unroll
        for (int t = 0; t < NT; ++t) ld4_at(Ap, rok[t] ? abase[t] + (uint32_t)(k0 + 4 * lk) : 0u, fa[t]);
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int s = 0; s < 4; ++s) U[t] = Mfma<T>::mma(fa[t][s], fb[s], U[t]);
        // every lane's read of this chunk precedes the next chunk's writes
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// X . U with X used as its transpose (X[row][k] stored at Xp[k * ldx + row]):
// a lane's four k of X are four rows of the stored block.  Per chunk of 16 k
// and output row tile, the 16 x 16 block is read along its stored rows (one
// 16-byte load per lane), transposed through the wave's LDS scratch and read
// back as the A fragment.  mu >= 16; the last partial chunk restarts at
// mu - 16 with the k already summed zeroed in U.
template <typename T, int RW, int NT, int LD>
__device__ __forceinline__ void tall_x_transX(typename Mfma<T>::v4 (&acc)[RW], const T* Xp, int ldx, int mu,
                                              const T* su, int wv, int m, int lr, int lk, T* scr) {
    constexpr int SL = 16;
    const int lane = lr + 16 * lk;
    const int kr = lane >> 2, c4 = 4 * (lane & 3);
    const int kfull = mu & ~15;
    const int nch = kfull / 16 + (kfull < mu ? 1 : 0);
    for (int c = 0; c < nch; ++c) {
        const bool last = c * 16 >= kfull;
        const int k0 = last ? mu - 16 : c * 16;
        const int kskip = last ? kfull - k0 : 0;
        T ub[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int k = k0 + 4 * lk + s;
            ub[s] = k >= k0 + kskip ? su[lr * LD + k] : T(0);
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int r0 = 16 * (wv + 4 * t);
            T xq[4] = {T(0), T(0), T(0), T(0)};
            const uint32_t o = (uint32_t)((k0 + kr) * ldx + r0 + c4);
            if (r0 + c4 + 4 <= m) {
                ld4_at(Xp, o, xq);
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (r0 + c4 + j < m) xq[j] = ld_at(Xp, o + (uint32_t)j);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) scr[(c4 + j) * SL + kr] = xq[j];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            T xf[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) xf[s] = scr[lr * SL + 4 * lk + s];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int s = 0; s < 4; ++s) acc[t] = Mfma<T>::mma(xf[s], ub[s], acc[t]);
        }
    }
}

template <typename T> struct TallCfg;
template <> struct TallCfg<float> {
    static constexpr int nbuf = 2, ld = kTallRows + 4, waves = 3;
};
template <> struct TallCfg<double> {
    static constexpr int nbuf = 1, ld = kTallRows + 6, waves = 2;
};

template <typename T, int NCT, bool LR>
__global__ __launch_bounds__(256, (TallCfg<T>::waves)) void tall_kernel(Bases<T> Bargs,
                                                                         const Task* __restrict__ tasks,
                                                                         int ntask,
                                                                         const Group* __restrict__ groups,
                                                                         const Contrib* __restrict__ contribs,
                                                                         int nvec) {
    using V4 = typename Mfma<T>::v4;
    constexpr int RW = kTallRows / 64;   // row tiles per wave
    constexpr int LD = TallCfg<T>::ld;
    constexpr int NB = TallCfg<T>::nbuf;
    __shared__ __attribute__((aligned(16))) T sU[NB][16 * LD];
    // per-wave transposition scratch of the row-major B path
    __shared__ __attribute__((aligned(16))) T sBt[4 * 256];
    __shared__ Group sG[LR ? kRecG : 1];
    __shared__ Contrib sC[LR ? kRecC : 1];
    (void)Bargs;

    int task, w, vec;
    tall_unit(NCT, nvec, task, w, vec);
    if (task >= ntask) return;               // the whole workgroup: no barrier is reached
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    // the wave index in a scalar register: the per-tile guards below are then
    // scalar branches, not exec-mask changes
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const Task tk = tasks[task];
    const int lr0 = lane & 15;
    const int lk0 = lane >> 4;
    const int ncv = min(tk.ncol, tk.n - tk.col0);
    const int nrm = (tk.m + 15) >> 4;
    const int nto = nrm > wv ? (nrm - wv + 3) >> 2 : 0;   // output row tiles of this wave
    Recs<LR> R;
    if constexpr (LR) {
        const int cb = stage_records(groups, contribs, tk.g0, tk.g1, sG, sC, tid, 256);
        __syncthreads();
        R = Recs<true>{sG, sC, tk.g0, cb};
    } else {
        R = Recs<false>{groups, contribs};
    }
    auto opaque = [](int x) { asm volatile("" : "+v"(x)); return x; };

    V4 acc[RW];
#pragma unroll
    for (int t = 0; t < RW; ++t) acc[t] = V4{0, 0, 0, 0};
    int buf = 0;

    for (int g = tk.g0; g < tk.g1; ++g) {
        const Group gr = R.group(g);
        const int mu = gr.mu;
        const int nru = (mu + 15) >> 4;
        const int ntu = nru > wv ? (nru - wv + 3) >> 2 : 0;   // U row tiles of this wave
        V4 U[RW];
#pragma unroll
        for (int t = 0; t < RW; ++t) U[t] = V4{0, 0, 0, 0};
        for (int c = gr.c0; c < gr.c1; ++c) {
            const Contrib ct = R.contrib(c);
            const T alpha = (T)ct.alpha;
            if (is_identity(ct.flags)) {
                const int lr = opaque(lr0), lk = opaque(lk0);
                const int gcol = tk.col0 + 16 * w + lr;
                const bool colok = 16 * w + lr < ncv;
                const bool ida = (ct.flags & F_ID_A) != 0, idb = (ct.flags & F_ID_B) != 0;
                const T* P = ida ? base_ptr<T>((ct.flags >> 3) & 7, vec) + ct.b_off
                                 : base_ptr<T>(ct.flags & 7, vec) + ct.a_off;
                const bool tp = ida ? (ct.flags & F_TRANS_B) != 0 : (ct.flags & F_TRANS_A) != 0;
                const int ld = ida ? ct.ldb : ct.lda;
#pragma unroll
                for (int t = 0; t < RW; ++t) {
                    const int j = wv + 4 * t;
                    if (j >= nru) continue;
                    T x[4];
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = 16 * j + Mfma<T>::row(lk, v);
                        const bool ok = row < mu && colok;
                        if (ida && idb)
                            x[v] = (row + (int)ct.a_off == gcol) ? T(1) : T(0);
                        else
                            x[v] = ld_at(P, ok ? (tp ? (uint32_t)(gcol * ld + row) : (uint32_t)(row * ld + gcol)) : 0u);
                    }
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = 16 * j + Mfma<T>::row(lk, v);
                        U[t][v] += (row < mu && colok) ? alpha * x[v] : T(0);
                    }
                }
                continue;
            }
            const T* Ap = base_ptr<T>(ct.flags & 7, vec) + ct.a_off;
            const T* Bp = base_ptr<T>((ct.flags >> 3) & 7, vec) + ct.b_off;
            const bool ta = (ct.flags & F_TRANS_A) != 0, tb = (ct.flags & F_TRANS_B) != 0;
            const int K = ct.k, lda = ct.lda, ldb = ct.ldb;
            int kstart = 0;
            {   // B row-major: through the wave's LDS scratch (FP64 up to three tiles per wave)
                if (!ta && !tb && K >= 16 && (sizeof(T) == 4 || ntu <= 3)) {
                    const int lr = opaque(lr0), lk = opaque(lk0);
                    T* scr = sBt + wv * 256;
                    const int ncolv = min(16, ncv - 16 * w);
                    const int bc0 = tk.col0 + 16 * w;
                    switch (ntu) {
                        case 1: tall_u_rowB<T, RW, 1>(U, Ap, Bp, lda, ldb, K, wv, mu, lr, lk, bc0, ncolv, alpha, scr); break;
                        case 2: tall_u_rowB<T, RW, 2>(U, Ap, Bp, lda, ldb, K, wv, mu, lr, lk, bc0, ncolv, alpha, scr); break;
                        case 3: tall_u_rowB<T, RW, 3>(U, Ap, Bp, lda, ldb, K, wv, mu, lr, lk, bc0, ncolv, alpha, scr); break;
                        case 4:
                            if constexpr (sizeof(T) == 4)
                                tall_u_rowB<T, RW, 4>(U, Ap, Bp, lda, ldb, K, wv, mu, lr, lk, bc0, ncolv, alpha, scr);
                            break;
                        case 5:
                            if constexpr (sizeof(T) == 4)
                                tall_u_rowB<T, RW, 5>(U, Ap, Bp, lda, ldb, K, wv, mu, lr, lk, bc0, ncolv, alpha, scr);
                            break;
                        default: break;
                    }
                    kstart = K;
                }
            }
            // the common case, over the full chunks (FP64 up to three tiles per wave: the
            // FP64 fragments of four or five would not fit the registers)
            if ((sizeof(T) == 4 || ntu <= 3) && !ta && tb) {
                const int kfull = K & ~15;
                const bool tail = kfull < K && K >= 4;   // the partial chunk as vector loads too
                const int lr = opaque(lr0), lk = opaque(lk0);
                const int gcol = tk.col0 + 16 * w + lr;
                const bool colok = 16 * w + lr < ncv;
                if (kfull > 0 || tail) {
                    switch (ntu) {
                        case 1:
                            tall_u_fast<T, RW, 1>(U, Ap, Bp, lda, ldb, kfull, wv, mu, lr, lk, gcol, colok, alpha);
                            if (tail) tall_u_tail<T, RW, 1>(U, Ap, Bp, lda, ldb, kfull, K, wv, mu, lr, lk, gcol, colok, alpha);
                            break;
                        case 2:
                            tall_u_fast<T, RW, 2>(U, Ap, Bp, lda, ldb, kfull, wv, mu, lr, lk, gcol, colok, alpha);
                            if (tail) tall_u_tail<T, RW, 2>(U, Ap, Bp, lda, ldb, kfull, K, wv, mu, lr, lk, gcol, colok, alpha);
                            break;
                        case 3:
                            tall_u_fast<T, RW, 3>(U, Ap, Bp, lda, ldb, kfull, wv, mu, lr, lk, gcol, colok, alpha);
                            if (tail) tall_u_tail<T, RW, 3>(U, Ap, Bp, lda, ldb, kfull, K, wv, mu, lr, lk, gcol, colok, alpha);
                            break;
                        case 4:
                            if constexpr (sizeof(T) == 4) {
                                tall_u_fast<T, RW, 4>(U, Ap, Bp, lda, ldb, kfull, wv, mu, lr, lk, gcol, colok, alpha);
                                if (tail) tall_u_tail<T, RW, 4>(U, Ap, Bp, lda, ldb, kfull, K, wv, mu, lr, lk, gcol, colok, alpha);
                            }
                            break;
                        case 5:
                            if constexpr (sizeof(T) == 4) {
                                tall_u_fast<T, RW, 5>(U, Ap, Bp, lda, ldb, kfull, wv, mu, lr, lk, gcol, colok, alpha);
                                if (tail) tall_u_tail<T, RW, 5>(U, Ap, Bp, lda, ldb, kfull, K, wv, mu, lr, lk, gcol, colok, alpha);
                            }
                            break;
                        default: break;
                    }
                }
                kstart = tail ? K : kfull;
            }
            for (int k0 = kstart; k0 < K; k0 += 16) {
                T fa[RW][4], fb[4];
                {
                    const int lr = opaque(lr0), lk = opaque(lk0);
                    const int gcol = tk.col0 + 16 * w + lr;
                    const bool colok = 16 * w + lr < ncv;
                    const int kb = k0 + 4 * lk;
                    const bool vec4 = k0 + 16 <= K;
                    // B first: every tile's MFMAs need it, so the A loads behind it can
                    // still be in flight when the first tile's products start
                    if (tb && vec4) {
                        ld4_at(Bp, colok ? (uint32_t)(gcol * ldb + kb) : 0u, fb);
                    } else {
#pragma unroll
                        for (int s = 0; s < 4; ++s) {
                            const int k = kb + s;
                            const bool ok = colok && k < K;
                            fb[s] = ld_at(Bp, ok ? (tb ? (uint32_t)(gcol * ldb + k) : (uint32_t)(k * ldb + gcol)) : 0u);
                        }
                    }
#pragma unroll
                    for (int t = 0; t < RW; ++t) {
                        const int j = wv + 4 * t;
                        if (j >= nru) continue;
                        const int row = 16 * j + lr;
                        const bool rok = row < mu;
                        if (!ta && vec4) {
                            ld4_at(Ap, rok ? (uint32_t)(row * lda + kb) : 0u, fa[t]);
                        } else {
#pragma unroll
                            for (int s = 0; s < 4; ++s) {
                                const int k = kb + s;
                                const bool ok = rok && k < K;
                                fa[t][s] = ld_at(Ap, ok ? (ta ? (uint32_t)(k * lda + row) : (uint32_t)(row * lda + k)) : 0u);
                            }
                        }
                    }
                    // loads at masked positions read element 0 of the operand (finite), so
                    // a zero factor clears them; the k mask matters only in the last chunk
                    const T acol = colok ? alpha : T(0);
                    if (vec4) {
#pragma unroll
                        for (int s = 0; s < 4; ++s) fb[s] *= acol;
                    } else {
#pragma unroll
                        for (int s = 0; s < 4; ++s) fb[s] = kb + s < K ? acol * fb[s] : T(0);
                    }
                }
#pragma unroll
                for (int t = 0; t < RW; ++t) {
                    if (wv + 4 * t >= nru) continue;
#pragma unroll
                    for (int s = 0; s < 4; ++s) U[t] = Mfma<T>::mma(fa[t][s], fb[s], U[t]);
                }
            }
        }
        {
            const int lk = opaque(lk0);
#pragma unroll
            for (int t = 0; t < RW; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (16 * (wv + 4 * t) + Mfma<T>::row(lk, v) >= mu) U[t][v] = T(0);
        }
        if (gr.xid_coef != 0.0) {   // identity X: output rows are U's rows (m == mu), same owner wave
            const T xi = (T)gr.xid_coef;
#pragma unroll
            for (int t = 0; t < RW; ++t) acc[t] += xi * U[t];
        }
        if (gr.flags & G_HAS_X) {
            T* su = sU[buf];
            const T xc = (T)gr.x_coef;
            {
                const int lr = opaque(lr0), lk = opaque(lk0);
#pragma unroll
                for (int t = 0; t < RW; ++t) {
                    const int j = wv + 4 * t;
                    if (j >= nru) continue;
#pragma unroll
                    for (int v = 0; v < 4; ++v) su[lr * LD + 16 * j + Mfma<T>::row(lk, v)] = xc * U[t][v];
                }
            }
            __syncthreads();
            const T* Xp = base_ptr<T>(gr.flags & 7, vec) + gr.x_off;
            const bool tx = (gr.flags & G_TRANS_X) != 0;
            const int ldx = gr.ldx;
            int qstart = 0;
            if (tx && mu >= 16 && (sizeof(T) == 4 || nto <= 3)) {   // X used as its transpose: through LDS
                const int lr = opaque(lr0), lk = opaque(lk0);
                T* scr = sBt + wv * 256;
                switch (nto) {
                    case 1: tall_x_transX<T, RW, 1, LD>(acc, Xp, ldx, mu, su, wv, tk.m, lr, lk, scr); break;
                    case 2: tall_x_transX<T, RW, 2, LD>(acc, Xp, ldx, mu, su, wv, tk.m, lr, lk, scr); break;
                    case 3: tall_x_transX<T, RW, 3, LD>(acc, Xp, ldx, mu, su, wv, tk.m, lr, lk, scr); break;
                    case 4:
                        if constexpr (sizeof(T) == 4) tall_x_transX<T, RW, 4, LD>(acc, Xp, ldx, mu, su, wv, tk.m, lr, lk, scr);
                        break;
                    case 5:
                        if constexpr (sizeof(T) == 4) tall_x_transX<T, RW, 5, LD>(acc, Xp, ldx, mu, su, wv, tk.m, lr, lk, scr);
                        break;
                    default: break;
                }
                qstart = nru;
            }
            if ((sizeof(T) == 4 || nto <= 3) && !tx) {   // row-major X over the full 16-row chunks of U
                const int qfull = mu >> 4;
                const bool tail = 16 * qfull < mu && mu >= 4;
                const int lr = opaque(lr0), lk = opaque(lk0);
                if (qfull > 0 || tail) {
                    switch (nto) {
                        case 1:
                            tall_x_fast<T, RW, 1, LD>(acc, Xp, ldx, qfull, su, wv, tk.m, lr, lk);
                            if (tail) tall_x_tail<T, RW, 1, LD>(acc, Xp, ldx, 16 * qfull, mu, su, wv, tk.m, lr, lk);
                            break;
                        case 2:
                            tall_x_fast<T, RW, 2, LD>(acc, Xp, ldx, qfull, su, wv, tk.m, lr, lk);
                            if (tail) tall_x_tail<T, RW, 2, LD>(acc, Xp, ldx, 16 * qfull, mu, su, wv, tk.m, lr, lk);
                            break;
                        case 3:
                            tall_x_fast<T, RW, 3, LD>(acc, Xp, ldx, qfull, su, wv, tk.m, lr, lk);
                            if (tail) tall_x_tail<T, RW, 3, LD>(acc, Xp, ldx, 16 * qfull, mu, su, wv, tk.m, lr, lk);
                            break;
                        case 4:
                            if constexpr (sizeof(T) == 4) {
                                tall_x_fast<T, RW, 4, LD>(acc, Xp, ldx, qfull, su, wv, tk.m, lr, lk);
                                if (tail) tall_x_tail<T, RW, 4, LD>(acc, Xp, ldx, 16 * qfull, mu, su, wv, tk.m, lr, lk);
                            }
                            break;
                        case 5:
                            if constexpr (sizeof(T) == 4) {
                                tall_x_fast<T, RW, 5, LD>(acc, Xp, ldx, qfull, su, wv, tk.m, lr, lk);
                                if (tail) tall_x_tail<T, RW, 5, LD>(acc, Xp, ldx, 16 * qfull, mu, su, wv, tk.m, lr, lk);
                            }
                            break;
                        default: break;
                    }
                }
                qstart = tail ? nru : qfull;
            }
            for (int q = qstart; q < nru; ++q) {
                const int lr = opaque(lr0), lk = opaque(lk0);
                // B fragment: U[16q + 4 lk + s][lr], s = 0..3 (four consecutive k of U^T's row lr)
                T ub[4];
                {
                    const T* p = su + lr * LD + 16 * q + 4 * lk;
                    if constexpr (sizeof(T) == 4) {
                        const float4 v = *reinterpret_cast<const float4*>(p);
                        ub[0] = v.x; ub[1] = v.y; ub[2] = v.z; ub[3] = v.w;
                    } else {
                        const double2 a = *reinterpret_cast<const double2*>(p);
                        const double2 b = *reinterpret_cast<const double2*>(p + 2);
                        ub[0] = a.x; ub[1] = a.y; ub[2] = b.x; ub[3] = b.y;
                    }
                }
                const bool full = 16 * q + 16 <= mu;
                T xf[RW][4];
#pragma unroll
                for (int t = 0; t < RW; ++t) {
                    const int i = wv + 4 * t;
                    if (i >= nrm) continue;
                    const int row = 16 * i + lr;
                    const bool rok = row < tk.m;
                    if (!tx && full) {
                        ld4_at(Xp, rok ? (uint32_t)(row * ldx + 16 * q + 4 * lk) : 0u, xf[t]);
                    } else {
#pragma unroll
                        for (int s = 0; s < 4; ++s) {
                            const int k = 16 * q + 4 * lk + s;
                            const bool ok = rok && k < mu;
                            xf[t][s] = ld_at(Xp, ok ? (tx ? (uint32_t)(k * ldx + row) : (uint32_t)(row * ldx + k)) : 0u);
                        }
                    }
                }
#pragma unroll
                for (int t = 0; t < RW; ++t) {
                    if (wv + 4 * t >= nrm) continue;
#pragma unroll
                    for (int s = 0; s < 4; ++s) acc[t] = Mfma<T>::mma(xf[t][s], ub[s], acc[t]);
                }
            }
            if constexpr (NB == 1) __syncthreads();   // the single buffer is rewritten by the next group
            else buf ^= 1;
        }
    }

    const int cbuf = tk.cbuf & 15;
    const bool accum = (tk.cbuf >> 8) & 1;
    const bool local = (tk.cbuf >> 9) & 1;
    T* Cp = const_cast<T*>(base_ptr<T>(cbuf, vec)) + tk.c_off + (local ? 0 : tk.col0);
    const int mycol = 16 * w + lr0;
    if (mycol < ncv) {
#pragma unroll
        for (int t = 0; t < RW; ++t) {
            const int i = wv + 4 * t;
            if (i >= nrm) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 16 * i + Mfma<T>::row(lk0, v);
                if (row < tk.m) {
                    T* d = Cp + (uint32_t)(row * tk.ldc + mycol);
                    *d = accum ? *d + acc[t][v] : acc[t][v];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// wave_kernel: tiles of at most 16*RT rows (and U rows) x 16*CT columns.  One
// wave per task, four independent tasks per workgroup, no LDS and no
// barrier: MFMA fragments come straight from global memory and the
// intermediate U stays in the accumulator registers (used as the B operand
// of X . U with X loaded in the matching k order).  The small register
// footprint allows many waves per SIMD, which is what hides the latency of
// the short, dependent products of small sector blocks.
// ---------------------------------------------------------------------------
template <typename T, int RT, int CT> struct WaveOcc {
    static constexpr int waves = sizeof(T) == 4 ? (RT * CT == 1 ? 6 : 5) : (RT * CT <= 2 ? 4 : 3);
};

template <typename T, int RT, int CT, bool LR>
__global__ __launch_bounds__(256, (WaveOcc<T, RT, CT>::waves)) void wave_kernel(Bases<T> Bargs, const Task* __restrict__ tasks, int ntask,
                                                   const Group* __restrict__ groups,
                                                   const Contrib* __restrict__ contribs, int nvec) {
    using V4 = typename Mfma<T>::v4;
    __shared__ Group sG[LR ? 4 : 1][LR ? kRecG : 1];
    __shared__ Contrib sC[LR ? 4 : 1][LR ? kRecC : 1];
    (void)Bargs;
    const int wv = threadIdx.x >> 6;
    int wg, vec;
    unit_vec(nvec, wg, vec);
    const int ti = wg * 4 + wv;
    if (ti >= ntask) return;
    const int lane = threadIdx.x & 63;
    const int lr = lane & 15;
    const int lk = lane >> 4;
    const Task tk = tasks[ti];
    const int ncv = min(tk.ncol, tk.n - tk.col0);
    Recs<LR> R;
    if constexpr (LR) {   // each wave stages its own task's records; in-order LDS within a wave
        const int cb = stage_records(groups, contribs, tk.g0, tk.g1, sG[wv], sC[wv], lane, 64);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        R = Recs<true>{sG[wv], sC[wv], tk.g0, cb};
    } else {
        R = Recs<false>{groups, contribs};
    }

    V4 acc[RT][CT];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < CT; ++j) acc[i][j] = V4{0, 0, 0, 0};

    for (int g = tk.g0; g < tk.g1; ++g) {
        const Group gr = R.group(g);
        const int mu = gr.mu;
        V4 U[RT][CT];
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
            for (int j = 0; j < CT; ++j) U[i][j] = V4{0, 0, 0, 0};
        for (int c = gr.c0; c < gr.c1; ++c) {
            const Contrib ct = R.contrib(c);
            const T alpha = (T)ct.alpha;
            if (is_identity(ct.flags)) {
                const bool ida = (ct.flags & F_ID_A) != 0, idb = (ct.flags & F_ID_B) != 0;
                const T* P = ida ? base_ptr<T>((ct.flags >> 3) & 7, vec) + ct.b_off
                                 : base_ptr<T>(ct.flags & 7, vec) + ct.a_off;
                const bool tp = ida ? (ct.flags & F_TRANS_B) != 0 : (ct.flags & F_TRANS_A) != 0;
                const int ld = ida ? ct.ldb : ct.lda;
                // loads first (clamped to offset 0 when out of range), masks after
                T x[RT][CT][4];
#pragma unroll
                for (int i = 0; i < RT; ++i)
#pragma unroll
                    for (int j = 0; j < CT; ++j) {
                        const int col = 16 * j + lr;
                        const int gc = tk.col0 + col;
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int row = 16 * i + Mfma<T>::row(lk, v);
                            const bool ok = row < mu && col < ncv;
                            if (ida && idb)
                                x[i][j][v] = ((int64_t)row + ct.a_off == gc) ? T(1) : T(0);
                            else
                                x[i][j][v] = ld_at(P, ok ? (tp ? (uint32_t)(gc * ld + row) : (uint32_t)(row * ld + gc)) : 0u);
                        }
                    }
#pragma unroll
                for (int i = 0; i < RT; ++i)
#pragma unroll
                    for (int j = 0; j < CT; ++j)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int row = 16 * i + Mfma<T>::row(lk, v);
                            const bool ok = row < mu && 16 * j + lr < ncv;
                            U[i][j][v] += ok ? alpha * x[i][j][v] : T(0);
                        }
                continue;
            }
            const T* Ap = base_ptr<T>(ct.flags & 7, vec) + ct.a_off;
            const T* Bp = base_ptr<T>((ct.flags >> 3) & 7, vec) + ct.b_off;
            const bool ta = (ct.flags & F_TRANS_A) != 0, tb = (ct.flags & F_TRANS_B) != 0;
            const int K = ct.k, lda = ct.lda, ldb = ct.ldb;
            for (int k0 = 0; k0 < K; k0 += 16) {
                // all fragment loads of the chunk first (clamped), masks at use
                T fa[RT][4], fb[CT][4];
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int k = k0 + 4 * lk + s;
#pragma unroll
                    for (int i = 0; i < RT; ++i) {
                        const int row = 16 * i + lr;
                        const bool ok = row < mu && k < K;
                        fa[i][s] = ld_at(Ap, ok ? (ta ? (uint32_t)(k * lda + row) : (uint32_t)(row * lda + k)) : 0u);
                    }
#pragma unroll
                    for (int j = 0; j < CT; ++j) {
                        const int gc = tk.col0 + 16 * j + lr;
                        const bool ok = 16 * j + lr < ncv && k < K;
                        fb[j][s] = ld_at(Bp, ok ? (tb ? (uint32_t)(gc * ldb + k) : (uint32_t)(k * ldb + gc)) : 0u);
                    }
                }
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int k = k0 + 4 * lk + s;
#pragma unroll
                    for (int i = 0; i < RT; ++i) fa[i][s] = (16 * i + lr < mu && k < K) ? alpha * fa[i][s] : T(0);
#pragma unroll
                    for (int j = 0; j < CT; ++j) fb[j][s] = (16 * j + lr < ncv && k < K) ? fb[j][s] : T(0);
                }
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int i = 0; i < RT; ++i)
#pragma unroll
                        for (int j = 0; j < CT; ++j) U[i][j] = Mfma<T>::mma(fa[i][s], fb[j][s], U[i][j]);
            }
        }
        if (gr.flags & G_HAS_X) {
            const T* Xp = base_ptr<T>(gr.flags & 7, vec) + gr.x_off;
            const bool tx = (gr.flags & G_TRANS_X) != 0;
            const T xc = (T)gr.x_coef;
            const int ldx = gr.ldx;
#pragma unroll
            for (int q = 0; q < RT; ++q) {      // U row tile = k tile of X . U
                T xf[RT][4];
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int k = 16 * q + Mfma<T>::row(lk, s);
#pragma unroll
                    for (int i = 0; i < RT; ++i) {
                        const int row = 16 * i + lr;
                        const bool ok = row < tk.m && k < mu;
                        xf[i][s] = ld_at(Xp, ok ? (tx ? (uint32_t)(k * ldx + row) : (uint32_t)(row * ldx + k)) : 0u);
                    }
                }
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int k = 16 * q + Mfma<T>::row(lk, s);
#pragma unroll
                    for (int i = 0; i < RT; ++i) xf[i][s] = (16 * i + lr < tk.m && k < mu) ? xc * xf[i][s] : T(0);
                }
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int i = 0; i < RT; ++i)
#pragma unroll
                        for (int j = 0; j < CT; ++j) acc[i][j] = Mfma<T>::mma(xf[i][s], U[q][j][s], acc[i][j]);
            }
        }
        if (gr.xid_coef != 0.0) {
            const T xi = (T)gr.xid_coef;
#pragma unroll
            for (int i = 0; i < RT; ++i)
#pragma unroll
                for (int j = 0; j < CT; ++j) acc[i][j] += xi * U[i][j];
        }
    }

    const int cbuf = tk.cbuf & 15;
    const bool accum = (tk.cbuf >> 8) & 1;
    const bool local = (tk.cbuf >> 9) & 1;
    T* Cp = const_cast<T*>(base_ptr<T>(cbuf, vec)) + tk.c_off + (local ? 0 : tk.col0);
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < CT; ++j) {
            const int col = 16 * j + lr;
            if (col >= ncv) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 16 * i + Mfma<T>::row(lk, v);
                if (row < tk.m) {
                    T* d = Cp + (uint32_t)(row * tk.ldc + col);
                    *d = accum ? *d + acc[i][j][v] : acc[i][j][v];
                }
            }
        }
}

template <typename T, bool LR>
static const void* chain_func(int cls) {
    constexpr int RS = kShortRows / 16, RL = kMaxRows / 16;
    if (cls >= kTallClass0) {   // tall classes: one workgroup per column slice
        switch (cls - kTallClass0 + 1) {
            case 1: return (const void*)&tall_kernel<T, 1, LR>;
            case 2: return (const void*)&tall_kernel<T, 2, LR>;
            case 3: return (const void*)&tall_kernel<T, 3, LR>;
            case 4: return (const void*)&tall_kernel<T, 4, LR>;
            case 5: return (const void*)&tall_kernel<T, 5, LR>;
            case 6: return (const void*)&tall_kernel<T, 6, LR>;
            default: return nullptr;
        }
    }
    if (cls >= kNumTileClass) {   // wave classes: four tasks per workgroup
        switch (cls - kNumTileClass) {
            case 0: return (const void*)&wave_kernel<T, 1, 1, LR>;
            case 1: return (const void*)&wave_kernel<T, 1, 2, LR>;
            case 2: return (const void*)&wave_kernel<T, 2, 1, LR>;
            case 3: return (const void*)&wave_kernel<T, 2, 2, LR>;
            default: return nullptr;
        }
    }
    // tile classes: four column slices per workgroup; five row tiles for
    // classes below kColClasses, six above
    switch (cls) {
        case 0: return (const void*)&slice_kernel<T, 1, RS, LR>;
        case 1: return (const void*)&slice_kernel<T, 2, RS, LR>;
        case 2: return (const void*)&slice_kernel<T, 3, RS, LR>;
        case 3: return (const void*)&slice_kernel<T, 4, RS, LR>;
        case 4: return (const void*)&slice_kernel<T, 5, RS, LR>;
        case 5: return (const void*)&slice_kernel<T, 6, RS, LR>;
        case 6: return (const void*)&slice_kernel<T, 1, RL, LR>;
        case 7: return (const void*)&slice_kernel<T, 2, RL, LR>;
        case 8: return (const void*)&slice_kernel<T, 3, RL, LR>;
        case 9: return (const void*)&slice_kernel<T, 4, RL, LR>;
        case 10: return (const void*)&slice_kernel<T, 5, RL, LR>;
        case 11: return (const void*)&slice_kernel<T, 6, RL, LR>;
        default: return nullptr;
    }
}

// workgroups of one vector's launch of class cls
static int chain_units(int cls, int ntask) {
    if (cls >= kTallClass0) return ntask * (cls - kTallClass0 + 1);
    if (cls >= kNumTileClass) return (ntask + 3) / 4;
    return (ntask * (cls % kColClasses + 1) + 3) / 4;
}

template <typename T>
static KernelDesc chain_desc(int cls, bool lds_records, int ntask, int nvec) {
    KernelDesc d{};
    if (ntask <= 0 || cls < 0 || cls >= kNumClass) return d;
    d.func = lds_records ? chain_func<T, true>(cls) : chain_func<T, false>(cls);
    d.gx = cls >= kTallClass0 ? grid_tall(ntask, cls - kTallClass0 + 1, nvec)
                              : grid_units(chain_units(cls, ntask), nvec);
    d.gy = 1;
    d.bx = 256;
    return d;
}
KernelDesc chain_desc_f64(int cls, bool lds_records, int ntask, int nvec) {
    return chain_desc<double>(cls, lds_records, ntask, nvec);
}
KernelDesc chain_desc_f32(int cls, bool lds_records, int ntask, int nvec) {
    return chain_desc<float>(cls, lds_records, ntask, nvec);
}

template <typename T>
static int launch_chain(int cls, bool lds_records, const Task* t, int ntask, const Group* g, const Contrib* c,
                        const Bases<T>& b, int nvec, void* stream) {
    if (ntask <= 0) return 0;
    const KernelDesc d = chain_desc<T>(cls, lds_records, ntask, nvec);
    if (!d.func) return (int)hipErrorInvalidValue;
    ChainArgs<T> a(b, t, ntask, g, c, nvec);
    return (int)hipLaunchKernel(d.func, dim3(d.gx, d.gy), dim3(d.bx), a.ptrs, 0, (hipStream_t)stream);
}

int launch_chain_f64(int cls, bool lds_records, const Task* t, int ntask, const Group* g, const Contrib* c,
                     const Bases<double>& b, int nvec, void* stream) {
    return launch_chain<double>(cls, lds_records, t, ntask, g, c, b, nvec, stream);
}
int launch_chain_f32(int cls, bool lds_records, const Task* t, int ntask, const Group* g, const Contrib* c,
                     const Bases<float>& b, int nvec, void* stream) {
    return launch_chain<float>(cls, lds_records, t, ntask, g, c, b, nvec, stream);
}

// One workgroup per split tile.  Each thread owns up to kRedPer elements of
// the tile (stride kRedThreads, so every load of one slot is coalesced) and
// keeps their sums in registers while it walks the slots.  The loads of a
// slot are unconditional (indices past the tile are clamped to its last
// element and their sums discarded), so they are all in flight together;
// each element is still summed in slot order.
// A tile of up to kMaxRows x kMaxCols elements takes one pass; taller tiles
// (tall classes) take several passes over element ranges of that size.
constexpr int kRedThreads = 512;
constexpr int kRedPer = (kMaxRows * kMaxCols + kRedThreads - 1) / kRedThreads;

template <typename T>
__global__ __launch_bounds__(kRedThreads) void reduce_kernel(const Reduce* __restrict__ red, Bases<T> b) {
    const Reduce r = red[blockIdx.x];
    const int vec = blockIdx.y;
    const int cbuf = r.cbuf & 15;
    const bool accum = (r.cbuf >> 8) & 1;
    const T* P = b.p[kPartialBuf] + r.poff + (int64_t)vec * b.vstride[kPartialBuf];
    T* Cp = b.p[cbuf] + r.c_off + (int64_t)vec * b.vstride[cbuf];
    const int slot = r.m * r.ncol;   // <= kTallRows * kMaxCols (checked on the host)
    const int tid = threadIdx.x;
    for (int e0 = 0; e0 < slot; e0 += kRedPer * kRedThreads) {
        T s[kRedPer];
#pragma unroll
        for (int i = 0; i < kRedPer; ++i) s[i] = 0;
        for (int q = 0; q < r.nslot; ++q) {
            const T* Pq = P + (int64_t)q * slot;
            T v[kRedPer];
#pragma unroll
            for (int i = 0; i < kRedPer; ++i) v[i] = Pq[min(e0 + tid + i * kRedThreads, slot - 1)];
#pragma unroll
            for (int i = 0; i < kRedPer; ++i) s[i] += v[i];
        }
#pragma unroll
        for (int i = 0; i < kRedPer; ++i) {
            const int e = e0 + tid + i * kRedThreads;
            if (e >= slot) continue;
            const int row = e / r.ncol, j = e - row * r.ncol;
            T* d = Cp + (int64_t)row * r.ldc + r.col0 + j;
            *d = accum ? *d + s[i] : s[i];
        }
    }
}

template <typename T>
static KernelDesc reduce_desc(int nred, int nvec) {
    KernelDesc d{};
    if (nred <= 0) return d;
    d.func = (const void*)&reduce_kernel<T>;
    d.gx = (unsigned)nred;
    d.gy = (unsigned)nvec;
    d.bx = kRedThreads;
    return d;
}
KernelDesc reduce_desc_f64(int nred, int nvec) { return reduce_desc<double>(nred, nvec); }
KernelDesc reduce_desc_f32(int nred, int nvec) { return reduce_desc<float>(nred, nvec); }

template <typename T>
static int launch_reduce(const Reduce* r, int nred, const Bases<T>& b, int nvec, void* stream) {
    if (nred <= 0) return 0;
    const KernelDesc d = reduce_desc<T>(nred, nvec);
    ReduceArgs<T> a(r, b);
    return (int)hipLaunchKernel(d.func, dim3(d.gx, d.gy), dim3(d.bx), a.ptrs, 0, (hipStream_t)stream);
}
int launch_reduce_f64(const Reduce* r, int nred, const Bases<double>& b, int nvec, void* stream) {
    return launch_reduce<double>(r, nred, b, nvec, stream);
}
int launch_reduce_f32(const Reduce* r, int nred, const Bases<float>& b, int nvec, void* stream) {
    return launch_reduce<float>(r, nred, b, nvec, stream);
}

// ---------------------------------------------------------------------------
// elementwise
// ---------------------------------------------------------------------------

__global__ void cast_d2f_kernel(const double* __restrict__ in, float* __restrict__ out, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (float)in[i];
}
__global__ void cast_f2d_kernel(const float* __restrict__ in, double* __restrict__ out, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (double)in[i];
}

static dim3 grid_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

int launch_cast_d2f(const double* in, float* out, int64_t n, void* stream) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL(cast_d2f_kernel, grid_for(n), dim3(256), 0, (hipStream_t)stream, in, out, n);
    return (int)hipGetLastError();
}
int launch_cast_f2d(const float* in, double* out, int64_t n, void* stream) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL(cast_f2d_kernel, grid_for(n), dim3(256), 0, (hipStream_t)stream, in, out, n);
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// H_eff diagonal
// ---------------------------------------------------------------------------

__global__ void diag_kernel(const DiagBlock* __restrict__ blocks, const DiagTerm* __restrict__ terms,
                            Bases<double> b, double* __restrict__ diag) {
    const DiagBlock bl = blocks[blockIdx.x];
    const int n = bl.ma * bl.mb;
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        const int i = e / bl.mb, j = e % bl.mb;
        double s = 0.0;
        for (int t = bl.c0; t < bl.c1; ++t) {
            const DiagTerm dt = terms[t];
            double x = 1.0, y = 1.0;
            if (dt.x_off >= 0) x = b.p[dt.xbuf][dt.x_off + (int64_t)i * dt.ldx + i];
            if (dt.y_off >= 0) y = b.p[dt.ybuf][dt.y_off + (int64_t)j * dt.ldy + j];
            s += dt.coef * x * y;
        }
        diag[bl.off + e] = s;
    }
}

int launch_diag(const DiagBlock* blocks, int nblock, const DiagTerm* terms, Bases<double> b,
                double* diag, void* stream) {
    if (nblock <= 0) return 0;
    hipLaunchKernelGGL(diag_kernel, dim3(nblock), dim3(256), 0, (hipStream_t)stream, blocks, terms,
                       b, diag);
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Davidson helpers
// ---------------------------------------------------------------------------

constexpr int kGramMax = 64;
constexpr int kChunk = 256 * 16;

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// partial[(chunk * nw + j) * kGramMax + i] = sum over the chunk of V_i * W_j
__global__ __launch_bounds__(256) void gram_partial_kernel(const double* __restrict__ V, int nv,
                                                           const double* __restrict__ W,
                                                           int64_t n, double* __restrict__ part) {
    __shared__ double red[4][kGramMax];
    const int j = blockIdx.y;
    const int64_t e0 = (int64_t)blockIdx.x * kChunk;
    double acc[kGramMax];
#pragma unroll
    for (int i = 0; i < kGramMax; ++i) acc[i] = 0.0;
    for (int t = 0; t < kChunk / 256; ++t) {
        const int64_t e = e0 + t * 256 + threadIdx.x;
        if (e < n) {
            const double w = W[(int64_t)j * n + e];
#pragma unroll
            for (int i = 0; i < kGramMax; ++i)
                if (i < nv) acc[i] += V[(int64_t)i * n + e] * w;
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < kGramMax; ++i) {
        if (i < nv) {
            const double s = wave_sum(acc[i]);
            if (lane == 0) red[wave][i] = s;
        }
    }
    __syncthreads();
    if (threadIdx.x < nv) {
        const int i = threadIdx.x;
        part[((int64_t)blockIdx.x * gridDim.y + j) * kGramMax + i] =
            red[0][i] + red[1][i] + red[2][i] + red[3][i];
    }
}

__global__ void gram_reduce_kernel(const double* __restrict__ part, int nchunk, int nv, int nw,
                                   double* __restrict__ G, int ldg) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nv * nw) return;
    const int i = idx / nw, j = idx % nw;
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += part[((int64_t)c * nw + j) * kGramMax + i];
    G[i * ldg + j] = s;
}

int launch_gram(const double* V, int nv, const double* W, int nw, int64_t n, double* G, int ldg,
                double* scratch, void* stream) {
    if (nv <= 0 || nw <= 0) return 0;
    if (nv > kGramMax) return (int)hipErrorInvalidValue;
    const int nchunk = (int)((n + kChunk - 1) / kChunk);
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(gram_partial_kernel, dim3(nchunk, nw), dim3(256), 0, s, V, nv, W, n, scratch);
    hipLaunchKernelGGL(gram_reduce_kernel, dim3((nv * nw + 255) / 256), dim3(256), 0, s, scratch,
                       nchunk, nv, nw, G, ldg);
    return (int)hipGetLastError();
}

constexpr int kCombMax = 32;

// Y_j[e] = sum_i C[i*ldc+j] V_i[e] + beta Y_j[e], j < ny <= 32, i < nv <= 64
__global__ __launch_bounds__(256) void combine_kernel(const double* __restrict__ V, int nv,
                                                      const double* __restrict__ C, int ldc,
                                                      double* __restrict__ Y, int ny, int64_t n,
                                                      double beta) {
    __shared__ double sc[kGramMax * kCombMax];
    for (int idx = threadIdx.x; idx < nv * ny; idx += blockDim.x)
        sc[(idx / ny) * kCombMax + idx % ny] = C[(idx / ny) * ldc + idx % ny];
    __syncthreads();
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        double acc[kCombMax];
#pragma unroll
        for (int j = 0; j < kCombMax; ++j) acc[j] = 0.0;
        for (int i = 0; i < nv; ++i) {
            const double v = V[(int64_t)i * n + e];
#pragma unroll
            for (int j = 0; j < kCombMax; ++j)
                if (j < ny) acc[j] += sc[i * kCombMax + j] * v;
        }
#pragma unroll
        for (int j = 0; j < kCombMax; ++j)
            if (j < ny) {
                double* y = Y + (int64_t)j * n + e;
                *y = (beta != 0.0 ? beta * *y : 0.0) + acc[j];
            }
    }
}

int launch_combine(const double* V, int nv, const double* C, int ldc, double* Y, int ny, int64_t n,
                   double beta, void* stream) {
    if (ny <= 0) return 0;
    if (nv > kGramMax || ny > kCombMax) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(combine_kernel, grid_for(n), dim3(256), 0, (hipStream_t)stream, V, nv, C,
                       ldc, Y, ny, n, beta);
    return (int)hipGetLastError();
}

__global__ void precond_kernel(const double* __restrict__ r, const double* __restrict__ d,
                               double theta, double clamp, double* __restrict__ t, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (clamp < 0.0) {
            t[i] = r[i];
            continue;
        }
        double den = theta - d[i];
        if (fabs(den) < clamp) den = den < 0 ? -clamp : clamp;
        t[i] = r[i] / den;
    }
}

int launch_precond(const double* r, const double* d, double theta, double clamp, double* t, int64_t n,
                   void* stream) {
    hipLaunchKernelGGL(precond_kernel, grid_for(n), dim3(256), 0, (hipStream_t)stream, r, d, theta,
                       clamp, t, n);
    return (int)hipGetLastError();
}

// Cyclic Jacobi with round-robin parallel ordering (disjoint rotations of a
// step are applied together).  N = n rounded up to even; padding rows hold
// a large diagonal and stay decoupled.
__global__ __launch_bounds__(256) void jacobi_kernel(const double* __restrict__ Ain, int n,
                                                     double* __restrict__ w, double* __restrict__ Zout) {
    constexpr int NM = 64;
    __shared__ double a[NM][NM + 1];
    __shared__ double z[NM][NM + 1];
    __shared__ double cs[NM / 2], sn[NM / 2];
    __shared__ int pp[NM / 2], qq[NM / 2];
    __shared__ double offn, totn;
    __shared__ int order[NM];
    const int N = (n + 1) & ~1;
    const int tid = threadIdx.x;
    double big = 0.0;
    for (int i = 0; i < n; ++i) big = fmax(big, fabs(Ain[i * n + i]));
    big = 4.0 * big + 1.0;
    for (int idx = tid; idx < N * N; idx += blockDim.x) {
        const int i = idx / N, j = idx % N;
        a[i][j] = (i < n && j < n) ? Ain[i * n + j] : (i == j ? big : 0.0);
        z[i][j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int sweep = 0; sweep < 60; ++sweep) {
        if (tid == 0) {
            double o = 0.0, t = 0.0;
            for (int i = 0; i < N; ++i)
                for (int j = 0; j < N; ++j) {
                    const double v = a[i][j] * a[i][j];
                    t += v;
                    if (i != j) o += v;
                }
            offn = o;
            totn = t;
        }
        __syncthreads();
        if (offn <= 1e-30 * totn || offn == 0.0) break;
        for (int r = 0; r < N - 1; ++r) {
            if (tid < N / 2) {
                int p, q;
                if (tid == 0) { p = N - 1; q = r; }
                else { p = (r + tid) % (N - 1); q = (r - tid + N - 1) % (N - 1); }
                if (p > q) { const int t = p; p = q; q = t; }
                const double apq = a[p][q];
                double c = 1.0, s = 0.0;
                if (apq != 0.0) {
                    const double th = (a[q][q] - a[p][p]) / (2.0 * apq);
                    const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                    c = 1.0 / sqrt(t * t + 1.0);
                    s = t * c;
                }
                pp[tid] = p; qq[tid] = q; cs[tid] = c; sn[tid] = s;
            }
            __syncthreads();
            for (int idx = tid; idx < (N / 2) * N; idx += blockDim.x) {   // rows
                const int k = idx / N, j = idx % N;
                const int p = pp[k], q = qq[k];
                const double c = cs[k], s = sn[k];
                const double ap = a[p][j], aq = a[q][j];
                a[p][j] = c * ap - s * aq;
                a[q][j] = s * ap + c * aq;
            }
            __syncthreads();
            for (int idx = tid; idx < (N / 2) * N; idx += blockDim.x) {   // columns
                const int k = idx / N, i = idx % N;
                const int p = pp[k], q = qq[k];
                const double c = cs[k], s = sn[k];
                const double ap = a[i][p], aq = a[i][q];
                a[i][p] = c * ap - s * aq;
                a[i][q] = s * ap + c * aq;
                const double zp = z[i][p], zq = z[i][q];
                z[i][p] = c * zp - s * zq;
                z[i][q] = s * zp + c * zq;
            }
            __syncthreads();
        }
    }
    if (tid == 0) {
        for (int i = 0; i < n; ++i) order[i] = i;
        // only the first n (unpadded) columns are eigenpairs of the input
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j)
                if (a[order[j]][order[j]] < a[order[i]][order[i]]) {
                    const int t = order[i]; order[i] = order[j]; order[j] = t;
                }
    }
    __syncthreads();
    for (int idx = tid; idx < n * n; idx += blockDim.x) {
        const int i = idx / n, j = idx % n;
        Zout[i * n + j] = z[i][order[j]];
    }
    if (tid < n) w[tid] = a[order[tid]][order[tid]];
}

int launch_jacobi(const double* A, int n, double* w, double* Z, void* stream) {
    if (n > 64 || n < 1) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, A, n, w, Z);
    return (int)hipGetLastError();
}

__global__ void nonfinite_kernel(const double* __restrict__ x, int64_t n, int* flag) {
    int bad = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        if (!isfinite(x[i])) bad = 1;
    if (bad) atomicAdd(flag, 1);
}

int launch_nonfinite(const double* x, int64_t n, int* flag, void* stream) {
    hipLaunchKernelGGL(nonfinite_kernel, grid_for(n), dim3(256), 0, (hipStream_t)stream, x, n, flag);
    return (int)hipGetLastError();
}

__global__ void psi_gather_kernel(const GatherBlock* __restrict__ blocks, const double* __restrict__ psi,
                                  int part, int64_t dim, double scale, double* __restrict__ out) {
    const GatherBlock B = blocks[blockIdx.x];
    const int64_t v = blockIdx.y;
    const double* src = psi + v * dim + B.src;
    double* dst = out + B.dst + part * B.pcol + v * B.vcol;
    const int64_t n = (int64_t)B.ma * B.mb;
    for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
        const int64_t i = e / B.mb, j = e - i * B.mb;
        dst[B.trans ? j * B.ld + i : i * B.ld + j] = scale * src[e];
    }
}

int launch_psi_gather(const GatherBlock* blocks, int nblock, int nvec, const double* psi, int part, int64_t dim,
                      double scale, double* out, void* stream) {
    if (nblock <= 0 || nvec <= 0) return 0;
    hipLaunchKernelGGL(psi_gather_kernel, dim3(nblock, nvec), dim3(256), 0, (hipStream_t)stream, blocks, psi, part,
                       dim, scale, out);
    return (int)hipGetLastError();
}

__global__ void evec_gather_kernel(const EvecBlock* __restrict__ blocks, const double* __restrict__ evec,
                                   double* __restrict__ iso) {
    const EvecBlock B = blocks[blockIdx.x];
    const int64_t n = (int64_t)B.d * B.k;
    for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
        const int64_t i = e / B.k, c = e - i * B.k;
        iso[B.dst + e] = evec[B.src + i + (B.d - 1 - c) * (int64_t)B.d];
    }
}

int launch_evec_gather(const EvecBlock* blocks, int nblock, const double* evec, double* iso, void* stream) {
    if (nblock <= 0) return 0;
    hipLaunchKernelGGL(evec_gather_kernel, dim3(nblock), dim3(256), 0, (hipStream_t)stream, blocks, evec, iso);
    return (int)hipGetLastError();
}

}  // namespace dmrgk
