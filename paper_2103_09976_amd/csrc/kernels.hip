// HIP kernels (gfx950) of the DMRG library.
//
// chain_kernel: the grouped, output-stationary sector-GEMM engine described
// in kernels.hpp.  One 256-thread workgroup (4 waves of 64) owns one output
// tile of up to 64*MT rows x 32 columns.  MFMA 16x16x4 (f64 or f32) tiles:
// wave w owns row tiles w, w+4, ...; both 16-column tiles.  The operands of
// A . B and of X . U go from global memory (L2 / MALL hits for the reused
// sector blocks) straight into MFMA fragments, one 16-k chunk ahead of the
// multiply; only the group intermediate U (mu x 32), needed by every output
// row, passes through LDS, with one barrier pair per group.
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

constexpr int LDU_S = kTN + 1;    // LDS row stride of U

// One MFMA k-step group covers 16 consecutive k.  Lane (r = l%16, g = l/16)
// supplies k = k0 + 4g + s at step s (s = 0..3): the four k of one lane are
// contiguous in a row-major operand, and any fixed permutation of k used by
// both operands leaves the product unchanged.
template <typename T>
struct Frag {
    T v[4];
};

// A fragment: rows row0..row0+15 of a (rows x K) operand, k0..k0+15.
// PAT 0: lane group g holds k = k0 + 4g + s; PAT 1: k = k0 + g + 4s.
template <typename T, int PAT = 0>
__device__ inline Frag<T> load_a(const T* __restrict__ p, int ld, bool tr, int row, int rows, int k0,
                                 int K, int g, T scale) {
    Frag<T> f;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int k = PAT == 0 ? k0 + 4 * g + s : k0 + g + 4 * s;
        T x = 0;
        if (row < rows && k < K) x = tr ? p[(int64_t)k * ld + row] : p[(int64_t)row * ld + k];
        f.v[s] = scale * x;
    }
    return f;
}

// B fragment: column col of a (K x cols) operand, k0..k0+15
template <typename T>
__device__ inline Frag<T> load_b(const T* __restrict__ p, int ld, bool tr, int col, int cols, int k0,
                                 int K, int g) {
    Frag<T> f;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int k = k0 + 4 * g + s;
        T x = 0;
        if (col < cols && k < K) x = tr ? p[(int64_t)col * ld + k] : p[(int64_t)k * ld + col];
        f.v[s] = x;
    }
    return f;
}

template <typename T, int MT>
__global__ __launch_bounds__(256) void chain_kernel(const Task* __restrict__ tasks,
                                                    const Group* __restrict__ groups,
                                                    const Contrib* __restrict__ contribs,
                                                    Bases<T> B) {
    using V4 = typename Mfma<T>::v4;
    constexpr int RC = 64 * MT;
    __shared__ T sU[RC * LDU_S];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int lr = lane & 15;
    const int lk = lane >> 4;
    const Task tk = tasks[blockIdx.x];
    const int vec = blockIdx.y;

    V4 acc[MT][2];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = V4{0, 0, 0, 0};

    for (int g = tk.g0; g < tk.g1; ++g) {
        const Group gr = groups[g];
        const int mu = gr.mu;
        V4 U[MT][2];
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) U[i][j] = V4{0, 0, 0, 0};

        for (int c = gr.c0; c < gr.c1; ++c) {
            const Contrib ct = contribs[c];
            const int abuf = ct.flags & 7, bbuf = (ct.flags >> 3) & 7;
            const T* Ap = B.p[abuf] + ct.a_off + (int64_t)vec * B.vstride[abuf];
            const T* Bp = B.p[bbuf] + ct.b_off + (int64_t)vec * B.vstride[bbuf];
            const T alpha = (T)ct.alpha;
            const bool ta = (ct.flags & F_TRANS_A) != 0, tb = (ct.flags & F_TRANS_B) != 0;
            if (ct.flags & (F_ID_A | F_ID_B)) {
                const bool ida = (ct.flags & F_ID_A) != 0, idb = (ct.flags & F_ID_B) != 0;
#pragma unroll
                for (int i = 0; i < MT; ++i) {
                    const int rt = wave + 4 * i;
                    if (16 * rt >= mu) continue;
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        const int col = tk.col0 + 16 * j + lr;
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int row = 16 * rt + Mfma<T>::row(lk, v);
                            T val = 0;
                            if (row < mu && col < tk.n) {
                                if (ida && idb)   // a_off: diagonal offset of the identity
                                    val = (row + ct.a_off == col) ? alpha : T(0);
                                else if (ida)
                                    val = alpha * (tb ? Bp[(int64_t)col * ct.ldb + row]
                                                      : Bp[(int64_t)row * ct.ldb + col]);
                                else
                                    val = alpha * (ta ? Ap[(int64_t)col * ct.lda + row]
                                                      : Ap[(int64_t)row * ct.lda + col]);
                            }
                            U[i][j][v] += val;
                        }
                    }
                }
                continue;
            }
            // U += alpha A . B, operands straight from global memory with the
            // next 16-k chunk prefetched while the current one is multiplied
            const int K = ct.k;
            const int n = tk.n, c0 = tk.col0;
            Frag<T> fa[MT], fb[2], na[MT], nb[2];
#pragma unroll
            for (int i = 0; i < MT; ++i) {
                const int rt = wave + 4 * i;
                if (16 * rt < mu) fa[i] = load_a(Ap, ct.lda, ta, 16 * rt + lr, mu, 0, K, lk, alpha);
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) fb[j] = load_b(Bp, ct.ldb, tb, c0 + 16 * j + lr, n, 0, K, lk);
            for (int k0 = 0; k0 < K; k0 += 16) {
                const int k1 = k0 + 16;
                if (k1 < K) {
#pragma unroll
                    for (int i = 0; i < MT; ++i) {
                        const int rt = wave + 4 * i;
                        if (16 * rt < mu) na[i] = load_a(Ap, ct.lda, ta, 16 * rt + lr, mu, k1, K, lk, alpha);
                    }
#pragma unroll
                    for (int j = 0; j < 2; ++j) nb[j] = load_b(Bp, ct.ldb, tb, c0 + 16 * j + lr, n, k1, K, lk);
                }
#pragma unroll
                for (int i = 0; i < MT; ++i) {
                    const int rt = wave + 4 * i;
                    if (16 * rt >= mu) continue;
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        U[i][0] = Mfma<T>::mma(fa[i].v[s], fb[0].v[s], U[i][0]);
                        U[i][1] = Mfma<T>::mma(fa[i].v[s], fb[1].v[s], U[i][1]);
                    }
                }
                if (k1 < K) {
#pragma unroll
                    for (int i = 0; i < MT; ++i) fa[i] = na[i];
                    fb[0] = nb[0];
                    fb[1] = nb[1];
                }
            }
        }

        if (gr.flags & G_HAS_X) {
            // U is shared by all output rows: park it in LDS
            __syncthreads();
#pragma unroll
            for (int i = 0; i < MT; ++i) {
                const int rt = wave + 4 * i;
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        sU[(16 * rt + Mfma<T>::row(lk, v)) * LDU_S + 16 * j + lr] = U[i][j][v];
            }
            __syncthreads();
            const int xbuf = gr.flags & 7;
            const bool tx = (gr.flags & G_TRANS_X) != 0;
            const T* Xp = B.p[xbuf] + gr.x_off + (int64_t)vec * B.vstride[xbuf];
            const T xc = (T)gr.x_coef;
            const int m = tk.m;
            Frag<T> fx[MT], nx[MT];
#pragma unroll
            for (int i = 0; i < MT; ++i) {
                const int rt = wave + 4 * i;
                if (16 * rt < m) fx[i] = load_a(Xp, gr.ldx, tx, 16 * rt + lr, m, 0, mu, lk, xc);
            }
            for (int k0 = 0; k0 < mu; k0 += 16) {
                const int k1 = k0 + 16;
                if (k1 < mu) {
#pragma unroll
                    for (int i = 0; i < MT; ++i) {
                        const int rt = wave + 4 * i;
                        if (16 * rt < m) nx[i] = load_a(Xp, gr.ldx, tx, 16 * rt + lr, m, k1, mu, lk, xc);
                    }
                }
                T b0[4], b1[4];
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    // rows of U at or beyond mu are zero in LDS (their U tiles were zero)
                    const int kr = k0 + 4 * lk + s;
                    b0[s] = sU[kr * LDU_S + lr];
                    b1[s] = sU[kr * LDU_S + 16 + lr];
                }
#pragma unroll
                for (int i = 0; i < MT; ++i) {
                    const int rt = wave + 4 * i;
                    if (16 * rt >= m) continue;
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        acc[i][0] = Mfma<T>::mma(fx[i].v[s], b0[s], acc[i][0]);
                        acc[i][1] = Mfma<T>::mma(fx[i].v[s], b1[s], acc[i][1]);
                    }
                }
                if (k1 < mu) {
#pragma unroll
                    for (int i = 0; i < MT; ++i) fx[i] = nx[i];
                }
            }
        }
        if (gr.xid_coef != 0.0) {
            const T xi = (T)gr.xid_coef;
#pragma unroll
            for (int i = 0; i < MT; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] += xi * U[i][j];
        }
    }

    const int cbuf = tk.cbuf & 15;
    const bool accum = (tk.cbuf >> 8) & 1;
    const int cshift = ((tk.cbuf >> 9) & 1) ? tk.col0 : 0;   // partial tiles store columns from 0
    T* Cp = B.p[cbuf] + tk.c_off - cshift + (int64_t)vec * B.vstride[cbuf];
#pragma unroll
    for (int i = 0; i < MT; ++i) {
        const int rt = wave + 4 * i;
        if (16 * rt >= tk.m) continue;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int col = tk.col0 + 16 * j + lr;
            if (col >= tk.n) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 16 * rt + Mfma<T>::row(lk, v);
                if (row < tk.m) {
                    T* d = Cp + (int64_t)row * tk.ldc + col;
                    *d = accum ? *d + acc[i][j][v] : acc[i][j][v];
                }
            }
        }
    }
}

// Wave-per-task variant for tiles of at most 16*RT rows: each wave owns a whole
// output tile (RT row tiles x 2 column tiles) and a whole group intermediate
// U, so no LDS and no barrier is needed.  The accumulator layout of U is used
// directly as the B operand of X . U: MFMA step (t, v) takes from lane group g
// the U row held in register v of row tile t, and X is loaded with the same k
// order (f32: k = 16t + 4g + v, f64: k = 16t + 4v + g).
template <typename T, int RT>
__global__ __launch_bounds__(256) void chain_wave_kernel(const Task* __restrict__ tasks, int ntask,
                                                         const Group* __restrict__ groups,
                                                         const Contrib* __restrict__ contribs,
                                                         Bases<T> B) {
    using V4 = typename Mfma<T>::v4;
    constexpr int XPAT = Mfma<T>::row(1, 0) == 4 ? 0 : 1;   // f32: rows 4g+v; f64: rows 4v+g
    const int lane = threadIdx.x & 63;
    const int ti = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (ti >= ntask) return;
    const int lr = lane & 15;
    const int lk = lane >> 4;
    const Task tk = tasks[ti];
    const int vec = blockIdx.y;

    V4 acc[RT][2];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = V4{0, 0, 0, 0};

    for (int g = tk.g0; g < tk.g1; ++g) {
        const Group gr = groups[g];
        const int mu = gr.mu;
        V4 U[RT][2];
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) U[i][j] = V4{0, 0, 0, 0};

        for (int c = gr.c0; c < gr.c1; ++c) {
            const Contrib ct = contribs[c];
            const int abuf = ct.flags & 7, bbuf = (ct.flags >> 3) & 7;
            const T* Ap = B.p[abuf] + ct.a_off + (int64_t)vec * B.vstride[abuf];
            const T* Bp = B.p[bbuf] + ct.b_off + (int64_t)vec * B.vstride[bbuf];
            const T alpha = (T)ct.alpha;
            const bool ta = (ct.flags & F_TRANS_A) != 0, tb = (ct.flags & F_TRANS_B) != 0;
            if (ct.flags & (F_ID_A | F_ID_B)) {
                const bool ida = (ct.flags & F_ID_A) != 0, idb = (ct.flags & F_ID_B) != 0;
#pragma unroll
                for (int i = 0; i < RT; ++i) {
                    if (16 * i >= mu) continue;
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        const int col = tk.col0 + 16 * j + lr;
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int row = 16 * i + Mfma<T>::row(lk, v);
                            T val = 0;
                            if (row < mu && col < tk.n) {
                                if (ida && idb)
                                    val = (row + ct.a_off == col) ? alpha : T(0);
                                else if (ida)
                                    val = alpha * (tb ? Bp[(int64_t)col * ct.ldb + row]
                                                      : Bp[(int64_t)row * ct.ldb + col]);
                                else
                                    val = alpha * (ta ? Ap[(int64_t)col * ct.lda + row]
                                                      : Ap[(int64_t)row * ct.lda + col]);
                            }
                            U[i][j][v] += val;
                        }
                    }
                }
                continue;
            }
            const int K = ct.k;
            const int n = tk.n, c0 = tk.col0;
            const int nrt = (mu + 15) >> 4;
            for (int k0 = 0; k0 < K; k0 += 16) {
                Frag<T> fb0 = load_b(Bp, ct.ldb, tb, c0 + lr, n, k0, K, lk);
                Frag<T> fb1 = load_b(Bp, ct.ldb, tb, c0 + 16 + lr, n, k0, K, lk);
                Frag<T> fa[RT];
#pragma unroll
                for (int i = 0; i < RT; ++i)
                    if (i < nrt) fa[i] = load_a(Ap, ct.lda, ta, 16 * i + lr, mu, k0, K, lk, alpha);
#pragma unroll
                for (int i = 0; i < RT; ++i) {
                    if (i >= nrt) continue;
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        U[i][0] = Mfma<T>::mma(fa[i].v[s], fb0.v[s], U[i][0]);
                        U[i][1] = Mfma<T>::mma(fa[i].v[s], fb1.v[s], U[i][1]);
                    }
                }
            }
        }

        if (gr.flags & G_HAS_X) {
            const int xbuf = gr.flags & 7;
            const bool tx = (gr.flags & G_TRANS_X) != 0;
            const T* Xp = B.p[xbuf] + gr.x_off + (int64_t)vec * B.vstride[xbuf];
            const T xc = (T)gr.x_coef;
            const int m = tk.m;
            const int nmt = (m + 15) >> 4;
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                if (16 * t >= mu) continue;
                Frag<T> fx[RT];
#pragma unroll
                for (int i = 0; i < RT; ++i)
                    if (i < nmt) fx[i] = load_a<T, XPAT>(Xp, gr.ldx, tx, 16 * i + lr, m, 16 * t, mu, lk, xc);
#pragma unroll
                for (int i = 0; i < RT; ++i) {
                    if (i >= nmt) continue;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        acc[i][0] = Mfma<T>::mma(fx[i].v[v], U[t][0][v], acc[i][0]);
                        acc[i][1] = Mfma<T>::mma(fx[i].v[v], U[t][1][v], acc[i][1]);
                    }
                }
            }
        }
        if (gr.xid_coef != 0.0) {
            const T xi = (T)gr.xid_coef;
#pragma unroll
            for (int i = 0; i < RT; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] += xi * U[i][j];
        }
    }

    const int cbuf = tk.cbuf & 15;
    const bool accum = (tk.cbuf >> 8) & 1;
    const int cshift = ((tk.cbuf >> 9) & 1) ? tk.col0 : 0;   // partial tiles store columns from 0
    T* Cp = B.p[cbuf] + tk.c_off - cshift + (int64_t)vec * B.vstride[cbuf];
#pragma unroll
    for (int i = 0; i < RT; ++i) {
        if (16 * i >= tk.m) continue;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int col = tk.col0 + 16 * j + lr;
            if (col >= tk.n) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 16 * i + Mfma<T>::row(lk, v);
                if (row < tk.m) {
                    T* d = Cp + (int64_t)row * tk.ldc + col;
                    *d = accum ? *d + acc[i][j][v] : acc[i][j][v];
                }
            }
        }
    }
}

template <typename T>
static int launch_chain(int cls, int variant, const Task* t, int ntask, const Group* g, const Contrib* c,
                        const Bases<T>& b, int nvec, void* stream) {
    if (ntask <= 0) return 0;
    dim3 grid(ntask, nvec), block(256);
    hipStream_t s = (hipStream_t)stream;
    dim3 wgrid((ntask + 3) / 4, nvec);
    if (variant == 1 && cls == 0)
        hipLaunchKernelGGL((chain_wave_kernel<T, 4>), wgrid, block, 0, s, t, ntask, g, c, b);
    else if (variant == 1 && cls == 1)
        hipLaunchKernelGGL((chain_wave_kernel<T, 8>), wgrid, block, 0, s, t, ntask, g, c, b);
    else if (cls == 0)
        hipLaunchKernelGGL((chain_kernel<T, 1>), grid, block, 0, s, t, g, c, b);
    else if (cls == 1)
        hipLaunchKernelGGL((chain_kernel<T, 2>), grid, block, 0, s, t, g, c, b);
    else
        hipLaunchKernelGGL((chain_kernel<T, 5>), grid, block, 0, s, t, g, c, b);
    return (int)hipGetLastError();
}

int launch_chain_f64(int cls, int variant, const Task* t, int ntask, const Group* g, const Contrib* c,
                     const Bases<double>& b, int nvec, void* stream) {
    return launch_chain<double>(cls, variant, t, ntask, g, c, b, nvec, stream);
}
int launch_chain_f32(int cls, int variant, const Task* t, int ntask, const Group* g, const Contrib* c,
                     const Bases<float>& b, int nvec, void* stream) {
    return launch_chain<float>(cls, variant, t, ntask, g, c, b, nvec, stream);
}

template <typename T>
__global__ __launch_bounds__(256) void reduce_kernel(const Reduce* __restrict__ red, Bases<T> b) {
    const Reduce r = red[blockIdx.x];
    const int vec = blockIdx.y;
    const int ncol = min(32, r.n - r.col0);
    const int cbuf = r.cbuf & 15;
    const bool accum = (r.cbuf >> 8) & 1;
    const T* P = b.p[kPartialBuf] + r.poff + (int64_t)vec * b.vstride[kPartialBuf];
    T* Cp = b.p[cbuf] + r.c_off + (int64_t)vec * b.vstride[cbuf];
    const int64_t slot = (int64_t)r.m * 32;
    for (int e = threadIdx.x; e < r.m * 32; e += blockDim.x) {
        const int row = e >> 5, j = e & 31;
        if (j >= ncol) continue;
        T s = 0;
        for (int q = 0; q < r.nslot; ++q) s += P[q * slot + e];
        T* d = Cp + (int64_t)row * r.ldc + r.col0 + j;
        *d = accum ? *d + s : s;
    }
}

template <typename T>
static int launch_reduce(const Reduce* r, int nred, const Bases<T>& b, int nvec, void* stream) {
    if (nred <= 0) return 0;
    hipLaunchKernelGGL(reduce_kernel<T>, dim3(nred, nvec), dim3(256), 0, (hipStream_t)stream, r, b);
    return (int)hipGetLastError();
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

}  // namespace dmrgk
