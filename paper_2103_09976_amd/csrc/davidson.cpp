// Block Davidson solution of the effective eigenproblem (Appendix A,
// H_eff Psi = E Psi; the paper solves it with Davidson's method).
//
// All vector algebra runs on the device in FP64: Gram products V^T W,
// Rayleigh-Ritz with a single-workgroup Jacobi eigensolver, Ritz vectors,
// residuals, the diagonal preconditioner t = r / (theta - diag H_eff) and
// classical Gram-Schmidt applied twice.  Only the small subspace matrix,
// residual norms and eigenvalues cross to the host each iteration.
//
// Mixed policy: H_eff psi runs in FP32 while the largest residual norm is
// above switch_tol; then the basis restarts from the Ritz vectors with FP64
// products and continues in FP64, so converged energies come from FP64
// products.  With fixed_iters the final energies are FP64 Rayleigh quotients
// of the Ritz vectors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "core.hpp"

using namespace dmrg;

extern "C" int64_t dmrg_heff_dim(const dmrg_heff* H);

namespace {

struct DavWs {
    Ctx* C;
    int64_t region = -1;
    double *V, *W, *X, *HX, *R, *diag, *small, *scratch, *V2, *W2;
    float *f_in, *f_out;
    int* flag;
};

struct Timer {
    hipEvent_t a, b;
    Timer() { hipEventCreate(&a); hipEventCreate(&b); }
    ~Timer() { hipEventDestroy(a); hipEventDestroy(b); }
};

}  // namespace

static dmrg_status matvec(dmrg_heff* H, DavWs& ws, int prec, const double* in, double* out, int n, int64_t dim,
                          void* stream, double* ms, int* cnt32) {
    Timer t;
    hipStream_t s = (hipStream_t)stream;
    hipEventRecord(t.a, s);
    dmrg_status st;
    if (prec == DMRG_PREC_F32) {
        DMRG_HIP(dmrgk::launch_cast_d2f(in, ws.f_in, (int64_t)n * dim, stream));
        st = dmrg_heff_apply(H, DMRG_PREC_F32, n, ws.f_in, ws.f_out, stream);
        if (st != DMRG_OK) return st;
        DMRG_HIP(dmrgk::launch_cast_f2d(ws.f_out, out, (int64_t)n * dim, stream));
        *cnt32 += n;
    } else {
        st = dmrg_heff_apply(H, DMRG_PREC_F64, n, in, out, stream);
        if (st != DMRG_OK) return st;
    }
    hipEventRecord(t.b, s);
    DMRG_HIP(hipMemsetAsync(ws.flag, 0, sizeof(int), s));
    DMRG_HIP(dmrgk::launch_nonfinite(out, (int64_t)n * dim, ws.flag, stream));
    int bad = 0;
    DMRG_HIP(hipMemcpyAsync(&bad, ws.flag, sizeof(int), hipMemcpyDeviceToHost, s));
    DMRG_HIP(hipStreamSynchronize(s));
    float e = 0.f;
    hipEventElapsedTime(&e, t.a, t.b);
    *ms += e;
    if (bad) return fail(DMRG_E_NONFINITE, "non-finite value in H_eff psi");
    return DMRG_OK;
}

// G[i*ld + j] = <A_i, B_j> copied to host (na x nb)
static dmrg_status gram_host(DavWs& ws, const double* A, int na, const double* B, int nb, int64_t dim,
                             std::vector<double>& out, void* stream) {
    DMRG_HIP(dmrgk::launch_gram(A, na, B, nb, dim, ws.small, nb, ws.scratch, stream));
    out.assign((size_t)na * nb, 0.0);
    DMRG_HIP(hipMemcpyAsync(out.data(), ws.small, out.size() * 8, hipMemcpyDeviceToHost, (hipStream_t)stream));
    DMRG_HIP(hipStreamSynchronize((hipStream_t)stream));
    return DMRG_OK;
}

// Y_j (+)= sum_i C[i*ny + j] A_i   (C on host, uploaded)
static dmrg_status combine(DavWs& ws, const double* A, int na, const std::vector<double>& Ch, double* Y, int ny,
                           int64_t dim, double beta, void* stream) {
    double* Cd = ws.small + 64 * 64;
    DMRG_HIP(hipMemcpyAsync(Cd, Ch.data(), Ch.size() * 8, hipMemcpyHostToDevice, (hipStream_t)stream));
    DMRG_HIP(hipStreamSynchronize((hipStream_t)stream));   // Ch is pageable and short-lived
    DMRG_HIP(dmrgk::launch_combine(A, na, Cd, ny, Y, ny, dim, beta, stream));
    return DMRG_OK;
}

// orthonormalise vector t against V[0:nv] (CGS2); returns its norm before normalisation
static dmrg_status orth_append(DavWs& ws, double* V, int nv, double* t, int64_t dim, double& nrm, void* stream) {
    std::vector<double> c;
    for (int pass = 0; pass < 2 && nv > 0; ++pass) {
        dmrg_status st = gram_host(ws, V, nv, t, 1, dim, c, stream);
        if (st != DMRG_OK) return st;
        for (double& x : c) x = -x;
        st = combine(ws, V, nv, c, t, 1, dim, 1.0, stream);
        if (st != DMRG_OK) return st;
    }
    dmrg_status st = gram_host(ws, t, 1, t, 1, dim, c, stream);
    if (st != DMRG_OK) return st;
    nrm = std::sqrt(std::max(0.0, c[0]));
    return DMRG_OK;
}

static dmrg_status scale_into(DavWs& ws, const double* src, double s, double* dst, int64_t dim, void* stream) {
    std::vector<double> c(1, s);
    return combine(ws, src, 1, c, dst, 1, dim, 0.0, stream);
}

extern "C" dmrg_status dmrg_davidson(dmrg_heff* H, int32_t k, double* psi_io, double* energies,
                                     const dmrg_dav_opts* opts, dmrg_dav_stats* stats, void* stream) {
    if (!H || !psi_io || !energies || !opts) return fail(DMRG_E_ARG, "null argument");
    if (k < 1 || k > 16) return fail(DMRG_E_ARG, "n_roots must be 1..16");
    const int msub = std::min(64, std::max(opts->max_subspace, 2 * k));
    if (msub < 2 * k) return fail(DMRG_E_ARG, "max_subspace too small");
    if (opts->precision != DMRG_PREC_F64 && opts->precision != DMRG_PREC_F32)
        return fail(DMRG_E_ARG, "bad precision");
    const int64_t dim = dmrg_heff_dim(H);
    Ctx* C = heff_ctx(H);
    hipStream_t s = (hipStream_t)stream;
    DavWs ws;
    ws.C = C;
    const int64_t nchunk = (dim + 4095) / 4096;
    const int keep = std::min(msub - k, std::max(2 * k, msub / 3));   // Ritz vectors kept at restart
    const int64_t bytes = ((int64_t)(2 * msub + 3 * k + 2 * keep) * dim + dim) * 8 + 2 * (int64_t)k * dim * 4 +
                          (int64_t)(64 * 64 * 2) * 8 + nchunk * 64 * 64 * 8 + 16384;
    ws.region = C->arena.alloc(bytes);
    if (ws.region < 0) return fail(DMRG_E_WORKSPACE, "arena too small for the Davidson workspace");
    char* p = C->arena.base + ws.region;
    auto take = [&](int64_t n) { char* q = p; p += (n + 255) / 256 * 256; return q; };
    ws.V = (double*)take((int64_t)msub * dim * 8);
    ws.W = (double*)take((int64_t)msub * dim * 8);
    ws.X = (double*)take((int64_t)k * dim * 8);
    ws.HX = (double*)take((int64_t)k * dim * 8);
    ws.R = (double*)take((int64_t)k * dim * 8);
    ws.diag = (double*)take(dim * 8);
    ws.V2 = (double*)take((int64_t)keep * dim * 8);
    ws.W2 = (double*)take((int64_t)keep * dim * 8);
    ws.small = (double*)take(64 * 64 * 2 * 8);
    ws.scratch = (double*)take(nchunk * 64 * 64 * 8);
    ws.f_in = (float*)take((int64_t)k * dim * 4);
    ws.f_out = (float*)take((int64_t)k * dim * 4);
    ws.flag = (int*)take(256);
    struct Release { Ctx* C; int64_t r; ~Release() { C->arena.release(r); } } rel{C, ws.region};

    Timer total;
    hipEventRecord(total.a, s);
    dmrg_dav_stats st_local{};
    double ms_mv = 0.0;
    int mv32 = 0, nmv = 0;
    dmrg_status st = dmrg_heff_diag(H, ws.diag, stream);
    if (st != DMRG_OK) return st;
    // start block: orthonormalised input vectors
    int nv = 0;
    for (int j = 0; j < k; ++j) {
        DMRG_HIP(hipMemcpyAsync(ws.V + (int64_t)nv * dim, psi_io + (int64_t)j * dim, dim * 8,
                                hipMemcpyDeviceToDevice, s));
        double nrm;
        st = orth_append(ws, ws.V, nv, ws.V + (int64_t)nv * dim, dim, nrm, stream);
        if (st != DMRG_OK) return st;
        if (!(nrm > 1e-12)) return fail(DMRG_E_ARG, "start vectors are linearly dependent");
        st = scale_into(ws, ws.V + (int64_t)nv * dim, 1.0 / nrm, ws.V + (int64_t)nv * dim, dim, stream);
        if (st != DMRG_OK) return st;
        ++nv;
    }
    int prec = opts->precision;
    const double clamp = opts->precond_clamp == 0.0 ? 0.1 : opts->precond_clamp;
    st = matvec(H, ws, prec, ws.V, ws.W, nv, dim, stream, &ms_mv, &mv32);
    if (st != DMRG_OK) return st;
    nmv += nv;
    std::vector<double> G((size_t)msub * msub, 0.0);
    auto refresh_G = [&](int c0, int c1) -> dmrg_status {
        std::vector<double> g;
        dmrg_status e = gram_host(ws, ws.V, nv, ws.W + (int64_t)c0 * dim, c1 - c0, dim, g, stream);
        if (e != DMRG_OK) return e;
        for (int i = 0; i < nv; ++i)
            for (int j = c0; j < c1; ++j) {
                const double x = g[(size_t)i * (c1 - c0) + (j - c0)];
                G[(size_t)i * msub + j] = x;
                if (i < c0) G[(size_t)j * msub + i] = x;   // projected matrix is symmetric
            }
        // new-new block: symmetrise
        for (int i = c0; i < c1; ++i)
            for (int j = i + 1; j < c1; ++j) {
                const double a = 0.5 * (G[(size_t)i * msub + j] + G[(size_t)j * msub + i]);
                G[(size_t)i * msub + j] = G[(size_t)j * msub + i] = a;
            }
        return DMRG_OK;
    };
    {
        std::vector<double> g;
        st = gram_host(ws, ws.V, nv, ws.W, nv, dim, g, stream);
        if (st != DMRG_OK) return st;
        for (int i = 0; i < nv; ++i)
            for (int j = 0; j < nv; ++j) G[(size_t)i * msub + j] = 0.5 * (g[(size_t)i * nv + j] + g[(size_t)j * nv + i]);
    }
    std::vector<double> theta(k, 0.0), res(k, 0.0);
    int it = 0;
    bool converged = false;
    for (;;) {
        // Rayleigh-Ritz
        std::vector<double> Gs((size_t)nv * nv);
        for (int i = 0; i < nv; ++i)
            for (int j = 0; j < nv; ++j) Gs[(size_t)i * nv + j] = G[(size_t)i * msub + j];
        double* Gd = ws.small;
        double* wd = ws.small + 64 * 64;
        double* Zd = ws.small + 64 * 64 + 64;
        DMRG_HIP(hipMemcpyAsync(Gd, Gs.data(), Gs.size() * 8, hipMemcpyHostToDevice, s));
        DMRG_HIP(dmrgk::launch_jacobi(Gd, nv, wd, Zd, stream));
        std::vector<double> w(nv), Z((size_t)nv * nv);
        DMRG_HIP(hipMemcpyAsync(w.data(), wd, nv * 8, hipMemcpyDeviceToHost, s));
        DMRG_HIP(hipMemcpyAsync(Z.data(), Zd, Z.size() * 8, hipMemcpyDeviceToHost, s));
        DMRG_HIP(hipStreamSynchronize(s));
        std::vector<double> Zk((size_t)nv * k), Zt((size_t)nv * k);
        for (int i = 0; i < nv; ++i)
            for (int j = 0; j < k; ++j) {
                Zk[(size_t)i * k + j] = Z[(size_t)i * nv + j];
                Zt[(size_t)i * k + j] = -w[j] * Z[(size_t)i * nv + j];
            }
        for (int j = 0; j < k; ++j) theta[j] = w[j];
        if ((st = combine(ws, ws.V, nv, Zk, ws.X, k, dim, 0.0, stream)) != DMRG_OK) return st;
        if ((st = combine(ws, ws.W, nv, Zk, ws.HX, k, dim, 0.0, stream)) != DMRG_OK) return st;
        if ((st = combine(ws, ws.W, nv, Zk, ws.R, k, dim, 0.0, stream)) != DMRG_OK) return st;
        if ((st = combine(ws, ws.V, nv, Zt, ws.R, k, dim, 1.0, stream)) != DMRG_OK) return st;
        std::vector<double> rr;
        if ((st = gram_host(ws, ws.R, k, ws.R, k, dim, rr, stream)) != DMRG_OK) return st;
        double rmax = 0.0;
        for (int j = 0; j < k; ++j) {
            res[j] = std::sqrt(std::max(0.0, rr[(size_t)j * k + j]));
            rmax = std::max(rmax, res[j]);
        }
        if (!std::isfinite(rmax)) return fail(DMRG_E_NONFINITE, "non-finite residual");
        const bool fixed = opts->fixed_iters > 0;
        converged = rmax <= opts->tol;
        if (fixed ? it >= opts->fixed_iters : (converged || it >= opts->max_iter)) break;
        // precision switch of the mixed policy
        bool restart = nv + k > msub;
        bool switched = false;
        if (prec == DMRG_PREC_F32 && !fixed && rmax <= opts->switch_tol) {
            prec = DMRG_PREC_F64;
            restart = true;
            switched = true;
        }
        if (restart && !switched && nv > keep) {
            // thick restart: V <- V Z[:, :keep], W <- W Z[:, :keep], G <- V^T W
            std::vector<double> Zr((size_t)nv * keep);
            for (int i = 0; i < nv; ++i)
                for (int j = 0; j < keep; ++j) Zr[(size_t)i * keep + j] = Z[(size_t)i * nv + j];
            for (int j0 = 0; j0 < keep; j0 += 32) {
                const int nj = std::min(32, keep - j0);
                std::vector<double> Cj((size_t)nv * nj);
                for (int i = 0; i < nv; ++i)
                    for (int j = 0; j < nj; ++j) Cj[(size_t)i * nj + j] = Zr[(size_t)i * keep + j0 + j];
                if ((st = combine(ws, ws.V, nv, Cj, ws.V2 + (int64_t)j0 * dim, nj, dim, 0.0, stream)) != DMRG_OK)
                    return st;
                if ((st = combine(ws, ws.W, nv, Cj, ws.W2 + (int64_t)j0 * dim, nj, dim, 0.0, stream)) != DMRG_OK)
                    return st;
            }
            DMRG_HIP(hipMemcpyAsync(ws.V, ws.V2, (int64_t)keep * dim * 8, hipMemcpyDeviceToDevice, s));
            DMRG_HIP(hipMemcpyAsync(ws.W, ws.W2, (int64_t)keep * dim * 8, hipMemcpyDeviceToDevice, s));
            nv = keep;
            std::vector<double> g;
            if ((st = gram_host(ws, ws.V, nv, ws.W, nv, dim, g, stream)) != DMRG_OK) return st;
            std::fill(G.begin(), G.end(), 0.0);
            for (int i = 0; i < nv; ++i)
                for (int j = 0; j < nv; ++j)
                    G[(size_t)i * msub + j] = 0.5 * (g[(size_t)i * nv + j] + g[(size_t)j * nv + i]);
            ++it;
            continue;
        }
        if (restart) {
            DMRG_HIP(hipMemcpyAsync(ws.V, ws.X, (int64_t)k * dim * 8, hipMemcpyDeviceToDevice, s));
            nv = k;
            if (switched) {
                st = matvec(H, ws, prec, ws.V, ws.W, k, dim, stream, &ms_mv, &mv32);
                if (st != DMRG_OK) return st;
                nmv += k;
            } else {
                DMRG_HIP(hipMemcpyAsync(ws.W, ws.HX, (int64_t)k * dim * 8, hipMemcpyDeviceToDevice, s));
            }
            std::vector<double> g;
            if ((st = gram_host(ws, ws.V, nv, ws.W, nv, dim, g, stream)) != DMRG_OK) return st;
            std::fill(G.begin(), G.end(), 0.0);
            for (int i = 0; i < nv; ++i)
                for (int j = 0; j < nv; ++j)
                    G[(size_t)i * msub + j] = 0.5 * (g[(size_t)i * nv + j] + g[(size_t)j * nv + i]);
            ++it;
            continue;
        }
        // corrections
        const int nv0 = nv;
        for (int j = 0; j < k; ++j) {
            if (res[j] <= opts->tol && !fixed) continue;
            double* t = ws.V + (int64_t)nv * dim;
            DMRG_HIP(dmrgk::launch_precond(ws.R + (int64_t)j * dim, ws.diag, theta[j], clamp, t, dim, stream));
            double n0;
            std::vector<double> c;
            if ((st = gram_host(ws, t, 1, t, 1, dim, c, stream)) != DMRG_OK) return st;
            n0 = std::sqrt(std::max(0.0, c[0]));
            if (!(n0 > 0.0)) continue;
            double nrm;
            if ((st = orth_append(ws, ws.V, nv, t, dim, nrm, stream)) != DMRG_OK) return st;
            if (!(nrm > 1e-12 * std::max(1.0, n0)) || !std::isfinite(nrm)) continue;
            if ((st = scale_into(ws, t, 1.0 / nrm, t, dim, stream)) != DMRG_OK) return st;
            ++nv;
        }
        if (nv == nv0) break;   // no new direction: the subspace is invariant
        st = matvec(H, ws, prec, ws.V + (int64_t)nv0 * dim, ws.W + (int64_t)nv0 * dim, nv - nv0, dim, stream,
                    &ms_mv, &mv32);
        if (st != DMRG_OK) return st;
        nmv += nv - nv0;
        if ((st = refresh_G(nv0, nv)) != DMRG_OK) return st;
        ++it;
    }
    // final energies: FP64 Rayleigh quotients when any FP32 product was used
    if (opts->precision == DMRG_PREC_F32 && (prec == DMRG_PREC_F32 || opts->fixed_iters > 0)) {
        st = matvec(H, ws, DMRG_PREC_F64, ws.X, ws.HX, k, dim, stream, &ms_mv, &mv32);
        if (st != DMRG_OK) return st;
        std::vector<double> xx, xh;
        if ((st = gram_host(ws, ws.X, k, ws.X, k, dim, xx, stream)) != DMRG_OK) return st;
        if ((st = gram_host(ws, ws.X, k, ws.HX, k, dim, xh, stream)) != DMRG_OK) return st;
        for (int j = 0; j < k; ++j) theta[j] = xh[(size_t)j * k + j] / xx[(size_t)j * k + j];
    }
    for (int j = 0; j < k; ++j) energies[j] = theta[j];
    DMRG_HIP(hipMemcpyAsync(psi_io, ws.X, (int64_t)k * dim * 8, hipMemcpyDeviceToDevice, s));
    hipEventRecord(total.b, s);
    DMRG_HIP(hipStreamSynchronize(s));
    float et = 0.f;
    hipEventElapsedTime(&et, total.a, total.b);
    st_local.iters = it;
    st_local.matvecs = nmv;
    st_local.matvecs_f32 = mv32;
    st_local.converged = converged ? 1 : 0;
    double rmax = 0.0;
    for (double r : res) rmax = std::max(rmax, r);
    st_local.max_residual = rmax;
    st_local.ms_total = et;
    st_local.ms_matvec = ms_mv;
    if (stats) *stats = st_local;
    return DMRG_OK;
}
