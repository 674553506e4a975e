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
#include <memory>
#include <vector>

#include "core.hpp"

using namespace dmrg;

extern "C" int64_t dmrg_heff_dim(const dmrg_heff* H);

namespace {

// Subspace dimension limit of the one-workgroup Jacobi eigensolver and of the
// Gram / combine kernels.
constexpr int kSubMax = 64;

struct DavWs {
    Ctx* C;
    int64_t region = -1;
    double *V, *W, *X, *HX, *R, *diag, *scratch, *V2, *W2;
    // small device matrices, each with its own slot: the projected matrix and
    // its eigenvectors (kSubMax^2 each), eigenvalues (kSubMax), combination
    // coefficients (kSubMax x 32) and Gram results (kSubMax^2)
    double *Gd, *Zd, *wd, *Cd, *gram;
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
    DMRG_HIP(dmrgk::launch_gram(A, na, B, nb, dim, ws.gram, nb, ws.scratch, stream));
    out.assign((size_t)na * nb, 0.0);
    DMRG_HIP(hipMemcpyAsync(out.data(), ws.gram, out.size() * 8, hipMemcpyDeviceToHost, (hipStream_t)stream));
    DMRG_HIP(hipStreamSynchronize((hipStream_t)stream));
    return DMRG_OK;
}

// Y_j (+)= sum_i C[i*ny + j] A_i   (C on host, uploaded)
static dmrg_status combine(DavWs& ws, const double* A, int na, const std::vector<double>& Ch, double* Y, int ny,
                           int64_t dim, double beta, void* stream) {
    double* Cd = ws.Cd;
    if (na > kSubMax || ny > 32) return fail(DMRG_E_ARG, "combination larger than the subspace limit");
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

// Workspace of a solve: V, W (max_subspace vectors each), Ritz vectors X, HX,
// residuals R (n_roots each), the H_eff diagonal, restart buffers V2, W2, the
// small matrices, Gram partials and the FP32 staging of mixed products.
static int64_t dav_bytes(int64_t dim, int k, int msub, int keep) {
    const int64_t nchunk = (dim + 4095) / 4096;
    return ((int64_t)(2 * msub + 3 * k + 2 * keep) * dim + dim) * 8 + 2 * (int64_t)k * dim * 4 +
           (int64_t)(4 * kSubMax * kSubMax + kSubMax) * 8 + nchunk * kSubMax * kSubMax * 8 + 16384;
}

static void dav_shape(int k, const dmrg_dav_opts* opts, int& msub, int& keep) {
    msub = std::min(kSubMax, std::max(opts->max_subspace, 2 * k));
    keep = std::min(msub - k, std::max(2 * k, msub / 3));   // Ritz vectors kept at a thick restart
}

int64_t dmrg::dav_workspace_bytes(int64_t dim, int k, const dmrg_dav_opts* opts) {
    int msub, keep;
    dav_shape(k, opts, msub, keep);
    return dav_bytes(dim, k, msub, keep);
}

// State of one block Davidson solve between calls (dmrg_davidson_start /
// _step / _finish).  Everything lives on the device except the projected
// matrix G, the last Ritz values, residual norms and eigenvectors Z.
struct dmrg_dav {
    dmrg_heff* H = nullptr;
    Ctx* C = nullptr;
    void* stream = nullptr;
    dmrg_dav_opts opts{};
    DavWs ws{};
    int k = 1, msub = 0, keep = 0, nv = 0, prec = 0, it = 0, nmv = 0, mv32 = 0;
    int64_t dim = 0;
    double clamp = 0.1, ms_mv = 0.0;
    bool done = false, converged = false;
    std::vector<double> G, theta, res, Z;
    Timer total;
    ~dmrg_dav() {
        if (ws.region >= 0) C->arena.release(ws.region);
    }
};

namespace {

dmrg_status refresh_G(dmrg_dav& D, int c0, int c1) {
    std::vector<double> g;
    const int64_t dim = D.dim;
    dmrg_status e = gram_host(D.ws, D.ws.V, D.nv, D.ws.W + (int64_t)c0 * dim, c1 - c0, dim, g, D.stream);
    if (e != DMRG_OK) return e;
    const int msub = D.msub;
    for (int i = 0; i < D.nv; ++i)
        for (int j = c0; j < c1; ++j) {
            const double x = g[(size_t)i * (c1 - c0) + (j - c0)];
            D.G[(size_t)i * msub + j] = x;
            if (i < c0) D.G[(size_t)j * msub + i] = x;   // projected matrix is symmetric
        }
    // new-new block: symmetrise
    for (int i = c0; i < c1; ++i)
        for (int j = i + 1; j < c1; ++j) {
            const double a = 0.5 * (D.G[(size_t)i * msub + j] + D.G[(size_t)j * msub + i]);
            D.G[(size_t)i * msub + j] = D.G[(size_t)j * msub + i] = a;
        }
    return DMRG_OK;
}

// G <- symmetrised V^T W of the current nv vectors (after a restart)
dmrg_status reset_G(dmrg_dav& D) {
    std::vector<double> g;
    dmrg_status st = gram_host(D.ws, D.ws.V, D.nv, D.ws.W, D.nv, D.dim, g, D.stream);
    if (st != DMRG_OK) return st;
    std::fill(D.G.begin(), D.G.end(), 0.0);
    for (int i = 0; i < D.nv; ++i)
        for (int j = 0; j < D.nv; ++j)
            D.G[(size_t)i * D.msub + j] = 0.5 * (g[(size_t)i * D.nv + j] + g[(size_t)j * D.nv + i]);
    return DMRG_OK;
}

// Rayleigh-Ritz on the current basis: Ritz values theta, vectors X, HX,
// residuals R = HX - theta X and their norms; then the termination test.
dmrg_status rayleigh_ritz(dmrg_dav& D) {
    DavWs& ws = D.ws;
    const int nv = D.nv, k = D.k, msub = D.msub;
    const int64_t dim = D.dim;
    hipStream_t s = (hipStream_t)D.stream;
    std::vector<double> Gs((size_t)nv * nv);
    for (int i = 0; i < nv; ++i)
        for (int j = 0; j < nv; ++j) Gs[(size_t)i * nv + j] = D.G[(size_t)i * msub + j];
    if (nv > kSubMax) return fail(DMRG_E_STATE, "subspace larger than the eigensolver limit");
    DMRG_HIP(hipMemcpyAsync(ws.Gd, Gs.data(), Gs.size() * 8, hipMemcpyHostToDevice, s));
    DMRG_HIP(dmrgk::launch_jacobi(ws.Gd, nv, ws.wd, ws.Zd, D.stream));
    std::vector<double> w(nv);
    D.Z.assign((size_t)nv * nv, 0.0);
    DMRG_HIP(hipMemcpyAsync(w.data(), ws.wd, nv * 8, hipMemcpyDeviceToHost, s));
    DMRG_HIP(hipMemcpyAsync(D.Z.data(), ws.Zd, D.Z.size() * 8, hipMemcpyDeviceToHost, s));
    DMRG_HIP(hipStreamSynchronize(s));
    std::vector<double> Zk((size_t)nv * k), Zt((size_t)nv * k);
    for (int i = 0; i < nv; ++i)
        for (int j = 0; j < k; ++j) {
            Zk[(size_t)i * k + j] = D.Z[(size_t)i * nv + j];
            Zt[(size_t)i * k + j] = -w[j] * D.Z[(size_t)i * nv + j];
        }
    for (int j = 0; j < k; ++j) D.theta[j] = w[j];
    dmrg_status st;
    if ((st = combine(ws, ws.V, nv, Zk, ws.X, k, dim, 0.0, D.stream)) != DMRG_OK) return st;
    if ((st = combine(ws, ws.W, nv, Zk, ws.HX, k, dim, 0.0, D.stream)) != DMRG_OK) return st;
    if ((st = combine(ws, ws.W, nv, Zk, ws.R, k, dim, 0.0, D.stream)) != DMRG_OK) return st;
    if ((st = combine(ws, ws.V, nv, Zt, ws.R, k, dim, 1.0, D.stream)) != DMRG_OK) return st;
    std::vector<double> rr;
    if ((st = gram_host(ws, ws.R, k, ws.R, k, dim, rr, D.stream)) != DMRG_OK) return st;
    double rmax = 0.0;
    for (int j = 0; j < k; ++j) {
        D.res[j] = std::sqrt(std::max(0.0, rr[(size_t)j * k + j]));
        rmax = std::max(rmax, D.res[j]);
    }
    if (!std::isfinite(rmax)) return fail(DMRG_E_NONFINITE, "non-finite residual");
    const bool fixed = D.opts.fixed_iters > 0;
    D.converged = rmax <= D.opts.tol;
    if (fixed ? D.it >= D.opts.fixed_iters : (D.converged || D.it >= D.opts.max_iter)) D.done = true;
    return DMRG_OK;
}

double max_res(const dmrg_dav& D) {
    double r = 0.0;
    for (double x : D.res) r = std::max(r, x);
    return r;
}

}  // namespace

extern "C" {

dmrg_status dmrg_davidson_start(dmrg_heff* H, int32_t k, const double* psi0, const dmrg_dav_opts* opts,
                                dmrg_dav** out, void* stream) {
    if (!H || !psi0 || !opts || !out) return fail(DMRG_E_ARG, "null argument");
    *out = nullptr;
    if (k < 1 || k > 16) return fail(DMRG_E_ARG, "n_roots must be 1..16");
    if (opts->precision != DMRG_PREC_F64 && opts->precision != DMRG_PREC_F32)
        return fail(DMRG_E_ARG, "bad precision");
    std::unique_ptr<dmrg_dav> D(new dmrg_dav());
    D->H = H;
    D->C = heff_ctx(H);
    D->stream = stream;
    D->opts = *opts;
    D->k = k;
    dav_shape(k, opts, D->msub, D->keep);
    if (D->msub < 2 * k) return fail(DMRG_E_ARG, "max_subspace too small");
    const int64_t dim = D->dim = dmrg_heff_dim(H);
    const int msub = D->msub, keep = D->keep;
    DavWs& ws = D->ws;
    ws.C = D->C;
    ws.region = D->C->arena.alloc(dav_bytes(dim, k, msub, keep));
    if (ws.region < 0) return fail(DMRG_E_WORKSPACE, "arena too small for the Davidson workspace");
    char* p = D->C->arena.base + ws.region;
    auto take = [&](int64_t n) { char* q = p; p += (n + 255) / 256 * 256; return q; };
    ws.V = (double*)take((int64_t)msub * dim * 8);
    ws.W = (double*)take((int64_t)msub * dim * 8);
    ws.X = (double*)take((int64_t)k * dim * 8);
    ws.HX = (double*)take((int64_t)k * dim * 8);
    ws.R = (double*)take((int64_t)k * dim * 8);
    ws.diag = (double*)take(dim * 8);
    ws.V2 = (double*)take((int64_t)keep * dim * 8);
    ws.W2 = (double*)take((int64_t)keep * dim * 8);
    ws.Gd = (double*)take(kSubMax * kSubMax * 8);
    ws.Zd = (double*)take(kSubMax * kSubMax * 8);
    ws.wd = (double*)take(kSubMax * 8);
    ws.Cd = (double*)take(kSubMax * 32 * 8);
    ws.gram = (double*)take(kSubMax * kSubMax * 8);
    ws.scratch = (double*)take(((dim + 4095) / 4096) * kSubMax * kSubMax * 8);
    ws.f_in = (float*)take((int64_t)k * dim * 4);
    ws.f_out = (float*)take((int64_t)k * dim * 4);
    ws.flag = (int*)take(256);
    hipStream_t s = (hipStream_t)stream;
    hipEventRecord(D->total.a, s);
    dmrg_status st = dmrg_heff_diag(H, ws.diag, stream);
    if (st != DMRG_OK) return st;
    // start block: orthonormalised input vectors
    int nv = 0;
    for (int j = 0; j < k; ++j) {
        DMRG_HIP(hipMemcpyAsync(ws.V + (int64_t)nv * dim, psi0 + (int64_t)j * dim, dim * 8,
                                hipMemcpyDeviceToDevice, s));
        double nrm;
        st = orth_append(ws, ws.V, nv, ws.V + (int64_t)nv * dim, dim, nrm, stream);
        if (st != DMRG_OK) return st;
        if (!(nrm > 1e-12)) return fail(DMRG_E_ARG, "start vectors are linearly dependent");
        st = scale_into(ws, ws.V + (int64_t)nv * dim, 1.0 / nrm, ws.V + (int64_t)nv * dim, dim, stream);
        if (st != DMRG_OK) return st;
        ++nv;
    }
    D->nv = nv;
    D->prec = opts->precision;
    D->clamp = opts->precond_clamp == 0.0 ? 0.1 : opts->precond_clamp;
    st = matvec(H, ws, D->prec, ws.V, ws.W, nv, dim, stream, &D->ms_mv, &D->mv32);
    if (st != DMRG_OK) return st;
    D->nmv += nv;
    D->G.assign((size_t)msub * msub, 0.0);
    D->theta.assign(k, 0.0);
    D->res.assign(k, 0.0);
    if ((st = reset_G(*D)) != DMRG_OK) return st;
    if ((st = rayleigh_ritz(*D)) != DMRG_OK) return st;
    *out = D.release();
    return DMRG_OK;
}

dmrg_status dmrg_davidson_step(dmrg_dav* Dp, int32_t* done, double* energies, double* max_residual) {
    if (!Dp) return fail(DMRG_E_ARG, "null argument");
    dmrg_dav& D = *Dp;
    DavWs& ws = D.ws;
    const int k = D.k;
    const int64_t dim = D.dim;
    hipStream_t s = (hipStream_t)D.stream;
    dmrg_status st = DMRG_OK;
    if (!D.done) {
        const bool fixed = D.opts.fixed_iters > 0;
        // precision switch of the mixed policy
        bool restart = D.nv + k > D.msub;
        bool switched = false;
        if (D.prec == DMRG_PREC_F32 && !fixed && max_res(D) <= D.opts.switch_tol) {
            D.prec = DMRG_PREC_F64;
            restart = true;
            switched = true;
        }
        if (restart && !switched && D.nv > D.keep) {
            // thick restart: V <- V Z[:, :keep], W <- W Z[:, :keep], G <- V^T W
            const int nv = D.nv, keep = D.keep;
            for (int j0 = 0; j0 < keep; j0 += 32) {
                const int nj = std::min(32, keep - j0);
                std::vector<double> Cj((size_t)nv * nj);
                for (int i = 0; i < nv; ++i)
                    for (int j = 0; j < nj; ++j) Cj[(size_t)i * nj + j] = D.Z[(size_t)i * nv + j0 + j];
                if ((st = combine(ws, ws.V, nv, Cj, ws.V2 + (int64_t)j0 * dim, nj, dim, 0.0, D.stream)) != DMRG_OK)
                    return st;
                if ((st = combine(ws, ws.W, nv, Cj, ws.W2 + (int64_t)j0 * dim, nj, dim, 0.0, D.stream)) != DMRG_OK)
                    return st;
            }
            DMRG_HIP(hipMemcpyAsync(ws.V, ws.V2, (int64_t)keep * dim * 8, hipMemcpyDeviceToDevice, s));
            DMRG_HIP(hipMemcpyAsync(ws.W, ws.W2, (int64_t)keep * dim * 8, hipMemcpyDeviceToDevice, s));
            D.nv = keep;
            if ((st = reset_G(D)) != DMRG_OK) return st;
        } else if (restart) {
            // restart from the Ritz vectors (and, at the precision switch, FP64 products of them)
            DMRG_HIP(hipMemcpyAsync(ws.V, ws.X, (int64_t)k * dim * 8, hipMemcpyDeviceToDevice, s));
            D.nv = k;
            if (switched) {
                st = matvec(D.H, ws, D.prec, ws.V, ws.W, k, dim, D.stream, &D.ms_mv, &D.mv32);
                if (st != DMRG_OK) return st;
                D.nmv += k;
            } else {
                DMRG_HIP(hipMemcpyAsync(ws.W, ws.HX, (int64_t)k * dim * 8, hipMemcpyDeviceToDevice, s));
            }
            if ((st = reset_G(D)) != DMRG_OK) return st;
        } else {
            // corrections t = r / (theta - diag), orthonormalised against V by CGS2
            const int nv0 = D.nv;
            for (int j = 0; j < k; ++j) {
                if (D.res[j] <= D.opts.tol && !fixed) continue;
                double* t = ws.V + (int64_t)D.nv * dim;
                DMRG_HIP(dmrgk::launch_precond(ws.R + (int64_t)j * dim, ws.diag, D.theta[j], D.clamp, t, dim,
                                               D.stream));
                std::vector<double> c;
                if ((st = gram_host(ws, t, 1, t, 1, dim, c, D.stream)) != DMRG_OK) return st;
                const double n0 = std::sqrt(std::max(0.0, c[0]));
                if (!(n0 > 0.0)) continue;
                double nrm;
                if ((st = orth_append(ws, ws.V, D.nv, t, dim, nrm, D.stream)) != DMRG_OK) return st;
                if (!(nrm > 1e-12 * std::max(1.0, n0)) || !std::isfinite(nrm)) continue;
                if ((st = scale_into(ws, t, 1.0 / nrm, t, dim, D.stream)) != DMRG_OK) return st;
                ++D.nv;
            }
            if (D.nv == nv0) {
                D.done = true;   // no new direction: the subspace is invariant
            } else {
                st = matvec(D.H, ws, D.prec, ws.V + (int64_t)nv0 * dim, ws.W + (int64_t)nv0 * dim, D.nv - nv0,
                            dim, D.stream, &D.ms_mv, &D.mv32);
                if (st != DMRG_OK) return st;
                D.nmv += D.nv - nv0;
                if ((st = refresh_G(D, nv0, D.nv)) != DMRG_OK) return st;
            }
        }
        if (!D.done) {
            ++D.it;
            if ((st = rayleigh_ritz(D)) != DMRG_OK) return st;
        }
    }
    if (done) *done = D.done ? 1 : 0;
    if (energies)
        for (int j = 0; j < k; ++j) energies[j] = D.theta[j];
    if (max_residual) *max_residual = max_res(D);
    return DMRG_OK;
}

dmrg_status dmrg_davidson_finish(dmrg_dav* Dp, double* psi_out, double* energies, dmrg_dav_stats* stats) {
    if (!Dp || !psi_out || !energies) return fail(DMRG_E_ARG, "null argument");
    dmrg_dav& D = *Dp;
    DavWs& ws = D.ws;
    const int k = D.k;
    const int64_t dim = D.dim;
    hipStream_t s = (hipStream_t)D.stream;
    dmrg_status st;
    // final energies: FP64 Rayleigh quotients when any FP32 product was used
    if (D.opts.precision == DMRG_PREC_F32 && (D.prec == DMRG_PREC_F32 || D.opts.fixed_iters > 0)) {
        st = matvec(D.H, ws, DMRG_PREC_F64, ws.X, ws.HX, k, dim, D.stream, &D.ms_mv, &D.mv32);
        if (st != DMRG_OK) return st;
        std::vector<double> xx, xh;
        if ((st = gram_host(ws, ws.X, k, ws.X, k, dim, xx, D.stream)) != DMRG_OK) return st;
        if ((st = gram_host(ws, ws.X, k, ws.HX, k, dim, xh, D.stream)) != DMRG_OK) return st;
        for (int j = 0; j < k; ++j) D.theta[j] = xh[(size_t)j * k + j] / xx[(size_t)j * k + j];
    }
    for (int j = 0; j < k; ++j) energies[j] = D.theta[j];
    DMRG_HIP(hipMemcpyAsync(psi_out, ws.X, (int64_t)k * dim * 8, hipMemcpyDeviceToDevice, s));
    hipEventRecord(D.total.b, s);
    DMRG_HIP(hipStreamSynchronize(s));
    float et = 0.f;
    hipEventElapsedTime(&et, D.total.a, D.total.b);
    if (stats) {
        dmrg_dav_stats x{};
        x.iters = D.it;
        x.matvecs = D.nmv;
        x.matvecs_f32 = D.mv32;
        x.converged = D.converged ? 1 : 0;
        x.max_residual = max_res(D);
        x.ms_total = et;
        x.ms_matvec = D.ms_mv;
        *stats = x;
    }
    return DMRG_OK;
}

void dmrg_davidson_free(dmrg_dav* D) { delete D; }

dmrg_status dmrg_davidson(dmrg_heff* H, int32_t k, double* psi_io, double* energies, const dmrg_dav_opts* opts,
                          dmrg_dav_stats* stats, void* stream) {
    if (!H || !psi_io || !energies || !opts) return fail(DMRG_E_ARG, "null argument");
    dmrg_dav* D = nullptr;
    dmrg_status st = dmrg_davidson_start(H, k, psi_io, opts, &D, stream);
    int32_t done = D ? (D->done ? 1 : 0) : 1;
    while (st == DMRG_OK && !done) st = dmrg_davidson_step(D, &done, nullptr, nullptr);
    if (st == DMRG_OK) st = dmrg_davidson_finish(D, psi_io, energies, stats);
    dmrg_davidson_free(D);
    return st;
}

}  // extern "C"
