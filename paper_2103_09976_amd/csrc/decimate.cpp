// Decimation of the two-site wavefunction (Appendix A: after the effective
// eigenproblem of a step, the reduced density matrix of the side that moves
// on is diagonalised and its heaviest eigenvectors become the block's new
// renormalized basis -- the MPS tensor of that site).
//
// Per enlarged sector q of that side (L' = Lb + d1, or R' = d2 + Rb), the
// wavefunction sub-blocks are gathered into one dense matrix Psi_q (the
// partner sector on the other side is fixed by the target; with noise, the
// perturbations, scaled by sqrt(noise), as further columns), the density
// matrix rho_q = Psi_q Psi_q^T (averaged over the roots) is one GEMM of the
// library's FP64 MFMA work-list kernels, and rho_q is diagonalised with
// rocSOLVER's divide-and-conquer symmetric eigensolver, its workspace carved
// out of the context arena.  The kept states are chosen on the host from all
// sectors' weights, and their eigenvectors are gathered into the isometry.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <map>

#include "core.hpp"

struct dmrg_iso {
    dmrg::Ctx* ctx = nullptr;
    int64_t region = -1;
    double* dev = nullptr;
    std::vector<int32_t> qn;
    std::vector<int64_t> rows, cols, offset;
    std::vector<double> weights;   // kept weights, block by block, descending within a block
    dmrg_decim_info info{};
};

namespace dmrg {

void release_solver(Ctx* C) {
    if (C->solver) {
        rocblas_destroy_handle((rocblas_handle)C->solver);
        C->solver = nullptr;
    }
}

}  // namespace dmrg

using namespace dmrg;

namespace {

// Kept states: the max_states heaviest over all sectors, extended by every
// state within kTieRel * w_M + kTieAbs * w_max of the last one's weight w_M
// (no multiplet of the spin symmetry is cut, also when a solver's residual
// splits it slightly, and the bond dimension stays max_states up to such
// partners), and no state of weight <= kFloorRel * w_max (no weightless
// basis state).
constexpr double kTieRel = 1e-5;
constexpr double kTieAbs = 1e-12;
constexpr double kFloorRel = 1e-14;

struct Sector {
    QN q;
    int d = 0;             // dimension of the enlarged sector
    int other = 0;         // dimension of its partner sector on the other side
    int64_t woff = 0;      // Psi_q: d x (n_vec * other), row-major
    int64_t roff = 0;      // rho_q: d x d (eigenvectors after the solve)
    int64_t doff = 0;      // its eigenvalues
};

// segments of enlarged sector q of a block with basis `old`: row offset of
// site state s (-1 when old has no sector q - q_s); returns the dimension
int enlarged(const Basis& old, const QN& q, std::array<int, 4>& seg) {
    int d = 0;
    for (int s = 0; s < 4; ++s) {
        const int k = old.find(q - kSiteQ[s]);
        if (k < 0) {
            seg[s] = -1;
            continue;
        }
        seg[s] = d;
        d += old.m[k];
    }
    return d;
}

// arena regions released on every exit path
struct Regions {
    Ctx* C;
    std::vector<int64_t> r;
    explicit Regions(Ctx* c) : C(c) {}
    int64_t take(int64_t bytes) {
        const int64_t o = C->arena.alloc(std::max<int64_t>(bytes, 8));
        if (o >= 0) r.push_back(o);
        return o;
    }
    ~Regions() {
        for (int64_t o : r) C->arena.release(o);
    }
};

dmrg_status solver_handle(Ctx* C, void* stream, rocblas_handle& h) {
    if (!C->solver) {
        rocblas_handle x = nullptr;
        if (rocblas_create_handle(&x) != rocblas_status_success) return fail(DMRG_E_HIP, "rocblas_create_handle failed");
        C->solver = x;
    }
    h = (rocblas_handle)C->solver;
    if (rocblas_set_stream(h, (hipStream_t)stream) != rocblas_status_success)
        return fail(DMRG_E_HIP, "rocblas_set_stream failed");
    return DMRG_OK;
}

}  // namespace

extern "C" {

dmrg_status dmrg_decimate(dmrg_heff* H, int32_t side, int32_t n_vec, const double* psi, double noise,
                          const double* xi, int32_t max_states, dmrg_iso** out, dmrg_decim_info* info,
                          void* stream) {
    if (!H || !psi || !out) return fail(DMRG_E_ARG, "null argument");
    *out = nullptr;
    if (side != DMRG_LEFT && side != DMRG_RIGHT) return fail(DMRG_E_ARG, "side must be DMRG_LEFT or DMRG_RIGHT");
    if (n_vec < 1 || n_vec > 64) return fail(DMRG_E_ARG, "n_vec must be 1..64");
    if (!std::isfinite(noise) || noise < 0.0 || (noise != 0.0 && !xi))
        return fail(DMRG_E_ARG, "noise must be finite and >= 0, with xi when > 0");
    const int nset = noise != 0.0 ? 2 : 1;   // column sets of Psi_q: the roots, then the perturbations
    Ctx* C = heff_ctx(H);
    if (C->dry) return fail(DMRG_E_STATE, "decimation has no workspace query");
    const OpSetImpl* Lb = nullptr;
    const OpSetImpl* Rb = nullptr;
    std::vector<PsiSub> subs;
    heff_psi_subblocks(H, Lb, Rb, subs);
    const int64_t dim = dmrg_heff_dim(H);
    hipStream_t s = (hipStream_t)stream;

    // sectors of the side that moves on, their partners and the gather plan
    std::map<QN, int> index;
    std::vector<Sector> sec;
    std::vector<std::array<int, 4>> segs_self, segs_other;
    for (const PsiSub& P : subs) {
        const QN ql = Lb->basis.q[P.a] + kSiteQ[P.s1];
        const QN qr = kSiteQ[P.s2] + Rb->basis.q[P.b];
        const QN q = side == DMRG_LEFT ? ql : qr;
        if (index.count(q)) continue;
        Sector S;
        S.q = q;
        std::array<int, 4> a, b;
        const int dl = enlarged(Lb->basis, ql, a);
        const int dr = enlarged(Rb->basis, qr, b);
        S.d = side == DMRG_LEFT ? dl : dr;
        S.other = side == DMRG_LEFT ? dr : dl;
        index[q] = (int)sec.size();
        sec.push_back(S);
        segs_self.push_back(side == DMRG_LEFT ? a : b);
        segs_other.push_back(side == DMRG_LEFT ? b : a);
    }
    if (sec.empty()) return fail(DMRG_E_ARG, "empty wavefunction");
    {   // sectors in sorted order (the isometry's blocks follow it)
        std::vector<int> perm(sec.size());
        for (size_t i = 0; i < perm.size(); ++i) perm[i] = (int)i;
        std::sort(perm.begin(), perm.end(), [&](int x, int y) { return sec[x].q < sec[y].q; });
        std::vector<Sector> s2;
        std::vector<std::array<int, 4>> a2, b2;
        for (int i : perm) {
            index[sec[i].q] = (int)s2.size();
            s2.push_back(sec[i]);
            a2.push_back(segs_self[i]);
            b2.push_back(segs_other[i]);
        }
        sec.swap(s2);
        segs_self.swap(a2);
        segs_other.swap(b2);
    }
    int64_t wel = 0, rel = 0, del = 0;
    int dmax = 0;
    for (Sector& S : sec) {
        S.woff = wel;
        wel += (int64_t)S.d * nset * n_vec * S.other;
        S.roff = rel;
        rel += (int64_t)S.d * S.d;
        S.doff = del;
        del += S.d;
        dmax = std::max(dmax, S.d);
    }
    if (wel != (int64_t)nset * n_vec * dim) return fail(DMRG_E_STATE, "wavefunction sub-blocks do not tile the sectors");
    std::vector<dmrgk::GatherBlock> gb;
    for (const PsiSub& P : subs) {
        const QN ql = Lb->basis.q[P.a] + kSiteQ[P.s1];
        const QN qr = kSiteQ[P.s2] + Rb->basis.q[P.b];
        const int k = index.at(side == DMRG_LEFT ? ql : qr);
        const Sector& S = sec[k];
        const int ld = nset * n_vec * S.other;
        dmrgk::GatherBlock g{};
        g.src = P.off;
        g.ma = P.ma;
        g.mb = P.mb;
        g.ld = ld;
        g.vcol = S.other;
        g.pcol = (int64_t)n_vec * S.other;
        if (side == DMRG_LEFT) {
            g.dst = S.woff + (int64_t)segs_self[k][P.s1] * ld + segs_other[k][P.s2];
            g.trans = 0;
        } else {
            g.dst = S.woff + (int64_t)segs_self[k][P.s2] * ld + segs_other[k][P.s1];
            g.trans = 1;
        }
        gb.push_back(g);
    }

    // rho_q = Psi_q Psi_q^T: one group per sector, identity X, contributions over k chunks
    WorkList wl;
    for (const Sector& S : sec) {
        const int64_t kw = (int64_t)nset * n_vec * S.other;
        const int g0 = (int)wl.groups.size();
        dmrgk::Group g{};
        g.xid_coef = 1.0;
        g.mu = S.d;
        g.c0 = (int)wl.contribs.size();
        const int64_t kc = 1 << 20;
        for (int64_t k0 = 0; k0 < kw; k0 += kc) {
            dmrgk::Contrib c{};
            c.a_off = S.woff + k0;
            c.lda = (int)kw;
            c.b_off = S.woff + k0;
            c.ldb = (int)kw;
            c.k = (int)std::min(kc, kw - k0);
            c.alpha = 1.0;
            c.flags = 0 | (0 << 3) | dmrgk::F_TRANS_B;
            wl.contribs.push_back(c);
        }
        g.c1 = (int)wl.contribs.size();
        wl.groups.push_back(g);
        emit_block_tasks(wl, 1, S.roff, S.d, S.d, S.d, g0, g0 + 1);
    }
    int64_t sz[dmrgk::kMaxBuf] = {0};
    sz[0] = wel;
    sz[1] = rel;
    dmrg_status st = validate_work(wl, sz);
    if (st != DMRG_OK) return st;

    rocblas_handle h = nullptr;
    st = solver_handle(C, stream, h);
    if (st != DMRG_OK) return st;
    Regions R(C);
    const int64_t r_w = R.take(wel * 8), r_rho = R.take(rel * 8), r_d = R.take(del * 8);
    const int64_t r_e = R.take((int64_t)dmax * 8), r_info = R.take((int64_t)sec.size() * 4);
    const int64_t r_gb = R.take((int64_t)gb.size() * sizeof(dmrgk::GatherBlock));
    if (r_w < 0 || r_rho < 0 || r_d < 0 || r_e < 0 || r_info < 0 || r_gb < 0)
        return fail(DMRG_E_WORKSPACE, "arena too small for the density matrices");
    char* base = C->arena.base;
    double* W = (double*)(base + r_w);
    double* rho = (double*)(base + r_rho);
    double* D = (double*)(base + r_d);
    double* E = (double*)(base + r_e);
    rocblas_int* dinfo = (rocblas_int*)(base + r_info);
    dmrgk::GatherBlock* dgb = (dmrgk::GatherBlock*)(base + r_gb);
    // rocSOLVER's workspace: the largest of its size queries, from the arena
    size_t ws = 0;
    {
        std::vector<int> dims;
        for (const Sector& S : sec) dims.push_back(S.d);
        std::sort(dims.begin(), dims.end());
        dims.erase(std::unique(dims.begin(), dims.end()), dims.end());
        if (rocblas_start_device_memory_size_query(h) != rocblas_status_success)
            return fail(DMRG_E_HIP, "rocBLAS size query failed");
        for (int d : dims) rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, d, rho, d, D, E, dinfo);
        if (rocblas_stop_device_memory_size_query(h, &ws) != rocblas_status_success)
            return fail(DMRG_E_HIP, "rocBLAS size query failed");
    }
    const int64_t r_ws = R.take((int64_t)ws);
    if (r_ws < 0) return fail(DMRG_E_WORKSPACE, "arena too small for the eigensolver workspace");
    if (rocblas_set_workspace(h, base + r_ws, std::max<size_t>(ws, 8)) != rocblas_status_success)
        return fail(DMRG_E_HIP, "rocblas_set_workspace failed");
    struct Unset {
        rocblas_handle h;
        ~Unset() { rocblas_set_workspace(h, nullptr, 0); }
    } unset{h};

    DevWork dw;
    st = upload_work(C, wl, dw, stream);
    if (st != DMRG_OK) return st;
    struct FreeWork {
        Ctx* C;
        DevWork& d;
        ~FreeWork() { free_work(C, d); }
    } fw{C, dw};
    // from here on, every exit waits for the queued work before the regions go back to the arena
    struct SyncOnExit {
        hipStream_t s;
        ~SyncOnExit() { (void)hipStreamSynchronize(s); }
    } sync_on_exit{s};
    DMRG_HIP(hipMemcpyAsync(dgb, gb.data(), gb.size() * sizeof(dmrgk::GatherBlock), hipMemcpyHostToDevice, s));
    DMRG_HIP(dmrgk::launch_psi_gather(dgb, (int)gb.size(), n_vec, psi, 0, dim, 1.0 / std::sqrt((double)n_vec), W,
                                      stream));
    if (nset == 2)
        DMRG_HIP(dmrgk::launch_psi_gather(dgb, (int)gb.size(), n_vec, xi, 1, dim, std::sqrt(noise / n_vec), W,
                                          stream));
    dmrgk::Bases<double> b{};
    b.p[0] = W;
    b.p[1] = rho;
    st = run_work_f64(dw, b, 1, stream);
    if (st != DMRG_OK) return st;
    for (size_t i = 0; i < sec.size(); ++i) {
        const Sector& S = sec[i];
        const rocblas_status rs = rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, S.d, rho + S.roff,
                                                   S.d, D + S.doff, E, dinfo + i);
        if (rs != rocblas_status_success) return fail(DMRG_E_HIP, "rocsolver_dsyevd failed");
    }
    std::vector<double> w(del);
    std::vector<rocblas_int> hinfo(sec.size());
    DMRG_HIP(hipMemcpyAsync(w.data(), D, del * 8, hipMemcpyDeviceToHost, s));
    DMRG_HIP(hipMemcpyAsync(hinfo.data(), dinfo, sec.size() * 4, hipMemcpyDeviceToHost, s));
    DMRG_HIP(hipStreamSynchronize(s));
    for (rocblas_int x : hinfo)
        if (x != 0) return fail(DMRG_E_HIP, "rocsolver_dsyevd did not converge");

    // selection over all sectors (eigenvalues ascending within a sector)
    double wmax = 0.0, total = 0.0;
    for (double x : w) {
        if (!std::isfinite(x)) return fail(DMRG_E_NONFINITE, "non-finite density-matrix weight");
        wmax = std::max(wmax, x);
        total += x;
    }
    if (!(wmax > 0.0)) return fail(DMRG_E_ARG, "the wavefunction is zero");
    const double floor = kFloorRel * wmax;
    std::vector<double> sorted;
    for (double x : w)
        if (x > floor) sorted.push_back(x);
    std::sort(sorted.begin(), sorted.end(), std::greater<double>());
    double cut = floor;
    if (max_states > 0 && (size_t)max_states < sorted.size())
        cut = std::max(sorted[max_states - 1] * (1.0 - kTieRel) - kTieAbs * wmax, floor);
    auto keep = [&](double x) { return cut <= floor ? x > floor : x >= cut; };

    dmrg_iso* iso = new dmrg_iso();
    iso->ctx = C;
    std::vector<dmrgk::EvecBlock> eb;
    int64_t iel = 0;
    double kept_w = 0.0;
    for (const Sector& S : sec) {
        int k = 0;
        for (int j = S.d - 1; j >= 0 && keep(w[S.doff + j]); --j) ++k;
        if (k == 0) continue;
        iso->qn.push_back(S.q.a);
        iso->qn.push_back(S.q.b);
        iso->rows.push_back(S.d);
        iso->cols.push_back(k);
        iso->offset.push_back(iel);
        for (int c = 0; c < k; ++c) {
            iso->weights.push_back(w[S.doff + S.d - 1 - c]);
            kept_w += w[S.doff + S.d - 1 - c];
        }
        eb.push_back(dmrgk::EvecBlock{S.roff, iel, S.d, k});
        iel += (int64_t)S.d * k;
    }
    iso->region = C->arena.alloc(iel * 8 + (int64_t)eb.size() * sizeof(dmrgk::EvecBlock));
    if (iso->region < 0) {
        delete iso;
        return fail(DMRG_E_WORKSPACE, "arena too small for the isometry");
    }
    iso->dev = (double*)(base + iso->region);
    dmrgk::EvecBlock* deb = (dmrgk::EvecBlock*)(iso->dev + iel);
    int e = (int)hipMemcpyAsync(deb, eb.data(), eb.size() * sizeof(dmrgk::EvecBlock), hipMemcpyHostToDevice, s);
    if (!e) e = dmrgk::launch_evec_gather(deb, (int)eb.size(), rho, iso->dev, stream);
    if (!e) e = (int)hipStreamSynchronize(s);
    if (e) {
        C->arena.release(iso->region);
        delete iso;
        return hip_fail(e, "isometry gather");
    }
    iso->info.kept = (int64_t)iso->weights.size();
    iso->info.n_blocks = (int32_t)eb.size();
    iso->info.weight_total = total;
    iso->info.trunc_err = total > 0 ? std::max(0.0, (total - kept_w) / total) : 0.0;
    if (info) *info = iso->info;
    *out = iso;
    return DMRG_OK;
}

dmrg_status dmrg_iso_bsm(const dmrg_iso* iso, dmrg_bsm* view) {
    if (!iso || !view) return fail(DMRG_E_ARG, "null argument");
    view->n_blocks = (int32_t)iso->rows.size();
    view->qn_row = iso->qn.data();
    view->qn_col = iso->qn.data();
    view->rows = iso->rows.data();
    view->cols = iso->cols.data();
    view->offset = iso->offset.data();
    view->dtype = DMRG_F64;
    view->data = iso->dev;
    return DMRG_OK;
}

int64_t dmrg_iso_weights(const dmrg_iso* iso, int64_t n, double* w) {
    if (!iso) return -1;
    const int64_t m = (int64_t)iso->weights.size();
    if (w)
        for (int64_t i = 0; i < std::min(n, m); ++i) w[i] = iso->weights[i];
    return m;
}

void dmrg_iso_free(dmrg_iso* iso) {
    if (!iso) return;
    if (iso->region >= 0) iso->ctx->arena.release(iso->region);
    delete iso;
}

}  // extern "C"
