// Host core of the DMRG library: status handling, arena, operator-set
// layout, site operators, isometry layout, work lists, weighted sums.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <tuple>

#include "core.hpp"

namespace dmrg {
static thread_local std::string g_last_error;
}

extern "C" const char* dmrg_last_error(void) { return dmrg::g_last_error.c_str(); }

namespace dmrg {

const QN kSiteQ[4] = {QN(0, 0), QN(1, 0), QN(0, 1), QN(1, 1)};

double wall_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

dmrg_status fail(dmrg_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

dmrg_status hip_fail(int err, const char* where) {
    g_last_error = std::string(where) + ": " + hipGetErrorString((hipError_t)err);
    return DMRG_E_HIP;
}

int Basis::find_slow(const QN& x) const {
    auto it = std::lower_bound(q.begin(), q.end(), x);
    if (it == q.end() || !(*it == x)) return -1;
    return (int)(it - q.begin());
}

void Basis::index() {
    amax = bmax = 0;
    for (const QN& x : q) {
        amax = std::max(amax, x.a);
        bmax = std::max(bmax, x.b);
    }
    tab.assign((size_t)(amax + 1) * (bmax + 1), -1);
    for (size_t i = 0; i < q.size(); ++i)
        if (q[i].a >= 0 && q[i].b >= 0) tab[(size_t)q[i].a * (bmax + 1) + q[i].b] = (int)i;
}

int OpSetImpl::skel_for(const QN& dq) {
    for (size_t i = 0; i < skels.size(); ++i)
        if (skels[i].dq == dq) return (int)i;
    Skel s;
    s.dq = dq;
    s.blk_of_ket.assign(basis.size(), -1);
    int64_t off = 0;
    for (int k = 0; k < basis.size(); ++k) {
        const int b = basis.find(basis.q[k] + dq);
        if (b < 0) continue;
        s.blk_of_ket[k] = (int)s.ket.size();
        s.ket.push_back(k);
        s.bra.push_back(b);
        s.off.push_back(off);
        off += (int64_t)basis.m[b] * basis.m[k];
    }
    s.size = off;
    skels.push_back(std::move(s));
    return (int)skels.size() - 1;
}

int OpSetImpl::family(char kind, const QN& dq, int par) {
    for (size_t i = 0; i < fams.size(); ++i)
        if (fams[i].kind == kind && fams[i].dq == dq) return (int)i;
    Family f;
    f.kind = kind;
    f.dq = dq;
    f.par = par;
    f.skel = skel_for(dq);
    fams.push_back(std::move(f));
    return (int)fams.size() - 1;
}

int OpSetImpl::add_op(char kind, int p, int q, const QN& dq, int par) {
    const int64_t key = okey(kind, p, q);
    auto it = lookup.find(key);
    if (it != lookup.end()) return it->second.first;
    const int f = family(kind, dq, par);
    Family& F = fams[f];
    const int idx = (int)F.keys.size();
    F.keys.push_back(key);
    F.index[key] = idx;
    lookup[key] = {f, idx};
    return f;
}

void OpSetImpl::layout() {
    int64_t off = 0;
    for (auto& F : fams) {
        F.stride = skels[F.skel].size;
        F.base = off;
        off += F.stride * (int64_t)F.keys.size();
        off = (off + 31) & ~int64_t(31);   // 256-byte alignment of every family
    }
    elems = off;
}

// ---------------------------------------------------------------------------
void Arena::init(void* p, int64_t n) {
    base = (char*)p;
    bytes = n;
    free_.clear();
    live_.clear();
    // align the usable start to 256 bytes
    const int64_t start = (int64_t)((256 - ((uintptr_t)p & 255)) & 255);
    if (n > start) free_[start] = n - start;
    used = peak = 0;
    high = start;
}

int64_t Arena::alloc(int64_t n) {
    if (n <= 0) n = 256;
    n = (n + 255) & ~int64_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second >= n) {
            const int64_t off = it->first, sz = it->second;
            free_.erase(it);
            if (sz > n) free_[off + n] = sz - n;
            live_[off] = n;
            used += n;
            peak = std::max(peak, used);
            high = std::max(high, off + n);
            return off;
        }
    }
    return -1;
}

void Arena::release(int64_t off) {
    auto it = live_.find(off);
    if (it == live_.end()) return;
    int64_t o = off, n = it->second;
    live_.erase(it);
    used -= n;
    auto nx = free_.lower_bound(o);
    if (nx != free_.end() && o + n == nx->first) {
        n += nx->second;
        free_.erase(nx);
    }
    auto pv = free_.lower_bound(o);
    if (pv != free_.begin()) {
        --pv;
        if (pv->first + pv->second == o) {
            o = pv->first;
            n += pv->second;
            free_.erase(pv);
        }
    }
    free_[o] = n;
}

dmrg_status alloc_set(Ctx* ctx, OpSetImpl& s) {
    if (s.basis.tab.empty()) s.basis.index();
    s.layout();
    const int64_t off = ctx->arena.alloc(std::max<int64_t>(s.elems, 1) * 8);
    if (off < 0)
        return fail(DMRG_E_WORKSPACE, "arena too small for an operator set of " +
                                          std::to_string(s.elems * 8) + " bytes");
    s.region = off;
    s.dev = (double*)(ctx->arena.base + off);
    return DMRG_OK;
}

int64_t set_bytes(const OpSetImpl& s) { return (std::max<int64_t>(s.elems, 1) * 8 + 255) / 256 * 256; }

void free_set(Ctx* ctx, OpSetImpl& s) {
    if (s.region >= 0) ctx->arena.release(s.region);
    s.region = -1;
    s.dev = nullptr;
}

// ---------------------------------------------------------------------------
QN Ref::dq() const {
    if (type == 0) return QN(0, 0);
    const QN d = set->fams[fam].dq;
    return trans ? -d : d;
}

int Ref::par() const { return type == 0 ? 0 : set->fams[fam].par; }

bool Ref::block(int k, int& bra, int64_t& off, int& ld, bool& tr) const {
    if (type == 0) {
        bra = k;
        off = -1;
        ld = 0;
        tr = false;
        return true;
    }
    const Family& F = set->fams[fam];
    const Skel& S = set->skels[F.skel];
    const Basis& B = set->basis;
    if (!trans) {
        const int b = S.blk_of_ket[k];
        if (b < 0) return false;
        bra = S.bra[b];
        off = F.base + (int64_t)idx * F.stride + S.off[b];
        ld = B.m[k];
        tr = false;
        return true;
    }
    const int k2 = B.find(B.q[k] - F.dq);
    if (k2 < 0) return false;
    const int b = S.blk_of_ket[k2];
    if (b < 0) return false;
    bra = k2;
    off = F.base + (int64_t)idx * F.stride + S.off[b];
    ld = B.m[k2];
    tr = true;
    return true;
}

// ---------------------------------------------------------------------------
M4 M4::operator*(const M4& o) const {
    M4 r;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double s = 0;
            for (int k = 0; k < 4; ++k) s += a[i][k] * o.a[k][j];
            r.a[i][j] = s;
        }
    return r;
}
M4 M4::operator+(const M4& o) const {
    M4 r;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) r.a[i][j] = a[i][j] + o.a[i][j];
    return r;
}
M4 M4::operator*(double s) const {
    M4 r;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) r.a[i][j] = a[i][j] * s;
    return r;
}
M4 M4::T() const {
    M4 r;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) r.a[i][j] = a[j][i];
    return r;
}
bool M4::zero() const {
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j)
            if (a[i][j] != 0.0) return false;
    return true;
}

static int proc1(int p, int i, int P) { return ((i - p) % P + P) % P == 0; }
static int proc2(int p, int i, int j, int P) {
    if (i > j) std::swap(i, j);
    const long long x = (long long)(j - 1) * j / 2 + i - p;
    return ((x % P) + P) % P == 0;
}

bool Ctx::pair_needed(int i, int j) const {
    if (n_proc <= 1) return true;
    return proc2(proc_id, i + 1, j + 1, n_proc) != 0;
}

M4 Ctx::c(int p) const {
    M4 r;
    if ((p & 1) == 0) {          // alpha: |0> -> |a>, |b> -> |ab>
        r.a[1][0] = 1.0;
        r.a[3][2] = 1.0;
    } else {                     // beta: |0> -> |b>, |a> -> -|ab>
        r.a[2][0] = 1.0;
        r.a[3][1] = -1.0;
    }
    return r;
}

M4 Ctx::site_H(int n) const {
    M4 r;
    const int o[2] = {2 * n, 2 * n + 1};
    for (int p : o)
        for (int q : o) {
            const double tt = t(p, q);
            if (tt != 0.0) r = r + c(p) * c(q).T() * tt;
            for (int rr : o)
                for (int s : o) {
                    const double vv = v(p, q, rr, s);
                    if (vv != 0.0) r = r + c(p) * c(rr) * c(s).T() * c(q).T() * (0.5 * vv);
                }
        }
    return r;
}

M4 Ctx::site_R(int n, int p) const {
    M4 r;
    const int o[2] = {2 * n, 2 * n + 1};
    for (int q : o) {
        const double tt = t(p, q);
        if (tt != 0.0) r = r + c(q).T() * (0.5 * tt);
        for (int rr : o)
            for (int s : o) {
                const double vv = v(p, q, rr, s);
                if (vv != 0.0) r = r + c(rr) * c(s).T() * c(q).T() * vv;
            }
    }
    return r;
}

M4 Ctx::site_Pd(int n, int p, int rr) const {
    M4 r;
    const int o[2] = {2 * n, 2 * n + 1};
    for (int q : o)
        for (int s : o) {
            const double vv = v(p, q, rr, s);
            if (vv != 0.0) r = r + c(q) * c(s) * vv;   // (a_s a_q)^T = a+_q a+_s
        }
    return r;
}

M4 Ctx::site_Q(int n, int p, int q) const {
    M4 r;
    const int o[2] = {2 * n, 2 * n + 1};
    for (int rr : o)
        for (int s : o) {
            const double vv = v(p, q, rr, s) - v(p, s, rr, q);
            if (vv != 0.0) r = r + c(rr) * c(s).T() * vv;
        }
    return r;
}

// ---------------------------------------------------------------------------
dmrg_status make_iso(const Basis& old, const dmrg_bsm* bsm, Iso& out, bool need_data) {
    if (!bsm || bsm->n_blocks <= 0 || !bsm->qn_col || !bsm->rows || !bsm->cols || !bsm->offset ||
        (need_data && !bsm->data))
        return fail(DMRG_E_ARG, "isometry descriptor incomplete");
    if (bsm->dtype != DMRG_F64) return fail(DMRG_E_ARG, "isometries must be float64");
    std::vector<std::pair<QN, int>> order;
    for (int b = 0; b < bsm->n_blocks; ++b) order.push_back({QN(bsm->qn_col[2 * b], bsm->qn_col[2 * b + 1]), b});
    std::sort(order.begin(), order.end(),
              [](const std::pair<QN, int>& x, const std::pair<QN, int>& y) { return x.first < y.first; });
    out.dev = (const double*)bsm->data;
    out.nb = Basis();
    out.off.clear();
    out.d.clear();
    out.seg.clear();
    for (size_t i = 0; i < order.size(); ++i) {
        const QN q = order[i].first;
        const int b = order[i].second;
        if (i > 0 && order[i - 1].first == q) return fail(DMRG_E_ARG, "duplicate isometry sector");
        if (bsm->qn_row && (bsm->qn_row[2 * b] != q.a || bsm->qn_row[2 * b + 1] != q.b))
            return fail(DMRG_E_ARG, "isometry block must map sector q to q");
        std::array<int, 4> seg;
        int d = 0;
        for (int s = 0; s < 4; ++s) {
            const int k = old.find(q - kSiteQ[s]);
            if (k < 0) { seg[s] = -1; continue; }
            seg[s] = d;
            d += old.m[k];
        }
        const int64_t m = bsm->cols[b];
        if (bsm->rows[b] != d)
            return fail(DMRG_E_ARG, "isometry rows " + std::to_string(bsm->rows[b]) +
                                        " != enlarged dimension " + std::to_string(d) + " of sector (" +
                                        std::to_string(q.a) + "," + std::to_string(q.b) + ")");
        if (m <= 0 || m > d) return fail(DMRG_E_ARG, "isometry columns out of range");
        out.nb.q.push_back(q);
        out.nb.m.push_back((int)m);
        out.nb.total += m;
        out.off.push_back(bsm->offset[b]);
        out.d.push_back(d);
        out.seg.push_back(seg);
    }
    return DMRG_OK;
}

// ---------------------------------------------------------------------------
void WorkList::clear() {
    for (auto& t : task) t.clear();
    groups.clear();
    contribs.clear();
    reduces.clear();
    partial_elems = 0;
}

size_t WorkList::ntasks() const {
    size_t n = 0;
    for (auto& t : task) n += t.size();
    return n;
}

int task_class_of(const WorkList& w, const dmrgk::Task& t) {
    int rows = t.m;
    for (int g = t.g0; g < t.g1; ++g) rows = std::max(rows, w.groups[g].mu);
    return dmrgk::task_class(rows, t.ncol, w.tall_min);
}

void reclassify(WorkList& w) {
    std::vector<dmrgk::Task> all;
    for (auto& T : w.task) {
        all.insert(all.end(), T.begin(), T.end());
        T.clear();
    }
    for (const dmrgk::Task& t : all) w.task[task_class_of(w, t)].push_back(t);
}

void emit_block_tasks(WorkList& w, int cbuf, int64_t c_off, int ldc, int m, int n, int g0, int g1,
                      bool accumulate) {
    if (m <= 0 || n <= 0) return;
    // near-equal column tiles of at most kMaxCols, widths in multiples of 16
    const int nt = (n + dmrgk::kMaxCols - 1) / dmrgk::kMaxCols;
    const int width = ((n + nt - 1) / nt + 15) / 16 * 16;
    for (int col0 = 0; col0 < n; col0 += width) {
        dmrgk::Task t{};
        t.c_off = c_off;
        t.ldc = ldc;
        t.m = m;
        t.n = n;
        t.col0 = col0;
        t.ncol = std::min(width, n - col0);
        t.g0 = g0;
        t.g1 = g1;
        t.cbuf = cbuf | (accumulate ? 256 : 0);
        w.task[task_class_of(w, t)].push_back(t);
    }
}

// Tiles taller than kTallRows are split exactly: output rows into row tiles,
// the inner dimension mu of X . U into chunks (a group becomes one group per
// chunk; its identity part follows the output rows).  Tiles up to kTallRows
// run whole on the tall kernel.
void split_large(WorkList& w) {
    const int CAP = dmrgk::kTallRows;
    bool need = false;
    for (auto& T : w.task)
        for (const dmrgk::Task& t : T) {
            if (t.m > CAP) need = true;
            for (int g = t.g0; g < t.g1 && !need; ++g) need = w.groups[g].mu > CAP;
            if (need) break;
        }
    if (!need) return;
    std::vector<dmrgk::Task> all;
    for (auto& T : w.task) {
        all.insert(all.end(), T.begin(), T.end());
        T.clear();
    }
    auto shift_contrib = [](dmrgk::Contrib c, int u0) {
        const bool ida = c.flags & dmrgk::F_ID_A, idb = c.flags & dmrgk::F_ID_B;
        if (ida && idb) c.a_off += u0;                       // diagonal offset of an identity
        else if (ida) c.b_off += (c.flags & dmrgk::F_TRANS_B) ? u0 : (int64_t)u0 * c.ldb;
        else c.a_off += (c.flags & dmrgk::F_TRANS_A) ? u0 : (int64_t)u0 * c.lda;
        return c;
    };
    std::map<std::tuple<int, int, int>, std::pair<int, int>> done;   // (g0, g1, r0) -> new range
    std::vector<dmrgk::Group> ng = w.groups;
    std::vector<dmrgk::Contrib> nc = w.contribs;
    for (const dmrgk::Task& t : all) {
        bool big = t.m > CAP;
        for (int g = t.g0; g < t.g1 && !big; ++g) big = w.groups[g].mu > CAP;
        if (!big) {
            w.task[task_class_of(w, t)].push_back(t);
            continue;
        }
        for (int r0 = 0; r0 < t.m; r0 += CAP) {
            const int rm = std::min(CAP, t.m - r0);
            auto key = std::make_tuple(t.g0, t.g1, r0);
            auto it = done.find(key);
            if (it == done.end()) {
                const int g0 = (int)ng.size();
                for (int g = t.g0; g < t.g1; ++g) {
                    const dmrgk::Group& G = w.groups[g];
                    if (G.flags & dmrgk::G_HAS_X) {
                        for (int u0 = 0; u0 < G.mu; u0 += CAP) {
                            dmrgk::Group H = G;
                            H.mu = std::min(CAP, G.mu - u0);
                            H.xid_coef = 0.0;
                            H.x_off += (G.flags & dmrgk::G_TRANS_X) ? (int64_t)u0 * G.ldx + r0
                                                                    : (int64_t)r0 * G.ldx + u0;
                            H.c0 = (int)nc.size();
                            for (int c = G.c0; c < G.c1; ++c) nc.push_back(shift_contrib(w.contribs[c], u0));
                            H.c1 = (int)nc.size();
                            ng.push_back(H);
                        }
                    }
                    if (G.xid_coef != 0.0) {
                        dmrgk::Group H = G;
                        H.flags &= ~(dmrgk::G_HAS_X | dmrgk::G_TRANS_X);
                        H.x_coef = 0.0;
                        H.mu = rm;
                        H.c0 = (int)nc.size();
                        for (int c = G.c0; c < G.c1; ++c) nc.push_back(shift_contrib(w.contribs[c], r0));
                        H.c1 = (int)nc.size();
                        ng.push_back(H);
                    }
                }
                it = done.emplace(key, std::make_pair(g0, (int)ng.size())).first;
            }
            dmrgk::Task u = t;
            u.c_off += (int64_t)r0 * t.ldc;
            u.m = rm;
            u.g0 = it->second.first;
            u.g1 = it->second.second;
            int rows = u.m;
            for (int g = u.g0; g < u.g1; ++g) rows = std::max(rows, ng[g].mu);
            w.task[dmrgk::task_class(rows, u.ncol, w.tall_min)].push_back(u);
        }
    }
    w.groups.swap(ng);
    w.contribs.swap(nc);
}

// Cost model of one group for a tile of m rows: MFMA work of the A.B
// products and of X.U, plus a fixed per-group and per-contribution overhead
// (fragment loads, the LDS round trip of U, barriers) in flop equivalents.
static double group_cost(const WorkList& w, const dmrgk::Group& G, int m, int ncol) {
    const int cols = (ncol + 15) / 16 * 16;
    double f = 16384.0;
    if (G.flags & dmrgk::G_HAS_X) f += 2.0 * m * G.mu * cols;
    for (int c = G.c0; c < G.c1; ++c) {
        const dmrgk::Contrib& q = w.contribs[c];
        f += 4096.0;
        if (!(q.flags & (dmrgk::F_ID_A | dmrgk::F_ID_B))) f += 2.0 * G.mu * q.k * cols;
    }
    return f;
}

double task_useful_flops(const WorkList& w, const dmrgk::Task& t) {
    const int cols = std::min(t.ncol, t.n - t.col0);
    double f = 0;
    for (int g = t.g0; g < t.g1; ++g) {
        const dmrgk::Group& G = w.groups[g];
        if (G.flags & dmrgk::G_HAS_X) f += 2.0 * t.m * G.mu * cols;
        for (int c = G.c0; c < G.c1; ++c) {
            const dmrgk::Contrib& q = w.contribs[c];
            if (!(q.flags & (dmrgk::F_ID_A | dmrgk::F_ID_B))) f += 2.0 * G.mu * q.k * cols;
        }
    }
    return f;
}

double task_cost(const WorkList& w, const dmrgk::Task& t) {
    double f = 0;
    for (int g = t.g0; g < t.g1; ++g) f += group_cost(w, w.groups[g], t.m, t.ncol);
    return f;
}

bool records_fit(const WorkList& w, const dmrgk::Task& t) {
    if (t.g1 - t.g0 > dmrgk::kRecG) return false;
    if (t.g1 <= t.g0) return true;
    for (int g = t.g0 + 1; g < t.g1; ++g)
        if (w.groups[g].c0 != w.groups[g - 1].c1) return false;
    return w.groups[t.g1 - 1].c1 - w.groups[t.g0].c0 <= dmrgk::kRecC;
}

void balance_work(WorkList& w, int target_tasks) {
    // the cost of every group of every task (it depends on the task's rows and
    // columns), computed on several threads; the sums and the cutting below run
    // in list order, so the result is the same for any thread count
    std::vector<const dmrgk::Task*> all;
    for (auto& T : w.task)
        for (const dmrgk::Task& t : T) all.push_back(&t);
    std::vector<size_t> goff(all.size() + 1, 0);
    for (size_t i = 0; i < all.size(); ++i) goff[i + 1] = goff[i] + (size_t)(all[i]->g1 - all[i]->g0);
    std::vector<double> gcost(goff.back()), tcost(all.size());
    {
        const unsigned nth = (unsigned)std::max<size_t>(
            1, std::min<size_t>({32, std::max(1u, std::thread::hardware_concurrency()), all.size() / 4096 + 1}));
        std::vector<std::thread> th;
        for (unsigned k = 0; k < nth; ++k)
            th.emplace_back([&, k]() {
                for (size_t i = k; i < all.size(); i += nth) {
                    const dmrgk::Task& t = *all[i];
                    double tc = 0;
                    for (int g = t.g0; g < t.g1; ++g)
                        tc += gcost[goff[i] + (g - t.g0)] = group_cost(w, w.groups[g], t.m, t.ncol);
                    tcost[i] = tc;
                }
            });
        for (auto& x : th) x.join();
    }
    double total = 0;
    for (double c : tcost) total += c;
    if (total <= 0 || target_tasks < 1) return;
    // chunks of at least kMinChunkCost: small problems are not cut into pieces
    // whose fixed cost (records, partial tile, reduction) exceeds their work
    const double kMinChunkCost = 4.0e6;
    const double cap = std::max(total / target_tasks, kMinChunkCost);
    std::vector<std::pair<double, dmrgk::Task>> out[dmrgk::kNumClass];
    int64_t poff = w.partial_elems;
    size_t ti = 0;
    for (auto& T : w.task) {
        for (const dmrgk::Task& t : T) {
            const double* gc = gcost.data() + goff[ti];
            const double tc = tcost[ti++];
            const int nchunk = (int)std::min<double>(std::ceil(tc / cap), t.g1 - t.g0);
            if (nchunk <= 1 && records_fit(w, t)) {
                out[task_class_of(w, t)].emplace_back(tc, t);
                continue;
            }
            // greedy cut at multiples of tc / nchunk, and wherever the next group would
            // overflow the records a task can stage (kRecG groups, kRecC contributions)
            const double per = tc / std::max(1, nchunk);
            int slot = 0;
            int a = t.g0;
            double run = 0, done = 0;
            const int64_t slot_elems = (int64_t)t.m * t.ncol;
            for (int g = t.g0; g < t.g1; ++g) {
                run += gc[g - t.g0];
                const bool last = g + 1 == t.g1;
                bool cut = last || done + run >= per * (slot + 1);
                if (!cut) {
                    const dmrgk::Group& N = w.groups[g + 1];
                    cut = g + 2 - a > dmrgk::kRecG || N.c1 - w.groups[a].c0 > dmrgk::kRecC ||
                          N.c0 != w.groups[g].c1;
                }
                if (!cut) continue;
                dmrgk::Task u = t;
                u.g0 = a;
                u.g1 = g + 1;
                u.c_off = poff + slot * slot_elems;
                u.ldc = t.ncol;
                u.cbuf = dmrgk::kPartialBuf | (1 << 9);
                out[task_class_of(w, u)].emplace_back(run, u);
                done += run;
                run = 0;
                a = g + 1;
                ++slot;
            }
            dmrgk::Reduce r;
            r.c_off = t.c_off;
            r.poff = poff;
            r.ldc = t.ldc;
            r.m = t.m;
            r.col0 = t.col0;
            r.ncol = t.ncol;
            r.nslot = slot;
            r.cbuf = t.cbuf & (15 | 256);
            w.reduces.push_back(r);
            poff += slot * slot_elems;
        }
    }
    w.partial_elems = poff;
    for (int c = 0; c < dmrgk::kNumClass; ++c) {
        std::stable_sort(out[c].begin(), out[c].end(),
                         [](const auto& x, const auto& y) { return x.first > y.first; });
        w.task[c].clear();
        for (auto& e : out[c]) w.task[c].push_back(e.second);
    }
}

// Every element a task can touch must lie inside its buffer: checked on the
// host before any work list reaches the device.  The kernels address an
// operand through a 64-bit block origin plus a 32-bit byte offset (scalar base
// + vector offset loads), with the in-block element index formed in 32-bit
// signed arithmetic; so the span of every operand, from its origin to the last
// element a task reads or writes, must stay below 2^32 bytes at 8-byte
// elements (the lists are shared by the FP64 and FP32 products).  A longer
// operand is reported as DMRG_E_UNSUPPORTED rather than wrapping silently.
dmrg_status validate_work(WorkList& w, const int64_t* size) {
    split_large(w);
    bool span_ok = true;
    auto in = [&](int buf, int64_t first, int64_t last) {
        if (last - first >= kMaxOperandSpan) {
            span_ok = false;
            return false;
        }
        return buf >= 0 && buf < dmrgk::kMaxBuf && first >= 0 && last < size[buf] && first <= last;
    };
    auto bad = [&](const char* what) {
        return span_ok ? fail(DMRG_E_STATE, std::string("work list: ") + what)
                       : fail(DMRG_E_UNSUPPORTED, std::string("work list: ") + what +
                                                      " (operand spans 2^32 bytes or more)");
    };
    for (int cls = 0; cls < dmrgk::kNumClass; ++cls) {
        const int cap = dmrgk::class_rows(cls);
        int lg0 = -1, lg1 = -1;
        for (const dmrgk::Task& t : w.task[cls]) {
            const bool local = (t.cbuf >> 9) & 1;
            if (t.m > cap || t.m < 1 || t.n < 1 || t.col0 < 0 || t.ncol < 1 || t.col0 + t.ncol > t.n ||
                t.ncol > dmrgk::class_cols(cls) || (local ? t.ldc != t.ncol : t.ldc < t.n))
                return fail(DMRG_E_STATE, "work list: bad task shape");
            if (local ? !in(t.cbuf & 15, t.c_off, t.c_off + (int64_t)t.m * t.ncol - 1)
                      : !in(t.cbuf & 15, t.c_off, t.c_off + (int64_t)(t.m - 1) * t.ldc + t.n - 1))
                return bad("output out of bounds");
            if (t.g0 == lg0 && t.g1 == lg1) continue;
            lg0 = t.g0;
            lg1 = t.g1;
            if (t.g0 < 0 || t.g1 > (int)w.groups.size() || t.g0 > t.g1)
                return fail(DMRG_E_STATE, "work list: bad group range");
            for (int g = t.g0; g < t.g1; ++g) {
                const dmrgk::Group& G = w.groups[g];
                if (G.mu < 1 || G.mu > cap) return fail(DMRG_E_STATE, "work list: group rows exceed class");
                if (!(G.flags & dmrgk::G_HAS_X) && G.xid_coef != 0.0 && G.mu != t.m)
                    return fail(DMRG_E_STATE, "work list: identity X with mismatched rows");
                if (G.flags & dmrgk::G_HAS_X) {
                    const bool tr = G.flags & dmrgk::G_TRANS_X;
                    const int64_t last = tr ? G.x_off + (int64_t)(G.mu - 1) * G.ldx + t.m - 1
                                            : G.x_off + (int64_t)(t.m - 1) * G.ldx + G.mu - 1;
                    if ((tr ? G.ldx < t.m : G.ldx < G.mu) || !in(G.flags & 7, G.x_off, last))
                        return bad("X operand out of bounds");
                }
                if (G.c0 < 0 || G.c1 > (int)w.contribs.size() || G.c0 > G.c1)
                    return fail(DMRG_E_STATE, "work list: bad contribution range");
                for (int c = G.c0; c < G.c1; ++c) {
                    const dmrgk::Contrib& q = w.contribs[c];
                    const bool ida = q.flags & dmrgk::F_ID_A, idb = q.flags & dmrgk::F_ID_B;
                    const bool ta = q.flags & dmrgk::F_TRANS_A, tb = q.flags & dmrgk::F_TRANS_B;
                    const int abuf = q.flags & 7, bbuf = (q.flags >> 3) & 7;
                    if (ida && idb) {
                        if (q.a_off < 0 || q.a_off > 1 << 20) return fail(DMRG_E_STATE, "work list: identity offset");
                        continue;
                    }
                    if (ida) {          // U += alpha B[0:mu, 0:n]
                        const int64_t last = tb ? q.b_off + (int64_t)(t.n - 1) * q.ldb + G.mu - 1
                                                : q.b_off + (int64_t)(G.mu - 1) * q.ldb + t.n - 1;
                        if (!in(bbuf, q.b_off, last)) return bad("B (A=I) out of bounds");
                        continue;
                    }
                    if (idb) {          // U += alpha A[0:mu, 0:n]
                        const int64_t last = ta ? q.a_off + (int64_t)(t.n - 1) * q.lda + G.mu - 1
                                                : q.a_off + (int64_t)(G.mu - 1) * q.lda + t.n - 1;
                        if (!in(abuf, q.a_off, last)) return bad("A (B=I) out of bounds");
                        continue;
                    }
                    if (q.k < 1) return fail(DMRG_E_STATE, "work list: empty contraction");
                    const int64_t la = ta ? q.a_off + (int64_t)(q.k - 1) * q.lda + G.mu - 1
                                          : q.a_off + (int64_t)(G.mu - 1) * q.lda + q.k - 1;
                    const int64_t lb = tb ? q.b_off + (int64_t)(t.n - 1) * q.ldb + q.k - 1
                                          : q.b_off + (int64_t)(q.k - 1) * q.ldb + t.n - 1;
                    if (!in(abuf, q.a_off, la)) return bad("A out of bounds");
                    if (!in(bbuf, q.b_off, lb)) return bad("B out of bounds");
                }
            }
        }
    }
    for (const dmrgk::Reduce& r : w.reduces) {
        if (r.m < 1 || r.m > dmrgk::kTallRows || r.ncol < 1 || r.ncol > dmrgk::kMaxCols || r.col0 < 0 ||
            r.col0 + r.ncol > r.ldc || r.nslot < 1)
            return fail(DMRG_E_STATE, "work list: bad reduction shape");
        if (!in(r.cbuf & 15, r.c_off, r.c_off + (int64_t)(r.m - 1) * r.ldc + r.col0 + r.ncol - 1))
            return fail(DMRG_E_STATE, "work list: reduction output out of bounds");
        if (!in(dmrgk::kPartialBuf, r.poff, r.poff + (int64_t)r.nslot * r.m * r.ncol - 1))
            return fail(DMRG_E_STATE, "work list: partial tiles out of bounds");
    }
    return DMRG_OK;
}

int64_t work_bytes(const WorkList& w) {
    int64_t bytes = 0;
    for (int c = 0; c < dmrgk::kNumClass; ++c) bytes += ((int64_t)w.task[c].size() * sizeof(dmrgk::Task) + 255) & ~int64_t(255);
    bytes += ((int64_t)w.groups.size() * sizeof(dmrgk::Group) + 255) & ~int64_t(255);
    bytes += ((int64_t)w.contribs.size() * sizeof(dmrgk::Contrib) + 255) & ~int64_t(255);
    bytes += ((int64_t)w.reduces.size() * sizeof(dmrgk::Reduce) + 255) & ~int64_t(255);
    return std::max<int64_t>(bytes, 256);
}

// Copies the selected parts of a list into one arena region: the tasks and
// reductions (with_tasks) and the groups and contributions (with_records).
static dmrg_status upload_parts(Ctx* ctx, const WorkList& w, DevWork& d, void* stream, bool with_tasks,
                                bool with_records, bool with_useful = true) {
    auto round = [](int64_t x) { return (x + 255) & ~int64_t(255); };
    int64_t bytes = 0;
    int64_t toff[dmrgk::kNumClass] = {};
    if (with_tasks)
        for (int c = 0; c < dmrgk::kNumClass; ++c) {
            toff[c] = bytes;
            bytes += round((int64_t)w.task[c].size() * sizeof(dmrgk::Task));
        }
    const int64_t goff = bytes;
    if (with_records) bytes += round((int64_t)w.groups.size() * sizeof(dmrgk::Group));
    const int64_t coff = bytes;
    if (with_records) bytes += round((int64_t)w.contribs.size() * sizeof(dmrgk::Contrib));
    const int64_t roff = bytes;
    if (with_tasks) bytes += round((int64_t)w.reduces.size() * sizeof(dmrgk::Reduce));
    const int64_t reg = ctx->arena.alloc(std::max<int64_t>(bytes, 256));
    if (reg < 0) return fail(DMRG_E_WORKSPACE, "arena too small for a work list of " + std::to_string(bytes) + " bytes");
    d.region = reg;
    char* base = ctx->arena.base + reg;
    hipStream_t s = (hipStream_t)stream;
    const bool dev = !ctx->dry;
    if (with_tasks) {
        for (int c = 0; c < dmrgk::kNumClass; ++c) {
            d.task[c] = (dmrgk::Task*)(base + toff[c]);
            d.ntask[c] = (int)w.task[c].size();
            d.useful[c] = 0;
            if (with_useful)
                for (const dmrgk::Task& t : w.task[c]) d.useful[c] += task_useful_flops(w, t);
            if (dev && !w.task[c].empty())
                DMRG_HIP(hipMemcpyAsync(d.task[c], w.task[c].data(), w.task[c].size() * sizeof(dmrgk::Task),
                                        hipMemcpyHostToDevice, s));
        }
        d.lds_records = true;
        for (const auto& T : w.task)
            for (const dmrgk::Task& t : T) d.lds_records = d.lds_records && records_fit(w, t);
        d.reduces = (dmrgk::Reduce*)(base + roff);
        d.nred = (int)w.reduces.size();
        if (dev && !w.reduces.empty())
            DMRG_HIP(hipMemcpyAsync(d.reduces, w.reduces.data(), w.reduces.size() * sizeof(dmrgk::Reduce),
                                    hipMemcpyHostToDevice, s));
    }
    if (with_records) {
        d.groups = (dmrgk::Group*)(base + goff);
        d.contribs = (dmrgk::Contrib*)(base + coff);
        if (dev && !w.groups.empty())
            DMRG_HIP(hipMemcpyAsync(d.groups, w.groups.data(), w.groups.size() * sizeof(dmrgk::Group),
                                    hipMemcpyHostToDevice, s));
        if (dev && !w.contribs.empty())
            DMRG_HIP(hipMemcpyAsync(d.contribs, w.contribs.data(), w.contribs.size() * sizeof(dmrgk::Contrib),
                                    hipMemcpyHostToDevice, s));
    }
    if (dev) DMRG_HIP(hipStreamSynchronize(s));   // host vectors may be released after return
    return DMRG_OK;
}

dmrg_status upload_work(Ctx* ctx, const WorkList& w, DevWork& d, void* stream) {
    return upload_parts(ctx, w, d, stream, true, true);
}

dmrg_status upload_records(Ctx* ctx, const WorkList& w, DevWork& d, void* stream) {
    return upload_parts(ctx, w, d, stream, false, true);
}

dmrg_status upload_tasks(Ctx* ctx, const WorkList& w, const DevWork& recs, DevWork& d, void* stream,
                         bool with_useful) {
    const dmrg_status st = upload_parts(ctx, w, d, stream, true, false, with_useful);
    d.groups = recs.groups;
    d.contribs = recs.contribs;
    return st;
}

int64_t task_bytes(const WorkList& w) {
    int64_t bytes = 0;
    for (const auto& T : w.task) bytes += ((int64_t)T.size() * sizeof(dmrgk::Task) + 255) & ~int64_t(255);
    return bytes + (((int64_t)w.reduces.size() * sizeof(dmrgk::Reduce) + 255) & ~int64_t(255));
}

void free_work(Ctx* ctx, DevWork& d) {
    if (d.region >= 0) ctx->arena.release(d.region);
    d = DevWork();
}

dmrg_status run_work_f64(const DevWork& d, const dmrgk::Bases<double>& b, int nvec, void* stream) {
    for (int c = dmrgk::kNumClass - 1; c >= 0; --c)
        DMRG_HIP(dmrgk::launch_chain_f64(c, d.lds_records, d.task[c], d.ntask[c], d.groups, d.contribs, b, nvec,
                                         stream));
    DMRG_HIP(dmrgk::launch_reduce_f64(d.reduces, d.nred, b, nvec, stream));
    return DMRG_OK;
}

dmrg_status run_work_f32(const DevWork& d, const dmrgk::Bases<float>& b, int nvec, void* stream) {
    for (int c = dmrgk::kNumClass - 1; c >= 0; --c)
        DMRG_HIP(dmrgk::launch_chain_f32(c, d.lds_records, d.task[c], d.ntask[c], d.groups, d.contribs, b, nvec,
                                         stream));
    DMRG_HIP(dmrgk::launch_reduce_f32(d.reduces, d.nred, b, nvec, stream));
    return DMRG_OK;
}

template <typename T, typename L, typename R>
static dmrg_status run_timed(const DevWork& d, const dmrgk::Bases<T>& b, float* ms, void* stream, L chain, R red) {
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t ev[2 * (dmrgk::kNumClass + 1)];
    for (auto& e : ev) DMRG_HIP(hipEventCreate(&e));
    dmrg_status st = DMRG_OK;
    for (int c = dmrgk::kNumClass - 1; c >= 0 && st == DMRG_OK; --c) {   // classes high -> low, then reduce
        hipEventRecord(ev[2 * c], s);
        const int e = chain(c, d.lds_records, d.task[c], d.ntask[c], d.groups, d.contribs, b, 1, stream);
        hipEventRecord(ev[2 * c + 1], s);
        if (e) st = hip_fail(e, "kernel launch");
    }
    if (st == DMRG_OK) {
        hipEventRecord(ev[2 * dmrgk::kNumClass], s);
        const int e = red(d.reduces, d.nred, b, 1, stream);
        hipEventRecord(ev[2 * dmrgk::kNumClass + 1], s);
        if (e) st = hip_fail(e, "kernel launch");
    }
    if (st == DMRG_OK && hipEventSynchronize(ev[2 * dmrgk::kNumClass + 1]) != hipSuccess)
        st = fail(DMRG_E_HIP, "event synchronize");
    for (int c = 0; c <= dmrgk::kNumClass && st == DMRG_OK; ++c) {
        const bool empty = c < dmrgk::kNumClass ? d.ntask[c] == 0 : d.nred == 0;
        float t = 0;
        if (!empty) hipEventElapsedTime(&t, ev[2 * c], ev[2 * c + 1]);
        ms[c] = t;
    }
    for (auto& e : ev) hipEventDestroy(e);
    return st;
}

dmrg_status run_work_timed_f64(const DevWork& d, const dmrgk::Bases<double>& b, float* ms, void* stream) {
    return run_timed<double>(d, b, ms, stream, dmrgk::launch_chain_f64, dmrgk::launch_reduce_f64);
}
dmrg_status run_work_timed_f32(const DevWork& d, const dmrgk::Bases<float>& b, float* ms, void* stream) {
    return run_timed<float>(d, b, ms, stream, dmrgk::launch_chain_f32, dmrgk::launch_reduce_f32);
}

// ---------------------------------------------------------------------------
// integral-weighted sums: one dense GEMM per input family,
//   out[n_req x stride] = W[n_req x n_ops] . family[n_ops x stride]
void plan_wsums(const OpSetImpl& src, WSumPlan& plan, OpSetImpl& temps) {
    std::map<int, std::vector<int>> by_fam;
    for (size_t i = 0; i < plan.reqs.size(); ++i) by_fam[plan.reqs[i].fam].push_back((int)i);
    plan.out.assign(plan.reqs.size(), {-1, -1});
    for (auto& kv : by_fam) {
        const Family& F = src.fams[kv.first];
        Family T;                      // a fresh temporary family per input family
        T.kind = 'T';
        T.dq = F.dq;
        T.par = F.par;
        T.skel = temps.skel_for(F.dq);
        temps.fams.push_back(T);
        const int tf = (int)temps.fams.size() - 1;
        for (int r : kv.second) {
            Family& TF = temps.fams[tf];
            const int idx = (int)TF.keys.size();
            const int64_t key = okey('T', tf, idx);
            TF.keys.push_back(key);
            TF.index[key] = idx;
            plan.out[r] = {tf, idx};
        }
    }
}

// The source family is the B operand [nin x stride]; its span from a
// contribution's origin must stay below kMaxOperandSpan, so the sum over the
// operator index is cut into chunks of at most kc operators (one contribution
// each, summed in order into the same tile).  Output rows go in groups of at
// most 64 (fewer for very large operators) for the same reason.
// DMRG_FAMILY_CHUNK_OPS lowers kc (a GPU test forces the chunked path).
void family_chunks(int64_t stride, int64_t& kc, int& rchunk) {
    kc = kMaxOperandSpan / std::max<int64_t>(stride, 1);
    if (const char* e = std::getenv("DMRG_FAMILY_CHUNK_OPS")) kc = std::min<int64_t>(kc, std::max(1, std::atoi(e)));
    rchunk = (int)std::min<int64_t>(64, kMaxOperandSpan / std::max<int64_t>(stride, 1));
}

int64_t wsum_work_bytes(const OpSetImpl& src, const WSumPlan& plan) {
    std::map<int, int> rows;   // input family -> requests
    for (const WSumReq& r : plan.reqs) rows[r.fam]++;
    int64_t worst = 0;
    for (auto& kv : rows) {
        const Family& F = src.fams[kv.first];
        const int64_t nin = (int64_t)F.keys.size();
        int64_t kc;
        int rchunk;
        family_chunks(F.stride, kc, rchunk);
        if (kc < 1 || rchunk < 1) continue;
        const int64_t ngroup = (kv.second + rchunk - 1) / rchunk;
        const int64_t ncontrib = ngroup * ((nin + kc - 1) / kc);
        const int64_t ntask = ngroup * ((F.stride + dmrgk::kMaxCols - 1) / dmrgk::kMaxCols);
        const int64_t b = ((nin * kv.second * 8 + 255) / 256 * 256) + ntask * (int64_t)sizeof(dmrgk::Task) +
                          ngroup * (int64_t)sizeof(dmrgk::Group) + ncontrib * (int64_t)sizeof(dmrgk::Contrib) +
                          (dmrgk::kNumClass + 3) * 256;
        worst = std::max(worst, b);
    }
    return worst;
}

dmrg_status family_gemm(Ctx* ctx, const std::vector<double>& W, const OpSetImpl& src, int sf,
                        const OpSetImpl& dst, int df, int row0, int nrows, void* stream) {
    const Family& F = src.fams[sf];
    const Family& D = dst.fams[df];
    const int nin = (int)F.keys.size();
    const int64_t stride = F.stride;
    if (nrows <= 0 || stride == 0) return DMRG_OK;
    if (D.stride != stride) return fail(DMRG_E_ARG, "family_gemm: skeleton mismatch");
    if (stride > INT32_MAX) return fail(DMRG_E_UNSUPPORTED, "operator larger than 2^31 elements");
    if ((int64_t)W.size() != (int64_t)nrows * nin) return fail(DMRG_E_ARG, "family_gemm: weight shape");
    if (nin == 0) {
        if (!ctx->dry)
            DMRG_HIP(hipMemsetAsync(dst.dev + D.base + (int64_t)row0 * stride, 0, (size_t)nrows * stride * 8,
                                    (hipStream_t)stream));
        return DMRG_OK;
    }
    const double t0 = wall_s();
    const int64_t wreg = ctx->arena.alloc((int64_t)W.size() * 8);
    if (wreg < 0) return fail(DMRG_E_WORKSPACE, "arena too small for integral weights");
    double* wdev = (double*)(ctx->arena.base + wreg);
    hipStream_t s = (hipStream_t)stream;
    int e = ctx->dry ? 0 : (int)hipMemcpyAsync(wdev, W.data(), W.size() * 8, hipMemcpyHostToDevice, s);
    if (e) { ctx->arena.release(wreg); return hip_fail(e, "weights upload"); }
    int64_t kc;
    int rchunk;
    family_chunks(stride, kc, rchunk);
    if (kc < 1) return fail(DMRG_E_UNSUPPORTED, "operator of 2^32 bytes or more");
    WorkList wl;
    for (int r0 = 0; r0 < nrows; r0 += rchunk) {
        const int rows = std::min(rchunk, nrows - r0);
        const int g0 = (int)wl.groups.size();
        dmrgk::Group g{};
        g.xid_coef = 1.0;
        g.mu = rows;
        g.c0 = (int)wl.contribs.size();
        for (int64_t k0 = 0; k0 < nin; k0 += kc) {
            dmrgk::Contrib c{};
            c.a_off = (int64_t)r0 * nin + k0;
            c.lda = nin;
            c.b_off = F.base + k0 * stride;
            c.ldb = (int)stride;
            c.k = (int)std::min<int64_t>(kc, nin - k0);
            c.alpha = 1.0;
            c.flags = 0 | (1 << 3);
            wl.contribs.push_back(c);
        }
        g.c1 = (int)wl.contribs.size();
        wl.groups.push_back(g);
        emit_block_tasks(wl, 3, D.base + (int64_t)(row0 + r0) * stride, (int)stride, rows, (int)stride,
                         g0, g0 + 1);
    }
    int64_t sz[dmrgk::kMaxBuf] = {0};
    sz[0] = (int64_t)W.size();
    sz[1] = src.elems;
    sz[3] = dst.elems;
    DevWork dw;
    dmrg_status st = validate_work(wl, sz);
    if (st == DMRG_OK) st = upload_work(ctx, wl, dw, stream);
    if (st != DMRG_OK) { ctx->arena.release(wreg); return st; }
    const double t1 = wall_s();
    ctx->tm[TM_WSUM_HOST] += t1 - t0;
    dmrgk::Bases<double> b{};
    b.p[0] = wdev;
    b.p[1] = src.dev;
    b.p[3] = dst.dev;
    if (!ctx->dry) {
        st = run_work_f64(dw, b, 1, stream);
        if (st == DMRG_OK) {
            e = (int)hipStreamSynchronize(s);
            if (e) st = hip_fail(e, "family gemm");
        }
    }
    ctx->tm[TM_WSUM_DEV] += wall_s() - t1;
    free_work(ctx, dw);
    ctx->arena.release(wreg);
    return st;
}

dmrg_status exec_wsums(Ctx* ctx, const OpSetImpl& src, const WSumPlan& plan, const OpSetImpl& temps,
                       void* stream) {
    std::map<int, std::vector<int>> rows_of;   // temp family -> request ids ordered by idx
    for (size_t i = 0; i < plan.reqs.size(); ++i) rows_of[plan.out[i].first].push_back((int)i);
    for (auto& kv : rows_of) {
        auto& v = kv.second;
        std::sort(v.begin(), v.end(), [&](int x, int y) { return plan.out[x].second < plan.out[y].second; });
        std::vector<double> W;
        for (int r : v) W.insert(W.end(), plan.reqs[r].w.begin(), plan.reqs[r].w.end());
        dmrg_status st = family_gemm(ctx, W, src, plan.reqs[v[0]].fam, temps, kv.first, 0, (int)v.size(), stream);
        if (st != DMRG_OK) return st;
    }
    return DMRG_OK;
}

}  // namespace dmrg
