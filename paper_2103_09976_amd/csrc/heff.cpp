// The effective Hamiltonian of the two-site middle step (Appendix A,
// effective eigenproblem) as a sum over the normal/complementary terms of the
// left-right decomposition across L' = Lb + d1 | R' = d2 + Rb:
//
//   H_eff = H^{L'} 1 + 1 H^{R'} + sum_{p in L'} (C_p R^{R'}_p - D_p R^{R'}_p+)
//         + sum_{p in R'} (R^{L'}_p+ D_p - R^{L'}_p C_p)
//         + sum_{p<r in L'} (A_pr P^{R'}_pr + h.c.) + sum_{pq in L'} B_pq Q^{R'}_pq
//
// with sigma = sum_terms X (P^{pi(Y)} Psi) Y^T.  Each operator of L' and R'
// stays delayed: per site transition, one block-level operator of Lb (Rb)
// or the identity.  The work list ("list of GEMMs generated once for each
// site", Section II.G) has one output tile per (psi sub-block, 32 columns);
// its groups are (term, left transition) and its contributions the right
// transitions, so each term runs as psi . Y^T summed in LDS, then X . (that).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <deque>
#include <fstream>
#include <memory>
#include <mutex>
#include <sstream>
#include <unordered_set>

#include "core.hpp"

// per-phase host timing on stderr when DMRG_VERBOSE is set
struct PhaseClock {
    bool on = std::getenv("DMRG_VERBOSE") != nullptr;
    std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
    void mark(const char* what) {
        if (!on) return;
        const auto n = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[dmrg] %-28s %8.3f s\n", what, std::chrono::duration<double>(n - t).count());
        t = n;
    }
};


using namespace dmrg;

// Parameters of the work list that the autotuner chooses: the number of
// equal-cost chunks heavy tasks are cut into, and the height from which tiles
// run on the tall kernel (97: only tiles the one-wave kernels cannot hold).
struct TuneParams {
    int balance = 131072;
    int tall_min = dmrgk::kMaxRows + 1;
};

// A product captured as a graph of kernel nodes (one per non-empty class,
// then the reduction), replayed with its nodes' arguments updated to the
// vectors of each call.
struct ProductGraph {
    int prec = -1, nvec = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipGraphNode_t> nodes;
    std::vector<int> cls;   // class of each node; dmrgk::kNumClass is the reduction
};

struct PsiBlock {
    int a, s1, s2, b;
    int ma, mb;
    int64_t off;
};

struct Term {
    double coef;
    TransOp X, Y;
    char kind;    // '2', '1', 'H'
};

struct dmrg_heff {
    Ctx* ctx = nullptr;
    const OpSetImpl* Lb = nullptr;
    const OpSetImpl* Rb = nullptr;
    OpSetImpl TL, TR, TML, TMR;
    Grown GL, GR;
    std::vector<PsiBlock> blocks;
    std::vector<int> blk_index;    // (a*4 + s1)*4 + s2 -> block or -1
    int64_t dim = 0;
    int n_roots = 1;
    DevWork work;
    DevWork recs;   // groups and contributions of work when held apart (autotuned lists)
    // diagonal
    int64_t diag_region = -1;
    dmrgk::DiagBlock* dblocks = nullptr;
    dmrgk::DiagTerm* dterms = nullptr;
    int n_dblocks = 0;
    // fp32 mirrors of buffers 0,1,4..7
    int64_t f32_region = -1;
    float* f32[8] = {nullptr};
    // partial tiles of split tasks (buffer 8), n_roots vectors
    int64_t part_region = -1;
    void* part = nullptr;
    int64_t part_elems = 0;
    int64_t flops = 0;
    int64_t op_bytes64 = 0;
    int n2 = 0, n1 = 0, nh = 0;
    size_t ntask = 0, ngroup = 0, ncontrib = 0;
    int precision = DMRG_PREC_F32;      // DMRG_PREC_F64: FP64 products only
    const dmrg_psi_layout* layout = nullptr;   // caller's layout during creation (NULL: default)
    int flags = 0;                      // DMRG_HEFF_GRAPH | DMRG_HEFF_AUTOTUNE
    // work-list parameters (defaults, tuned or cached) and the tuning record
    TuneParams tune;
    int tuned = 0;
    std::vector<TuneParams> cand;
    std::vector<float> cand_ms;
    std::unique_ptr<WorkList> base;     // the list before splitting, kept while tuning
    int64_t buf_elems[dmrgk::kMaxBuf] = {0};
    // captured products: one graph per (precision, vector batch)
    std::deque<ProductGraph> graphs;
    int64_t graph_launches = 0;
};

namespace dmrg {

static TransOp transpose_left(const TransOp& T) {
    TransOp R;
    R.dq = -T.dq;
    R.par = T.par;
    for (const Comp& c : T.comps) {
        Comp d = c;
        d.sb = c.sk;
        d.sk = c.sb;
        if (c.ref.type == 1) d.ref.trans = !c.ref.trans;
        const int dn = c.ref.dq().n();
        if (c.sgn_par && (dn & 1)) d.coef = -c.coef;
        R.comps.push_back(d);
    }
    return R;
}

static TransOp transpose_right(const TransOp& T) {
    TransOp R;
    R.dq = -T.dq;
    R.par = T.par;
    for (const Comp& c : T.comps) {
        Comp d = c;
        d.sb = c.sk;
        d.sk = c.sb;
        if (c.ref.type == 1) d.ref.trans = !c.ref.trans;
        R.comps.push_back(d);
    }
    return R;
}

static TransOp identity_op() {
    TransOp T;
    T.dq = QN(0, 0);
    T.par = 0;
    for (int s = 0; s < 4; ++s) T.comps.push_back(Comp{s, s, Ref(), 1.0, 0});
    return T;
}

// Replace every site transition holding two or more non-identity components
// by one operator of `out` (sum of the components, signs folded per block).
static dmrg_status materialize(Ctx* C, std::vector<TransOp*> ops, const OpSetImpl& base, const OpSetImpl& temps,
                               OpSetImpl& out, void* stream) {
    struct Job { TransOp* T; std::vector<int> comps; int sb, sk; int fam, idx; QN dq; };
    std::vector<Job> jobs;
    out.basis = base.basis;
    out.kind = 2;
    for (TransOp* T : ops) {
        std::map<std::pair<int, int>, std::vector<int>> by;
        for (size_t i = 0; i < T->comps.size(); ++i)
            if (T->comps[i].ref.type == 1) by[{T->comps[i].sb, T->comps[i].sk}].push_back((int)i);
        for (auto& kv : by) {
            if (kv.second.size() < 2) continue;
            Job j;
            j.T = T;
            j.comps = kv.second;
            j.sb = kv.first.first;
            j.sk = kv.first.second;
            j.dq = T->comps[kv.second[0]].ref.dq();
            const int f = out.family('M', j.dq, T->comps[kv.second[0]].ref.par());
            Family& F = out.fams[f];
            j.fam = f;
            j.idx = (int)F.keys.size();
            const int64_t key = okey('M', (int)jobs.size(), -1);
            F.keys.push_back(key);
            F.index[key] = j.idx;
            jobs.push_back(j);
        }
    }
    if (jobs.empty()) return DMRG_OK;
    dmrg_status st = alloc_set(C, out);
    if (st != DMRG_OK) return st;
    WorkList wl;
    const Basis& B = base.basis;
    for (const Job& j : jobs) {
        const Family& F = out.fams[j.fam];
        const Skel& S = out.skels[F.skel];
        for (size_t b = 0; b < S.ket.size(); ++b) {
            const int a = S.ket[b], a2 = S.bra[b];
            const int g0 = (int)wl.groups.size();
            dmrgk::Group g{};
            g.xid_coef = 1.0;
            g.mu = B.m[a2];
            g.c0 = (int)wl.contribs.size();
            for (int ci : j.comps) {
                const Comp& cp = j.T->comps[ci];
                int bra, ld;
                int64_t off;
                bool tr;
                if (!cp.ref.block(a, bra, off, ld, tr) || bra != a2) continue;
                const double sg = (cp.sgn_par && (B.q[a].n() & 1)) ? -1.0 : 1.0;
                dmrgk::Contrib c{};
                c.a_off = off;
                c.lda = ld;
                c.k = B.m[a];
                c.alpha = cp.coef * sg;
                c.flags = ((cp.ref.set == &base) ? 0 : 1) | (tr ? dmrgk::F_TRANS_A : 0) | dmrgk::F_ID_B;
                wl.contribs.push_back(c);
            }
            g.c1 = (int)wl.contribs.size();
            int ng = 0;
            if (g.c1 > g.c0) { wl.groups.push_back(g); ng = 1; }
            emit_block_tasks(wl, 3, F.base + (int64_t)j.idx * F.stride + S.off[b], B.m[a], B.m[a2], B.m[a], g0,
                             g0 + ng);
        }
    }
    int64_t sz[dmrgk::kMaxBuf] = {0};
    sz[0] = base.elems;
    sz[1] = temps.elems > 0 ? temps.elems : base.elems;
    sz[3] = out.elems;
    DevWork dw;
    st = validate_work(wl, sz);
    if (st == DMRG_OK) st = upload_work(C, wl, dw, stream);
    if (st != DMRG_OK) return st;
    {
    dmrgk::Bases<double> bs{};
    bs.p[0] = base.dev;
    bs.p[1] = temps.dev ? temps.dev : base.dev;
    bs.p[3] = out.dev;
    if (!C->dry) {
        st = run_work_f64(dw, bs, 1, stream);
        if (st == DMRG_OK) {
            const int e = (int)hipStreamSynchronize((hipStream_t)stream);
            if (e) st = hip_fail(e, "materialize");
        }
    }
    free_work(C, dw);
    }
    if (st != DMRG_OK) return st;
    // rewrite the transitions
    std::map<TransOp*, std::vector<const Job*>> per;
    for (const Job& j : jobs) per[j.T].push_back(&j);
    for (auto& kv : per) {
        TransOp* T = kv.first;
        std::vector<char> drop(T->comps.size(), 0);
        std::vector<Comp> add;
        for (const Job* j : kv.second) {
            for (int ci : j->comps) drop[ci] = 1;
            Comp c;
            c.sb = j->sb;
            c.sk = j->sk;
            c.ref.type = 1;
            c.ref.set = &out;
            c.ref.fam = j->fam;
            c.ref.idx = j->idx;
            c.ref.trans = false;
            c.coef = 1.0;
            c.sgn_par = 0;
            add.push_back(c);
        }
        std::vector<Comp> keep;
        for (size_t i = 0; i < T->comps.size(); ++i)
            if (!drop[i]) keep.push_back(T->comps[i]);
        keep.insert(keep.end(), add.begin(), add.end());
        T->comps.swap(keep);
    }
    return DMRG_OK;
}

static int buf_of(const dmrg_heff* H, const OpSetImpl* s) {
    if (s == H->Lb) return 0;
    if (s == H->Rb) return 1;
    if (s == &H->TL) return 4;
    if (s == &H->TR) return 5;
    if (s == &H->TML) return 6;
    if (s == &H->TMR) return 7;
    return -1;
}

}  // namespace dmrg

// Splits, balances and checks a work list under the given parameters.
static dmrg_status finalize_list(dmrg_heff* H, WorkList& wl, const TuneParams& tp) {
    wl.tall_min = tp.tall_min;
    reclassify(wl);
    split_large(wl);
    balance_work(wl, tp.balance);
    int64_t sz[dmrgk::kMaxBuf];
    for (int i = 0; i < dmrgk::kMaxBuf; ++i) sz[i] = H->buf_elems[i];
    sz[dmrgk::kPartialBuf] = wl.partial_elems;
    return validate_work(wl, sz);
}

// Shape key of an H_eff for the tuning cache: orbitals, electrons, share,
// roots and every sector dimension of both blocks (FNV-1a).
static std::string shape_key(const dmrg_heff* H) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](int64_t x) {
        for (int i = 0; i < 8; ++i) {
            h ^= (uint64_t)((x >> (8 * i)) & 255);
            h *= 1099511628211ull;
        }
    };
    const Ctx* C = H->ctx;
    mix(C->K); mix(C->na); mix(C->nb); mix(C->n_proc); mix(C->proc_id); mix(H->n_roots);
    for (const OpSetImpl* S : {H->Lb, H->Rb})
        for (int i = 0; i < S->basis.size(); ++i) {
            mix(S->basis.q[i].a);
            mix(S->basis.q[i].b);
            mix(S->basis.m[i]);
        }
    char buf[32];
    std::snprintf(buf, sizeof(buf), "%016llx", (unsigned long long)h);
    return buf;
}

// Process-wide tuning cache; DMRG_TUNE_CACHE names a file that is read once
// and appended to ("key balance tall_min" per line).
static std::mutex g_tune_mu;
static std::map<std::string, TuneParams> g_tune;
static bool g_tune_loaded = false;

static void lookup_tuning(dmrg_heff* H) {
    H->tune = TuneParams();
    if (const char* e = std::getenv("DMRG_BALANCE")) H->tune.balance = std::max(1, std::atoi(e));
    if (const char* e = std::getenv("DMRG_TALL_MIN")) H->tune.tall_min = std::max(1, std::atoi(e));
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_tune_loaded) {
        g_tune_loaded = true;
        if (const char* f = std::getenv("DMRG_TUNE_CACHE")) {
            std::ifstream in(f);
            std::string key;
            TuneParams tp;
            while (in >> key >> tp.balance >> tp.tall_min) g_tune[key] = tp;
        }
    }
    auto it = g_tune.find(shape_key(H));
    if (it != g_tune.end()) {
        H->tune = it->second;
        H->tuned = 2;
    }
}

static void store_tuning(const dmrg_heff* H) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const std::string key = shape_key(H);
    g_tune[key] = H->tune;
    if (const char* f = std::getenv("DMRG_TUNE_CACHE")) {
        std::ofstream out(f, std::ios::app);
        out << key << " " << H->tune.balance << " " << H->tune.tall_min << "\n";
    }
}

// The caller's wavefunction layout: every sub-block (a, s1, s2) once, tiling
// [0, dim) exactly; the offsets replace the default ones.
static dmrg_status apply_layout(dmrg_heff* H, const Basis& lb) {
    const dmrg_psi_layout* L = H->layout;
    const size_t n = H->blocks.size();
    if (L->n_blocks != (int32_t)n || !L->qn_left || !L->site1 || !L->site2 || !L->offset)
        return fail(DMRG_E_ARG, "psi layout: expected " + std::to_string(n) + " sub-blocks");
    std::vector<int64_t> off(n, -1);
    for (int i = 0; i < L->n_blocks; ++i) {
        const int a = lb.find(QN(L->qn_left[2 * i], L->qn_left[2 * i + 1]));
        const int s1 = L->site1[i], s2 = L->site2[i];
        if (a < 0 || s1 < 0 || s1 > 3 || s2 < 0 || s2 > 3) return fail(DMRG_E_ARG, "psi layout: unknown sub-block");
        const int bi = H->blk_index[(a * 4 + s1) * 4 + s2];
        if (bi < 0) return fail(DMRG_E_ARG, "psi layout: sub-block outside the target sector");
        if (off[bi] >= 0) return fail(DMRG_E_ARG, "psi layout: sub-block listed twice");
        off[bi] = L->offset[i];
    }
    std::vector<std::pair<int64_t, size_t>> order;
    for (size_t b = 0; b < n; ++b) order.push_back({off[b], b});
    std::sort(order.begin(), order.end());
    int64_t end = 0;
    for (auto& o : order) {
        if (o.first != end) return fail(DMRG_E_ARG, "psi layout: sub-blocks must tile [0, dim) without gaps");
        const PsiBlock& B = H->blocks[o.second];
        end += (int64_t)B.ma * B.mb;
    }
    for (size_t b = 0; b < n; ++b) H->blocks[b].off = off[b];
    return DMRG_OK;
}

static dmrg_status build_heff(dmrg_heff* H, void* stream) {
    Ctx* C = H->ctx;
    const int K = C->K, KL = H->Lb->nsites;   // dots d1 = KL, d2 = KL + 1
    const OpSetImpl& Lb = *H->Lb;
    const OpSetImpl& Rb = *H->Rb;
    std::vector<int> lp, rp;
    for (int p = 0; p < 2 * (KL + 1); ++p) lp.push_back(p);
    for (int p = 2 * (KL + 1); p < 2 * K; ++p) rp.push_back(p);
    PhaseClock clk;
    grow_left(C, Lb, KL, rp, H->GL);
    grow_right_compl(C, Rb, KL + 1, lp, H->GR);
    clk.mark("grow L' R'");
    // weighted sums of Lb / Rb operators
    {
        WSumPlan pl, pr;
        compact(H->GL.ops, Lb, pl);
        compact(H->GR.ops, Rb, pr);
        H->TL.basis = Lb.basis;
        H->TL.kind = 2;
        H->TR.basis = Rb.basis;
        H->TR.kind = 2;
        plan_wsums(Lb, pl, H->TL);
        plan_wsums(Rb, pr, H->TR);
        dmrg_status st = alloc_set(C, H->TL);
        if (st == DMRG_OK) st = alloc_set(C, H->TR);
        if (st == DMRG_OK) st = exec_wsums(C, Lb, pl, H->TL, stream);
        if (st == DMRG_OK) st = exec_wsums(C, Rb, pr, H->TR, stream);
        if (st != DMRG_OK) return st;
        resolve(H->GL.ops, pl, H->TL);
        resolve(H->GR.ops, pr, H->TR);
    }
    clk.mark("weighted sums");
    // working copies of L'/R' operators for the terms (multi-component
    // transitions of H and R materialised; GL itself stays for renormalization)
    std::unordered_map<int64_t, TransOp> Lx, Rx;
    for (size_t i = 0; i < H->GL.keys.size(); ++i) Lx[H->GL.keys[i]] = H->GL.ops[i];
    for (size_t i = 0; i < H->GR.keys.size(); ++i) Rx[H->GR.keys[i]] = H->GR.ops[i];
    {
        std::vector<TransOp*> ml, mr;
        for (auto& kv : Lx) ml.push_back(&kv.second);
        for (auto& kv : Rx) mr.push_back(&kv.second);
        dmrg_status st = materialize(C, ml, Lb, H->TL, H->TML, stream);
        if (st == DMRG_OK) st = materialize(C, mr, Rb, H->TR, H->TMR, stream);
        if (st != DMRG_OK) return st;
    }
    clk.mark("materialize");
    auto L = [&](char k, int p, int q) -> const TransOp* {
        auto it = Lx.find(okey(k, p, q));
        return it == Lx.end() ? nullptr : &it->second;
    };
    auto R = [&](char k, int p, int q) -> const TransOp* {
        auto it = Rx.find(okey(k, p, q));
        return it == Rx.end() ? nullptr : &it->second;
    };
    std::vector<Term> terms;
    terms.push_back(Term{1.0, *L('H', -1, -1), identity_op(), 'H'});
    terms.push_back(Term{1.0, identity_op(), *R('H', -1, -1), 'H'});
    for (int p : lp) {
        const TransOp *c = L('C', p, -1), *r = R('R', p, -1);
        if (!c || !r) continue;
        terms.push_back(Term{1.0, *c, *r, '1'});
        terms.push_back(Term{-1.0, transpose_left(*c), transpose_right(*r), '1'});
    }
    for (int p : rp) {
        const TransOp *r = L('R', p, -1), *c = R('C', p, -1);
        if (!c || !r) continue;
        terms.push_back(Term{1.0, transpose_left(*r), transpose_right(*c), '1'});
        terms.push_back(Term{-1.0, *r, *c, '1'});
    }
    for (size_t i = 0; i < lp.size(); ++i)
        for (size_t j = i + 1; j < lp.size(); ++j) {
            const int p = lp[i], r = lp[j];
            const TransOp *a = L('A', p, r), *d = R('D', p, r);
            if (!a || !d) continue;
            terms.push_back(Term{1.0, *a, transpose_right(*d), '2'});
            terms.push_back(Term{1.0, transpose_left(*a), *d, '2'});
        }
    for (int p : lp)
        for (int q : lp) {
            const TransOp *b = L('B', p, q), *Q = R('Q', p, q);
            if (!b || !Q) continue;
            terms.push_back(Term{1.0, *b, *Q, '2'});
        }
    if (C->e_core != 0.0) terms.push_back(Term{C->e_core, identity_op(), identity_op(), 'H'});
    for (const Term& t : terms) {
        if (t.kind == '2') H->n2++;
        else if (t.kind == '1') H->n1++;
        else H->nh++;
    }
    clk.mark("terms");
    // wavefunction layout
    const Basis& lb = Lb.basis;
    const Basis& rb = Rb.basis;
    const QN tgt(C->na, C->nb);
    H->blk_index.assign((size_t)lb.size() * 16, -1);
    int64_t off = 0;
    for (int a = 0; a < lb.size(); ++a)
        for (int s1 = 0; s1 < 4; ++s1)
            for (int s2 = 0; s2 < 4; ++s2) {
                const int b = rb.find(tgt - lb.q[a] - kSiteQ[s1] - kSiteQ[s2]);
                if (b < 0) continue;
                H->blk_index[(a * 4 + s1) * 4 + s2] = (int)H->blocks.size();
                H->blocks.push_back(PsiBlock{a, s1, s2, b, lb.m[a], rb.m[b], off});
                off += (int64_t)lb.m[a] * rb.m[b];
            }
    H->dim = off;
    if (H->layout) {
        dmrg_status ls = apply_layout(H, lb);
        if (ls != DMRG_OK) return ls;
    }
    // per term: components by bra site state
    struct TI { std::vector<const Comp*> x[4], y[4]; int piY; };
    std::vector<TI> ti(terms.size());
    for (size_t t = 0; t < terms.size(); ++t) {
        for (int sb = 0; sb < 4; ++sb) {
            int n = 0;
            for (const Comp& c : terms[t].Y.comps) n += (c.sb == sb);
            if (n > 64) return fail(DMRG_E_STATE, "more than 64 right components on one transition");
        }
        for (const Comp& c : terms[t].X.comps) ti[t].x[c.sb].push_back(&c);
        for (const Comp& c : terms[t].Y.comps) ti[t].y[c.sb].push_back(&c);
        ti[t].piY = terms[t].Y.par;
    }
    const size_t NT = terms.size();
    // validity of an output block (a', s1', s2', b')
    auto out_block = [&](int a2, int s1, int s2, int b2) -> int {
        if (a2 < 0) return -1;
        const int bi = H->blk_index[(a2 * 4 + s1) * 4 + s2];
        return (bi >= 0 && H->blocks[bi].b == b2) ? bi : -1;
    };
    // X comp maps source sector a -> bra (or -1)
    auto xmap = [&](const Comp* xc, int a, int64_t& off, int& ld, bool& tr) -> int {
        if (xc->ref.type == 0) { off = -1; ld = 0; tr = false; return a; }
        int bra;
        if (!xc->ref.block(a, bra, off, ld, tr)) return -1;
        return bra;
    };
    auto ymap = xmap;
    struct Local {
        WorkList wl;
        std::vector<dmrgk::DiagBlock> dbl;
        std::vector<dmrgk::DiagTerm> dtm;
        std::vector<std::pair<int64_t, int64_t>> ops;   // (operator block key, elements)
        std::vector<std::vector<std::pair<int64_t, int64_t>>> opshard;   // ops by key hash, sorted, unique
        std::vector<double> lfx, lfy, rfx, rfy;
    };
    const size_t nblk = H->blocks.size();
    unsigned nth = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
    if (const char* e = std::getenv("DMRG_HOST_THREADS")) nth = (unsigned)std::max(1, std::min(32, std::atoi(e)));
    if (nblk < 64) nth = 1;
    const unsigned nshard = nth;
    auto shard_of = [nshard](int64_t key) {
        return (unsigned)(((uint64_t)key * 0x9E3779B97F4A7C15ull >> 40) % nshard);
    };
    auto work = [&](size_t o0, size_t o1, Local& Lc) {
        Lc.lfx.assign(NT, 0.0); Lc.lfy.assign(NT, 0.0); Lc.rfx.assign(NT, 0.0); Lc.rfy.assign(NT, 0.0);
        WorkList& wl = Lc.wl;
        auto note = [&](int buf, int64_t o, int64_t n) { Lc.ops.emplace_back(((int64_t)buf << 56) ^ o, n); };
        for (size_t o = o0; o < o1; ++o) {
            const PsiBlock& O = H->blocks[o];
            const int g0 = (int)wl.groups.size();
            dmrgk::DiagBlock db{};
            db.off = O.off;
            db.ma = O.ma;
            db.mb = O.mb;
            db.c0 = (int)Lc.dtm.size();
            for (size_t t = 0; t < NT; ++t) {
                const auto& xs = ti[t].x[O.s1];
                const auto& ys = ti[t].y[O.s2];
                if (xs.empty() || ys.empty()) continue;
                if (ys.size() > 64) continue;   // guarded below at term construction
                const Term& T = terms[t];
                struct Src { const Comp* x = nullptr; double xid = 0.0, xco = 0.0; int a = -1, ld = 0; int64_t off = 0; bool tr = false; };
                Src src[4];
                for (const Comp* xc : xs) {
                    int a;
                    if (xc->ref.type == 0) a = O.a;
                    else {
                        a = lb.find(lb.q[O.a] - xc->ref.dq());
                        if (a < 0) continue;
                    }
                    int64_t off; int ld; bool tr;
                    if (xmap(xc, a, off, ld, tr) != O.a) continue;
                    const int s1 = xc->sk;
                    Src& S = src[s1];
                    S.a = a;
                    double xco = T.coef * xc->coef;
                    if (xc->sgn_par && (lb.q[a].n() & 1)) xco = -xco;
                    if (ti[t].piY && ((lb.q[a].n() + kSiteQ[s1].n()) & 1)) xco = -xco;
                    if (xc->ref.type == 0) S.xid += xco;
                    else { S.x = xc; S.xco = xco; S.off = off; S.ld = ld; S.tr = tr; }
                }
                uint64_t yused = 0;
                for (int s1 = 0; s1 < 4; ++s1) {
                    const Src& S = src[s1];
                    if (S.a < 0 || (!S.x && S.xid == 0.0)) continue;
                    const int a = S.a;
                    dmrgk::Group g{};
                    g.mu = lb.m[a];
                    g.c0 = (int)wl.contribs.size();
                    g.xid_coef = S.xid;
                    int xb = -1;
                    if (S.x) {
                        xb = buf_of(H, S.x->ref.set);
                        g.x_off = S.off;
                        g.ldx = S.ld;
                        g.x_coef = S.xco;
                        g.flags = xb | dmrgk::G_HAS_X | (S.tr ? dmrgk::G_TRANS_X : 0);
                    }
                    for (size_t yi = 0; yi < ys.size(); ++yi) {
                        const Comp* yc = ys[yi];
                        int b;
                        if (yc->ref.type == 0) b = O.b;
                        else {
                            b = rb.find(rb.q[O.b] - yc->ref.dq());
                            if (b < 0) continue;
                        }
                        int64_t yoff; int ldy; bool ytr;
                        if (ymap(yc, b, yoff, ldy, ytr) != O.b) continue;
                        const int s2 = yc->sk;
                        const int bi = out_block(a, s1, s2, b);
                        if (bi < 0) continue;
                        const PsiBlock& I = H->blocks[bi];
                        dmrgk::Contrib c{};
                        c.a_off = I.off;
                        c.lda = I.mb;
                        c.k = I.mb;
                        c.alpha = yc->coef;
                        c.flags = 2;
                        if (yc->ref.type == 0) {
                            c.flags |= dmrgk::F_ID_B;
                        } else {
                            const int yb = buf_of(H, yc->ref.set);
                            c.b_off = yoff;
                            c.ldb = ldy;
                            c.flags |= (yb << 3) | (ytr ? 0 : dmrgk::F_TRANS_B);
                            note(yb, yoff, (int64_t)O.mb * I.mb);
                            yused |= 1ull << yi;
                            // right-first: psi_I . Y^T once per (y, I); the U block it feeds
                            // is counted at its first consumer (left component order)
                            bool first = false;
                            for (const Comp& xq : T.X.comps) {
                                if (xq.sk != s1) continue;
                                int64_t o_; int l_; bool t_;
                                const int aa = xmap(&xq, a, o_, l_, t_);
                                if (aa < 0 || out_block(aa, xq.sb, O.s2, O.b) < 0) continue;
                                first = (aa == O.a && xq.sb == O.s1);
                                break;
                            }
                            if (first) Lc.rfy[t] += 2.0 * I.ma * I.mb * O.mb;
                        }
                        wl.contribs.push_back(c);
                        if (S.x) {
                            // left-first: X . psi_I once per (x, I), counted at the first right
                            // component (term order) that consumes T(a', s1', s2, b)
                            bool first = false;
                            for (const Comp& yq : T.Y.comps) {
                                if (yq.sk != s2) continue;
                                int64_t o_; int l_; bool t_;
                                const int bb = ymap(&yq, b, o_, l_, t_);
                                if (bb < 0 || out_block(O.a, O.s1, yq.sb, bb) < 0) continue;
                                first = (&yq == yc);
                                break;
                            }
                            if (first) Lc.lfx[t] += 2.0 * O.ma * I.ma * I.mb;
                        }
                        if (I.a == O.a && s1 == O.s1 && s2 == O.s2 && I.b == O.b) {
                            dmrgk::DiagTerm d{};
                            d.y_off = -1;
                            if (yc->ref.type != 0) {
                                d.y_off = yoff;
                                d.ldy = ldy;
                                d.ybuf = buf_of(H, yc->ref.set);
                            }
                            if (S.x) {
                                d.coef = S.xco * yc->coef;
                                d.x_off = S.off;
                                d.ldx = S.ld;
                                d.xbuf = xb;
                                Lc.dtm.push_back(d);
                            }
                            if (S.xid != 0.0) {
                                d.coef = S.xid * yc->coef;
                                d.x_off = -1;
                                Lc.dtm.push_back(d);
                            }
                        }
                    }
                    g.c1 = (int)wl.contribs.size();
                    if (g.c1 == g.c0) continue;
                    wl.groups.push_back(g);
                    if (S.x) {
                        Lc.rfx[t] += 2.0 * O.ma * lb.m[a] * O.mb;
                        note(xb, S.off, (int64_t)O.ma * lb.m[a]);
                    }
                }
                // left-first: T . Y^T once per (output, y)
                for (size_t yi = 0; yi < ys.size(); ++yi)
                    if (yused >> yi & 1) {
                        const Comp* yc = ys[yi];
                        const int b = rb.find(rb.q[O.b] - yc->ref.dq());
                        Lc.lfy[t] += 2.0 * O.ma * rb.m[b] * O.mb;
                    }
            }
            db.c1 = (int)Lc.dtm.size();
            Lc.dbl.push_back(db);
            emit_block_tasks(wl, 3, O.off, O.mb, O.ma, O.mb, g0, (int)wl.groups.size());
        }
        // a key names one block of one operator, so its size is the same wherever
        // noted; the distinct keys go to the shards the merge counts them in
        std::sort(Lc.ops.begin(), Lc.ops.end());
        Lc.opshard.assign(nshard, {});
        for (size_t j = 0; j < Lc.ops.size(); ++j)
            if (j == 0 || Lc.ops[j].first != Lc.ops[j - 1].first)
                Lc.opshard[shard_of(Lc.ops[j].first)].push_back(Lc.ops[j]);
        std::vector<std::pair<int64_t, int64_t>>().swap(Lc.ops);
    };
    std::vector<Local> loc(nth);
    {
        // interleaved chunks balance the uneven cost of output blocks
        std::vector<std::vector<std::pair<size_t, size_t>>> chunks(nth);
        const size_t cs = 8;
        size_t k = 0;
        for (size_t o = 0; o < nblk; o += cs, ++k) chunks[k % nth].push_back({o, std::min(nblk, o + cs)});
        std::vector<std::vector<Local>> parts(nth);
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nth; ++t)
            th.emplace_back([&, t]() {
                for (auto& r : chunks[t]) {
                    parts[t].emplace_back();
                    work(r.first, r.second, parts[t].back());
                }
            });
        for (auto& x : th) x.join();
        // reassemble in output-block order (chunk k went to thread k % nth)
        std::vector<Local> ordered;
        std::vector<size_t> pos(nth, 0);
        for (size_t kk = 0; kk < k; ++kk) ordered.push_back(std::move(parts[kk % nth][pos[kk % nth]++]));
        loc.swap(ordered);
    }
    clk.mark("work list: blocks");
    // Merge the chunks in output-block order: prefix offsets first, then the
    // copies (with group / contribution / diagonal-term indices shifted) run
    // on the worker threads, each on its own chunks.
    WorkList wl;
    std::vector<dmrgk::DiagBlock> dbl;
    std::vector<dmrgk::DiagTerm> dtm;
    std::vector<double> lfx(NT, 0.0), lfy(NT, 0.0), rfx(NT, 0.0), rfy(NT, 0.0);
    int64_t op_bytes = 0;
    {
        const size_t nl = loc.size();
        std::vector<size_t> go(nl + 1, 0), co(nl + 1, 0), bo(nl + 1, 0), to(nl + 1, 0);
        std::vector<size_t> ko((nl + 1) * dmrgk::kNumClass, 0);
        for (size_t i = 0; i < nl; ++i) {
            const Local& Lc = loc[i];
            go[i + 1] = go[i] + Lc.wl.groups.size();
            co[i + 1] = co[i] + Lc.wl.contribs.size();
            bo[i + 1] = bo[i] + Lc.dbl.size();
            to[i + 1] = to[i] + Lc.dtm.size();
            for (int c = 0; c < dmrgk::kNumClass; ++c)
                ko[(i + 1) * dmrgk::kNumClass + c] = ko[i * dmrgk::kNumClass + c] + Lc.wl.task[c].size();
            for (size_t t = 0; t < NT; ++t) {
                lfx[t] += Lc.lfx[t];
                lfy[t] += Lc.lfy[t];
                rfx[t] += Lc.rfx[t];
                rfy[t] += Lc.rfy[t];
            }
        }
        if (co[nl] > (size_t)INT32_MAX || go[nl] > (size_t)INT32_MAX || to[nl] > (size_t)INT32_MAX)
            return fail(DMRG_E_UNSUPPORTED, "work list beyond 2^31 groups or contributions");
        wl.groups.resize(go[nl]);
        wl.contribs.resize(co[nl]);
        dbl.resize(bo[nl]);
        dtm.resize(to[nl]);
        for (int c = 0; c < dmrgk::kNumClass; ++c) wl.task[c].resize(ko[nl * dmrgk::kNumClass + c]);
        const unsigned nw = std::max(1u, std::min<unsigned>(nth, (unsigned)nl));
        auto copy_part = [&](unsigned w) {
            for (size_t i = w; i < nl; i += nw) {
                const Local& Lc = loc[i];
                const int goff = (int)go[i], coff = (int)co[i], doff = (int)to[i];
                for (int c = 0; c < dmrgk::kNumClass; ++c) {
                    dmrgk::Task* d = wl.task[c].data() + ko[i * dmrgk::kNumClass + c];
                    for (dmrgk::Task t : Lc.wl.task[c]) {
                        t.g0 += goff;
                        t.g1 += goff;
                        *d++ = t;
                    }
                }
                dmrgk::Group* dg = wl.groups.data() + go[i];
                for (dmrgk::Group g : Lc.wl.groups) {
                    g.c0 += coff;
                    g.c1 += coff;
                    *dg++ = g;
                }
                std::copy(Lc.wl.contribs.begin(), Lc.wl.contribs.end(), wl.contribs.begin() + co[i]);
                dmrgk::DiagBlock* db = dbl.data() + bo[i];
                for (dmrgk::DiagBlock x : Lc.dbl) {
                    x.c0 += doff;
                    x.c1 += doff;
                    *db++ = x;
                }
                std::copy(Lc.dtm.begin(), Lc.dtm.end(), dtm.begin() + to[i]);
            }
        };
        // bytes of the distinct operator blocks: each shard of keys gathered
        // from every chunk, sorted and deduplicated on a thread of its own
        std::vector<int64_t> shard_bytes(nshard, 0);
        auto count_shard = [&](unsigned sh) {
            std::vector<std::pair<int64_t, int64_t>> mine;
            size_t n = 0;
            for (const Local& Lc : loc) n += Lc.opshard[sh].size();
            mine.reserve(n);
            for (const Local& Lc : loc) mine.insert(mine.end(), Lc.opshard[sh].begin(), Lc.opshard[sh].end());
            std::sort(mine.begin(), mine.end());
            int64_t sum = 0;
            for (size_t j = 0; j < mine.size(); ++j)
                if (j == 0 || mine[j].first != mine[j - 1].first) sum += mine[j].second;
            shard_bytes[sh] = sum;
        };
        auto run = [&](unsigned n, auto&& f) {
            std::vector<std::thread> th;
            for (unsigned w = 0; w < n; ++w) th.emplace_back([&, w]() { f(w); });
            for (auto& x : th) x.join();
        };
        run(nw, copy_part);
        run(nshard, count_shard);
        for (int64_t b : shard_bytes) op_bytes += b;
        run(nw, [&](unsigned w) {
            for (size_t i = w; i < nl; i += nw) loc[i] = Local();
        });
    }
    clk.mark("work list: merge");
    std::vector<double> lf(NT), rf(NT);
    for (size_t t = 0; t < NT; ++t) {
        lf[t] = lfx[t] + lfy[t];
        rf[t] = rfx[t] + rfy[t];
    }
    double F = 0.0;
    for (size_t t = 0; t < terms.size(); ++t) F += std::min(lf[t], rf[t]);
    H->flops = (int64_t)F;
    H->op_bytes64 = op_bytes * 8;
    H->ntask = wl.ntasks();
    H->ngroup = wl.groups.size();
    H->ncontrib = wl.contribs.size();
    {
        int64_t sz[dmrgk::kMaxBuf] = {0};
        sz[0] = Lb.elems;
        sz[1] = Rb.elems;
        sz[2] = sz[3] = H->dim;
        sz[4] = H->TL.elems;
        sz[5] = H->TR.elems;
        sz[6] = H->TML.elems;
        sz[7] = H->TMR.elems;
        for (int i = 0; i < dmrgk::kMaxBuf; ++i) H->buf_elems[i] = sz[i];
        lookup_tuning(H);
        if ((H->flags & DMRG_HEFF_AUTOTUNE) && H->tuned == 0) {
            // the candidates differ only in their tasks: tiles above kTallRows are
            // split here, once, and the tuner shares the groups and contributions
            wl.tall_min = H->tune.tall_min;
            reclassify(wl);
            split_large(wl);
            H->base.reset(new WorkList(std::move(wl)));
            wl = WorkList();
        } else {
            dmrg_status vs = finalize_list(H, wl, H->tune);
            if (vs != DMRG_OK) return vs;
        }
        for (const auto& d : dtm) {
            if (d.x_off >= 0 && (d.xbuf < 0 || d.xbuf >= 8 || d.x_off >= sz[d.xbuf])) return fail(DMRG_E_STATE, "diag X");
            if (d.y_off >= 0 && (d.ybuf < 0 || d.ybuf >= 8 || d.y_off >= sz[d.ybuf])) return fail(DMRG_E_STATE, "diag Y");
        }
    }
    clk.mark("validate");
    if (clk.on) {
        // work per task (flops of its groups) -> load-balance picture
        for (int c = 0; c < dmrgk::kNumClass; ++c) {
            double tot = 0, mx = 0;
            std::vector<double> w;
            for (const dmrgk::Task& t : wl.task[c]) {
                const double f = task_cost(wl, t);
                tot += f;
                mx = std::max(mx, f);
                w.push_back(f);
            }
            std::sort(w.begin(), w.end());
            if (!w.empty())
                std::fprintf(stderr, "[dmrg] class %d: tasks %zu work %.3f TF max %.3f GF median %.3f GF p99 %.3f GF\n", c,
                             w.size(), tot / 1e12, mx / 1e9, w[w.size() / 2] / 1e9, w[w.size() * 99 / 100] / 1e9);
            // operand layouts of the class's products (flops): A.B with A row-major and B
            // transposed, other A.B layouts, X.U with X row-major, X transposed; identities
            double f_ab = 0, f_ab_other = 0, f_x = 0, f_xt = 0;
            size_t n_id = 0;
            for (const dmrgk::Task& t : wl.task[c]) {
                const int cols = std::min(t.ncol, t.n - t.col0);
                for (int g = t.g0; g < t.g1; ++g) {
                    const dmrgk::Group& G = wl.groups[g];
                    if (G.flags & dmrgk::G_HAS_X)
                        ((G.flags & dmrgk::G_TRANS_X) ? f_xt : f_x) += 2.0 * t.m * G.mu * cols;
                    for (int q = G.c0; q < G.c1; ++q) {
                        const dmrgk::Contrib& k = wl.contribs[q];
                        if (k.flags & (dmrgk::F_ID_A | dmrgk::F_ID_B)) { ++n_id; continue; }
                        const bool fast = !(k.flags & dmrgk::F_TRANS_A) && (k.flags & dmrgk::F_TRANS_B);
                        (fast ? f_ab : f_ab_other) += 2.0 * G.mu * k.k * cols;
                    }
                }
            }
            if (!w.empty())
                std::fprintf(stderr, "[dmrg]   layouts: A.B row/trans %.3f TF, other %.3f TF; X.U row %.3f TF, "
                             "trans %.3f TF; identity contributions %zu\n", f_ab / 1e12, f_ab_other / 1e12,
                             f_x / 1e12, f_xt / 1e12, n_id);
        }
    }
    if (clk.on)
        std::fprintf(stderr, "[dmrg] tasks %zu groups %zu contribs %zu reductions %zu partial %.1f MB diag terms %zu\n",
                     wl.ntasks(), wl.groups.size(), wl.contribs.size(), wl.reduces.size(),
                     wl.partial_elems * 8.0 * H->n_roots / 1e6, dtm.size());
    if (!H->base) {   // an autotuned list is uploaded by the tuner
        H->part_elems = wl.partial_elems;
        if (H->part_elems > 0) {
            H->part_region = C->arena.alloc(H->part_elems * 8 * H->n_roots);
            if (H->part_region < 0) return fail(DMRG_E_WORKSPACE, "arena too small for partial tiles");
            H->part = C->arena.base + H->part_region;
        }
        dmrg_status st = upload_work(C, wl, H->work, stream);
        if (st != DMRG_OK) return st;
    }
    clk.mark("upload");
    // diagonal lists
    {
        const int64_t bytes = ((int64_t)dbl.size() * sizeof(dmrgk::DiagBlock) + 255) / 256 * 256 +
                              (int64_t)std::max<size_t>(dtm.size(), 1) * sizeof(dmrgk::DiagTerm);
        H->diag_region = C->arena.alloc(bytes);
        if (H->diag_region < 0) return fail(DMRG_E_WORKSPACE, "arena too small for diagonal lists");
        char* base = C->arena.base + H->diag_region;
        H->dblocks = (dmrgk::DiagBlock*)base;
        H->dterms = (dmrgk::DiagTerm*)(base + ((int64_t)dbl.size() * sizeof(dmrgk::DiagBlock) + 255) / 256 * 256);
        H->n_dblocks = (int)dbl.size();
        if (!C->dry) {
            DMRG_HIP(hipMemcpy(H->dblocks, dbl.data(), dbl.size() * sizeof(dmrgk::DiagBlock), hipMemcpyHostToDevice));
            if (!dtm.empty())
                DMRG_HIP(hipMemcpy(H->dterms, dtm.data(), dtm.size() * sizeof(dmrgk::DiagTerm), hipMemcpyHostToDevice));
        }
    }
    clk.mark("diagonal lists");
    return DMRG_OK;
}

static dmrgk::Bases<double> bases64(const dmrg_heff* H) {
    dmrgk::Bases<double> b{};
    b.p[dmrgk::kPartialBuf] = (double*)H->part;
    b.vstride[dmrgk::kPartialBuf] = H->part_elems;
    b.p[0] = H->Lb->dev;
    b.p[1] = H->Rb->dev;
    b.p[4] = H->TL.dev;
    b.p[5] = H->TR.dev;
    b.p[6] = H->TML.dev;
    b.p[7] = H->TMR.dev;
    for (int i = 0; i < dmrgk::kMaxBuf; ++i)
        if (!b.p[i]) b.p[i] = H->Lb->dev;
    return b;
}

static dmrg_status ensure_f32(dmrg_heff* H, void* stream) {
    if (H->f32_region >= 0) return DMRG_OK;
    const OpSetImpl* sets[8] = {H->Lb, H->Rb, nullptr, nullptr, &H->TL, &H->TR, &H->TML, &H->TMR};
    int64_t off[8] = {0};
    int64_t total = 0;
    for (int i = 0; i < 8; ++i) {
        if (!sets[i] || !sets[i]->dev) continue;
        off[i] = total;
        total += (sets[i]->elems * 4 + 255) / 256 * 256;
    }
    H->f32_region = H->ctx->arena.alloc(std::max<int64_t>(total, 256));
    if (H->f32_region < 0) return fail(DMRG_E_WORKSPACE, "arena too small for FP32 operator copies");
    char* base = H->ctx->arena.base + H->f32_region;
    for (int i = 0; i < 8; ++i) {
        if (!sets[i] || !sets[i]->dev) continue;
        H->f32[i] = (float*)(base + off[i]);
        if (!H->ctx->dry) DMRG_HIP(dmrgk::launch_cast_d2f(sets[i]->dev, H->f32[i], sets[i]->elems, stream));
    }
    return DMRG_OK;
}

static dmrgk::Bases<float> bases32(const dmrg_heff* H) {
    dmrgk::Bases<float> b{};
    for (int i = 0; i < 8; ++i) b.p[i] = H->f32[i] ? H->f32[i] : H->f32[0];
    b.p[dmrgk::kPartialBuf] = H->part ? (float*)H->part : H->f32[0];
    b.vstride[dmrgk::kPartialBuf] = H->part_elems;
    return b;
}

// ---------------------------------------------------------------------------
// graph replay of a product: the class launches and the reduction as kernel
// nodes in launch order; each call rewrites the nodes' arguments (the vector
// pointers) and launches the instantiated graph on the caller's stream
template <typename T>
static hipKernelNodeParams node_params(const dmrgk::KernelDesc& kd, void** args) {
    hipKernelNodeParams p{};
    p.func = const_cast<void*>(kd.func);
    p.gridDim = dim3(kd.gx, kd.gy);
    p.blockDim = dim3(kd.bx);
    p.sharedMemBytes = 0;
    p.kernelParams = args;
    p.extra = nullptr;
    return p;
}

template <typename T>
static dmrg_status run_graph(dmrg_heff* H, int prec, const dmrgk::Bases<T>& b, int nvec, void* stream) {
    const DevWork& d = H->work;
    constexpr bool f64 = sizeof(T) == 8;
    ProductGraph* pg = nullptr;
    for (ProductGraph& g : H->graphs)
        if (g.prec == prec && g.nvec == nvec) pg = &g;
    auto chain = [&](int c) {
        return f64 ? dmrgk::chain_desc_f64(c, d.lds_records, d.ntask[c], nvec)
                   : dmrgk::chain_desc_f32(c, d.lds_records, d.ntask[c], nvec);
    };
    auto reduce = [&]() { return f64 ? dmrgk::reduce_desc_f64(d.nred, nvec) : dmrgk::reduce_desc_f32(d.nred, nvec); };
    if (!pg) {
        H->graphs.emplace_back();
        pg = &H->graphs.back();
        pg->prec = prec;
        pg->nvec = nvec;
        DMRG_HIP(hipGraphCreate(&pg->graph, 0));
        hipGraphNode_t prev = nullptr;
        for (int c = dmrgk::kNumClass - 1; c >= 0; --c) {
            if (d.ntask[c] == 0) continue;
            const dmrgk::KernelDesc kd = chain(c);
            dmrgk::ChainArgs<T> a(b, d.task[c], d.ntask[c], d.groups, d.contribs, nvec);
            const hipKernelNodeParams p = node_params<T>(kd, a.ptrs);
            hipGraphNode_t n;
            DMRG_HIP(hipGraphAddKernelNode(&n, pg->graph, prev ? &prev : nullptr, prev ? 1 : 0, &p));
            pg->nodes.push_back(n);
            pg->cls.push_back(c);
            prev = n;
        }
        if (d.nred > 0) {
            dmrgk::ReduceArgs<T> a(d.reduces, b);
            const hipKernelNodeParams p = node_params<T>(reduce(), a.ptrs);
            hipGraphNode_t n;
            DMRG_HIP(hipGraphAddKernelNode(&n, pg->graph, prev ? &prev : nullptr, prev ? 1 : 0, &p));
            pg->nodes.push_back(n);
            pg->cls.push_back(dmrgk::kNumClass);
        }
        if (pg->nodes.empty()) return DMRG_OK;
        DMRG_HIP(hipGraphInstantiate(&pg->exec, pg->graph, nullptr, nullptr, 0));
    } else {
        for (size_t i = 0; i < pg->nodes.size(); ++i) {
            const int c = pg->cls[i];
            if (c < dmrgk::kNumClass) {
                dmrgk::ChainArgs<T> a(b, d.task[c], d.ntask[c], d.groups, d.contribs, nvec);
                const hipKernelNodeParams p = node_params<T>(chain(c), a.ptrs);
                DMRG_HIP(hipGraphExecKernelNodeSetParams(pg->exec, pg->nodes[i], &p));
            } else {
                dmrgk::ReduceArgs<T> a(d.reduces, b);
                const hipKernelNodeParams p = node_params<T>(reduce(), a.ptrs);
                DMRG_HIP(hipGraphExecKernelNodeSetParams(pg->exec, pg->nodes[i], &p));
            }
        }
    }
    if (!pg->exec) return DMRG_OK;
    DMRG_HIP(hipGraphLaunch(pg->exec, (hipStream_t)stream));
    ++H->graph_launches;
    return DMRG_OK;
}

static void drop_graphs(dmrg_heff* H) {
    for (ProductGraph& g : H->graphs) {
        if (g.exec) hipGraphExecDestroy(g.exec);
        if (g.graph) hipGraphDestroy(g.graph);
    }
    H->graphs.clear();
}

// ---------------------------------------------------------------------------
// autotuner: every candidate work list (balance target x tall threshold) is
// built, uploaded and timed on one FP32 product of zero vectors (the
// kernels' work does not depend on the values); the fastest is kept and
// cached under the H_eff's shape key
static dmrg_status autotune(dmrg_heff* H, void* stream) {
    Ctx* C = H->ctx;
    hipStream_t s = (hipStream_t)stream;
    // Two stages: the chunk count first (tall kernel from 97 rows), then, with
    // the fastest count, the tall kernel from 81 rows if tiles of 81..96 rows
    // exist.  Lower heights (65, 49) were slower on every workload measured:
    // the slice kernels serve those tiles better.
    bool mid = false;
    for (const auto& T : H->base->task)
        for (const dmrgk::Task& t : T) {
            int rows = t.m;
            for (int g = t.g0; g < t.g1; ++g) rows = std::max(rows, H->base->groups[g].mu);
            if (rows > dmrgk::kShortRows && rows <= dmrgk::kMaxRows) mid = true;
        }
    H->cand.clear();
    H->cand_ms.clear();
    WorkList& base = *H->base;
    // every candidate's tasks index the same groups and contributions: one copy
    // on the device, held by H from here on (released with it on any failure)
    dmrg_status st = upload_records(C, base, H->recs, stream);
    if (st != DMRG_OK) return st;
    // candidates are timed on the vector batch the products run on: n_roots
    // vectors at once (the partial tiles are sized for that many)
    const int nr = H->n_roots;
    const int64_t vreg = C->arena.alloc(H->dim * 4 * 2 * nr);
    if (vreg < 0) return fail(DMRG_E_WORKSPACE, "arena too small for the autotuner's vectors");
    float* x = (float*)(C->arena.base + vreg);
    float* y = x + H->dim * nr;
    if (!C->dry) DMRG_HIP(hipMemsetAsync(x, 0, H->dim * 4 * 2 * nr, s));
    hipEvent_t e0, e1;
    DMRG_HIP(hipEventCreate(&e0));
    DMRG_HIP(hipEventCreate(&e1));
    size_t best = 0;
    int64_t biggest = 0;
    TuneParams biggest_tp{};
    // a candidate's list: the base's tasks, with its groups and contributions
    // lent (moved, not copied) for the time of the call
    auto with_list = [&](const TuneParams& tp, auto&& use) {
        WorkList w;
        for (int c = 0; c < dmrgk::kNumClass; ++c) w.task[c] = base.task[c];
        w.groups.swap(base.groups);
        w.contribs.swap(base.contribs);
        dmrg_status r = finalize_list(H, w, tp);
        if (r == DMRG_OK) r = use(w);
        base.groups.swap(w.groups);
        base.contribs.swap(w.contribs);
        return r;
    };
    float margin = 1.f;   // a candidate is kept if faster than margin x the best so far
    // uploads and (unless dry) times one FP32 product (n_roots vectors) of a candidate
    auto trial = [&](const TuneParams& tp) {
        if (st != DMRG_OK) return;
        float best_ms = 0.f;
        bool skipped = false;
        st = with_list(tp, [&](const WorkList& w) -> dmrg_status {
            DevWork dw;
            int64_t preg = -1;
            dmrg_status r = upload_tasks(C, w, H->recs, dw, stream, false);
            // the partial tiles at the size the chosen list takes (8-byte
            // elements, n_roots vectors): a candidate that does not fit is
            // skipped, unless none has fitted yet
            if (r == DMRG_OK && w.partial_elems > 0) {
                preg = C->arena.alloc(w.partial_elems * 8 * H->n_roots);
                if (preg < 0) {
                    free_work(C, dw);
                    if (H->cand.empty()) return fail(DMRG_E_WORKSPACE, "arena too small for the autotuner's partial tiles");
                    skipped = true;
                    return DMRG_OK;
                }
            }
            const int64_t need = task_bytes(w) + w.partial_elems * 8 * H->n_roots;
            if (need > biggest) {
                biggest = need;
                biggest_tp = tp;
            }
            if (r == DMRG_OK && !C->dry) {
                dmrgk::Bases<float> b = bases32(H);
                b.p[dmrgk::kPartialBuf] = preg >= 0 ? (float*)(C->arena.base + preg) : H->f32[0];
                b.vstride[dmrgk::kPartialBuf] = w.partial_elems;
                b.p[2] = x;
                b.p[3] = y;
                b.vstride[2] = b.vstride[3] = H->dim;
                // a warm-up, then the best of two timed runs (one when the
                // warm-up took over 100 ms)
                best_ms = 1e30f;
                int runs = 2;
                for (int k = -1; k < runs && r == DMRG_OK; ++k) {
                    hipEventRecord(e0, s);
                    r = run_work_f32(dw, b, nr, stream);
                    hipEventRecord(e1, s);
                    if (r == DMRG_OK && hipEventSynchronize(e1) != hipSuccess) r = fail(DMRG_E_HIP, "autotune timing");
                    float ms = 0.f;
                    hipEventElapsedTime(&ms, e0, e1);
                    if (k < 0) {
                        if (ms > 100.f) runs = 1;
                    } else {
                        best_ms = std::min(best_ms, ms);
                    }
                }
            }
            free_work(C, dw);
            if (preg >= 0) C->arena.release(preg);
            return r;
        });
        if (st != DMRG_OK || skipped) return;
        H->cand.push_back(tp);
        H->cand_ms.push_back(best_ms);
        if (best_ms < H->cand_ms[best] * margin) best = H->cand.size() - 1;
    };
    const int kBalances[] = {65536, 131072, 262144, 524288};
    for (int bal : kBalances) trial(TuneParams{bal, dmrgk::kMaxRows + 1});
    // the lower threshold must win by more than 0.5 % (a tie keeps the first
    // stage's list, so the choice does not flip on timing noise)
    margin = 0.995f;
    if (mid) {
        if (C->dry) {
            // the choice is made on the device: size the rebuild for the largest
            // of every candidate the second stage could time
            for (int bal : kBalances) trial(TuneParams{bal, dmrgk::kShortRows + 1});
        } else if (st == DMRG_OK) {
            trial(TuneParams{H->cand[best].balance, dmrgk::kShortRows + 1});
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    C->arena.release(vreg);
    if (st != DMRG_OK) return st;
    H->tune = C->dry ? biggest_tp : H->cand[best];
    H->tuned = 1;
    // the chosen list: the base's records themselves (no copy), then the base goes
    WorkList w;
    for (int c = 0; c < dmrgk::kNumClass; ++c) w.task[c].swap(base.task[c]);
    w.groups.swap(base.groups);
    w.contribs.swap(base.contribs);
    H->base.reset();
    st = finalize_list(H, w, H->tune);
    if (st != DMRG_OK) return st;
    H->part_elems = w.partial_elems;
    if (H->part_elems > 0) {
        H->part_region = C->arena.alloc(H->part_elems * 8 * H->n_roots);
        if (H->part_region < 0) return fail(DMRG_E_WORKSPACE, "arena too small for partial tiles");
        H->part = C->arena.base + H->part_region;
    }
    st = upload_tasks(C, w, H->recs, H->work, stream);
    if (st == DMRG_OK && !C->dry) store_tuning(H);
    return st;
}

Ctx* heff_ctx(const dmrg_heff* H) { return H->ctx; }

void dmrg::heff_psi_subblocks(const dmrg_heff* H, const OpSetImpl*& Lb, const OpSetImpl*& Rb, std::vector<PsiSub>& out) {
    Lb = H->Lb;
    Rb = H->Rb;
    out.clear();
    for (const PsiBlock& B : H->blocks) out.push_back(PsiSub{B.a, B.s1, B.s2, B.b, B.ma, B.mb, B.off});
}

extern "C" {

static dmrg_status check_heff_args(const dmrg_ctx* ctx, const dmrg_opset* left, const dmrg_opset* right,
                                   int32_t n_roots, int32_t precision) {
    if (!ctx->has_ints) return fail(DMRG_E_STATE, "integrals not set");
    const int K = ctx->K, KL = left->nsites;
    if (left->side != DMRG_LEFT || left->kind != 0 || KL < 1)
        return fail(DMRG_E_ARG, "left must be a normal left block of at least one site");
    if (right->side != DMRG_RIGHT || right->kind != 1 || right->nsites < 1 || right->nsites != K - KL - 2)
        return fail(DMRG_E_ARG, "right must be a complementary right block of the K - 2 - KL sites after the dots");
    if (n_roots < 1 || n_roots > 32) return fail(DMRG_E_ARG, "n_roots must be 1..32");
    if (precision != DMRG_PREC_F64 && precision != DMRG_PREC_F32) return fail(DMRG_E_ARG, "bad precision");
    return DMRG_OK;
}

dmrg_status dmrg_heff_create(dmrg_ctx* ctx, const dmrg_opset* left, const dmrg_opset* right,
                             const dmrg_psi_layout* layout, int32_t n_roots, int32_t precision, int32_t flags,
                             dmrg_heff** out, void* stream) {
    if (!ctx || !left || !right || !out) return fail(DMRG_E_ARG, "null argument");
    *out = nullptr;
    dmrg_status st = check_heff_args(ctx, left, right, n_roots, precision);
    if (st != DMRG_OK) return st;
    if (flags & ~(DMRG_HEFF_GRAPH | DMRG_HEFF_AUTOTUNE)) return fail(DMRG_E_ARG, "unknown flags");
    if ((flags & DMRG_HEFF_AUTOTUNE) && precision != DMRG_PREC_F32)
        return fail(DMRG_E_ARG, "the autotuner times FP32 products: create with DMRG_PREC_F32");
    dmrg_heff* H = new dmrg_heff();
    H->ctx = ctx;
    H->Lb = left;
    H->Rb = right;
    H->n_roots = n_roots;
    H->precision = precision;
    H->layout = layout;
    H->flags = flags;
    st = build_heff(H, stream);
    H->layout = nullptr;
    PhaseClock clk;
    if (st == DMRG_OK && precision == DMRG_PREC_F32) st = ensure_f32(H, stream);
    clk.mark("FP32 copies");
    if (st == DMRG_OK && H->base && H->tuned == 0) st = autotune(H, stream);
    clk.mark("autotune");
    H->base.reset();
    if (st == DMRG_OK && !ctx->dry) {
        const int e = (int)hipStreamSynchronize((hipStream_t)stream);
        if (e) st = hip_fail(e, "heff create");
    }
    clk.mark("create: synchronize");
    if (st != DMRG_OK) {
        dmrg_heff_free(H);
        return st;
    }
    *out = H;
    return DMRG_OK;
}

int64_t dmrg_heff_dim(const dmrg_heff* H) { return H ? H->dim : -1; }

int32_t dmrg_heff_psi_layout(const dmrg_heff* H, int32_t n, int32_t* qn_left, int32_t* site1, int32_t* site2,
                             int32_t* qn_right, int64_t* rows, int64_t* cols, int64_t* offset) {
    if (!H) return fail(DMRG_E_ARG, "null argument");
    const Basis& lb = H->Lb->basis;
    const Basis& rb = H->Rb->basis;
    const int nb = (int)H->blocks.size();
    for (int i = 0; i < nb && i < n; ++i) {
        const PsiBlock& B = H->blocks[i];
        if (qn_left) { qn_left[2 * i] = lb.q[B.a].a; qn_left[2 * i + 1] = lb.q[B.a].b; }
        if (qn_right) { qn_right[2 * i] = rb.q[B.b].a; qn_right[2 * i + 1] = rb.q[B.b].b; }
        if (site1) site1[i] = B.s1;
        if (site2) site2[i] = B.s2;
        if (rows) rows[i] = B.ma;
        if (cols) cols[i] = B.mb;
        if (offset) offset[i] = B.off;
    }
    return nb;
}


int64_t dmrg_heff_flops(const dmrg_heff* H) { return H ? H->flops : -1; }
int64_t dmrg_heff_bytes(const dmrg_heff* H, int32_t precision) {
    if (!H) return -1;
    const int64_t es = precision == DMRG_PREC_F32 ? 4 : 8;
    return H->op_bytes64 / 8 * es + 2 * H->dim * es;
}
int32_t dmrg_heff_terms(const dmrg_heff* H, int32_t* n2, int32_t* n1, int32_t* nh) {
    if (!H) return -1;
    if (n2) *n2 = H->n2;
    if (n1) *n1 = H->n1;
    if (nh) *nh = H->nh;
    return H->n2 + H->n1 + H->nh;
}

}  // extern "C"

// H_eff psi with the partial tiles of split tasks in `partial` (bytes of
// room: partial_bytes), or in H's own buffer when partial is NULL.  Vectors
// go in batches of as many as the partial buffer holds (n_roots for H's own).
dmrg_status heff_apply_impl(dmrg_heff* H, int32_t precision, int32_t n_vec, const void* psi, void* sigma,
                            void* partial, int64_t partial_bytes, void* stream) {
    // the static-scratch variant never instantiates a graph (that may allocate)
    const bool graph = (H ? (H->flags & DMRG_HEFF_GRAPH) : 0) && !partial;
    if (!H || !psi || !sigma) return fail(DMRG_E_ARG, "null argument");
    if (n_vec < 1 || n_vec > 65535) return fail(DMRG_E_ARG, "bad n_vec");
    if (psi == sigma) return fail(DMRG_E_ARG, "psi and sigma must not alias");
    if (precision != DMRG_PREC_F64 && precision != DMRG_PREC_F32) return fail(DMRG_E_ARG, "bad precision");
    const int64_t es = precision == DMRG_PREC_F64 ? 8 : 4;
    int batch = H->part_elems > 0 ? H->n_roots : n_vec;
    if (partial && H->part_elems > 0) {
        const int64_t per_vec = H->part_elems * es;
        if (per_vec > partial_bytes)
            return fail(DMRG_E_WORKSPACE, "the split tiles of one product need " + std::to_string(per_vec) +
                                              " bytes of scratch; the static scratch holds " +
                                              std::to_string(partial_bytes));
        batch = (int)std::min<int64_t>(n_vec, partial_bytes / per_vec);
    }
    void* part = partial ? partial : H->part;
    for (int v0 = 0; v0 < n_vec; v0 += batch) {
        const int nv = std::min(batch, n_vec - v0);
        dmrg_status st;
        if (precision == DMRG_PREC_F64) {
            dmrgk::Bases<double> b = bases64(H);
            if (part) b.p[dmrgk::kPartialBuf] = (double*)part;
            b.p[2] = (double*)psi + (int64_t)v0 * H->dim;
            b.p[3] = (double*)sigma + (int64_t)v0 * H->dim;
            b.vstride[2] = b.vstride[3] = H->dim;
            st = graph ? run_graph<double>(H, precision, b, nv, stream) : run_work_f64(H->work, b, nv, stream);
        } else {
            if (H->f32_region < 0) return fail(DMRG_E_STATE, "H_eff was created for FP64 products only");
            dmrgk::Bases<float> b = bases32(H);
            if (part) b.p[dmrgk::kPartialBuf] = (float*)part;
            b.p[2] = (float*)psi + (int64_t)v0 * H->dim;
            b.p[3] = (float*)sigma + (int64_t)v0 * H->dim;
            b.vstride[2] = b.vstride[3] = H->dim;
            st = graph ? run_graph<float>(H, precision, b, nv, stream) : run_work_f32(H->work, b, nv, stream);
        }
        if (st != DMRG_OK) return st;
    }
    return DMRG_OK;
}

extern "C" {

dmrg_status dmrg_heff_apply(dmrg_heff* H, int32_t precision, int32_t n_vec, const void* psi, void* sigma,
                            void* stream) {
    return heff_apply_impl(H, precision, n_vec, psi, sigma, nullptr, 0, stream);
}

int32_t dmrg_heff_profile(dmrg_heff* H, int32_t precision, const void* psi, void* sigma, int32_t n, float* ms,
                          double* flops, int32_t* kind, void* stream) {
    if (!H || !psi || !sigma || !ms || !flops || !kind) return fail(DMRG_E_ARG, "null argument");
    if (psi == sigma) return fail(DMRG_E_ARG, "psi and sigma must not alias");
    if (n < dmrgk::kNumClass + 1) return fail(DMRG_E_ARG, "n below DMRG_HEFF_LAUNCHES");
    float t[dmrgk::kNumClass + 1] = {0};
    dmrg_status st;
    if (precision == DMRG_PREC_F64) {
        dmrgk::Bases<double> b = bases64(H);
        b.p[2] = (double*)psi;
        b.p[3] = (double*)sigma;
        b.vstride[2] = b.vstride[3] = H->dim;
        st = run_work_timed_f64(H->work, b, t, stream);
    } else if (precision == DMRG_PREC_F32) {
        if (H->f32_region < 0) return fail(DMRG_E_STATE, "H_eff was created for FP64 products only");
        dmrgk::Bases<float> b = bases32(H);
        b.p[2] = (float*)psi;
        b.p[3] = (float*)sigma;
        b.vstride[2] = b.vstride[3] = H->dim;
        st = run_work_timed_f32(H->work, b, t, stream);
    } else {
        return fail(DMRG_E_ARG, "bad precision");
    }
    if (st != DMRG_OK) return st;
    for (int i = 0; i <= dmrgk::kNumClass; ++i) {
        ms[i] = t[i];
        flops[i] = i < dmrgk::kNumClass ? H->work.useful[i] : 0.0;
        kind[i] = i | (H->work.lds_records && i < dmrgk::kNumClass ? 256 : 0);
    }
    return dmrgk::kNumClass + 1;
}

dmrg_status dmrg_heff_diag(dmrg_heff* H, double* diag, void* stream) {
    if (!H || !diag) return fail(DMRG_E_ARG, "null argument");
    DMRG_HIP(dmrgk::launch_diag(H->dblocks, H->n_dblocks, H->dterms, bases64(H), diag, stream));
    return DMRG_OK;
}

dmrg_status dmrg_heff_renormalize(dmrg_heff* H, const dmrg_bsm* isometry, dmrg_opset** out, void* stream) {
    if (!H || !isometry || !out) return fail(DMRG_E_ARG, "null argument");
    *out = nullptr;
    dmrg_opset* o = new dmrg_opset();
    o->side = DMRG_LEFT;
    o->kind = 0;
    dmrg_status st = renormalize_grown(H->ctx, *H->Lb, &H->TL, isometry, H->GL, *o, stream);
    if (st != DMRG_OK) {
        if (o->region >= 0) free_set(H->ctx, *o);
        delete o;
        return st;
    }
    o->orbs = H->Lb->orbs;
    const int d1 = H->Lb->nsites;
    o->orbs.push_back(2 * d1);
    o->orbs.push_back(2 * d1 + 1);
    o->nsites = H->Lb->nsites + 1;
    o->ctx = H->ctx;
    *out = o;
    return DMRG_OK;
}

dmrg_status dmrg_heff_get_info(const dmrg_heff* H, dmrg_heff_info* info) {
    if (!H || !info) return fail(DMRG_E_ARG, "null argument");
    dmrg_heff_info x{};
    x.flags = H->flags;
    x.balance_target = H->tune.balance;
    x.tall_min_rows = H->tune.tall_min;
    x.tuned = H->tuned;
    x.n_candidates = (int32_t)std::min<size_t>(H->cand.size(), 8);
    for (int i = 0; i < x.n_candidates; ++i) {
        x.candidate_ms[i] = i < (int)H->cand_ms.size() ? H->cand_ms[i] : 0.f;
        x.candidate_balance[i] = H->cand[i].balance;
        x.candidate_tall_min[i] = H->cand[i].tall_min;
    }
    x.graphs = (int32_t)H->graphs.size();
    x.graph_launches = H->graph_launches;
    int64_t nt = 0;
    for (int c = 0; c < dmrgk::kNumClass; ++c) nt += H->work.ntask[c];
    x.tasks = nt;
    x.reductions = H->work.nred;
    x.partial_elems = H->part_elems;
    *info = x;
    return DMRG_OK;
}

void dmrg_heff_free(dmrg_heff* H) {
    if (!H) return;
    Ctx* C = H->ctx;
    drop_graphs(H);
    free_work(C, H->work);
    free_work(C, H->recs);
    free_set(C, H->TL);
    free_set(C, H->TR);
    free_set(C, H->TML);
    free_set(C, H->TMR);
    if (H->diag_region >= 0) C->arena.release(H->diag_region);
    if (H->f32_region >= 0) C->arena.release(H->f32_region);
    if (H->part_region >= 0) C->arena.release(H->part_region);
    delete H;
}

}  // extern "C"
