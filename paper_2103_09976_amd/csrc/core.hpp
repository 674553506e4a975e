// Host-side data model of the DMRG library.
//
// Blocks and their renormalized operators (Appendix A of the paper):
//  * Basis: sectors (n_alpha, n_beta), sorted, with their dimensions;
//  * Skel: the block layout of every operator of one shift dq on a basis
//    (blocks ket q -> bra q+dq, row-major, contiguous);
//  * Family: operators of one kind and one shift, stored back to back
//    (stride = skeleton size) so an integral-weighted sum over a family is a
//    dense GEMM over the operator index;
//  * OpSet: a block = basis + families, one contiguous arena region.
//
// Operators on a block grown by one site are kept delayed ("transition
// form", the delayed contraction of the blocking step): a list of
// components (site bra state, site ket state, reference to an old-block
// operator or the identity, coefficient, parity flag), never materialised on
// the enlarged basis.  Renormalization and H_eff consume this form directly.
#pragma once
#include <array>
#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/dmrg.h"
#include "kernels.hpp"

namespace dmrg {

struct QN {
    int a = 0, b = 0;
    QN() = default;
    QN(int x, int y) : a(x), b(y) {}
    QN operator+(const QN& o) const { return {a + o.a, b + o.b}; }
    QN operator-(const QN& o) const { return {a - o.a, b - o.b}; }
    QN operator-() const { return {-a, -b}; }
    bool operator==(const QN& o) const { return a == o.a && b == o.b; }
    bool operator!=(const QN& o) const { return !(*this == o); }
    bool operator<(const QN& o) const { return a < o.a || (a == o.a && b < o.b); }
    int n() const { return a + b; }
};

// one-electron quantum number of spin-orbital p
inline QN qe(int p) { return (p & 1) ? QN(0, 1) : QN(1, 0); }
extern const QN kSiteQ[4];    // |0>, |a>, |b>, |ab>

struct Basis {
    std::vector<QN> q;
    std::vector<int> m;
    int64_t total = 0;
    // O(1) sector lookup table over (n_alpha, n_beta), built by index()
    std::vector<int> tab;
    int amax = -1, bmax = -1;
    int find(const QN& x) const {
        if (!tab.empty()) {
            if (x.a < 0 || x.b < 0 || x.a > amax || x.b > bmax) return -1;
            return tab[(size_t)x.a * (bmax + 1) + x.b];
        }
        return find_slow(x);
    }
    int find_slow(const QN& x) const;
    void index();
    int size() const { return (int)q.size(); }
};

struct Skel {
    QN dq;
    std::vector<int> ket, bra;     // per block
    std::vector<int64_t> off;      // element offset of block within one operator
    std::vector<int> blk_of_ket;   // ket sector -> block index or -1
    int64_t size = 0;
};

struct Family {
    char kind;          // 'H','C','A','B','R','D'(P^+),'Q','T'(temporary)
    QN dq;
    int par = 0;
    int skel = 0;
    std::vector<int64_t> keys;
    std::unordered_map<int64_t, int> index;
    int64_t base = 0;   // element offset (within the set's region) of operator 0
    int64_t stride = 0;
};

inline int64_t okey(char kind, int p, int q) {
    return ((int64_t)(unsigned char)kind << 40) | ((int64_t)(p + 1) << 20) | (int64_t)(q + 1);
}

// element offsets are in units of double within the set region
struct OpSetImpl {
    Basis basis;
    std::vector<Skel> skels;
    std::vector<Family> fams;
    std::unordered_map<int64_t, std::pair<int, int>> lookup;   // key -> (fam, idx)
    std::vector<int> orbs;     // spin-orbitals of the block (increasing)
    int side = 0;              // DMRG_LEFT / DMRG_RIGHT
    int kind = 0;              // 0 normal, 1 complementary, 2 temporaries
    int nsites = 0;
    int64_t region = -1;       // arena byte offset
    int64_t elems = 0;         // doubles in the region
    double* dev = nullptr;     // device pointer of the region

    int skel_for(const QN& dq);
    int family(char kind, const QN& dq, int par);
    int add_op(char kind, int p, int q, const QN& dq, int par);
    void layout();             // assign bases/strides, elems
    bool has(char kind, int p, int q) const { return lookup.count(okey(kind, p, q)) != 0; }
};

// device arena (caller-owned memory), first-fit allocator
struct Arena {
    char* base = nullptr;
    int64_t bytes = 0;
    std::map<int64_t, int64_t> free_;   // offset -> size
    std::map<int64_t, int64_t> live_;
    int64_t used = 0, peak = 0;
    int64_t high = 0;                   // highest end offset ever allocated
    void init(void* p, int64_t n);
    int64_t alloc(int64_t n);           // -1 on failure
    void release(int64_t off);
};

struct Ctx;

// reference to a block operator used as a component
struct Ref {
    int type = 0;                  // 0 identity, 1 operator
    const OpSetImpl* set = nullptr;
    int fam = -1, idx = -1;
    bool trans = false;
    QN dq() const;                 // shift of the referenced (possibly transposed) operator
    int par() const;
    // block with ket sector k: returns false if absent.  bra sector, offset
    // (elements within the set region), leading dimension, transposed flag.
    bool block(int k, int& bra, int64_t& off, int& ld, bool& tr) const;
};

struct Comp {
    int sb, sk;          // site bra / ket state (0..3)
    Ref ref;
    double coef;
    int sgn_par;         // multiply by (-1)^{n(ket block sector)} when 1
};

struct TransOp {
    QN dq;               // total shift on the enlarged space
    int par = 0;
    std::vector<Comp> comps;
};

// 4x4 site matrices (row = bra state)
struct M4 {
    double a[4][4] = {{0}};
    M4 operator*(const M4& o) const;
    M4 operator+(const M4& o) const;
    M4 operator*(double s) const;
    M4 T() const;
    bool zero() const;
};

// host wall clock (seconds), for the per-phase timing printed under DMRG_VERBOSE
double wall_s();
// indices of Ctx::tm, accumulated over a block build
enum { TM_GROW = 0, TM_PLAN, TM_WSUM_HOST, TM_WSUM_DEV, TM_REN_HOST, TM_REN_DEV, TM_N };

struct Ctx {
    int device = 0;
    Arena arena;
    double tm[TM_N] = {0};
    // Dry run (workspace queries): every arena allocation and release happens
    // as in a real call, but no device work is issued and no device memory is
    // touched; the arena's high-water mark then gives the size the call needs.
    bool dry = false;
    // rocBLAS handle of the decimation's eigensolver (created on first use,
    // released by dmrg_destroy)
    void* solver = nullptr;
    bool has_ints = false;
    int K = 0, na = 0, nb = 0;
    double e_core = 0.0;
    int n_proc = 1, proc_id = 1;
    std::vector<double> h, g;     // masked spatial integrals
    double t(int p, int q) const {
        if ((p & 1) != (q & 1)) return 0.0;
        return h[(size_t)(p >> 1) * K + (q >> 1)];
    }
    double v(int p, int q, int r, int s) const {
        if ((p & 1) != (q & 1) || (r & 1) != (s & 1)) return 0.0;
        const size_t K1 = K;
        return g[(((size_t)(p >> 1) * K1 + (q >> 1)) * K1 + (r >> 1)) * K1 + (s >> 1)];
    }
    // spatial pair (i, j) kept by this sub-Hamiltonian (always true for n_proc == 1)
    bool pair_needed(int i, int j) const;
    // site operators of spatial orbital n
    M4 c(int p) const;            // a+_p on its site
    M4 site_H(int n) const;
    M4 site_R(int n, int p) const;
    M4 site_Pd(int n, int p, int r) const;   // P_pr^+ restricted to the site
    M4 site_Q(int n, int p, int q) const;
};

// status helpers
dmrg_status fail(dmrg_status s, const std::string& msg);
dmrg_status hip_fail(int err, const char* where);
#define DMRG_HIP(call)                                              \
    do {                                                            \
        int _e = (int)(call);                                       \
        if (_e != 0) return ::dmrg::hip_fail(_e, #call);            \
    } while (0)

// sector layout of an isometry (enlarged rows by site state then old sector)
struct Iso {
    const double* dev = nullptr;
    Basis nb;                          // new basis
    std::vector<int64_t> off;          // per new sector: element offset of U_q
    std::vector<int> d;                // rows
    std::vector<std::array<int, 4>> seg;   // row offset of segment s (-1 absent)
};
// need_data = false (dry runs): the isometry's device data may be NULL
dmrg_status make_iso(const Basis& old, const dmrg_bsm* bsm, Iso& out, bool need_data = true);
// arena bytes of a Davidson workspace (davidson.cpp)
int64_t dav_workspace_bytes(int64_t dim, int k, const dmrg_dav_opts* opts);

// allocate + lay out an opset region
dmrg_status alloc_set(Ctx* ctx, OpSetImpl& s);
void free_set(Ctx* ctx, OpSetImpl& s);
// arena bytes of a laid-out set (as alloc_set takes them)
int64_t set_bytes(const OpSetImpl& s);

// ------------- work lists ---------------------------------------------------
struct WorkList {
    std::vector<dmrgk::Task> task[dmrgk::kNumClass];
    std::vector<dmrgk::Group> groups;
    std::vector<dmrgk::Contrib> contribs;
    std::vector<dmrgk::Reduce> reduces;   // sums of split tasks' partial tiles
    int64_t partial_elems = 0;            // per-vector size of the partial buffer
    int tall_min = dmrgk::kMaxRows + 1;   // tiles of this many rows or more run on the tall kernel
    void clear();
    size_t ntasks() const;
};

// device copy of a work list (in the arena)
struct DevWork {
    int64_t region = -1;
    dmrgk::Task* task[dmrgk::kNumClass] = {};
    int ntask[dmrgk::kNumClass] = {};
    dmrgk::Group* groups = nullptr;
    dmrgk::Contrib* contribs = nullptr;
    dmrgk::Reduce* reduces = nullptr;
    int nred = 0;
    bool lds_records = false;               // every task's records fit the kernels' LDS staging
    double useful[dmrgk::kNumClass] = {};   // useful MFMA flops per class (one vector)
};
dmrg_status upload_work(Ctx* ctx, const WorkList& w, DevWork& d, void* stream);
// the groups and contributions alone, and the tasks and reductions alone (their
// groups and contributions those of recs: lists that differ only in their tasks
// share one copy of the records)
dmrg_status upload_records(Ctx* ctx, const WorkList& w, DevWork& d, void* stream);
// (with_useful = false leaves DevWork::useful at zero: lists that are only timed)
dmrg_status upload_tasks(Ctx* ctx, const WorkList& w, const DevWork& recs, DevWork& d, void* stream,
                         bool with_useful = true);
int64_t task_bytes(const WorkList& w);   // arena bytes upload_tasks takes
// arena bytes upload_work takes for a list
int64_t work_bytes(const WorkList& w);
// splits tiles above kMaxRows rows, then checks every operand of every task on the
// host; size[b] = elements of buffer b
dmrg_status validate_work(WorkList& w, const int64_t* size);
// Largest span (elements, origin to last element) of one operand of a task:
// 2^32 bytes of 8-byte elements (the kernels' in-block byte offsets are 32-bit).
constexpr int64_t kMaxOperandSpan = (int64_t(1) << 32) / 8;
// Integral-weighted temporaries of one growth batch (bytes): operators are
// grown and transformed in batches whose temporaries stay below this.
constexpr int64_t kGrowBatchBytes = int64_t(8) << 30;
void split_large(WorkList& w);
// Splits the group ranges of expensive tasks into chunks of about
// 1/target_tasks of the total cost each (chunks write partial tiles that a
// reduction sums in fixed order), then orders every class by decreasing cost.
void balance_work(WorkList& w, int target_tasks);
// re-sorts every task into its class under w.tall_min
void reclassify(WorkList& w);
double task_cost(const WorkList& w, const dmrgk::Task& t);
// the task's records fit the LDS staging (kRecG groups, kRecC contiguous contributions)
bool records_fit(const WorkList& w, const dmrgk::Task& t);
// class of a task: by its columns and the largest of its rows and group mu
int task_class_of(const WorkList& w, const dmrgk::Task& t);
void free_work(Ctx* ctx, DevWork& d);
dmrg_status run_work_f64(const DevWork& d, const dmrgk::Bases<double>& b, int nvec, void* stream);
dmrg_status run_work_f32(const DevWork& d, const dmrgk::Bases<float>& b, int nvec, void* stream);
// as run_work_*, one vector, with HIP events around each launch: ms[c] for
// class c, ms[kNumClass] for the reduction (0 for empty launches)
dmrg_status run_work_timed_f64(const DevWork& d, const dmrgk::Bases<double>& b, float* ms, void* stream);
dmrg_status run_work_timed_f32(const DevWork& d, const dmrgk::Bases<float>& b, float* ms, void* stream);
double task_useful_flops(const WorkList& w, const dmrgk::Task& t);

// emit the tasks of one output block (m x n at c_off) with the given group range
void emit_block_tasks(WorkList& w, int cbuf, int64_t c_off, int ldc, int m, int n, int g0, int g1,
                      bool accumulate = false);

// ------------- weighted sums ------------------------------------------------
// out (family in `temps`) = sum_k w_k * ops[k] of input family `fam` in `src`
struct WSumReq {
    int fam;                      // input family (in src)
    std::vector<double> w;        // weight per operator of the family
    int out_idx = -1;             // index of the result in the temp family
};
struct WSumPlan {
    std::vector<WSumReq> reqs;
    std::vector<std::pair<int, int>> out;   // (temp family, idx) per request
};
// registers one output family per input family in `temps` (before alloc_set)
void plan_wsums(const OpSetImpl& src, WSumPlan& plan, OpSetImpl& temps);
// dst family df rows [row0, row0+nrows) = W[nrows x nin] . src family sf
dmrg_status family_gemm(Ctx* ctx, const std::vector<double>& W, const OpSetImpl& src, int sf,
                        const OpSetImpl& dst, int df, int row0, int nrows, void* stream);
// runs the GEMMs once `temps` is allocated; synchronises the stream
dmrg_status exec_wsums(Ctx* ctx, const OpSetImpl& src, const WSumPlan& plan, const OpSetImpl& temps,
                       void* stream);
// largest transient arena bytes (weights + work list) of one family GEMM of exec_wsums
int64_t wsum_work_bytes(const OpSetImpl& src, const WSumPlan& plan);
// rows of one family GEMM group, operators per contribution (span bound)
void family_chunks(int64_t stride, int64_t& kc, int& rchunk);

// operators of a block grown by one site, in transition form
struct Grown {
    std::vector<int64_t> keys;
    std::vector<TransOp> ops;
    std::vector<char> kinds;
    std::vector<std::pair<int, int>> idx;
    void add(char kind, int p, int q, const QN& dq, int par, TransOp&& T) {
        T.dq = dq;
        T.par = par;
        keys.push_back(okey(kind, p, q));
        kinds.push_back(kind);
        idx.push_back({p, q});
        ops.push_back(std::move(T));
    }
};

void grow_left(const Ctx* C, const OpSetImpl& X, int n, const std::vector<int>& outside, Grown& G);
void grow_right_compl(const Ctx* C, const OpSetImpl& Y, int n, const std::vector<int>& before, Grown& G);
// req_begin (optional): request index at which each operator's sums start, plus the total
void compact(std::vector<TransOp>& ops, const OpSetImpl& old, WSumPlan& plan, std::vector<int>* req_begin = nullptr);
// operators i0..i1-1; their requests are plan.reqs[idx - rbase]
void resolve(std::vector<TransOp>& ops, const WSumPlan& plan, const OpSetImpl& temps, size_t i0 = 0,
             size_t i1 = SIZE_MAX, int rbase = 0);
// transformation of grown operators (refs into old / temps) through an isometry
dmrg_status renormalize_grown(Ctx* C, const OpSetImpl& old, const OpSetImpl* temps, const dmrg_bsm* iso,
                              const Grown& G, OpSetImpl& nw, void* stream);

}  // namespace dmrg

struct dmrg_heff;
dmrg::Ctx* heff_ctx(const dmrg_heff* H);
namespace dmrg {
// wavefunction sub-block (a, s1, s2, b) of an H_eff: a, b index the sectors
// of its left / right block; m_a x m_b row-major at element `off`
struct PsiSub { int a, s1, s2, b, ma, mb; int64_t off; };
void heff_psi_subblocks(const dmrg_heff* H, const OpSetImpl*& Lb, const OpSetImpl*& Rb, std::vector<PsiSub>& out);
void release_solver(Ctx* C);
}  // namespace dmrg

struct dmrg_ctx : dmrg::Ctx {};
struct dmrg_opset : dmrg::OpSetImpl {
    dmrg::Ctx* ctx = nullptr;
};
