// Blocking and transformation (Appendix A of the paper) in delayed form,
// the edge-to-middle build, the normal -> complementary middle transform,
// and the context / integral entry points of the C ABI.
//
// Operator identities used (non-spin-adapted forms of the normal /
// complementary operators of Appendix B; spin-orbitals p,q,r,s; t, v the
// spin-resolved integrals).  For a bipartition X|Y (X first in the
// Jordan-Wigner order) the product O_X O_Y has matrix
// kron(O_X P^{pi(O_Y)}, O_Y), P = (-1)^{n} on X.
//   H = H^X + H^Y + sum_{p in X}(C_p R^Y_p - D_p R^Y_p+) + sum_{p in Y}(R^X_p+ D_p - R^X_p C_p)
//       + sum_{p<r in X}(A_pr P^Y_pr + h.c.) + sum_{pq in X} B_pq Q^Y_pq        (NC)
//     or the mirror with two-index operators grouped on Y's normal side (CN);
//   R^{XY}_p = R^X_p + R^Y_p + sum_{u in Y} Q^X_pu a_u + sum_{r in Y} P^X_pr a+_r
//              + sum_{u in X} a_u Q^Y_pu + sum_{r in X} a+_r P^Y_pr;
//   P^{XY}_pr and Q^{XY}_pq for a complementary block grown by a site X:
//              the site part, the old part, and mixed one-index products.
// The one-body term enters each R as t/2.  Two-index complementary operators
// are stored as P^+ ('D', same skeleton as A) and Q; index symmetry
// P_rp = -P_pr, Q_qp = Q_pq^T is used through transposed references.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <iterator>
#include <map>
#include <tuple>

#include "core.hpp"

namespace dmrg {

static M4 I4() {
    M4 r;
    for (int i = 0; i < 4; ++i) r.a[i][i] = 1.0;
    return r;
}

static Ref ID() { return Ref(); }

static Ref OP(const OpSetImpl& S, char kind, int p, int q, bool tr = false) {
    Ref r;
    auto it = S.lookup.find(okey(kind, p, q));
    if (it == S.lookup.end()) {
        r.type = -1;
        return r;
    }
    r.type = 1;
    r.set = &S;
    r.fam = it->second.first;
    r.idx = it->second.second;
    r.trans = tr;
    return r;
}

// kron(old-block operator, site operator): left growth (old block first)
static void kl(TransOp& T, const Ref& x, const M4& s, int pis, double c) {
    if (x.type < 0 || c == 0.0) return;
    for (int sb = 0; sb < 4; ++sb)
        for (int sk = 0; sk < 4; ++sk)
            if (s.a[sb][sk] != 0.0) T.comps.push_back(Comp{sb, sk, x, c * s.a[sb][sk], pis});
}

// kron(site operator, old-block operator): right growth (site first)
static void kr(TransOp& T, const M4& s, const Ref& y, double c) {
    if (y.type < 0 || c == 0.0) return;
    const int py = y.par();
    for (int sb = 0; sb < 4; ++sb)
        for (int sk = 0; sk < 4; ++sk)
            if (s.a[sb][sk] != 0.0) {
                const double sg = (py && (kSiteQ[sk].n() & 1)) ? -1.0 : 1.0;
                T.comps.push_back(Comp{sb, sk, y, c * s.a[sb][sk] * sg, 0});
            }
}



// ---------------------------------------------------------------------------
// left block (normal operators) grown by site n at its right end
void grow_left(const Ctx* C, const OpSetImpl& X, int n, const std::vector<int>& outside, Grown& G) {
    const std::vector<int>& xo = X.orbs;
    const int so[2] = {2 * n, 2 * n + 1};
    std::vector<int> zo = xo;
    zo.push_back(so[0]);
    zo.push_back(so[1]);
    auto need = [&](int p, int q) { return C->pair_needed(p >> 1, q >> 1); };
    auto site = [&](int p) { return (p >> 1) == n; };
    const M4 I = I4();
    for (int p : xo) { TransOp T; kl(T, OP(X, 'C', p, -1), I, 0, 1.0); G.add('C', p, -1, qe(p), 1, std::move(T)); }
    for (int p : so) { TransOp T; kl(T, ID(), C->c(p), 1, 1.0); G.add('C', p, -1, qe(p), 1, std::move(T)); }
    for (size_t i = 0; i < zo.size(); ++i)
        for (size_t j = i + 1; j < zo.size(); ++j) {
            const int p = zo[i], r = zo[j];
            if (!need(p, r)) continue;
            TransOp T;
            if (site(p) && site(r)) kl(T, ID(), C->c(p) * C->c(r), 0, 1.0);
            else if (site(r)) kl(T, OP(X, 'C', p, -1), C->c(r), 1, 1.0);
            else kl(T, OP(X, 'A', p, r), I, 0, 1.0);
            G.add('A', p, r, qe(p) + qe(r), 0, std::move(T));
        }
    for (int p : zo)
        for (int q : zo) {
            if (!need(p, q)) continue;
            TransOp T;
            if (site(p) && site(q)) kl(T, ID(), C->c(p) * C->c(q).T(), 0, 1.0);
            else if (site(q)) kl(T, OP(X, 'C', p, -1), C->c(q).T(), 1, 1.0);
            else if (site(p)) kl(T, OP(X, 'C', q, -1, true), C->c(p), 1, -1.0);
            else kl(T, OP(X, 'B', p, q), I, 0, 1.0);
            G.add('B', p, q, qe(p) - qe(q), 0, std::move(T));
        }
    {
        TransOp T;
        kl(T, OP(X, 'H', -1, -1), I, 0, 1.0);
        kl(T, ID(), C->site_H(n), 0, 1.0);
        for (int p : xo) {
            const M4 Rn = C->site_R(n, p);
            kl(T, OP(X, 'C', p, -1), Rn, 1, 1.0);
            kl(T, OP(X, 'C', p, -1, true), Rn.T(), 1, -1.0);
        }
        for (int p : so) {
            kl(T, OP(X, 'R', p, -1, true), C->c(p).T(), 1, 1.0);
            kl(T, OP(X, 'R', p, -1), C->c(p), 1, -1.0);
        }
        for (size_t i = 0; i < xo.size(); ++i)
            for (size_t j = i + 1; j < xo.size(); ++j) {
                const int p = xo[i], r = xo[j];
                if (!need(p, r)) continue;
                const M4 Pd = C->site_Pd(n, p, r);
                kl(T, OP(X, 'A', p, r), Pd.T(), 0, 1.0);
                kl(T, OP(X, 'A', p, r, true), Pd, 0, 1.0);
            }
        for (int p : xo)
            for (int q : xo)
                if (need(p, q)) kl(T, OP(X, 'B', p, q), C->site_Q(n, p, q), 0, 1.0);
        G.add('H', -1, -1, QN(0, 0), 0, std::move(T));
    }
    for (int p : outside) {
        TransOp T;
        kl(T, OP(X, 'R', p, -1), I, 0, 1.0);
        kl(T, ID(), C->site_R(n, p), 1, 1.0);
        for (int u : so)
            for (int r : xo)
                for (int s : xo) {
                    if (!need(r, s)) continue;
                    const double w = C->v(p, u, r, s) - C->v(p, s, r, u);
                    if (w != 0.0) kl(T, OP(X, 'B', r, s), C->c(u).T(), 1, w);
                }
        for (int r : so)
            for (size_t i = 0; i < xo.size(); ++i)
                for (size_t j = i + 1; j < xo.size(); ++j) {
                    const int q = xo[i], s = xo[j];
                    if (!need(q, s)) continue;
                    const double w = C->v(p, q, r, s) - C->v(p, s, r, q);
                    if (w != 0.0) kl(T, OP(X, 'A', q, s, true), C->c(r), 1, w);
                }
        for (int u : xo) kl(T, OP(X, 'C', u, -1, true), C->site_Q(n, p, u), 0, 1.0);
        for (int r : xo) kl(T, OP(X, 'C', r, -1), C->site_Pd(n, p, r).T(), 0, 1.0);
        G.add('R', p, -1, -qe(p), 1, std::move(T));
    }
}

// right block (normal operators, CN) grown by site n at its left end
static void grow_right_normal(const Ctx* C, const OpSetImpl& Y, int n, const std::vector<int>& before,
                              Grown& G) {
    const std::vector<int>& yo = Y.orbs;
    const int so[2] = {2 * n, 2 * n + 1};
    std::vector<int> zo = {so[0], so[1]};
    zo.insert(zo.end(), yo.begin(), yo.end());
    auto site = [&](int p) { return (p >> 1) == n; };
    const M4 I = I4();
    for (int p : so) { TransOp T; kr(T, C->c(p), ID(), 1.0); G.add('C', p, -1, qe(p), 1, std::move(T)); }
    for (int p : yo) { TransOp T; kr(T, I, OP(Y, 'C', p, -1), 1.0); G.add('C', p, -1, qe(p), 1, std::move(T)); }
    for (size_t i = 0; i < zo.size(); ++i)
        for (size_t j = i + 1; j < zo.size(); ++j) {
            const int p = zo[i], r = zo[j];
            TransOp T;
            if (site(p) && site(r)) kr(T, C->c(p) * C->c(r), ID(), 1.0);
            else if (site(p)) kr(T, C->c(p), OP(Y, 'C', r, -1), 1.0);
            else kr(T, I, OP(Y, 'A', p, r), 1.0);
            G.add('A', p, r, qe(p) + qe(r), 0, std::move(T));
        }
    for (int p : zo)
        for (int q : zo) {
            TransOp T;
            if (site(p) && site(q)) kr(T, C->c(p) * C->c(q).T(), ID(), 1.0);
            else if (site(p)) kr(T, C->c(p), OP(Y, 'C', q, -1, true), 1.0);
            else if (site(q)) kr(T, C->c(q).T(), OP(Y, 'C', p, -1), -1.0);
            else kr(T, I, OP(Y, 'B', p, q), 1.0);
            G.add('B', p, q, qe(p) - qe(q), 0, std::move(T));
        }
    {
        TransOp T;
        kr(T, C->site_H(n), ID(), 1.0);
        kr(T, I, OP(Y, 'H', -1, -1), 1.0);
        for (int p : so) {
            kr(T, C->c(p), OP(Y, 'R', p, -1), 1.0);
            kr(T, C->c(p).T(), OP(Y, 'R', p, -1, true), -1.0);
        }
        for (int p : yo) {
            const M4 Rn = C->site_R(n, p);
            kr(T, Rn.T(), OP(Y, 'C', p, -1, true), 1.0);
            kr(T, Rn, OP(Y, 'C', p, -1), -1.0);
        }
        for (size_t i = 0; i < yo.size(); ++i)
            for (size_t j = i + 1; j < yo.size(); ++j) {
                const int p = yo[i], r = yo[j];
                const M4 Pd = C->site_Pd(n, p, r);
                kr(T, Pd.T(), OP(Y, 'A', p, r), 1.0);
                kr(T, Pd, OP(Y, 'A', p, r, true), 1.0);
            }
        for (int p : yo)
            for (int q : yo) kr(T, C->site_Q(n, p, q), OP(Y, 'B', p, q), 1.0);
        G.add('H', -1, -1, QN(0, 0), 0, std::move(T));
    }
    for (int p : before) {
        TransOp T;
        kr(T, C->site_R(n, p), ID(), 1.0);
        kr(T, I, OP(Y, 'R', p, -1), 1.0);
        for (int u : yo) {
            kr(T, C->site_Q(n, p, u), OP(Y, 'C', u, -1, true), 1.0);
            kr(T, C->site_Pd(n, p, u).T(), OP(Y, 'C', u, -1), 1.0);
        }
        for (int u : so)
            for (int r : yo)
                for (int s : yo) {
                    const double w = C->v(p, u, r, s) - C->v(p, s, r, u);
                    if (w != 0.0) kr(T, C->c(u).T(), OP(Y, 'B', r, s), w);
                }
        for (int r : so)
            for (size_t i = 0; i < yo.size(); ++i)
                for (size_t j = i + 1; j < yo.size(); ++j) {
                    const int q = yo[i], s = yo[j];
                    const double w = C->v(p, q, r, s) - C->v(p, s, r, q);
                    if (w != 0.0) kr(T, C->c(r), OP(Y, 'A', q, s, true), w);
                }
        G.add('R', p, -1, -qe(p), 1, std::move(T));
    }
}

// right block (complementary operators) grown by site n at its left end
void grow_right_compl(const Ctx* C, const OpSetImpl& Y, int n, const std::vector<int>& before, Grown& G) {
    const std::vector<int>& yo = Y.orbs;
    const int so[2] = {2 * n, 2 * n + 1};
    auto need = [&](int p, int q) { return C->pair_needed(p >> 1, q >> 1); };
    const M4 I = I4();
    for (int p : so) { TransOp T; kr(T, C->c(p), ID(), 1.0); G.add('C', p, -1, qe(p), 1, std::move(T)); }
    for (int p : yo) { TransOp T; kr(T, I, OP(Y, 'C', p, -1), 1.0); G.add('C', p, -1, qe(p), 1, std::move(T)); }
    {
        TransOp T;
        kr(T, C->site_H(n), ID(), 1.0);
        kr(T, I, OP(Y, 'H', -1, -1), 1.0);
        for (int p : so) {
            kr(T, C->c(p), OP(Y, 'R', p, -1), 1.0);
            kr(T, C->c(p).T(), OP(Y, 'R', p, -1, true), -1.0);
        }
        for (int p : yo) {
            const M4 Rn = C->site_R(n, p);
            kr(T, Rn.T(), OP(Y, 'C', p, -1, true), 1.0);
            kr(T, Rn, OP(Y, 'C', p, -1), -1.0);
        }
        const M4 A = C->c(so[0]) * C->c(so[1]);
        kr(T, A, OP(Y, 'D', so[0], so[1], true), 1.0);
        kr(T, A.T(), OP(Y, 'D', so[0], so[1]), 1.0);
        for (int p : so)
            for (int q : so) kr(T, C->c(p) * C->c(q).T(), OP(Y, 'Q', p, q), 1.0);
        G.add('H', -1, -1, QN(0, 0), 0, std::move(T));
    }
    for (int p : before) {
        TransOp T;
        kr(T, C->site_R(n, p), ID(), 1.0);
        kr(T, I, OP(Y, 'R', p, -1), 1.0);
        for (int u : yo) {
            kr(T, C->site_Q(n, p, u), OP(Y, 'C', u, -1, true), 1.0);
            kr(T, C->site_Pd(n, p, u).T(), OP(Y, 'C', u, -1), 1.0);
        }
        for (int u : so) {
            kr(T, C->c(u).T(), OP(Y, 'Q', p, u), 1.0);
            if (p < u) kr(T, C->c(u), OP(Y, 'D', p, u, true), 1.0);
            else kr(T, C->c(u), OP(Y, 'D', u, p, true), -1.0);
        }
        G.add('R', p, -1, -qe(p), 1, std::move(T));
    }
    for (size_t i = 0; i < before.size(); ++i)
        for (size_t j = i + 1; j < before.size(); ++j) {
            const int p = before[i], r = before[j];
            if (!need(p, r)) continue;
            TransOp T;
            kr(T, C->site_Pd(n, p, r), ID(), 1.0);
            kr(T, I, OP(Y, 'D', p, r), 1.0);
            for (int u : so)
                for (int w : yo) {
                    const double c = -(C->v(p, w, r, u) - C->v(p, u, r, w));
                    if (c != 0.0) kr(T, C->c(u), OP(Y, 'C', w, -1), c);
                }
            G.add('D', p, r, qe(p) + qe(r), 0, std::move(T));
        }
    for (int p : before)
        for (int q : before) {
            if (!need(p, q)) continue;
            TransOp T;
            kr(T, C->site_Q(n, p, q), ID(), 1.0);
            kr(T, I, OP(Y, 'Q', p, q), 1.0);
            for (int r : so)
                for (int s : yo) {
                    const double w = C->v(p, q, r, s) - C->v(p, s, r, q);
                    if (w != 0.0) kr(T, C->c(r), OP(Y, 'C', s, -1, true), w);
                }
            for (int s : so)
                for (int r : yo) {
                    const double w = C->v(p, q, r, s) - C->v(p, s, r, q);
                    if (w != 0.0) kr(T, C->c(s).T(), OP(Y, 'C', r, -1), -w);
                }
            G.add('Q', p, q, qe(q) - qe(p), 0, std::move(T));
        }
}

// ---------------------------------------------------------------------------
// compaction: components of one transition that refer to operators of the
// same family of `old` (same orientation and sign rule) are replaced by one
// integral-weighted sum (GEMM over the operator index); identity components of
// one transition are merged.
void compact(std::vector<TransOp>& ops, const OpSetImpl& old, WSumPlan& plan, std::vector<int>* req_begin) {
    for (TransOp& T : ops) {
        if (req_begin) req_begin->push_back((int)plan.reqs.size());
        std::map<std::tuple<int, int, int, int, int>, std::vector<int>> grp;
        std::map<std::tuple<int, int, int>, double> idc;
        std::vector<Comp> out;
        for (size_t i = 0; i < T.comps.size(); ++i) {
            const Comp& c = T.comps[i];
            if (c.ref.type == 0) {
                idc[std::make_tuple(c.sb, c.sk, c.sgn_par)] += c.coef;
                continue;
            }
            if (c.ref.type == 1 && c.ref.set == &old)
                grp[std::make_tuple(c.sb, c.sk, c.ref.fam, (int)c.ref.trans, c.sgn_par)].push_back((int)i);
            else
                out.push_back(c);
        }
        for (auto& kv : grp) {
            const auto& lst = kv.second;
            if (lst.size() == 1) {
                out.push_back(T.comps[lst[0]]);
                continue;
            }
            const int fam = std::get<2>(kv.first);
            WSumReq r;
            r.fam = fam;
            r.w.assign(old.fams[fam].keys.size(), 0.0);
            for (int i : lst) r.w[T.comps[i].ref.idx] += T.comps[i].coef;
            bool any = false;
            for (double x : r.w) any |= (x != 0.0);
            if (!any) continue;
            plan.reqs.push_back(std::move(r));
            Comp c;
            c.sb = std::get<0>(kv.first);
            c.sk = std::get<1>(kv.first);
            c.ref.type = 2;
            c.ref.idx = (int)plan.reqs.size() - 1;
            c.ref.trans = std::get<3>(kv.first) != 0;
            c.coef = 1.0;
            c.sgn_par = std::get<4>(kv.first);
            out.push_back(c);
        }
        for (auto& kv : idc)
            if (kv.second != 0.0) {
                Comp c;
                c.sb = std::get<0>(kv.first);
                c.sk = std::get<1>(kv.first);
                c.ref = Ref();
                c.coef = kv.second;
                c.sgn_par = std::get<2>(kv.first);
                out.push_back(c);
            }
        T.comps.swap(out);
    }
    if (req_begin) req_begin->push_back((int)plan.reqs.size());
}

void resolve(std::vector<TransOp>& ops, const WSumPlan& plan, const OpSetImpl& temps, size_t i0, size_t i1,
             int rbase) {
    i1 = std::min(i1, ops.size());
    for (size_t i = i0; i < i1; ++i)
        for (Comp& c : ops[i].comps)
            if (c.ref.type == 2) {
                const auto o = plan.out[c.ref.idx - rbase];
                c.ref.type = 1;
                c.ref.set = &temps;
                c.ref.fam = o.first;
                c.ref.idx = o.second;
            }
}

// ---------------------------------------------------------------------------
// transformation: O_new[q' <- q] = sum_{(s',s)} U_{q',s'}^T (sum_k c_k Z_k) U_{q,s}
// the new set: one operator per grown operator, in the new basis (allocated)
static dmrg_status layout_new_set(Ctx* C, const Iso& iso, const Grown& G, OpSetImpl& nw) {
    nw.basis = iso.nb;
    nw.basis.index();
    nw.skels.clear();
    nw.fams.clear();
    nw.lookup.clear();
    for (size_t i = 0; i < G.keys.size(); ++i)
        nw.add_op(G.kinds[i], G.idx[i].first, G.idx[i].second, G.ops[i].dq, G.ops[i].par);
    return alloc_set(C, nw);
}

// Rows of a new-basis block above which its transformation runs in two
// passes (DMRG_TWO_PASS_ROWS overrides; a GPU test lowers it).
static int two_pass_rows() {
    const char* e = std::getenv("DMRG_TWO_PASS_ROWS");
    return e ? std::max(1, std::atoi(e)) : dmrgk::kTallRows;
}

// Transformation of grown operators i0..i1-1 into their rows of nw:
//   O_new[q' <- q] = sum_{s'} U_{q',s'}^T T_{s'},  T_{s'} = sum_{s, k} c_k Z_k U_{q,s}
// (Appendix A, operator transformation, with the blocked operator kept as its
// site transitions (s', s) and old-block components Z_k).  A block whose new
// bra dimension fits the tall tile runs in one pass: T stays in registers /
// LDS and U^T T follows at once.  A taller block would recompute T for every
// row tile of the output, so it runs in two: T_{s'} is first formed in a
// temporary buffer (buffer 4), then U^T T is a plain product of it.  The
// operators are taken in sub-ranges whose temporaries stay below
// kGrowBatchBytes.
static dmrg_status renormalize_sub(Ctx* C, const OpSetImpl& old, const OpSetImpl* temps, const Iso& iso,
                                   const Grown& G, size_t i0, size_t i1, OpSetImpl& nw, int two_rows,
                                   void* stream) {
    dmrg_status st = DMRG_OK;
    const double t0 = wall_s();
    WorkList wl, wl1;   // wl1: first pass of the two-pass blocks (into the temporaries)
    int64_t toff = 0;   // elements of the temporaries
    const Basis& ob = old.basis;
    const Basis& nb = nw.basis;
    for (size_t i = i0; i < i1; ++i) {
        const auto fi = nw.lookup.at(G.keys[i]);
        const Family& F = nw.fams[fi.first];
        const Skel& S = nw.skels[F.skel];
        const TransOp& T = G.ops[i];
        std::map<std::pair<int, int>, std::vector<int>> bucket;
        for (size_t c = 0; c < T.comps.size(); ++c) bucket[{T.comps[c].sb, T.comps[c].sk}].push_back((int)c);
        for (size_t b = 0; b < S.ket.size(); ++b) {
            const int kq = S.ket[b], kb = S.bra[b];
            const int mq = nb.m[kq], mqb = nb.m[kb];
            const bool two = mqb > two_rows;
            const int g0 = (int)wl.groups.size();
            // contributions of bucket (sb, sk): sum_k c_k Z_k U_{q,sk} (the A.B products of T_sb)
            auto add_contribs = [&](WorkList& w, int sb, int sk, const std::vector<int>& comps) {
                const int a = ob.find(nb.q[kq] - kSiteQ[sk]);
                const int a2 = ob.find(nb.q[kb] - kSiteQ[sb]);
                if (a < 0 || a2 < 0) return;
                for (int ci : comps) {
                    const Comp& cp = T.comps[ci];
                    const double sg = (cp.sgn_par && (ob.q[a].n() & 1)) ? -1.0 : 1.0;
                    dmrgk::Contrib c{};
                    c.b_off = iso.off[kq] + (int64_t)iso.seg[kq][sk] * mq;
                    c.ldb = mq;
                    c.k = ob.m[a];
                    c.alpha = cp.coef * sg;
                    if (cp.ref.type == 0) {
                        if (a != a2) continue;
                        c.flags = dmrgk::F_ID_A | (2 << 3);
                    } else {
                        int bra, ld;
                        int64_t off;
                        bool tr;
                        if (!cp.ref.block(a, bra, off, ld, tr) || bra != a2) continue;
                        const int abuf = (cp.ref.set == &old) ? 0 : 1;
                        c.a_off = off;
                        c.lda = ld;
                        c.flags = abuf | (2 << 3) | (tr ? dmrgk::F_TRANS_A : 0);
                    }
                    w.contribs.push_back(c);
                }
            };
            if (!two) {
                for (auto& kv : bucket) {
                    const int sb = kv.first.first;
                    const int a2 = ob.find(nb.q[kb] - kSiteQ[sb]);
                    if (a2 < 0 || ob.find(nb.q[kq] - kSiteQ[kv.first.second]) < 0) continue;
                    dmrgk::Group g{};
                    g.x_off = iso.off[kb] + (int64_t)iso.seg[kb][sb] * mqb;
                    g.ldx = mqb;
                    g.mu = ob.m[a2];
                    g.x_coef = 1.0;
                    g.flags = 2 | dmrgk::G_TRANS_X | dmrgk::G_HAS_X;
                    g.c0 = (int)wl.contribs.size();
                    add_contribs(wl, sb, kv.first.second, kv.second);
                    g.c1 = (int)wl.contribs.size();
                    if (g.c1 > g.c0) wl.groups.push_back(g);
                }
            } else {
                for (int sb = 0; sb < 4; ++sb) {
                    const int a2 = ob.find(nb.q[kb] - kSiteQ[sb]);
                    if (a2 < 0) continue;
                    // first pass: T_sb = sum over the buckets (sb, *) into the temporaries
                    dmrgk::Group g1{};
                    g1.xid_coef = 1.0;
                    g1.mu = ob.m[a2];
                    g1.c0 = (int)wl1.contribs.size();
                    for (auto& kv : bucket)
                        if (kv.first.first == sb) add_contribs(wl1, sb, kv.first.second, kv.second);
                    g1.c1 = (int)wl1.contribs.size();
                    if (g1.c1 == g1.c0) continue;
                    const int gi = (int)wl1.groups.size();
                    wl1.groups.push_back(g1);
                    emit_block_tasks(wl1, 4, toff, mq, ob.m[a2], mq, gi, gi + 1);
                    // second pass: O_new += U_{q',sb}^T T_sb
                    dmrgk::Group g{};
                    g.x_off = iso.off[kb] + (int64_t)iso.seg[kb][sb] * mqb;
                    g.ldx = mqb;
                    g.mu = ob.m[a2];
                    g.x_coef = 1.0;
                    g.flags = 2 | dmrgk::G_TRANS_X | dmrgk::G_HAS_X;
                    g.c0 = (int)wl.contribs.size();
                    dmrgk::Contrib c{};
                    c.a_off = toff;
                    c.lda = mq;
                    c.alpha = 1.0;
                    c.flags = 4 | dmrgk::F_ID_B;
                    wl.contribs.push_back(c);
                    g.c1 = (int)wl.contribs.size();
                    wl.groups.push_back(g);
                    toff += (int64_t)ob.m[a2] * mq;
                }
            }
            emit_block_tasks(wl, 3, F.base + (int64_t)fi.second * F.stride + S.off[b], mq, mqb, mq, g0,
                             (int)wl.groups.size());
        }
    }
    if (wl.ntasks() == 0) return DMRG_OK;
    int64_t sz[dmrgk::kMaxBuf] = {0};
    sz[0] = old.elems;
    sz[1] = temps ? temps->elems : 0;
    for (size_t i = 0; i < iso.off.size(); ++i)
        sz[2] = std::max<int64_t>(sz[2], iso.off[i] + (int64_t)iso.d[i] * iso.nb.m[i]);
    sz[3] = nw.elems;
    sz[4] = toff;
    int64_t treg = -1;
    if (toff > 0) {
        treg = C->arena.alloc(toff * 8);
        if (treg < 0) return fail(DMRG_E_WORKSPACE, "arena too small for transformation temporaries");
    }
    DevWork dw, dw1;
    st = validate_work(wl, sz);
    if (st == DMRG_OK && toff > 0) st = validate_work(wl1, sz);
    if (st == DMRG_OK && toff > 0) st = upload_work(C, wl1, dw1, stream);
    if (st == DMRG_OK) st = upload_work(C, wl, dw, stream);
    const double t1 = wall_s();
    C->tm[TM_REN_HOST] += t1 - t0;
    dmrgk::Bases<double> bs{};
    bs.p[0] = old.dev;
    bs.p[1] = temps ? temps->dev : old.dev;
    bs.p[2] = const_cast<double*>(iso.dev);
    bs.p[3] = nw.dev;
    bs.p[4] = treg >= 0 ? (double*)(C->arena.base + treg) : old.dev;
    if (st == DMRG_OK && !C->dry) {
        if (toff > 0) st = run_work_f64(dw1, bs, 1, stream);
        if (st == DMRG_OK) st = run_work_f64(dw, bs, 1, stream);
        if (st == DMRG_OK) {
            const int e = (int)hipStreamSynchronize((hipStream_t)stream);
            if (e) st = hip_fail(e, "renormalization");
        }
    }
    free_work(C, dw);
    free_work(C, dw1);
    if (treg >= 0) C->arena.release(treg);
    C->tm[TM_REN_DEV] += wall_s() - t1;
    return st;
}

// temporaries (elements) of the two-pass blocks of grown operator i
static int64_t two_pass_elems(const OpSetImpl& old, const Grown& G, size_t i, const OpSetImpl& nw, int two_rows) {
    const auto fi = nw.lookup.at(G.keys[i]);
    const Skel& S = nw.skels[nw.fams[fi.first].skel];
    const Basis& ob = old.basis;
    const Basis& nb = nw.basis;
    int64_t e = 0;
    for (size_t b = 0; b < S.ket.size(); ++b) {
        const int kq = S.ket[b], kb = S.bra[b];
        if (nb.m[kb] <= two_rows) continue;
        for (int sb = 0; sb < 4; ++sb) {
            const int a2 = ob.find(nb.q[kb] - kSiteQ[sb]);
            if (a2 >= 0) e += (int64_t)ob.m[a2] * nb.m[kq];
        }
    }
    return e;
}

static dmrg_status renormalize_range(Ctx* C, const OpSetImpl& old, const OpSetImpl* temps, const Iso& iso,
                                     const Grown& G, size_t i0, size_t i1, OpSetImpl& nw, void* stream) {
    const int two_rows = two_pass_rows();
    size_t a = i0;
    while (a < i1) {
        size_t b = a;
        int64_t e = 0;
        while (b < i1) {
            const int64_t x = two_pass_elems(old, G, b, nw, two_rows);
            if (b > a && (e + x) * 8 > kGrowBatchBytes) break;
            e += x;
            ++b;
        }
        dmrg_status st = renormalize_sub(C, old, temps, iso, G, a, b, nw, two_rows, stream);
        if (st != DMRG_OK) return st;
        a = b;
    }
    return DMRG_OK;
}

dmrg_status renormalize_grown(Ctx* C, const OpSetImpl& old, const OpSetImpl* temps, const dmrg_bsm* iso_desc,
                              const Grown& G, OpSetImpl& nw, void* stream) {
    Iso iso;
    dmrg_status st = make_iso(old.basis, iso_desc, iso, !C->dry);
    if (st == DMRG_OK) st = layout_new_set(C, iso, G, nw);
    if (st == DMRG_OK) st = renormalize_range(C, old, temps, iso, G, 0, G.ops.size(), nw, stream);
    return st;
}

// One growth step + transformation: old -> nw.  The integral-weighted sums of
// the grown operators (temporaries in the old basis) are formed and consumed
// in batches of operators whose temporaries fit half of the free arena, so
// the transient memory stays bounded when thousands of operators grow at once.
dmrg_status grow_and_renormalize(Ctx* C, OpSetImpl& old, Grown& G, const dmrg_bsm* iso_desc,
                                 OpSetImpl& nw, void* stream) {
    const double t0 = wall_s();
    WSumPlan plan;
    std::vector<int> rb;
    compact(G.ops, old, plan, &rb);
    Iso iso;
    dmrg_status st = make_iso(old.basis, iso_desc, iso, !C->dry);
    if (st == DMRG_OK) st = layout_new_set(C, iso, G, nw);
    if (st != DMRG_OK) return st;
    C->tm[TM_PLAN] += wall_s() - t0;
    // The budget is a fixed size, not a share of the free arena, so that the
    // sequence of allocations does not depend on the arena's size and a dry
    // run (dmrg_query_workspace) reproduces it exactly.  DMRG_GROW_BATCH_BYTES
    // overrides it (a GPU test sets 1: one operator's temporaries at a time).
    const char* env = std::getenv("DMRG_GROW_BATCH_BYTES");
    const int64_t budget = env ? std::atoll(env) : kGrowBatchBytes;
    const size_t n = G.ops.size();
    size_t i0 = 0;
    while (i0 < n && st == DMRG_OK) {
        size_t i1 = i0;
        int64_t bytes = 0;
        while (i1 < n) {
            int64_t b = 0;
            for (int r = rb[i1]; r < rb[i1 + 1]; ++r) b += old.fams[plan.reqs[r].fam].stride * (int64_t)sizeof(double);
            if (i1 > i0 && bytes + b > budget) break;
            bytes += b;
            ++i1;
        }
        WSumPlan sub;
        sub.reqs.assign(plan.reqs.begin() + rb[i0], plan.reqs.begin() + rb[i1]);
        OpSetImpl temps;
        temps.basis = old.basis;
        temps.kind = 2;
        plan_wsums(old, sub, temps);
        st = alloc_set(C, temps);
        if (st == DMRG_OK) st = exec_wsums(C, old, sub, temps, stream);
        if (st == DMRG_OK) {
            resolve(G.ops, sub, temps, i0, i1, rb[i0]);
            st = renormalize_range(C, old, &temps, iso, G, i0, i1, nw, stream);
        }
        free_set(C, temps);
        i0 = i1;
    }
    return st;
}

// The operators of block `cur` grown by its next site, in transition form
// (left block of n sites: site n, with R_p kept for every p to its right;
// right block of n sites: site K-1-n, with R_p, P, Q for every p to its left).
static void grow_ops(const Ctx* C, const OpSetImpl& cur, Grown& G) {
    const int K = C->K;
    if (cur.side == DMRG_LEFT) {
        const int n = cur.nsites;
        std::vector<int> outside;
        for (int p = 2 * (n + 1); p < 2 * K; ++p) outside.push_back(p);
        grow_left(C, cur, n, outside, G);
    } else {
        const int n = K - 1 - cur.nsites;
        std::vector<int> before;
        for (int p = 0; p < 2 * n; ++p) before.push_back(p);
        if (cur.kind == 1) grow_right_compl(C, cur, n, before, G);
        else grow_right_normal(C, cur, n, before, G);
    }
}

// spin-orbitals and site count of the grown block
static void grown_meta(const Ctx* C, const OpSetImpl& cur, OpSetImpl& nw) {
    nw.side = cur.side;
    nw.kind = cur.kind;
    nw.nsites = cur.nsites + 1;
    if (cur.side == DMRG_LEFT) {
        const int n = cur.nsites;
        nw.orbs = cur.orbs;
        nw.orbs.push_back(2 * n);
        nw.orbs.push_back(2 * n + 1);
    } else {
        const int n = C->K - 1 - cur.nsites;
        nw.orbs = {2 * n, 2 * n + 1};
        nw.orbs.insert(nw.orbs.end(), cur.orbs.begin(), cur.orbs.end());
    }
}

// One blocking + transformation step: cur grown by its next site through iso.
static dmrg_status grow_step(Ctx* C, OpSetImpl& cur, const dmrg_bsm* iso, OpSetImpl& nw, void* stream) {
    Grown G;
    const double tg = wall_s();
    grow_ops(C, cur, G);
    C->tm[TM_GROW] += wall_s() - tg;
    grown_meta(C, cur, nw);
    return grow_and_renormalize(C, cur, G, iso, nw, stream);
}

static dmrg_status vacuum(Ctx* C, OpSetImpl& S, int side, int kind, void* stream) {
    S = OpSetImpl();
    S.basis.q = {QN(0, 0)};
    S.basis.m = {1};
    S.basis.total = 1;
    S.side = side;
    S.kind = kind;
    S.add_op('H', -1, -1, QN(0, 0), 0);
    const int n = 2 * C->K;
    for (int p = 0; p < n; ++p) S.add_op('R', p, -1, -qe(p), 1);
    if (kind == 1) {
        for (int p = 0; p < n; ++p)
            for (int r = p + 1; r < n; ++r)
                if (C->pair_needed(p >> 1, r >> 1)) S.add_op('D', p, r, qe(p) + qe(r), 0);
        for (int p = 0; p < n; ++p)
            for (int q = 0; q < n; ++q)
                if (C->pair_needed(p >> 1, q >> 1)) S.add_op('Q', p, q, qe(q) - qe(p), 0);
    }
    dmrg_status st = alloc_set(C, S);
    if (st != DMRG_OK) return st;
    if (!C->dry) DMRG_HIP(hipMemsetAsync(S.dev, 0, (size_t)std::max<int64_t>(S.elems, 1) * 8, (hipStream_t)stream));
    return DMRG_OK;
}

}  // namespace dmrg

// ===========================================================================
// C ABI
// ===========================================================================
using namespace dmrg;

extern "C" {

const char* dmrg_status_string(dmrg_status s) {
    switch (s) {
        case DMRG_OK: return "ok";
        case DMRG_E_ARG: return "invalid argument";
        case DMRG_E_SYMMETRY: return "integral symmetry violated";
        case DMRG_E_WORKSPACE: return "arena too small";
        case DMRG_E_HIP: return "HIP error";
        case DMRG_E_NONFINITE: return "non-finite value";
        case DMRG_E_STATE: return "call out of order";
        case DMRG_E_UNSUPPORTED: return "unsupported size";
        default: return "unknown status";
    }
}

dmrg_status dmrg_create(dmrg_ctx** out, int32_t device, void* arena, int64_t arena_bytes) {
    if (!out) return fail(DMRG_E_ARG, "out is null");
    *out = nullptr;
    if (!arena || arena_bytes < (1 << 20)) return fail(DMRG_E_ARG, "arena must be at least 1 MiB");
    DMRG_HIP(hipSetDevice(device));
    dmrg_ctx* c = new dmrg_ctx();
    c->device = device;
    c->arena.init(arena, arena_bytes);
    *out = c;
    return DMRG_OK;
}

void dmrg_destroy(dmrg_ctx* ctx) {
    if (!ctx) return;
    release_solver(ctx);
    delete ctx;
}

int64_t dmrg_arena_used(const dmrg_ctx* ctx) { return ctx ? ctx->arena.used : 0; }
int64_t dmrg_arena_peak(const dmrg_ctx* ctx) { return ctx ? ctx->arena.peak : 0; }

static int proc1(int p, int i, int P) { return ((i - p) % P + P) % P == 0; }
static int proc2(int p, int i, int j, int P) {
    if (i > j) std::swap(i, j);
    const long long x = (long long)(j - 1) * j / 2 + i - p;
    return ((x % P) + P) % P == 0;
}

// Sub-Hamiltonian proc_id (1-based) of n_proc with the NC assignment
// (Section II.B): t_ij scaled by [proc(p,i) + proc(p,j)] / 2, v_ijkl kept when
// the sorted tuple is owned (proc(p, j) if j = k, else proc(p, i, j)).
static void apply_share_mask(Ctx* ctx) {
    const int K = ctx->K, n_proc = ctx->n_proc, proc_id = ctx->proc_id;
    if (n_proc <= 1) return;
    const size_t K1 = K;
    for (int i = 0; i < K; ++i)
        for (int j = 0; j < K; ++j)
            ctx->h[i * K1 + j] *= 0.5 * (proc1(proc_id, i + 1, n_proc) + proc1(proc_id, j + 1, n_proc));
    for (int i = 0; i < K; ++i)
        for (int j = 0; j < K; ++j)
            for (int k = 0; k < K; ++k)
                for (int l = 0; l < K; ++l) {
                    int s[4] = {i + 1, j + 1, k + 1, l + 1};
                    std::sort(s, s + 4);
                    const int own = (s[1] == s[2]) ? proc1(proc_id, s[1], n_proc) : proc2(proc_id, s[0], s[1], n_proc);
                    if (!own) ctx->g[((i * K1 + j) * K1 + k) * K1 + l] = 0.0;
                }
}

dmrg_status dmrg_set_integrals(dmrg_ctx* ctx, int32_t K, int32_t n_elec, int32_t two_sz, const double* h1e,
                               const double* g2e, double e_core, int32_t n_proc, int32_t proc_id) {
    if (!ctx || !h1e || !g2e) return fail(DMRG_E_ARG, "null argument");
    if (K < 4 || K > 512) return fail(DMRG_E_ARG, "K must satisfy 4 <= K <= 512");
    if ((n_elec + two_sz) % 2 || n_elec < 0 || std::abs(two_sz) > n_elec || n_elec > 2 * K)
        return fail(DMRG_E_ARG, "inconsistent n_elec / two_sz");
    if (n_proc < 1 || proc_id < 1 || proc_id > n_proc) return fail(DMRG_E_ARG, "bad n_proc / proc_id");
    const size_t K1 = K;
    for (int i = 0; i < K; ++i)
        for (int j = 0; j < K; ++j)
            if (std::fabs(h1e[i * K1 + j] - h1e[j * K1 + i]) > 1e-12)
                return fail(DMRG_E_SYMMETRY, "h1e not symmetric");
    auto G = [&](int i, int j, int k, int l) { return g2e[((i * K1 + j) * K1 + k) * K1 + l]; };
    for (int i = 0; i < K; ++i)
        for (int j = 0; j < K; ++j)
            for (int k = 0; k < K; ++k)
                for (int l = 0; l < K; ++l) {
                    const double x = G(i, j, k, l);
                    if (std::fabs(x - G(j, i, k, l)) > 1e-12 || std::fabs(x - G(i, j, l, k)) > 1e-12 ||
                        std::fabs(x - G(k, l, i, j)) > 1e-12)
                        return fail(DMRG_E_SYMMETRY, "g2e not 8-fold symmetric");
                }
    ctx->K = K;
    ctx->na = (n_elec + two_sz) / 2;
    ctx->nb = (n_elec - two_sz) / 2;
    ctx->e_core = e_core;
    ctx->n_proc = n_proc;
    ctx->proc_id = proc_id;
    ctx->h.assign(h1e, h1e + K1 * K1);
    ctx->g.assign(g2e, g2e + K1 * K1 * K1 * K1);
    apply_share_mask(ctx);
    ctx->has_ints = true;
    return DMRG_OK;
}

dmrg_status dmrg_build_block(dmrg_ctx* ctx, int32_t side, int32_t n_sites, const dmrg_bsm* isometries,
                             int32_t scheme, dmrg_opset** out, void* stream) {
    if (!ctx || !out || !isometries) return fail(DMRG_E_ARG, "null argument");
    *out = nullptr;
    if (!ctx->has_ints) return fail(DMRG_E_STATE, "integrals not set");
    if (side != DMRG_LEFT && side != DMRG_RIGHT) return fail(DMRG_E_ARG, "bad side");
    if (n_sites < 1 || n_sites > ctx->K - 2) return fail(DMRG_E_ARG, "bad n_sites");
    if (scheme != DMRG_SCHEME_NC && scheme != DMRG_SCHEME_CN) return fail(DMRG_E_ARG, "bad scheme");
    const int kind = (side == DMRG_RIGHT && scheme == DMRG_SCHEME_NC) ? 1 : 0;
    OpSetImpl cur;
    dmrg_status st = vacuum(ctx, cur, side, kind, stream);
    if (st != DMRG_OK) return st;
    for (int m = 0; m < TM_N; ++m) ctx->tm[m] = 0.0;
    for (int j = 0; j < n_sites; ++j) {
        OpSetImpl nw;
        st = grow_step(ctx, cur, &isometries[j], nw, stream);
        if (st != DMRG_OK) {
            free_set(ctx, cur);
            free_set(ctx, nw);
            return st;
        }
        if (std::getenv("DMRG_VERBOSE")) {
            size_t nops = 0;
            for (auto& F : nw.fams) nops += F.keys.size();
            std::fprintf(stderr, "[dmrg] %s site %d: M=%lld sectors=%d ops=%zu set=%.2f GB arena=%.2f GB peak=%.2f GB"
                                 " | cumulative s: grow %.2f plan %.2f wsum host %.2f dev %.2f renorm host %.2f dev %.2f\n",
                         side == DMRG_LEFT ? "left" : "right", j, (long long)nw.basis.total, nw.basis.size(), nops,
                         nw.elems * 8.0 / 1e9, ctx->arena.used / 1e9, ctx->arena.peak / 1e9, ctx->tm[TM_GROW],
                         ctx->tm[TM_PLAN], ctx->tm[TM_WSUM_HOST], ctx->tm[TM_WSUM_DEV], ctx->tm[TM_REN_HOST],
                         ctx->tm[TM_REN_DEV]);
        }
        free_set(ctx, cur);
        cur = std::move(nw);
    }
    dmrg_opset* o = new dmrg_opset();
    static_cast<OpSetImpl&>(*o) = std::move(cur);
    o->ctx = ctx;
    *out = o;
    return DMRG_OK;
}

dmrg_status dmrg_normal_to_complementary(dmrg_ctx* ctx, dmrg_opset* right, void* stream) {
    if (!ctx || !right) return fail(DMRG_E_ARG, "null argument");
    if (right->side != DMRG_RIGHT || right->kind != 0) return fail(DMRG_E_ARG, "needs a normal right block");
    const int K = ctx->K;
    const int first = K - right->nsites;
    std::vector<int> before;
    for (int p = 0; p < 2 * first; ++p) before.push_back(p);
    OpSetImpl nw;
    nw.basis = right->basis;
    nw.side = DMRG_RIGHT;
    nw.kind = 1;
    nw.orbs = right->orbs;
    nw.nsites = right->nsites;
    // copied families (same order => one copy per family)
    std::vector<std::pair<int, int>> copies;
    for (size_t f = 0; f < right->fams.size(); ++f) {
        const Family& F = right->fams[f];
        if (F.kind != 'H' && F.kind != 'C' && F.kind != 'R') continue;
        int nf = -1;
        for (int64_t key : F.keys) {
            const int p = (int)((key >> 20) & 0xFFFFF) - 1, q = (int)(key & 0xFFFFF) - 1;
            nf = nw.add_op(F.kind, p, q, F.dq, F.par);
        }
        copies.push_back({(int)f, nf});
    }
    for (int p : before)
        for (int r : before)
            if (p < r && ctx->pair_needed(p >> 1, r >> 1)) nw.add_op('D', p, r, qe(p) + qe(r), 0);
    for (int p : before)
        for (int q : before)
            if (ctx->pair_needed(p >> 1, q >> 1)) nw.add_op('Q', p, q, qe(q) - qe(p), 0);
    dmrg_status st = alloc_set(ctx, nw);
    if (st != DMRG_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    for (auto& cp : copies) {
        const Family& A = right->fams[cp.first];
        const Family& B = nw.fams[cp.second];
        if (A.keys.size() != B.keys.size() || A.stride != B.stride) {
            free_set(ctx, nw);
            return fail(DMRG_E_STATE, "family copy mismatch");
        }
        if (A.stride * (int64_t)A.keys.size() > 0 && !ctx->dry)
            DMRG_HIP(hipMemcpyAsync(nw.dev + B.base, right->dev + A.base, A.stride * A.keys.size() * 8,
                                    hipMemcpyDeviceToDevice, s));
    }
    for (size_t f = 0; f < nw.fams.size(); ++f) {
        const Family& D = nw.fams[f];
        if (D.kind != 'Q' && D.kind != 'D') continue;
        const char in_kind = D.kind == 'Q' ? 'B' : 'A';
        int sf = -1;
        for (size_t g = 0; g < right->fams.size(); ++g)
            if (right->fams[g].kind == in_kind && right->fams[g].dq == D.dq) sf = (int)g;
        if (sf < 0) {
            if (D.stride * (int64_t)D.keys.size() > 0 && !ctx->dry)
                DMRG_HIP(hipMemsetAsync(nw.dev + D.base, 0, D.stride * D.keys.size() * 8, s));
            continue;
        }
        const Family& S = right->fams[sf];
        std::vector<double> W((size_t)D.keys.size() * S.keys.size(), 0.0);
        for (size_t i = 0; i < D.keys.size(); ++i) {
            const int p = (int)((D.keys[i] >> 20) & 0xFFFFF) - 1, q = (int)(D.keys[i] & 0xFFFFF) - 1;
            for (size_t k = 0; k < S.keys.size(); ++k) {
                const int r = (int)((S.keys[k] >> 20) & 0xFFFFF) - 1, t = (int)(S.keys[k] & 0xFFFFF) - 1;
                // Q_pq = sum_rs (v_pqrs - v_psrq) B_rs ;  P+_pr = sum_{q<s} (v_pqrs - v_psrq) A_qs
                W[i * S.keys.size() + k] = (D.kind == 'Q') ? ctx->v(p, q, r, t) - ctx->v(p, t, r, q)
                                                           : ctx->v(p, r, q, t) - ctx->v(p, t, q, r);
            }
        }
        st = family_gemm(ctx, W, *right, sf, nw, (int)f, 0, (int)D.keys.size(), stream);
        if (st != DMRG_OK) {
            free_set(ctx, nw);
            return st;
        }
    }
    const int e = ctx->dry ? 0 : (int)hipStreamSynchronize(s);
    if (e) return hip_fail(e, "middle transform");
    free_set(ctx, *right);
    static_cast<OpSetImpl&>(*right) = std::move(nw);
    return DMRG_OK;
}

dmrg_status dmrg_renormalize(dmrg_ctx* ctx, const dmrg_opset* in, const dmrg_bsm* isometry, dmrg_opset** out,
                             void* stream) {
    if (!ctx || !in || !isometry || !out) return fail(DMRG_E_ARG, "null argument");
    *out = nullptr;
    if (!ctx->has_ints) return fail(DMRG_E_STATE, "integrals not set");
    if (in->ctx != ctx) return fail(DMRG_E_ARG, "operator set of another context");
    if (in->kind != 0 && in->kind != 1) return fail(DMRG_E_ARG, "not a block operator set");
    if (in->nsites + 1 > ctx->K - 2) return fail(DMRG_E_ARG, "the block cannot grow past the two dots");
    OpSetImpl& cur = const_cast<dmrg_opset&>(*in);   // read only: the grown operators refer to it
    OpSetImpl nw;
    dmrg_status st = grow_step(ctx, cur, isometry, nw, stream);
    if (st != DMRG_OK) {
        free_set(ctx, nw);
        return st;
    }
    dmrg_opset* o = new dmrg_opset();
    static_cast<OpSetImpl&>(*o) = std::move(nw);
    o->ctx = ctx;
    *out = o;
    return DMRG_OK;
}

// ---------------------------------------------------------------------------
// workspace queries: the call itself, run dry (arena bookkeeping only, no
// device work) on the context's arena, whose state is restored afterwards
namespace {
struct DryScope {
    Ctx* C;
    Arena saved;
    bool was;
    explicit DryScope(Ctx* c) : C(c), saved(c->arena), was(c->dry) {
        C->dry = true;
        Arena& A = C->arena;
        const int64_t huge = int64_t(1) << 60;
        // the tail of the arena becomes unbounded, so every allocation succeeds
        int64_t tail = A.bytes;
        auto it = A.free_.empty() ? A.free_.end() : std::prev(A.free_.end());
        if (it != A.free_.end() && it->first + it->second == A.bytes) {
            tail = it->first;
            A.free_.erase(it);
        }
        A.free_[tail] = huge - tail;
        A.bytes = huge;
        A.high = 0;
        for (auto& kv : A.live_) A.high = std::max(A.high, kv.first + kv.second);
    }
    ~DryScope() {
        C->arena = saved;
        C->dry = was;
    }
};

// generic nonzero integrals for a sizing run without a context: h_ij = x_i +
// x_j, g_ijkl = (x_i + x_j)(x_k + x_l), 8-fold symmetric, with no
// cancellation among the integral combinations the operators use
void generic_integrals(Ctx& c) {
    const int K = c.K;
    std::vector<double> x(K);
    for (int i = 0; i < K; ++i) x[i] = 1.0 + 0.7071067811865476 * (i + 1) + 0.013 * ((i + 1) * (i + 1) % 7);
    c.h.assign((size_t)K * K, 0.0);
    c.g.assign((size_t)K * K * K * K, 0.0);
    for (int i = 0; i < K; ++i)
        for (int j = 0; j < K; ++j) c.h[(size_t)i * K + j] = x[i] + x[j];
    for (int i = 0; i < K; ++i)
        for (int j = 0; j < K; ++j)
            for (int k = 0; k < K; ++k)
                for (int l = 0; l < K; ++l)
                    c.g[(((size_t)i * K + j) * K + k) * K + l] = (x[i] + x[j]) * (x[k] + x[l]);
}
}  // namespace

dmrg_status dmrg_query_workspace(const dmrg_ctx* cctx, int32_t what, const void* args, int64_t* bytes) {
    if (!args || !bytes) return fail(DMRG_E_ARG, "null argument");
    *bytes = 0;
    dmrg_ctx* ctx = const_cast<dmrg_ctx*>(cctx);
    dmrg_ctx local;
    if (!ctx) {
        if (what != DMRG_WS_BLOCK && what != DMRG_WS_DAVIDSON)
            return fail(DMRG_E_ARG, "this query needs the context of the operator sets");
        local.arena.init(reinterpret_cast<void*>(uintptr_t(1) << 12), 0);
        ctx = &local;
        if (what == DMRG_WS_BLOCK) {
            const dmrg_ws_block* a = (const dmrg_ws_block*)args;
            if (a->K < 4 || a->K > 512) return fail(DMRG_E_ARG, "K must satisfy 4 <= K <= 512");
            if ((a->n_elec + a->two_sz) % 2 || a->n_elec < 0 || std::abs(a->two_sz) > a->n_elec)
                return fail(DMRG_E_ARG, "inconsistent n_elec / two_sz");
            if (a->n_proc < 1 || a->proc_id < 1 || a->proc_id > a->n_proc)
                return fail(DMRG_E_ARG, "bad n_proc / proc_id");
            local.K = a->K;
            local.na = (a->n_elec + a->two_sz) / 2;
            local.nb = (a->n_elec - a->two_sz) / 2;
            local.n_proc = a->n_proc;
            local.proc_id = a->proc_id;
            generic_integrals(local);
            apply_share_mask(&local);
            local.has_ints = true;
        }
    }
    DryScope dry(ctx);
    dmrg_status st = DMRG_OK;
    switch (what) {
        case DMRG_WS_BLOCK: {
            const dmrg_ws_block* a = (const dmrg_ws_block*)args;
            dmrg_opset* o = nullptr;
            st = dmrg_build_block(ctx, a->side, a->n_sites, a->isometries, a->scheme, &o, nullptr);
            dmrg_opset_free(o);
            break;
        }
        case DMRG_WS_TRANSFORM: {
            const dmrg_ws_transform* a = (const dmrg_ws_transform*)args;
            if (!a->right) return fail(DMRG_E_ARG, "null argument");
            dmrg_opset copy;
            static_cast<OpSetImpl&>(copy) = static_cast<const OpSetImpl&>(*a->right);
            copy.ctx = ctx;
            st = dmrg_normal_to_complementary(ctx, &copy, nullptr);
            free_set(ctx, copy);
            break;
        }
        case DMRG_WS_HEFF: {
            const dmrg_ws_heff* a = (const dmrg_ws_heff*)args;
            dmrg_heff* H = nullptr;
            st = dmrg_heff_create(ctx, a->left, a->right, nullptr, a->n_roots, a->precision, 0, &H, nullptr);
            dmrg_heff_free(H);
            break;
        }
        case DMRG_WS_DAVIDSON: {
            const dmrg_ws_davidson* a = (const dmrg_ws_davidson*)args;
            if (a->dim < 1 || a->n_roots < 1 || a->n_roots > 16) return fail(DMRG_E_ARG, "bad dim / n_roots");
            if (ctx->arena.alloc(dav_workspace_bytes(a->dim, a->n_roots, &a->opts)) < 0)
                st = fail(DMRG_E_WORKSPACE, "dry run");
            break;
        }
        case DMRG_WS_RENORMALIZE: {
            const dmrg_ws_renorm* a = (const dmrg_ws_renorm*)args;
            dmrg_opset* o = nullptr;
            st = dmrg_renormalize(ctx, a->in, a->isometry, &o, nullptr);
            dmrg_opset_free(o);
            break;
        }
        default:
            return fail(DMRG_E_ARG, "unknown workspace query");
    }
    if (st != DMRG_OK) return st;
    *bytes = ctx->arena.high;
    return DMRG_OK;
}

int32_t dmrg_opset_basis(const dmrg_opset* s, int32_t n, int32_t* qn, int64_t* dims) {
    if (!s) return -1;
    const int ns = s->basis.size();
    for (int i = 0; i < ns && i < n; ++i) {
        if (qn) { qn[2 * i] = s->basis.q[i].a; qn[2 * i + 1] = s->basis.q[i].b; }
        if (dims) dims[i] = s->basis.m[i];
    }
    return ns;
}

dmrg_status dmrg_opset_block(const dmrg_opset* s, char kind, int32_t p, int32_t q, const int32_t* qn_ket,
                             double* out, int64_t out_elems) {
    if (!s || !qn_ket || !out) return fail(DMRG_E_ARG, "null argument");
    auto it = s->lookup.find(okey(kind, p, q));
    if (it == s->lookup.end()) return fail(DMRG_E_ARG, "operator not present");
    const Family& F = s->fams[it->second.first];
    const Skel& S = s->skels[F.skel];
    const int k = s->basis.find(QN(qn_ket[0], qn_ket[1]));
    if (k < 0 || S.blk_of_ket[k] < 0) return fail(DMRG_E_ARG, "block not present");
    const int b = S.blk_of_ket[k];
    const int64_t n = (int64_t)s->basis.m[S.bra[b]] * s->basis.m[k];
    if (out_elems < n) return fail(DMRG_E_ARG, "output too small");
    DMRG_HIP(hipMemcpy(out, s->dev + F.base + (int64_t)it->second.second * F.stride + S.off[b], n * 8,
                       hipMemcpyDeviceToHost));
    return DMRG_OK;
}

void dmrg_opset_free(dmrg_opset* s) {
    if (!s) return;
    if (s->ctx) free_set(s->ctx, *s);
    delete s;
}

}  // extern "C"
