"""O2 -- renormalized-operator oracle (plain NumPy FP64).  TEST INFRASTRUCTURE ONLY.

Follows the paper's serial algorithm (Appendix A) in its three steps,
with every operator kept as a dictionary of dense sector blocks:

1. blocking (Appendix A, blocking formula): an operator of a block grown by
   one site is a sum of products (old-block operator) x (site operator); each
   product is *materialised* as a matrix on the enlarged basis;
2. transformation (Appendix A, operator transformation): O_new = U^T O U per
   sector, U the site isometry;
3. solving: H_eff psi = sum over the normal/complementary terms of the
   left-right decomposition (Appendix B, NC partition; written here in the
   non-spin-adapted form) of X^{L'} (P^{pi(Y)} Psi) Y^{R'T}.

No product of two renormalized operators of one block is ever formed, so the
result equals W^T H W psi also when the bases are truncated.

Sign rule.  For a bipartition X|Y (X first in the Jordan-Wigner order) and a
product O = O_X O_Y, <x'y'|O|xy> = (-1)^{pi(O_Y) n(x)} <x'|O_X|x> <y'|O_Y|y>,
with the product state |x>|y> = (x creation string)(y creation string)|0>.

Non-spin-adapted operators (spin-orbitals p,q,r,s; t and v spin-resolved):
  C_p = a+_p, D_p = a_p, A_pr = a+_p a+_r, B_pq = a+_p a_q
  R^S_p = 1/2 sum_{q in S} t_pq a_q + sum_{qrs in S} v_pqrs a+_r a_s a_q
  P^S_pr = sum_{qs in S} v_pqrs a_s a_q
  Q^S_pq = sum_{rs in S} (v_pqrs - v_psrq) a+_r a_s
  H = H^L + H^R + sum_{p in L}(C_p R^R_p - D_p R^R_p+) + sum_{p in R}(R^L_p+ D_p - R^L_p C_p)
        + sum_{p<r in L}(A_pr P^R_pr + h.c.) + sum_{pq in L} B_pq Q^R_pq
The one-body term is split as 1/2 t into each one-index complementary
operator; these forms are pinned against O1 (fci) in the tests.
"""
from __future__ import annotations

from typing import Dict, List, Optional, Tuple

import numpy as np

Q = Tuple[int, int]
SITE_Q: Tuple[Q, ...] = ((0, 0), (1, 0), (0, 1), (1, 1))
ZQ: Q = (0, 0)


def qadd(a, b):
    return (a[0] + b[0], a[1] + b[1])


def qneg(a):
    return (-a[0], -a[1])


def e(p: int) -> Q:
    """Quantum number of one electron in spin-orbital p."""
    return (1, 0) if p % 2 == 0 else (0, 1)


# ---------------------------------------------------------------------------
# block-sparse operators
# ---------------------------------------------------------------------------

class Op:
    """Operator with definite shift dq and parity; blocks[q_ket] is m_{q+dq} x m_q."""

    __slots__ = ("dq", "par", "blocks")

    def __init__(self, dq: Q, par: int, blocks: Optional[Dict[Q, np.ndarray]] = None):
        self.dq = dq
        self.par = par
        self.blocks = blocks if blocks is not None else {}

    @property
    def T(self) -> "Op":
        return Op(qneg(self.dq), self.par,
                  {qadd(q, self.dq): b.T for q, b in self.blocks.items()})

    def scaled(self, c: float) -> "Op":
        return Op(self.dq, self.par, {q: c * b for q, b in self.blocks.items()})

    def __add__(self, other: "Op") -> "Op":
        assert self.dq == other.dq and self.par == other.par
        out = {q: b.copy() for q, b in self.blocks.items()}
        for q, b in other.blocks.items():
            out[q] = out[q] + b if q in out else b.copy()
        return Op(self.dq, self.par, out)

    def __sub__(self, other):
        return self + other.scaled(-1.0)


def identity(basis: Dict[Q, int]) -> Op:
    return Op(ZQ, 0, {q: np.eye(m) for q, m in basis.items()})


def weighted_sums(W: np.ndarray, ops: List[Op], dq: Q, par: int) -> List[Op]:
    """[sum_k W[i,k] ops[k] for each row i] (all ops share dq and parity)."""
    keys = set()
    for o in ops:
        assert o.dq == dq and o.par == par
        keys.update(o.blocks)
    outs = [dict() for _ in range(W.shape[0])]
    for q in keys:
        shape = None
        for o in ops:
            if q in o.blocks:
                shape = o.blocks[q].shape
                break
        stack = np.stack([o.blocks[q] if q in o.blocks else np.zeros(shape) for o in ops])
        res = np.tensordot(W, stack, axes=(1, 0))
        for i in range(W.shape[0]):
            outs[i][q] = res[i]
    return [Op(dq, par, b) for b in outs]


# ---------------------------------------------------------------------------
# the site: 4x4 matrices on |0>, |a>, |b>, |ab> = a+_a a+_b |0>
# ---------------------------------------------------------------------------

def _site_c() -> Tuple[np.ndarray, np.ndarray]:
    ca = np.zeros((4, 4))
    cb = np.zeros((4, 4))
    ca[1, 0] = 1.0      # |0>  -> |a>
    ca[3, 2] = 1.0      # |b>  -> a+_a a+_b |0> = |ab>
    cb[2, 0] = 1.0      # |0>  -> |b>
    cb[3, 1] = -1.0     # |a>  -> a+_b a+_a |0> = -|ab>
    return ca, cb


SITE_BASIS: Dict[Q, int] = {q: 1 for q in SITE_Q}


def site_op(M: np.ndarray, dq: Q, par: int) -> Op:
    """Op on the site basis from a 4x4 matrix that shifts by dq."""
    blocks = {}
    for s, qs in enumerate(SITE_Q):
        qb = qadd(qs, dq)
        if qb in SITE_Q:
            sb = SITE_Q.index(qb)
            if M[sb, s] != 0.0:
                blocks[qs] = np.array([[M[sb, s]]])
    # every nonzero must be compatible with dq
    for sb in range(4):
        for s in range(4):
            if M[sb, s] != 0.0:
                assert qadd(SITE_Q[s], dq) == SITE_Q[sb], "site op breaks its shift"
    return Op(dq, par, blocks)


class Integrals:
    """Spin-orbital view of spatial (h, g) with t and v as in Appendix B."""

    def __init__(self, h: np.ndarray, g: np.ndarray):
        self.h = h
        self.g = g
        K = h.shape[0]
        self.K = K
        n = 2 * K
        self.t = np.zeros((n, n))
        self.v = np.zeros((n, n, n, n))
        for s in range(2):
            self.t[s::2, s::2] = h
            for s2 in range(2):
                self.v[s::2, s::2, s2::2, s2::2] = g


class Site:
    """Exact 4x4 operators of spatial site n (spin-orbitals 2n, 2n+1)."""

    def __init__(self, n: int, ints: Integrals):
        self.n = n
        self.ints = ints
        ca, cb = _site_c()
        self.c = {2 * n: ca, 2 * n + 1: cb}
        self.d = {p: m.T for p, m in self.c.items()}
        self.orbs = [2 * n, 2 * n + 1]

    def C(self, p):
        return site_op(self.c[p], e(p), 1)

    def D(self, p):
        return site_op(self.d[p], qneg(e(p)), 1)

    def A(self, p, r):
        return site_op(self.c[p] @ self.c[r], qadd(e(p), e(r)), 0)

    def B(self, p, q):
        return site_op(self.c[p] @ self.d[q], qadd(e(p), qneg(e(q))), 0)

    def H(self):
        t, v = self.ints.t, self.ints.v
        M = np.zeros((4, 4))
        for p in self.orbs:
            for q in self.orbs:
                M += t[p, q] * self.c[p] @ self.d[q]
                for r in self.orbs:
                    for s in self.orbs:
                        M += 0.5 * v[p, q, r, s] * self.c[p] @ self.c[r] @ self.d[s] @ self.d[q]
        return site_op(M, ZQ, 0)

    def R(self, p):
        t, v = self.ints.t, self.ints.v
        M = np.zeros((4, 4))
        for q in self.orbs:
            M += 0.5 * t[p, q] * self.d[q]
            for r in self.orbs:
                for s in self.orbs:
                    M += v[p, q, r, s] * self.c[r] @ self.d[s] @ self.d[q]
        return site_op(M, qneg(e(p)), 1)

    def P(self, p, r):
        v = self.ints.v
        M = np.zeros((4, 4))
        for q in self.orbs:
            for s in self.orbs:
                M += v[p, q, r, s] * self.d[s] @ self.d[q]
        return site_op(M, qneg(qadd(e(p), e(r))), 0)

    def Qc(self, p, q):
        v = self.ints.v
        M = np.zeros((4, 4))
        for r in self.orbs:
            for s in self.orbs:
                M += (v[p, q, r, s] - v[p, s, r, q]) * self.c[r] @ self.d[s]
        return site_op(M, qadd(e(q), qneg(e(p))), 0)


# ---------------------------------------------------------------------------
# enlarged basis and the materialised product
# ---------------------------------------------------------------------------

class Enlarged:
    """Basis of a block grown by one site, segments ordered by site state.

    ``site_first`` False: old block then site (left block grows at its right
    end); True: site then old block (right block grows at its left end).
    Each sector q holds segments (qx, qy, dx, dy, offset) where x is the
    first part and y the second.
    """

    def __init__(self, old: Dict[Q, int], site_first: bool):
        self.site_first = site_first
        self.segs: Dict[Q, List[Tuple[Q, Q, int, int, int]]] = {}
        acc: Dict[Q, List] = {}
        for s, qs in enumerate(SITE_Q):
            for qo, m in sorted(old.items()):
                q = qadd(qo, qs)
                if site_first:
                    acc.setdefault(q, []).append((s, qs, qo, 1, m))
                else:
                    acc.setdefault(q, []).append((s, qo, qs, m, 1))
        for q in sorted(acc):
            off = 0
            lst = []
            for (s, qx, qy, dx, dy) in sorted(acc[q], key=lambda t: t[0]):
                lst.append((qx, qy, dx, dy, off))
                off += dx * dy
            self.segs[q] = lst
        self.dims = {q: sum(dx * dy for (_, _, dx, dy, _) in l) for q, l in self.segs.items()}

    def kron(self, A: Op, B: Op) -> Op:
        """Materialise the product (A on the first part)(B on the second part)."""
        dq = qadd(A.dq, B.dq)
        out = {}
        for q, segs in self.segs.items():
            qb = qadd(q, dq)
            if qb not in self.segs:
                continue
            bra = {(qx, qy): off for (qx, qy, _, _, off) in self.segs[qb]}
            blk = None
            for (qx, qy, dx, dy, off) in segs:
                if qx not in A.blocks or qy not in B.blocks:
                    continue
                key = (qadd(qx, A.dq), qadd(qy, B.dq))
                if key not in bra:
                    continue
                sign = -1.0 if (B.par and (qx[0] + qx[1]) % 2) else 1.0
                sub = sign * _kron(A.blocks[qx], B.blocks[qy])
                if blk is None:
                    blk = np.zeros((self.dims[qb], self.dims[q]))
                ro = bra[key]
                blk[ro:ro + sub.shape[0], off:off + sub.shape[1]] += sub
            if blk is not None:
                out[q] = blk
        return Op(dq, (A.par + B.par) % 2, out)


def _kron(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    # one factor is a 1x1 site block, so the Kronecker product is a scaling
    if a.shape == (1, 1):
        return a[0, 0] * b
    if b.shape == (1, 1):
        return a * b[0, 0]
    return np.kron(a, b)


def ksum(enl: Enlarged, terms) -> Op:
    """sum_k c_k * (A_k x B_k) for terms (c, A, B), materialised."""
    acc = None
    for (c, A, B) in terms:
        k = enl.kron(A, B)
        if acc is None:
            acc = k.scaled(c)
            continue
        assert k.dq == acc.dq and k.par == acc.par
        for q, b in k.blocks.items():
            if q in acc.blocks:
                acc.blocks[q] += c * b
            else:
                acc.blocks[q] = c * b
    return acc


def renormalize(op: Op, U: Dict[Q, np.ndarray]) -> Op:
    """U^T O U per sector (Appendix A, operator transformation)."""
    out = {}
    for q, blk in op.blocks.items():
        qb = qadd(q, op.dq)
        if q in U and qb in U:
            out[q] = U[qb].T @ blk @ U[q]
    return Op(op.dq, op.par, out)


# ---------------------------------------------------------------------------
# blocks
# ---------------------------------------------------------------------------

class Block:
    """A block of consecutive sites with its basis and operators.

    kind 'normal': C_p, A_pr (p<r), B_pq (all p, q) for p in block, H, R_p
    for p outside.  kind 'compl' (right block only): C_p for p in block, H,
    R_p, P_pr (p<r), Q_pq for p, q before the block.
    """

    def __init__(self, basis, orbs, ops, kind):
        self.basis = basis
        self.orbs = orbs            # spin-orbitals of the block, increasing
        self.ops = ops
        self.kind = kind

    def C(self, p):
        return self.ops[("C", p)]

    def D(self, p):
        return self.ops[("C", p)].T

    def A(self, p, r):
        return self.ops[("A", p, r)]

    def B(self, p, q):
        return self.ops[("B", p, q)]

    def aa(self, s, q):
        """(a_s a_q) on the block = (a+_q a+_s)^T."""
        if s == q:
            return None
        if q < s:
            return self.ops[("A", q, s)].T
        return self.ops[("A", s, q)].T.scaled(-1.0)


def vacuum_block(K: int, left: bool) -> Block:
    basis = {ZQ: 1}
    ops = {("H",): Op(ZQ, 0, {ZQ: np.zeros((1, 1))})}
    for p in range(2 * K):
        ops[("R", p)] = Op(qneg(e(p)), 1, {})
    return Block(basis, [], ops, "normal")


def _Qw(ints, p, u, rs_pairs):
    v = ints.v
    return np.array([v[p, u, r, s] - v[p, s, r, u] for (r, s) in rs_pairs])


def _class_sums(blk: Block, ints: Integrals, outs, kind):
    """Weighted sums of a block's normal operators, grouped by shift class.

    kind 'Q': outs = [(p, u)] -> sum_{rs in block} (v_purs - v_psru) B_rs
    kind 'P': outs = [(p, r)] -> sum_{qs in block} v_pqrs (a_s a_q)
    Returns {(p, u): Op or None}.
    """
    v = ints.v
    res = {}
    orbs = blk.orbs
    if kind == "Q":
        for (p, u) in outs:
            dq = qadd(e(u), qneg(e(p)))
            keys = [(r, s) for r in orbs for s in orbs if qadd(e(r), qneg(e(s))) == dq]
            if not keys:
                res[(p, u)] = None
                continue
            w = np.array([[v[p, u, r, s] - v[p, s, r, u] for (r, s) in keys]])
            res[(p, u)] = weighted_sums(w, [blk.B(r, s) for (r, s) in keys], dq, 0)[0]
    else:
        for (p, r) in outs:
            dq = qneg(qadd(e(p), e(r)))
            keys = [(q, s) for q in orbs for s in orbs if q < s and qadd(e(q), e(s)) == qneg(dq)]
            if not keys:
                res[(p, r)] = None
                continue
            # sum_{q,s} v_pqrs a_s a_q = sum_{q<s} (v_pqrs - v_psrq) (A_qs)^T
            w = np.array([[v[p, q, r, s] - v[p, s, r, q] for (q, s) in keys]])
            res[(p, r)] = weighted_sums(w, [blk.A(q, s).T for (q, s) in keys], dq, 0)[0]
    return res


def grow_left(X: Block, site: Site, ints: Integrals, outside: List[int]):
    """NC left block X grown by site at its right end; enlarged (unrenormalized)
    operators of Z = X + site.  ``outside``: spin-orbitals p with R_p kept."""
    enl = Enlarged(X.basis, site_first=False)
    IX, IY = identity(X.basis), identity(SITE_BASIS)
    ops = {}
    zorbs = X.orbs + site.orbs
    for p in X.orbs:
        ops[("C", p)] = enl.kron(X.C(p), IY)
    for p in site.orbs:
        ops[("C", p)] = enl.kron(IX, site.C(p))
    for i, p in enumerate(zorbs):
        for r in zorbs[i + 1:]:
            if r in site.orbs and p in site.orbs:
                ops[("A", p, r)] = enl.kron(IX, site.A(p, r))
            elif r in site.orbs:
                ops[("A", p, r)] = enl.kron(X.C(p), site.C(r))
            else:
                ops[("A", p, r)] = enl.kron(X.A(p, r), IY)
    for p in zorbs:
        for q in zorbs:
            if p in site.orbs and q in site.orbs:
                ops[("B", p, q)] = enl.kron(IX, site.B(p, q))
            elif q in site.orbs:
                ops[("B", p, q)] = enl.kron(X.C(p), site.D(q))
            elif p in site.orbs:
                ops[("B", p, q)] = enl.kron(X.D(q), site.C(p)).scaled(-1.0)
            else:
                ops[("B", p, q)] = enl.kron(X.B(p, q), IY)
    # block Hamiltonian, NC form: X normal, site complementary
    terms = [(1.0, X.ops[("H",)], IY), (1.0, IX, site.H())]
    for p in X.orbs:
        Rn = site.R(p)
        terms += [(1.0, X.C(p), Rn), (-1.0, X.D(p), Rn.T)]
    for p in site.orbs:
        RX = X.ops[("R", p)]
        terms += [(1.0, RX.T, site.D(p)), (-1.0, RX, site.C(p))]
    for i, p in enumerate(X.orbs):
        for r in X.orbs[i + 1:]:
            Pn = site.P(p, r)
            terms += [(1.0, X.A(p, r), Pn), (1.0, X.A(p, r).T, Pn.T)]
    for p in X.orbs:
        for q in X.orbs:
            terms.append((1.0, X.B(p, q), site.Qc(p, q)))
    ops[("H",)] = ksum(enl, terms)
    # R_p for p after Z
    QX = _class_sums(X, ints, [(p, u) for p in outside for u in site.orbs], "Q")
    PX = _class_sums(X, ints, [(p, r) for p in outside for r in site.orbs], "P")
    for p in outside:
        terms = [(1.0, X.ops[("R", p)], IY), (1.0, IX, site.R(p))]
        for u in site.orbs:
            if QX[(p, u)] is not None:
                terms.append((1.0, QX[(p, u)], site.D(u)))
            if PX[(p, u)] is not None:
                terms.append((1.0, PX[(p, u)], site.C(u)))
        for u in X.orbs:
            terms.append((1.0, X.D(u), site.Qc(p, u)))
            terms.append((1.0, X.C(u), site.P(p, u)))
        ops[("R", p)] = ksum(enl, terms)
    return enl, Block(enl.dims, zorbs, ops, "normal")


def grow_right_normal(Y: Block, site: Site, ints: Integrals, outside: List[int]):
    """CN right block Y grown by site at its left end (Z = site + Y)."""
    enl = Enlarged(Y.basis, site_first=True)
    IX, IY = identity(SITE_BASIS), identity(Y.basis)
    ops = {}
    zorbs = site.orbs + Y.orbs
    for p in site.orbs:
        ops[("C", p)] = enl.kron(site.C(p), IY)
    for p in Y.orbs:
        ops[("C", p)] = enl.kron(IX, Y.C(p))
    for i, p in enumerate(zorbs):
        for r in zorbs[i + 1:]:
            if p in site.orbs and r in site.orbs:
                ops[("A", p, r)] = enl.kron(site.A(p, r), IY)
            elif p in site.orbs:
                ops[("A", p, r)] = enl.kron(site.C(p), Y.C(r))
            else:
                ops[("A", p, r)] = enl.kron(IX, Y.A(p, r))
    for p in zorbs:
        for q in zorbs:
            if p in site.orbs and q in site.orbs:
                ops[("B", p, q)] = enl.kron(site.B(p, q), IY)
            elif p in site.orbs:
                ops[("B", p, q)] = enl.kron(site.C(p), Y.D(q))
            elif q in site.orbs:
                ops[("B", p, q)] = enl.kron(site.D(q), Y.C(p)).scaled(-1.0)
            else:
                ops[("B", p, q)] = enl.kron(IX, Y.B(p, q))
    # block Hamiltonian, CN form: site complementary, Y normal
    terms = [(1.0, site.H(), IY), (1.0, IX, Y.ops[("H",)])]
    for p in site.orbs:
        RY = Y.ops[("R", p)]
        terms += [(1.0, site.C(p), RY), (-1.0, site.D(p), RY.T)]
    for p in Y.orbs:
        Rn = site.R(p)
        terms += [(1.0, Rn.T, Y.D(p)), (-1.0, Rn, Y.C(p))]
    for i, p in enumerate(Y.orbs):
        for r in Y.orbs[i + 1:]:
            Pn = site.P(p, r)
            terms += [(1.0, Pn, Y.A(p, r)), (1.0, Pn.T, Y.A(p, r).T)]
    for p in Y.orbs:
        for q in Y.orbs:
            terms.append((1.0, site.Qc(p, q), Y.B(p, q)))
    ops[("H",)] = ksum(enl, terms)
    QY = _class_sums(Y, ints, [(p, u) for p in outside for u in site.orbs], "Q")
    PY = _class_sums(Y, ints, [(p, r) for p in outside for r in site.orbs], "P")
    for p in outside:
        terms = [(1.0, site.R(p), IY), (1.0, IX, Y.ops[("R", p)])]
        for u in Y.orbs:
            terms.append((1.0, site.Qc(p, u), Y.D(u)))
            terms.append((1.0, site.P(p, u), Y.C(u)))
        for u in site.orbs:
            if QY[(p, u)] is not None:
                terms.append((1.0, site.D(u), QY[(p, u)]))
            if PY[(p, u)] is not None:
                terms.append((1.0, site.C(u), PY[(p, u)]))
        ops[("R", p)] = ksum(enl, terms)
    return enl, Block(enl.dims, zorbs, ops, "normal")


def _cP(Y: Block, p, r):
    """P_pr of a complementary block for any order (P_rp = -P_pr, P_pp = 0)."""
    if p == r:
        return None
    if p < r:
        return Y.ops[("P", p, r)]
    return Y.ops[("P", r, p)].scaled(-1.0)


def grow_right_compl(Y: Block, site: Site, ints: Integrals, before: List[int]):
    """Complementary right block Y grown by site at its left end (Z = site + Y).
    ``before``: spin-orbitals before Z (R_p, P, Q indices)."""
    enl = Enlarged(Y.basis, site_first=True)
    IX, IY = identity(SITE_BASIS), identity(Y.basis)
    v = ints.v
    ops = {}
    zorbs = site.orbs + Y.orbs
    for p in site.orbs:
        ops[("C", p)] = enl.kron(site.C(p), IY)
    for p in Y.orbs:
        ops[("C", p)] = enl.kron(IX, Y.C(p))
    # block Hamiltonian, NC form: site normal, Y complementary
    terms = [(1.0, site.H(), IY), (1.0, IX, Y.ops[("H",)])]
    for p in site.orbs:
        RY = Y.ops[("R", p)]
        terms += [(1.0, site.C(p), RY), (-1.0, site.D(p), RY.T)]
    for p in Y.orbs:
        Rn = site.R(p)
        terms += [(1.0, Rn.T, Y.D(p)), (-1.0, Rn, Y.C(p))]
    p0, p1 = site.orbs
    PY = Y.ops[("P", p0, p1)]
    terms += [(1.0, site.A(p0, p1), PY), (1.0, site.A(p0, p1).T, PY.T)]
    for p in site.orbs:
        for q in site.orbs:
            terms.append((1.0, site.B(p, q), Y.ops[("Q", p, q)]))
    ops[("H",)] = ksum(enl, terms)
    # weighted sums of Y's one-index operators
    yo = Y.orbs

    def csum(w, dq_c):
        keys = [s for s in yo if e(s) == dq_c]
        ww = np.array([[w(s) for s in keys]])
        return weighted_sums(ww, [Y.C(s) for s in keys], dq_c, 1)[0]

    for p in before:
        terms = [(1.0, site.R(p), IY), (1.0, IX, Y.ops[("R", p)])]
        for u in yo:
            terms.append((1.0, site.Qc(p, u), Y.D(u)))
            terms.append((1.0, site.P(p, u), Y.C(u)))
        for u in site.orbs:
            terms.append((1.0, site.D(u), Y.ops[("Q", p, u)]))
            Pu = _cP(Y, p, u)
            if Pu is not None:
                terms.append((1.0, site.C(u), Pu))
        ops[("R", p)] = ksum(enl, terms)
    for i, p in enumerate(before):
        for r in before[i + 1:]:
            terms = [(1.0, site.P(p, r), IY), (1.0, IX, Y.ops[("P", p, r)])]
            for u in site.orbs:
                # sum_{w in Y} (v_pwru - v_purw) D_w = (sum_w (...) C_w)^T
                dq_c = qadd(e(p), e(r))
                dq_c = qadd(dq_c, qneg(e(u)))
                if dq_c in ((1, 0), (0, 1)):
                    S = csum(lambda w: v[p, w, r, u] - v[p, u, r, w], dq_c)
                    terms.append((1.0, site.D(u), S.T))
            ops[("P", p, r)] = ksum(enl, terms)
    for p in before:
        for q in before:
            terms = [(1.0, site.Qc(p, q), IY), (1.0, IX, Y.ops[("Q", p, q)])]
            for u in site.orbs:
                # r = u in site: sum_{s in Y} (v_pqus - v_psuq) D_s
                dq_c = qadd(qadd(e(p), qneg(e(q))), e(u))
                if dq_c in ((1, 0), (0, 1)):
                    S = csum(lambda s: v[p, q, u, s] - v[p, s, u, q], dq_c)
                    terms.append((1.0, site.C(u), S.T))
                # s = u in site: -sum_{r in Y} (v_pqru - v_purq) C_r
                dq_c2 = qadd(qadd(e(q), qneg(e(p))), e(u))
                if dq_c2 in ((1, 0), (0, 1)):
                    S2 = csum(lambda r: v[p, q, r, u] - v[p, u, r, q], dq_c2)
                    terms.append((-1.0, site.D(u), S2))
            ops[("Q", p, q)] = ksum(enl, terms)
    return enl, Block(enl.dims, zorbs, ops, "compl")


def vacuum_compl(before: List[int]) -> Block:
    basis = {ZQ: 1}
    ops = {("H",): Op(ZQ, 0, {ZQ: np.zeros((1, 1))})}
    for p in before:
        ops[("R", p)] = Op(qneg(e(p)), 1, {})
    for i, p in enumerate(before):
        for r in before[i + 1:]:
            ops[("P", p, r)] = Op(qneg(qadd(e(p), e(r))), 0, {})
    for p in before:
        for q in before:
            ops[("Q", p, q)] = Op(qadd(e(q), qneg(e(p))), 0, {})
    return Block(basis, [], ops, "compl")


def to_complementary(Y: Block, ints: Integrals, before: List[int]) -> Block:
    """Normal -> complementary transform of a right block (mixed NC/CN middle):
    Q_pq = sum_{rs in Y}(v_pqrs - v_psrq) B_rs, P_pr = sum_{qs in Y} v_pqrs a_s a_q."""
    ops = {("H",): Y.ops[("H",)]}
    for p in Y.orbs:
        ops[("C", p)] = Y.ops[("C", p)]
    for p in before:
        ops[("R", p)] = Y.ops[("R", p)]
    QY = _class_sums(Y, ints, [(p, q) for p in before for q in before], "Q")
    for (p, q), o in QY.items():
        ops[("Q", p, q)] = o if o is not None else Op(qadd(e(q), qneg(e(p))), 0, {})
    pairs = [(p, r) for i, p in enumerate(before) for r in before[i + 1:]]
    PY = _class_sums(Y, ints, pairs, "P")
    for (p, r), o in PY.items():
        ops[("P", p, r)] = o if o is not None else Op(qneg(qadd(e(p), e(r))), 0, {})
    return Block(Y.basis, Y.orbs, ops, "compl")


def renorm_block(enl_block: Block, U: Dict[Q, np.ndarray], dims: Dict[Q, int]) -> Block:
    ops = {k: renormalize(o, U) for k, o in enl_block.ops.items()}
    return Block(dict(dims), enl_block.orbs, ops, enl_block.kind)


# ---------------------------------------------------------------------------
# the middle step
# ---------------------------------------------------------------------------

def build_left(prob, ints: Integrals, nsites: int) -> Block:
    """NC left block of sites [0, nsites) through the problem's isometries."""
    K = prob.K
    X = vacuum_block(K, True)
    for j in range(nsites):
        site = Site(j, ints)
        outside = list(range(2 * (j + 1), 2 * K))
        _, Z = grow_left(X, site, ints, outside)
        X = renorm_block(Z, prob.left_iso[j], prob.left_dims[j + 1])
    return X


def build_right(prob, ints: Integrals, nsites: int, scheme: str) -> Block:
    """Right block of sites [K-nsites, K), 'CN' (normal ops) or 'NC' (complementary)."""
    K = prob.K
    if scheme == "CN":
        Y = vacuum_block(K, False)
    else:
        Y = vacuum_compl(list(range(0, 2 * K)))
    for j in range(nsites):
        n = K - 1 - j
        site = Site(n, ints)
        before = list(range(0, 2 * n))
        if scheme == "CN":
            _, Z = grow_right_normal(Y, site, ints, before)
        else:
            _, Z = grow_right_compl(Y, site, ints, before)
        Y = renorm_block(Z, prob.right_iso[j], prob.right_dims[j + 1])
    return Y


class TwoSiteHeff:
    """H_eff of a two-site step as an explicit term list over L' x R'.

    Lb: normal left block of sites [0, KL); Rb: complementary right block of
    sites [KL + 2, K); the dots are d1 = KL and d2 = KL + 1 (Appendix A,
    effective eigenproblem, with the NC partition of Appendix B).
    """

    def __init__(self, Lb: Block, Rb: Block, ints: Integrals, KL: int, K: int, target: Q,
                 e_core: float = 0.0):
        self.ints = ints
        self.K, self.KL, self.target = K, KL, target
        d1, d2 = KL, KL + 1
        lp_orbs = list(range(0, 2 * (KL + 1)))
        rp_orbs = list(range(2 * (KL + 1), 2 * K))
        self.Lb, self.Rb = Lb, Rb
        self.lb_dims, self.rb_dims = dict(Lb.basis), dict(Rb.basis)
        self.enl_L, Lp = grow_left(Lb, Site(d1, ints), ints, rp_orbs)
        self.enl_R, Rp = grow_right_compl(Rb, Site(d2, ints), ints, lp_orbs)
        self.Lp, self.Rp = Lp, Rp
        terms = [(1.0, Lp.ops[("H",)], identity(self.enl_R.dims)),
                 (1.0, identity(self.enl_L.dims), Rp.ops[("H",)])]
        for p in lp_orbs:
            R = Rp.ops[("R", p)]
            terms += [(1.0, Lp.C(p), R), (-1.0, Lp.D(p), R.T)]
        for p in rp_orbs:
            R = Lp.ops[("R", p)]
            terms += [(1.0, R.T, Rp.D(p)), (-1.0, R, Rp.C(p))]
        for i, p in enumerate(lp_orbs):
            for r in lp_orbs[i + 1:]:
                P = Rp.ops[("P", p, r)]
                terms += [(1.0, Lp.A(p, r), P), (1.0, Lp.A(p, r).T, P.T)]
        for p in lp_orbs:
            for q in lp_orbs:
                terms.append((1.0, Lp.B(p, q), Rp.ops[("Q", p, q)]))
        self.terms = terms
        self.e_core = e_core
        self._layout()

    def _layout(self):
        lb, rb = self.lb_dims, self.rb_dims
        tgt = self.target
        self.blocks = []
        off = 0
        loff = {}
        for QL, segs in self.enl_L.segs.items():
            for (qa, qs, dx, dy, o) in segs:
                loff[(qa, qs)] = (QL, o)
        roff = {}
        for QR, segs in self.enl_R.segs.items():
            for (qs, qb, dx, dy, o) in segs:
                roff[(qs, qb)] = (QR, o)
        for a in sorted(lb):
            for s1, q1 in enumerate(SITE_Q):
                for s2, q2 in enumerate(SITE_Q):
                    b = (tgt[0] - a[0] - q1[0] - q2[0], tgt[1] - a[1] - q1[1] - q2[1])
                    if b in rb:
                        QL, ro = loff[(a, q1)]
                        QR, co = roff[(q2, b)]
                        self.blocks.append((QL, QR, ro, co, lb[a], rb[b], off))
                        off += lb[a] * rb[b]
        self.dim = off

    def to_matrix(self, psi):
        M = {}
        for (QL, QR, ro, co, ma, mb, off) in self.blocks:
            if (QL, QR) not in M:
                M[(QL, QR)] = np.zeros((self.enl_L.dims[QL], self.enl_R.dims[QR]))
            M[(QL, QR)][ro:ro + ma, co:co + mb] = psi[off:off + ma * mb].reshape(ma, mb)
        return M

    def from_matrix(self, M):
        out = np.zeros(self.dim)
        for (QL, QR, ro, co, ma, mb, off) in self.blocks:
            if (QL, QR) in M:
                out[off:off + ma * mb] = M[(QL, QR)][ro:ro + ma, co:co + mb].ravel()
        return out

    def apply(self, psi: np.ndarray, terms=None) -> np.ndarray:
        """sigma = sum_terms X (P^{pi(Y)} Psi) Y^T (+ e_core psi)."""
        Psi = self.to_matrix(psi)
        S: Dict[Tuple[Q, Q], np.ndarray] = {}
        for (c, X, Y) in (self.terms if terms is None else terms):
            for (QL, QR), blk in Psi.items():
                if QL not in X.blocks or QR not in Y.blocks:
                    continue
                QL2, QR2 = qadd(QL, X.dq), qadd(QR, Y.dq)
                sign = -1.0 if (Y.par and (QL[0] + QL[1]) % 2) else 1.0
                contrib = (c * sign) * (X.blocks[QL] @ blk @ Y.blocks[QR].T)
                key = (QL2, QR2)
                S[key] = S[key] + contrib if key in S else contrib
        out = self.from_matrix(S)
        if self.e_core:
            out = out + self.e_core * psi
        return out


class MiddleHeff(TwoSiteHeff):
    """H_eff of the middle step of a problem (dots K/2 - 1, K/2), with the
    right block built in the NC scheme or in the CN scheme and then turned
    complementary (Section III.A)."""

    def __init__(self, prob, scheme: str = "CN", h1e=None, g2e=None):
        self.prob = prob
        h = prob.h1e if h1e is None else h1e
        g = prob.g2e if g2e is None else g2e
        ints = Integrals(h, g)
        K, KL = prob.K, prob.KL
        Lb = build_left(prob, ints, KL)
        Rb = build_right(prob, ints, prob.KR, scheme)
        if scheme == "CN":
            Rb = to_complementary(Rb, ints, list(range(0, 2 * (KL + 2))))
        super().__init__(Lb, Rb, ints, KL, K, prob.target, prob.e_core)

    def renormalize_left(self) -> Block:
        """Post-solve renormalization of the L' operators into the next basis."""
        return renorm_block(self.Lp, self.prob.next_iso, self.prob.next_dims)
