"""O1 -- determinant-space (FCI) oracle.  TEST INFRASTRUCTURE ONLY.

What it computes, by definition:

* H = sum_pq t_pq a+_p a_q + 1/2 sum_pqrs v_pqrs a+_p a+_r a_s a_q
  (Appendix B, ab initio Hamiltonian) over spin-orbitals p = 2 i + sigma,
  with t_pq = h_ij [sigma_p = sigma_q] and
  v_pqrs = g_ijkl [sigma_p = sigma_q][sigma_r = sigma_s] (chemists' order);
* determinants are bit strings over the 2K spin-orbitals; the state of a
  bit string is the product of creation operators in increasing
  spin-orbital order acting on the vacuum;
* the two-site embedding W maps the middle-site product basis
  |a> |s1> |s2> |b> (Appendix A, two-site wavefunction) into determinant
  space; H_eff = W^T H W (Appendix A, effective Hamiltonian matrix elements).

H is applied through E_pq = a+_p a_q and the identity
a+_p a+_r a_s a_q = E_pq E_rs - delta_qr E_ps, which is exact operator algebra.
"""
from __future__ import annotations

from itertools import combinations
from typing import Dict, List, Tuple

import numpy as np

Q = Tuple[int, int]


def spin_integrals(h: np.ndarray, g: np.ndarray):
    """Spin-orbital t[p,q] and v[p,q,r,s] from spatial h, g (dense)."""
    K = h.shape[0]
    n = 2 * K
    t = np.zeros((n, n))
    v = np.zeros((n, n, n, n))
    for s in range(2):
        t[s::2, s::2] = h
        for s2 in range(2):
            v[s::2, s::2, s2::2, s2::2] = g
    return t, v


def determinants(K: int, na: int, nb: int) -> np.ndarray:
    """Sorted bit strings with na alpha (even bits) and nb beta (odd bits)."""
    out = []
    for oa in combinations(range(K), na):
        ma = sum(1 << (2 * i) for i in oa)
        for ob in combinations(range(K), nb):
            out.append(ma | sum(1 << (2 * i + 1) for i in ob))
    return np.array(sorted(out), dtype=np.int64)


def _popcount_below(d: np.ndarray, p: int) -> np.ndarray:
    mask = np.int64((1 << p) - 1)
    return np.bitwise_count(d & mask).astype(np.int64)


def excitation(dets: np.ndarray, p: int, q: int):
    """Index map of E_pq = a+_p a_q on the determinant list.

    Returns (src, dst, sign): E_pq |dets[src]> = sign |dets[dst]>.
    """
    bq = np.int64(1 << q)
    bp = np.int64(1 << p)
    occ_q = (dets & bq) != 0
    src = np.nonzero(occ_q)[0]
    d1 = dets[src] & ~bq
    s1 = _popcount_below(dets[src], q)
    ok = (d1 & bp) == 0
    src, d1, s1 = src[ok], d1[ok], s1[ok]
    s2 = _popcount_below(d1, p)
    d2 = d1 | bp
    dst = np.searchsorted(dets, d2)
    sign = np.where((s1 + s2) % 2 == 0, 1.0, -1.0)
    return src, dst, sign


class FCIHamiltonian:
    """Matrix-free H on the (N_alpha, N_beta) determinant space."""

    def __init__(self, h: np.ndarray, g: np.ndarray, na: int, nb: int, e_core: float = 0.0):
        self.K = h.shape[0]
        self.h, self.g = h, g
        self.e_core = e_core
        self.dets = determinants(self.K, na, nb)
        self.dim = self.dets.size
        n = 2 * self.K
        t, v = spin_integrals(h, g)
        self.pairs = [(p, q) for p in range(n) for q in range(n) if p % 2 == q % 2]
        self.E = [excitation(self.dets, p, q) for (p, q) in self.pairs]
        P = len(self.pairs)
        V = np.empty((P, P))
        for a, (p, q) in enumerate(self.pairs):
            for b, (r, s) in enumerate(self.pairs):
                V[a, b] = v[p, q, r, s]
        self.V = V
        # one-body coefficient after the delta_qr E_ps term: t_ps - 1/2 sum_q v_pqqs
        kmat = np.einsum('pqqs->ps', v)
        self.t1 = np.array([t[p, q] - 0.5 * kmat[p, q] for (p, q) in self.pairs])

    def _apply_E(self, a: int, x: np.ndarray) -> np.ndarray:
        src, dst, sign = self.E[a]
        y = np.zeros_like(x)
        if x.ndim == 1:
            np.add.at(y, dst, sign * x[src])
        else:
            np.add.at(y, dst, sign[:, None] * x[src])
        return y

    def matvec(self, x: np.ndarray) -> np.ndarray:
        Y = np.stack([self._apply_E(b, x) for b in range(len(self.pairs))])
        Z = np.tensordot(self.V, Y, axes=(1, 0))
        out = self.e_core * x
        for a in range(len(self.pairs)):
            out = out + self._apply_E(a, self.t1[a] * x + 0.5 * Z[a])
        return out

    def dense(self, chunk: int = 256) -> np.ndarray:
        Hm = np.empty((self.dim, self.dim))
        for c0 in range(0, self.dim, chunk):
            c1 = min(self.dim, c0 + chunk)
            X = np.zeros((self.dim, c1 - c0))
            X[np.arange(c0, c1), np.arange(c1 - c0)] = 1.0
            Hm[:, c0:c1] = self.matvec(X)
        return Hm


def fci_ground_energy(h, g, na, nb, e_core=0.0) -> float:
    """Lowest eigenvalue of the FCI matrix (LAPACK eigh on the dense matrix)."""
    H = FCIHamiltonian(h, g, na, nb, e_core)
    return float(np.linalg.eigvalsh(H.dense())[0])


# ---------------------------------------------------------------------------
# two-site embedding W
# ---------------------------------------------------------------------------

SITE_BITS = (0b00, 0b01, 0b10, 0b11)      # |0>, |a>, |b>, |ab> on one site
SITE_Q = ((0, 0), (1, 0), (0, 1), (1, 1))


def _block_states(dims_seq: List[Dict[Q, int]], isos: List[Dict[Q, np.ndarray]],
                  from_left: bool) -> Dict[Q, Dict[int, np.ndarray]]:
    """Renormalized block states as vectors over the block's own bit strings.

    Returns {q: {bitstring: row vector over the m_q states}} for the last
    block in the sequence.  Bits are relative to the block's first orbital.
    A left block grows by appending a site at its high end, a right block by
    prepending a site at its low end; in both cases the creation string of
    the product state is already in increasing order, so no sign appears.
    """
    states: Dict[Q, Dict[int, np.ndarray]] = {(0, 0): {0: np.ones(1)}}
    nsite = 0
    for j, iso in enumerate(isos):
        old = dims_seq[j]
        new: Dict[Q, Dict[int, np.ndarray]] = {}
        for q, U in iso.items():
            acc: Dict[int, np.ndarray] = {}
            row = 0
            for s, qs in enumerate(SITE_Q):
                qo = (q[0] - qs[0], q[1] - qs[1])
                if qo not in old:
                    continue
                m_old = old[qo]
                seg = U[row:row + m_old]            # m_old x m_new
                row += m_old
                for bits, vec in states[qo].items():
                    if from_left:
                        nb = bits | (SITE_BITS[s] << (2 * nsite))
                    else:
                        nb = SITE_BITS[s] | (bits << 2)
                    acc[nb] = acc.get(nb, 0.0) + vec @ seg
            assert row == U.shape[0]
            new[q] = acc
        states = new
        nsite += 1
    return states


def embedding(prob) -> Tuple[np.ndarray, np.ndarray]:
    """W (FCI dim x psi dim) for the middle step of a problem; plus dets."""
    K, KL = prob.K, prob.KL
    na, nb = prob.target
    dets = determinants(K, na, nb)
    index = {int(d): i for i, d in enumerate(dets)}
    Ls = _block_states(prob.left_dims, prob.left_iso, True)
    Rs = _block_states(prob.right_dims, prob.right_iso, False)
    lb, rb = prob.left_dims[KL], prob.right_dims[prob.KR]
    cols = []
    off = 0
    blocks = []
    for a in sorted(lb):
        for s1, q1 in enumerate(SITE_Q):
            for s2, q2 in enumerate(SITE_Q):
                b = (na - a[0] - q1[0] - q2[0], nb - a[1] - q1[1] - q2[1])
                if b in rb:
                    blocks.append((a, s1, s2, b, off))
                    off += lb[a] * rb[b]
    W = np.zeros((dets.size, off))
    shift_d1 = 2 * KL
    shift_d2 = 2 * (KL + 1)
    shift_r = 2 * (KL + 2)
    for (a, s1, s2, b, o) in blocks:
        ma, mb = lb[a], rb[b]
        for lbits, lvec in Ls[a].items():
            for rbits, rvec in Rs[b].items():
                d = lbits | (SITE_BITS[s1] << shift_d1) | (SITE_BITS[s2] << shift_d2) \
                    | (rbits << shift_r)
                W[index[d], o:o + ma * mb] += np.outer(lvec, rvec).ravel()
    return W, dets


def heff_apply_definition(prob, psi: np.ndarray, W=None, H=None) -> np.ndarray:
    """H_eff psi = W^T H W psi with H from the (possibly masked) integrals."""
    if W is None:
        W, _ = embedding(prob)
    if H is None:
        H = FCIHamiltonian(prob.h1e, prob.g2e, *prob.target, prob.e_core)
    return W.T @ H.matvec(W @ psi)
