"""Seeded synthetic inputs for the two-site DMRG middle-site step.

This module produces *inputs only*: one- and two-electron integrals, the
bond-dimension profile of the left and right blocks, the per-site isometries
(the MPS tensors A[k] of the paper's Appendix A, in left/right canonical form)
and a start wavefunction.  It holds none of the method's arithmetic (no
operators, no blocking, no renormalization, no H_eff); both the CPU oracle and
the GPU path consume what it returns.

Stand-in for the paper's benzene / FeMo-cofactor integral files (Results
section, data availability footnote), which are not available: the integrals
follow a fixed recipe with the shapes (K orbitals, N electrons, S_z) of those
systems.

Conventions (interfaces shared by every consumer):

* spatial orbital i = 0..K-1, spin-orbital p = 2*i + sigma (alpha = 0,
  beta = 1);
* sector label q = (n_alpha, n_beta);
* site basis order: |0>, |a>, |b>, |ab> with quantum numbers
  (0,0), (1,0), (0,1), (1,1);
* middle step: left block Lb = sites [0, KL), dots d1 = KL, d2 = KL + 1,
  right block Rb = [KL + 2, K) with KL = K//2 - 1;
* enlarged basis of a block grown by one site: within each sector q the
  rows are ordered by site state (0, a, b, ab), each segment holding the old
  block's sector q - q_site in that block's own order;
* wavefunction layout: sub-blocks (a, s1, s2, b) ordered by left sector a
  (sorted q), then s1, then s2; b is the unique right sector completing the
  target (N_alpha, N_beta); each sub-block is m_a x m_b, row-major.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from math import comb
from typing import Dict, List, Optional, Tuple

import numpy as np

Q = Tuple[int, int]
SITE_Q: Tuple[Q, ...] = ((0, 0), (1, 0), (0, 1), (1, 1))


def qadd(a: Q, b: Q) -> Q:
    return (a[0] + b[0], a[1] + b[1])


def qsub(a: Q, b: Q) -> Q:
    return (a[0] - b[0], a[1] - b[1])


# ---------------------------------------------------------------------------
# integrals
# ---------------------------------------------------------------------------

def make_integrals(K: int, seed: int) -> Tuple[np.ndarray, np.ndarray]:
    """Return (h1e[K,K], g2e[K,K,K,K]) in chemists' order (ij|kl).

    h_ii = -2 + 4 i / K + N(0, 0.1);  h_ij (i<j) = N(0, 0.05) exp(-|i-j|/4),
    mirrored;  g_ijkl = sum_P L^P_ij L^P_kl with 2K symmetric factors L^P
    whose upper triangle (diagonal included) is N(0, 0.1 exp(-|i-j|/4)).
    N(0, s) has standard deviation s.  Draw order: h diagonal, h upper
    triangle row-major, then L P-major / upper-triangle row-major.

    g is formed on the pair space (i<=j) x (k<=l), symmetrised there and
    scattered to all eight index permutations, so the 8-fold symmetry holds
    bit for bit.
    """
    rng = np.random.default_rng(seed)
    h = np.zeros((K, K))
    h[np.arange(K), np.arange(K)] = -2.0 + 4.0 * np.arange(K) / K + rng.normal(0.0, 0.1, K)
    iu, ju = np.triu_indices(K, 1)
    h[iu, ju] = rng.normal(0.0, 0.05, iu.size) * np.exp(-np.abs(iu - ju) / 4.0)
    h[ju, iu] = h[iu, ju]

    ip, jp = np.triu_indices(K, 0)          # pairs i <= j, row-major
    npair = ip.size
    decay = np.exp(-np.abs(ip - jp) / 4.0)
    L = np.empty((2 * K, npair))
    for P in range(2 * K):
        L[P] = rng.normal(0.0, 1.0, npair) * (0.1 * decay)
    G = L.T @ L
    G = 0.5 * (G + G.T)                       # exact symmetry in the pair space
    g = np.empty((K, K, K, K))
    for a in range(npair):
        i, j = ip[a], jp[a]
        row = G[a]
        blk = np.zeros((K, K))
        blk[ip, jp] = row
        blk[jp, ip] = row
        g[i, j] = blk
        g[j, i] = blk
    return h, g


# ---------------------------------------------------------------------------
# bond dimensions
# ---------------------------------------------------------------------------

def _full_dims(nsite: int) -> Dict[Q, int]:
    return {(na, nb): comb(nsite, na) * comb(nsite, nb)
            for na in range(nsite + 1) for nb in range(nsite + 1)}


def allocate_dims(K: int, target: Q, nsite: int, prev: Dict[Q, int],
                  M: Optional[int]) -> Dict[Q, int]:
    """Sector dimensions of a block of ``nsite`` sites counted from an edge.

    Weight of sector q: number of full-space determinants through q,
    C(j,na) C(j,nb) C(K-j,Na-na) C(K-j,Nb-nb).  Cap: min(full dimension,
    enlarged dimension sum_s prev[q - s]).  If the caps sum to at most M
    (or M is None) every sector takes its cap; otherwise M is spread by
    water-filling in proportion to the weights under the caps, floors are
    taken and the remainder goes by largest fractional part (ties by q in
    lexicographic order).  Zero sectors are dropped.
    """
    Na, Nb = target
    full = _full_dims(nsite)
    w: Dict[Q, float] = {}
    cap: Dict[Q, int] = {}
    for q, f in sorted(full.items()):
        wt = f * comb(K - nsite, Na - q[0]) * comb(K - nsite, Nb - q[1]) \
            if (0 <= Na - q[0] <= K - nsite and 0 <= Nb - q[1] <= K - nsite) else 0
        if wt == 0:
            continue
        enl = sum(prev.get(qsub(q, s), 0) for s in SITE_Q)
        c = min(f, enl)
        if c <= 0:
            continue
        w[q] = float(wt)
        cap[q] = c
    if M is None or sum(cap.values()) <= M:
        return dict(sorted(cap.items()))
    # water-filling
    keys = sorted(cap, key=lambda q: (cap[q] / w[q], q))
    rem_m = float(M)
    rem_w = sum(w.values())
    x: Dict[Q, float] = {}
    lam = None
    for idx, q in enumerate(keys):
        if lam is None and cap[q] <= rem_m * w[q] / rem_w:
            x[q] = float(cap[q])
            rem_m -= cap[q]
            rem_w -= w[q]
        else:
            if lam is None:
                lam = rem_m / rem_w
            x[q] = min(float(cap[q]), lam * w[q])
    m = {q: int(np.floor(x[q])) for q in x}
    left = M - sum(m.values())
    order = sorted((q for q in x if m[q] < cap[q]), key=lambda q: (-(x[q] - m[q]), q))
    for q in order:
        if left <= 0:
            break
        m[q] += 1
        left -= 1
    return {q: v for q, v in sorted(m.items()) if v > 0}


def enlarged_segments(old: Dict[Q, int], q: Q) -> List[Tuple[int, Q, int]]:
    """Segments (site state s, old sector, dim) of enlarged sector q, in order."""
    out = []
    for s, qs in enumerate(SITE_Q):
        qo = qsub(q, qs)
        if qo in old:
            out.append((s, qo, old[qo]))
    return out


def random_isometry(rng: np.random.Generator, d: int, m: int) -> np.ndarray:
    """Q factor of the QR of a d x m Gaussian, columns signed so diag(R) > 0."""
    a = rng.standard_normal((d, m))
    qm, r = np.linalg.qr(a)
    sgn = np.sign(np.diag(r))
    sgn[sgn == 0] = 1.0
    return qm * sgn[None, :]


# ---------------------------------------------------------------------------
# problem
# ---------------------------------------------------------------------------

@dataclass
class Problem:
    name: str
    K: int
    target: Q
    M: Optional[int]
    h1e: np.ndarray
    g2e: np.ndarray
    e_core: float
    KL: int
    left_dims: List[Dict[Q, int]]            # [j] = dims of block of sites [0, j)
    right_dims: List[Dict[Q, int]]           # [j] = dims of block of sites [K-j, K)
    left_iso: List[Dict[Q, np.ndarray]]      # [j] = isometry adding site j to [0, j)
    right_iso: List[Dict[Q, np.ndarray]]     # [j] = isometry adding site K-1-j to [K-j, K)
    next_iso: Dict[Q, np.ndarray]            # isometry adding site d1 to Lb (renormalization)
    next_dims: Dict[Q, int]
    psi: np.ndarray                          # start wavefunction, wavefunction layout
    n_proc: int = 1
    proc_id: int = 1
    meta: dict = field(default_factory=dict)

    @property
    def KR(self) -> int:
        return self.K - self.KL - 2

    @property
    def lb_dims(self) -> Dict[Q, int]:
        return self.left_dims[self.KL]

    @property
    def rb_dims(self) -> Dict[Q, int]:
        return self.right_dims[self.KR]


def psi_blocks(lb: Dict[Q, int], rb: Dict[Q, int], target: Q):
    """Wavefunction sub-blocks (a, s1, s2, b, m_a, m_b) in layout order."""
    out = []
    for a in sorted(lb):
        for s1, q1 in enumerate(SITE_Q):
            for s2, q2 in enumerate(SITE_Q):
                b = qsub(qsub(qsub(target, a), q1), q2)
                if b in rb:
                    out.append((a, s1, s2, b, lb[a], rb[b]))
    return out


def psi_dim(lb, rb, target) -> int:
    return sum(ma * mb for (_, _, _, _, ma, mb) in psi_blocks(lb, rb, target))


def make_problem(K: int, n_elec: int, two_sz: int, M: Optional[int], seed_base: int,
                 name: str = "", n_proc: int = 1, proc_id: int = 1,
                 zero_g: bool = False) -> Problem:
    """Build the inputs of one middle-site step.

    Seeds: integrals seed_base+1, isometries seed_base+2, wavefunction
    seed_base+3 (seed_base = 1000 c for config c).
    """
    assert K % 2 == 0 and K >= 4
    Na = (n_elec + two_sz) // 2
    Nb = (n_elec - two_sz) // 2
    assert Na + Nb == n_elec and Na - Nb == two_sz
    target = (Na, Nb)
    h, g = make_integrals(K, seed_base + 1)
    if zero_g:
        g = np.zeros_like(g)
    KL = K // 2 - 1
    KR = K - KL - 2
    rng = np.random.default_rng(seed_base + 2)

    def grow(nsites: int):
        dims = [{(0, 0): 1}]
        isos = []
        for j in range(nsites):
            new = allocate_dims(K, target, j + 1, dims[-1], M)
            iso = {}
            for q, m in new.items():
                d = sum(dd for (_, _, dd) in enlarged_segments(dims[-1], q))
                iso[q] = random_isometry(rng, d, m)
            dims.append(new)
            isos.append(iso)
        return dims, isos

    left_dims, left_iso = grow(KL)
    right_dims, right_iso = grow(KR)
    # isometry for the renormalization of L' = Lb + d1 into the next left block
    nd = allocate_dims(K, target, KL + 1, left_dims[KL], M)
    next_iso = {}
    for q, m in nd.items():
        d = sum(dd for (_, _, dd) in enlarged_segments(left_dims[KL], q))
        next_iso[q] = random_isometry(rng, d, m)

    dim = psi_dim(left_dims[KL], right_dims[KR], target)
    rng3 = np.random.default_rng(seed_base + 3)
    psi = rng3.standard_normal(dim)
    psi /= np.linalg.norm(psi)
    return Problem(name=name, K=K, target=target, M=M, h1e=h, g2e=g, e_core=0.0, KL=KL,
                   left_dims=left_dims, right_dims=right_dims, left_iso=left_iso,
                   right_iso=right_iso, next_iso=next_iso, next_dims=nd, psi=psi,
                   n_proc=n_proc, proc_id=proc_id)


# The five workloads: shapes of the paper's benchmark systems with the
# integral recipe above (the integral files themselves are not available).
CONFIGS = {
    "C1": dict(K=8, n_elec=8, two_sz=0, M=None, seed_base=1000),
    "C2": dict(K=24, n_elec=24, two_sz=0, M=500, seed_base=2000),
    "C3": dict(K=54, n_elec=54, two_sz=0, M=2000, seed_base=3000),
    "C4": dict(K=76, n_elec=113, two_sz=1, M=1500, seed_base=4000),
    "C5": dict(K=108, n_elec=30, two_sz=0, M=6000, seed_base=5000, n_proc=16, proc_id=1),
}


# Reduced-M twins of the three largest workloads: the same orbital count,
# electron count, spin projection and sub-Hamiltonian share, with a bond
# dimension small enough for the CPU oracle (whose cost grows as K^4 in the
# number of operator constructions, not with M).  Their stored products are
# written by tests/golden/make_golden.py.
TWINS = {
    "C3T": dict(K=54, n_elec=54, two_sz=0, M=48, seed_base=3100),
    "C4T": dict(K=76, n_elec=113, two_sz=1, M=48, seed_base=4100),
    "C5T": dict(K=108, n_elec=30, two_sz=0, M=48, seed_base=5100, n_proc=16, proc_id=1),
}
TWIN_ROOTS = {"C3T": 1, "C4T": 8, "C5T": 1}


def config_problem(name: str, **over) -> Problem:
    kw = dict(CONFIGS[name] if name in CONFIGS else TWINS[name])
    kw.update(over)
    return make_problem(name=name, **kw)


def random_vectors(dim: int, n: int, seed: int) -> np.ndarray:
    """n seeded Gaussian vectors (rows), each normalised."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, dim))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v


# ---------------------------------------------------------------------------
# two-site sweeps
# ---------------------------------------------------------------------------

@dataclass
class SweepInputs:
    """Inputs of a run of two-site sweeps over sites 0..K-1.

    The starting MPS is the left block of site 0 (left_iso0, its sector
    dimensions left_dims1) and right blocks of n = 1..K-3 sites built through
    random isometries (right_iso[n-1] adds site K-n to the block of n-1
    sites; right_dims[n] are the dimensions of the block of n sites).
    """
    name: str
    K: int
    target: Q
    M: Optional[int]
    h1e: np.ndarray
    g2e: np.ndarray
    e_core: float
    left_dims1: Dict[Q, int]
    left_iso0: Dict[Q, np.ndarray]
    right_dims: List[Dict[Q, int]]
    right_iso: List[Dict[Q, np.ndarray]]
    seed_base: int


def make_sweep_inputs(K: int, n_elec: int, two_sz: int, M: Optional[int], seed_base: int,
                      name: str = "") -> SweepInputs:
    """Seeds: integrals seed_base+1 (as make_problem), isometries seed_base+2."""
    assert K >= 4
    Na = (n_elec + two_sz) // 2
    Nb = (n_elec - two_sz) // 2
    assert Na + Nb == n_elec and Na - Nb == two_sz
    target = (Na, Nb)
    h, g = make_integrals(K, seed_base + 1)
    rng = np.random.default_rng(seed_base + 2)

    def iso_for(old: Dict[Q, int], new: Dict[Q, int]) -> Dict[Q, np.ndarray]:
        out = {}
        for q, m in new.items():
            d = sum(dd for (_, _, dd) in enlarged_segments(old, q))
            out[q] = random_isometry(rng, d, m)
        return out

    vac = {(0, 0): 1}
    l1 = allocate_dims(K, target, 1, vac, M)
    liso = iso_for(vac, l1)
    rdims = [vac]
    riso = []
    for n in range(1, K - 2):
        new = allocate_dims(K, target, n, rdims[-1], M)
        riso.append(iso_for(rdims[-1], new))
        rdims.append(new)
    return SweepInputs(name=name, K=K, target=target, M=M, h1e=h, g2e=g, e_core=0.0,
                       left_dims1=l1, left_iso0=liso, right_dims=rdims, right_iso=riso,
                       seed_base=seed_base)


def sweep_seed(inp: SweepInputs, sweep: int, backward: bool, KL: int) -> int:
    """Seed of the Davidson start vector at one step of a sweep."""
    return inp.seed_base + 10 + 1000 * sweep + 2 * KL + (1 if backward else 0)

