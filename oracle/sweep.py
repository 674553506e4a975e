"""O4 -- decimation and two-site sweeps (plain NumPy FP64).  TEST INFRASTRUCTURE ONLY.

Follows the paper's serial two-site algorithm (Appendix A): after the
effective eigenproblem of a step is solved, the two-site wavefunction Psi
(rows: states of the enlarged left block L' = Lb + d1, columns: states of the
enlarged right block R' = d2 + Rb) is decimated -- the reduced density matrix
of the side that moves on is diagonalised and its eigenvectors of largest
weight become the new renormalized basis (the MPS tensor of that site) --
and the grown block's operators are transformed into that basis (operator
transformation, as in blockops.renormalize).  A sweep moves the dots from
the left end to the right end and back.

Readings fixed here (the paper does not spell them out):

* density matrix of the left side rho_L = sum over roots of Psi Psi^T / n,
  of the right side rho_R = sum Psi^T Psi / n (equal weights for several
  roots); noise adds noise * Xi Xi^T / n per root (Xi^T Xi on the right) for
  a given perturbation Xi: a positive semidefinite term that does not depend
  on the sign of a root;
* kept states: the M largest weights over all sectors, plus every further
  state whose weight lies within tie_rel * w_M + tie_abs * w_max of the M-th
  weight w_M (so no multiplet of the spin symmetry is cut, also when a
  solver's residual splits it slightly, while the bond dimension stays M up
  to such partners), minus every state of weight at most floor_rel * w_max
  (no basis state without weight is kept); with M None, or M at least the
  number of states above that floor, every such state is kept;
* truncation error: discarded weight / total weight;
* each step solves for the lowest root(s) of H_eff from a seeded start
  vector; the last step of a half-sweep is solved again at the start of the
  next half-sweep.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Tuple

import numpy as np
import scipy.sparse.linalg as spla

from .blockops import (Block, Integrals, Site, TwoSiteHeff, grow_left, grow_right_compl, renorm_block,
                       vacuum_block, vacuum_compl)

Q = Tuple[int, int]


@dataclass
class Decimation:
    U: Dict[Q, np.ndarray]            # enlarged sector -> isometry (d_q x k_q), columns by descending weight
    dims: Dict[Q, int]                # kept states per sector
    weights: Dict[Q, np.ndarray]      # kept weights per sector, descending
    all_weights: np.ndarray           # every weight, descending
    trunc_err: float                  # discarded / total weight
    kept: int = 0


def density_matrices(H: TwoSiteHeff, psis: List[np.ndarray], side: str, noise: float = 0.0,
                     xis: Optional[List[np.ndarray]] = None) -> Dict[Q, np.ndarray]:
    """Reduced density matrix of the enlarged left (side 'left') or right
    ('right') block, per sector, averaged over the given wavefunctions, plus
    noise times the same form of the perturbations."""
    rho: Dict[Q, np.ndarray] = {}
    terms = [(1.0, p) for p in psis] + ([(noise, x) for x in xis] if noise else [])
    for c, psi in terms:
        for (QL, QR), X in H.to_matrix(psi).items():
            q, R = (QL, X @ X.T) if side == "left" else (QR, X.T @ X)
            rho[q] = rho[q] + c * R if q in rho else c * R
    return {q: r / len(psis) for q, r in sorted(rho.items())}


TIE_REL = 1e-5
TIE_ABS = 1e-12
FLOOR_REL = 1e-14


def select_states(rho: Dict[Q, np.ndarray], M: Optional[int], tie_rel: float = TIE_REL,
                  floor_rel: float = FLOOR_REL, tie_abs: float = TIE_ABS) -> Decimation:
    """Diagonalise each sector's density matrix and keep the heaviest states."""
    eig = {}
    allw = []
    for q, r in rho.items():
        w, V = np.linalg.eigh(r)
        eig[q] = (w[::-1], V[:, ::-1])        # descending weight
        allw.append(w)
    allw = np.sort(np.concatenate(allw))[::-1] if allw else np.zeros(0)
    total = float(allw.sum())
    wmax = float(allw[0]) if allw.size else 0.0
    floor = floor_rel * wmax
    if M is None or M >= int(np.sum(allw > floor)):
        cut = floor
    else:
        wM = float(allw[M - 1])
        cut = max(wM - tie_rel * wM - tie_abs * wmax, floor)
    U, dims, wk = {}, {}, {}
    kept_w = 0.0
    for q, (w, V) in eig.items():
        # keep w >= cut (or w > floor when the cut sits on the floor)
        k = int(np.sum(w > floor)) if cut <= floor else int(np.sum(w >= cut))
        if k == 0:
            continue
        U[q] = V[:, :k].copy()
        dims[q] = k
        wk[q] = w[:k].copy()
        kept_w += float(w[:k].sum())
    kept = sum(dims.values())
    err = (total - kept_w) / total if total > 0 else 0.0
    return Decimation(U=U, dims=dims, weights=wk, all_weights=allw, trunc_err=max(err, 0.0), kept=kept)


def decimate(H: TwoSiteHeff, psis: List[np.ndarray], side: str, M: Optional[int], noise: float = 0.0,
             xis: Optional[List[np.ndarray]] = None, tie_rel: float = TIE_REL) -> Decimation:
    """Decimation of one step (Appendix A): the new basis of the side that
    moves on, from the density matrix of the (optionally perturbed) roots."""
    return select_states(density_matrices(H, psis, side, noise, xis), M, tie_rel)


def lowest_roots(H: TwoSiteHeff, v0: np.ndarray, n_roots: int = 1, dense_max: int = 200):
    """Lowest n_roots eigenpairs of H_eff: LAPACK on the dense matrix for
    small dimensions, else ARPACK (Lanczos) from the seeded start vector."""
    dim = H.dim
    if dim <= dense_max:
        Hm = np.stack([H.apply(c) for c in np.eye(dim)], axis=1)
        w, V = np.linalg.eigh(0.5 * (Hm + Hm.T))
        return w[:n_roots], V[:, :n_roots].T
    op = spla.LinearOperator((dim, dim), matvec=H.apply, dtype=np.float64)
    w, V = spla.eigsh(op, k=n_roots, which="SA", v0=v0[0], tol=1e-13, ncv=max(2 * n_roots + 1, 20))
    order = np.argsort(w)
    return w[order], V[:, order].T


@dataclass
class Step:
    sweep: int
    backward: bool
    KL: int
    dim: int
    energies: List[float]
    kept: int = 0                      # bond dimension after the decimation (0: none)
    dims: Dict[Q, int] = field(default_factory=dict)
    trunc_err: float = 0.0


def sweeps(inp, n_sweeps: int, start: Callable[[int, int, int], np.ndarray], M: Optional[int] = None,
           n_roots: int = 1, noise: float = 0.0, noise_vec: Optional[Callable[[int, int], np.ndarray]] = None,
           tie_rel: float = TIE_REL, seed_of: Optional[Callable[[int, bool, int], int]] = None,
           schedule: Optional[List[Tuple[Optional[int], float]]] = None) -> List[Step]:
    """Two-site sweeps from the starting MPS of ``inp`` (left block of site 0,
    right blocks of 1..K-3 sites).  start(dim, seed, n) gives the start
    vectors, seed_of(sweep, backward, KL) their seed; noise_vec(dim, seed)
    the perturbations (one per root) when noise != 0.  schedule: (M, noise)
    of every sweep (the bond-dimension schedule of a production run), which
    then sets the sweep count.  Returns every step."""
    K, tgt = inp.K, inp.target
    ints = Integrals(inp.h1e, inp.g2e)
    _, Z = grow_left(vacuum_block(K, True), Site(0, ints), ints, list(range(2, 2 * K)))
    L: Dict[int, Block] = {1: renorm_block(Z, inp.left_iso0, inp.left_dims1)}
    R: Dict[int, Block] = {}
    Y = vacuum_compl(list(range(0, 2 * K)))
    for n in range(1, K - 2):
        site = K - n
        _, Z = grow_right_compl(Y, Site(site, ints), ints, list(range(0, 2 * site)))
        Y = renorm_block(Z, inp.right_iso[n - 1], inp.right_dims[n])
        R[n] = Y
    out: List[Step] = []
    last = K - 3
    if schedule is not None:
        n_sweeps = len(schedule)
    for sw in range(n_sweeps):
        if schedule is not None:
            M, noise = schedule[sw]
        for backward in (False, True):
            order = range(1, last + 1) if not backward else range(last, 0, -1)
            for KL in order:
                H = TwoSiteHeff(L[KL], R[K - KL - 2], ints, KL, K, tgt, inp.e_core)
                seed = seed_of(sw, backward, KL)
                E, V = lowest_roots(H, start(H.dim, seed, n_roots), n_roots)
                st = Step(sweep=sw, backward=backward, KL=KL, dim=H.dim, energies=[float(x) for x in E])
                xis = None
                if noise:
                    xis = [noise_vec(H.dim, seed + 500 + r) for r in range(n_roots)]
                if not backward and KL < last:
                    d = decimate(H, list(V), "left", M, noise, xis, tie_rel)
                    L[KL + 1] = renorm_block(H.Lp, d.U, d.dims)
                    st.kept, st.dims, st.trunc_err = d.kept, dict(d.dims), d.trunc_err
                elif backward and KL > 1:
                    d = decimate(H, list(V), "right", M, noise, xis, tie_rel)
                    R[K - KL - 1] = renorm_block(H.Rp, d.U, d.dims)
                    st.kept, st.dims, st.trunc_err = d.kept, dict(d.dims), d.trunc_err
                out.append(st)
    return out
