"""Two-site DMRG sweeps driven over the C ABI (Appendix A of the paper).

Each step of a sweep is: blocking of the two dots and the work list of H_eff
(dmrg_heff_create), the effective eigenproblem (dmrg_davidson), decimation of
the side that moves on (dmrg_decimate) and the transformation of its grown
block into the decimated basis (dmrg_heff_renormalize for the left block,
dmrg_renormalize for the right one).  The dots move from the left end
(KL = 1) to the right end (KL = K - 3) and back; the last step of a
half-sweep is solved again at the start of the next one.  Right blocks hold
complementary operators (NC partition) at every position.

This module only sequences library calls and moves vectors between host and
device: every step of the arithmetic runs in the library's kernels.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Tuple

import numpy as np

from . import dmrg as D


@dataclass
class SweepStep:
    sweep: int
    backward: bool
    KL: int
    dim: int
    energies: List[float]
    kept: int = 0                       # bond dimension after the decimation (0: none)
    dims: Dict[Tuple[int, int], int] = field(default_factory=dict)
    trunc_err: float = 0.0
    davidson: dict = field(default_factory=dict)
    ms: Dict[str, float] = field(default_factory=dict)


def run_sweeps(ctx: "D.Context", inp, n_sweeps: int, max_states: Optional[int],
               start: Callable[[int, int, int], np.ndarray], seed_of: Callable[[int, bool, int], int],
               n_roots: int = 1, tol: float = 1e-9, precision: int = D.DMRG_PREC_F64,
               noise: float = 0.0, noise_vec: Optional[Callable[[int, int], np.ndarray]] = None,
               max_iter: int = 500, max_subspace: int = 24, diag_guess: bool = True,
               on_step: Optional[Callable[[SweepStep], None]] = None,
               schedule: Optional[List[Tuple[Optional[int], float]]] = None) -> List[SweepStep]:
    """Sweeps from the starting MPS of ``inp`` (integrals, the isometry of
    site 0, random isometries of the right blocks of 1..K-3 sites).

    start(dim, seed, n) returns seeded vectors ([n, dim], host), seed_of(sweep,
    backward, KL) their seed; with diag_guess, root j's Davidson start is the
    basis state of the j-th lowest diagonal element of H_eff plus 0.1 times
    the seeded vector, else the seeded vector alone.  noise_vec(dim, seed)
    gives one perturbation per root when noise != 0.  max_states None keeps
    every state with weight.  schedule: (max_states, noise) of every sweep
    (a bond-dimension schedule), which then sets the sweep count.  Returns
    every step."""
    import time
    import torch
    dev = ctx.device
    K = inp.K
    n_elec = inp.target[0] + inp.target[1]
    ctx.set_integrals(inp.h1e, inp.g2e, n_elec, inp.target[0] - inp.target[1], inp.e_core)
    L: Dict[int, D.OpSet] = {1: ctx.build_block(D.DMRG_LEFT, [D.Isometry(inp.left_iso0, dev)], D.DMRG_SCHEME_NC)}
    R: Dict[int, D.OpSet] = {1: ctx.build_block(D.DMRG_RIGHT, [D.Isometry(inp.right_iso[0], dev)],
                                                D.DMRG_SCHEME_NC)}
    for n in range(2, K - 2):
        R[n] = ctx.renormalize(R[n - 1], D.Isometry(inp.right_iso[n - 1], dev))
    last = K - 3
    if schedule is not None:
        n_sweeps = len(schedule)
    out: List[SweepStep] = []
    try:
        for sw in range(n_sweeps):
            if schedule is not None:
                max_states, noise = schedule[sw]
            M = 0 if max_states is None else int(max_states)
            for backward in (False, True):
                order = range(1, last + 1) if not backward else range(last, 0, -1)
                for KL in order:
                    t0 = time.perf_counter()
                    H = ctx.heff_create(L[KL], R[K - KL - 2], n_roots=n_roots, precision=precision)
                    try:
                        seed = seed_of(sw, backward, KL)
                        psi = torch.from_numpy(np.ascontiguousarray(start(H.dim, seed, n_roots))).to(dev)
                        if diag_guess:
                            # root j starts on the basis state of the j-th lowest diagonal element
                            # (plus the seeded vector at 1/10 weight): a random start alone has
                            # let Davidson settle on an excited root when the ground state's
                            # overlap with it was small
                            dg = torch.empty(H.dim, dtype=torch.float64, device=dev)
                            H.diag(dg)
                            idx = torch.topk(dg, min(n_roots, H.dim), largest=False).indices
                            psi = 0.1 * psi.view(n_roots, H.dim)
                            psi[torch.arange(idx.numel(), device=dev), idx] += 1.0
                            psi = psi.reshape(-1).contiguous()
                        torch.cuda.synchronize()
                        t1 = time.perf_counter()
                        E, stats = H.davidson(psi, n_roots=n_roots, tol=tol, max_iter=max_iter,
                                              max_subspace=max(max_subspace, 3 * n_roots), precision=precision)
                        torch.cuda.synchronize()
                        t2 = time.perf_counter()
                        st = SweepStep(sweep=sw, backward=backward, KL=KL, dim=H.dim,
                                       energies=[float(x) for x in E], davidson=stats)
                        st.ms = {"heff_create": 1e3 * (t1 - t0), "davidson": 1e3 * (t2 - t1)}
                        xi = None
                        if noise:
                            xs = [noise_vec(H.dim, seed + 500 + r) for r in range(n_roots)]
                            xi = torch.from_numpy(np.ascontiguousarray(np.stack(xs))).to(dev)
                        move = (not backward and KL < last) or (backward and KL > 1)
                        if move:
                            side = D.DMRG_LEFT if not backward else D.DMRG_RIGHT
                            iso = H.decimate(psi, side, M, n_vec=n_roots, noise=noise, xi=xi)
                            t3 = time.perf_counter()
                            try:
                                if not backward:
                                    new = H.renormalize(iso)
                                    if KL + 1 in L:
                                        L[KL + 1].free()
                                    L[KL + 1] = new
                                else:
                                    new = ctx.renormalize(R[K - KL - 2], iso)
                                    if K - KL - 1 in R:
                                        R[K - KL - 1].free()
                                    R[K - KL - 1] = new
                                torch.cuda.synchronize()
                                t4 = time.perf_counter()
                                st.kept = int(iso.info["kept"])
                                st.trunc_err = float(iso.info["trunc_err"])
                                st.dims = iso.dims
                                st.ms["decimate"] = 1e3 * (t3 - t2)
                                st.ms["renormalize"] = 1e3 * (t4 - t3)
                            finally:
                                iso.free()
                    finally:
                        H.free()
                    out.append(st)
                    if on_step is not None:
                        on_step(st)
    finally:
        for b in list(L.values()) + list(R.values()):
            b.free()
    return out
