"""Sum of sub-Hamiltonians: integral masking.  TEST INFRASTRUCTURE ONLY.

Section II.B of the paper writes H = sum_p H^(p) with

  H^(p) = 1/2 sum [proc(p,i) + proc(p,j)] t_ij a+ a
        + 1/2 sum proc(p,i,j,k,l) v_ijkl a+ a+ a a,

proc(p, i) = [p = i mod P], proc(p, i, j) = [p = (j-1)j/2 + i mod P] for
i <= j (symmetric in i, j), indices 1-based, p = 1..P (p = P is residue 0),
and for the NC partition proc(p, i, j, k, l) = proc(p, j) if j = k else
proc(p, i, j) on the sorted tuple i <= j <= k <= l.
"""
from __future__ import annotations

import numpy as np


def proc1(p: int, i: int, P: int) -> bool:
    return (i - p) % P == 0


def proc2(p: int, i: int, j: int, P: int) -> bool:
    if i > j:
        i, j = j, i
    return ((j - 1) * j // 2 + i - p) % P == 0


def proc4_nc(p: int, idx, P: int) -> bool:
    a, b, c, d = sorted(idx)
    if b == c:
        return proc1(p, b, P)
    return proc2(p, a, b, P)


def masked_integrals(h: np.ndarray, g: np.ndarray, P: int, p: int):
    """(t^(p), v^(p)) of sub-Hamiltonian p (1-based) out of P, NC assignment."""
    K = h.shape[0]
    w1 = np.array([1.0 if proc1(p, i + 1, P) else 0.0 for i in range(K)])
    hp = 0.5 * (w1[:, None] + w1[None, :]) * h
    mask = np.zeros((K, K, K, K))
    for i in range(K):
        for j in range(K):
            for k in range(K):
                for l in range(K):
                    if proc4_nc(p, (i + 1, j + 1, k + 1, l + 1), P):
                        mask[i, j, k, l] = 1.0
    return hp, g * mask


def owned_pairs(p: int, P: int, n: int):
    """Spatial pairs (i <= j, 0-based, both < n) owned by sub-Hamiltonian p."""
    return [(i, j) for j in range(n) for i in range(j + 1) if proc2(p, i + 1, j + 1, P)]
