"""Dense Jordan-Wigner matrices on a full Fock space (test helper).

An independent construction of fermion operators used to pin the oracle:
a+_p = Z x ... x Z x sigma+ x 1 x ... x 1 with Z = diag(1, -1) on every mode
before p.  The Fock basis index is sum_p n_p 2^p, and |n> =
(a+_0)^{n_0} (a+_1)^{n_1} ... |0>, i.e. creation operators in increasing
mode order, which is the determinant convention of the oracle.
"""
import numpy as np


def creation_ops(nmodes: int):
    dim = 1 << nmodes
    ops = []
    for p in range(nmodes):
        M = np.zeros((dim, dim))
        for idx in range(dim):
            if idx >> p & 1:
                continue
            # number of occupied modes before p
            sign = -1.0 if bin(idx & ((1 << p) - 1)).count("1") % 2 else 1.0
            M[idx | (1 << p), idx] = sign
        ops.append(M)
    return ops


def hamiltonian(t: np.ndarray, v: np.ndarray, cs=None):
    n = t.shape[0]
    cs = creation_ops(n) if cs is None else cs
    ds = [c.T for c in cs]
    H = np.zeros_like(cs[0])
    for p in range(n):
        for q in range(n):
            if t[p, q]:
                H += t[p, q] * cs[p] @ ds[q]
    for p in range(n):
        for q in range(n):
            for r in range(n):
                for s in range(n):
                    if v[p, q, r, s]:
                        H += 0.5 * v[p, q, r, s] * cs[p] @ cs[r] @ ds[s] @ ds[q]
    return H


def sector_indices(nmodes: int, na: int, nb: int):
    out = []
    for idx in range(1 << nmodes):
        a = sum(idx >> p & 1 for p in range(0, nmodes, 2))
        b = sum(idx >> p & 1 for p in range(1, nmodes, 2))
        if a == na and b == nb:
            out.append(idx)
    return np.array(out)
