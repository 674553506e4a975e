"""Writes the stored expected values of the GPU parity tests (calls only oracle/ and synth).

For each workload the oracle's H_eff psi of the seeded start vector(s)
(Appendix A effective eigenproblem, two-site product built from Appendix B's
Hamiltonian) is saved as float64 .npy; for the 8-orbital workload also the
FCI ground energy (lowest eigenvalue of the determinant-space matrix).

* C1, C2: the full 8-orbital and the 24-orbital M = 500 workloads (scheme CN);
* C3T: 54 orbitals, 54 electrons, S_z = 0 at M = 48, scheme CN with the middle
  transform;
* C4T: 76 orbitals, 113 electrons, S_z = 1/2 at M = 48, eight seeded start
  vectors (the 8-root block), scheme CN with the middle transform;
* C5T: 108 orbitals, 30 electrons, S_z = 0 at M = 48, sub-Hamiltonian 1 of 16
  (integrals masked by oracle.share, eq. sub-h / proc-def-nc), scheme NC;
* C2E: the lowest 1 and 8 eigenvalues of the 24-orbital H_eff by ARPACK on the
  oracle's product (reference energies of the Davidson tests).

Usage: python -m tests.golden.make_golden [NAME ...]   (default: all)
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import blockops, fci, share  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
ALL = ("C1", "C2", "C3T", "C4T", "C5T", "C2E")


def twin_vectors(p, name):
    """The seeded start vectors of a twin: the problem's psi, or for an n-root
    block n seeded Gaussian vectors (seed = seed_base + 4), one per row."""
    n = synth.TWIN_ROOTS.get(name, 1)
    if n == 1:
        return p.psi[None, :]
    return synth.random_vectors(p.psi.size, n, synth.TWINS[name]["seed_base"] + 4)


def arpack_energies(name="C2", roots=(1, 8)):
    """Lowest eigenvalues of the oracle's H_eff (scheme CN) by ARPACK (scipy's
    eigsh on the oracle's product, tol 1e-12): the reference energies of the
    1- and 8-root Davidson tests at the 24-orbital workload."""
    import scipy.sparse.linalg as sla
    t0 = time.time()
    p = synth.config_problem(name)
    H = blockops.MiddleHeff(p, "CN")
    n = p.psi.size
    op = sla.LinearOperator((n, n), matvec=H.apply, dtype=float)
    out = {"source": "scipy.sparse.linalg.eigsh(oracle.blockops.MiddleHeff(scheme=CN), which=SA, tol=1e-12)"}
    for k in roots:
        w = sla.eigsh(op, k=k, which="SA", tol=1e-12, v0=p.psi.copy(), ncv=max(2 * k + 1, 24))[0]
        out[f"energies_{k}"] = [float(x) for x in np.sort(w)]
    out["seconds"] = round(time.time() - t0, 1)
    return out


def run(name):
    if name == "C2E":
        return arpack_energies()
    t0 = time.time()
    p = synth.config_problem(name)
    m = {"dim": int(p.psi.size)}
    if p.n_proc > 1:
        hp, gp = share.masked_integrals(p.h1e, p.g2e, p.n_proc, p.proc_id)
        H = blockops.MiddleHeff(p, "NC", hp, gp)
        m["source"] = (f"oracle.blockops.MiddleHeff(scheme=NC, integrals of share {p.proc_id}/{p.n_proc})"
                       ".apply(seeded start vector)")
    else:
        H = blockops.MiddleHeff(p, "CN")
        m["source"] = "oracle.blockops.MiddleHeff(scheme=CN).apply(seeded start vector(s))"
    if name in synth.TWINS:
        X = twin_vectors(p, name)
        sigma = np.stack([H.apply(x) for x in X])
        m["vectors"] = int(X.shape[0])
        np.save(os.path.join(HERE, f"{name}_sigma.npy"), sigma if X.shape[0] > 1 else sigma[0])
    else:
        sigma = H.apply(p.psi)
        np.save(os.path.join(HERE, f"{name}_sigma.npy"), sigma)
    m["sigma_norm"] = float(np.linalg.norm(sigma))
    m["seconds"] = round(time.time() - t0, 1)
    if name == "C1":
        m["fci_ground_energy"] = float(fci.fci_ground_energy(p.h1e, p.g2e, *p.target))
    return m


def main(names=ALL):
    path = os.path.join(HERE, "golden.json")
    for name in names:
        m = run(name)
        print(name, m, flush=True)
        meta = json.load(open(path)) if os.path.exists(path) else {}
        meta[name] = m
        with open(path, "w") as f:
            json.dump(meta, f, indent=1)


if __name__ == "__main__":
    main(tuple(sys.argv[1:]) or ALL)
