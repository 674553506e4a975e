"""Writes the stored expected values of the GPU parity tests (calls only oracle/ and synth).

For each workload the oracle's H_eff psi of the seeded start vector
(Appendix A effective eigenproblem, two-site product built from Appendix B's
Hamiltonian) is saved as float64 .npy; for the 8-orbital workload also the
FCI ground energy (lowest eigenvalue of the determinant-space matrix).

Usage: python -m tests.golden.make_golden
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import blockops, fci  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main(names=("C1", "C2")):
    meta = {}
    for name in names:
        t0 = time.time()
        p = synth.config_problem(name)
        H = blockops.MiddleHeff(p, "CN")
        sigma = H.apply(p.psi)
        np.save(os.path.join(HERE, f"{name}_sigma.npy"), sigma)
        m = {"dim": int(p.psi.size), "sigma_norm": float(np.linalg.norm(sigma)),
             "psi_norm": float(np.linalg.norm(p.psi)), "seconds": round(time.time() - t0, 1),
             "source": "oracle.blockops.MiddleHeff(scheme=CN).apply(seeded start vector)"}
        if name == "C1":
            m["fci_ground_energy"] = float(fci.fci_ground_energy(p.h1e, p.g2e, *p.target))
        meta[name] = m
        print(name, m, flush=True)
    with open(os.path.join(HERE, "golden.json"), "w") as f:
        json.dump(meta, f, indent=1)


if __name__ == "__main__":
    main()
