"""Pins of O1 (determinant-space Hamiltonian) against things other than itself.

* a 2-orbital, 2-electron S_z = 0 matrix written out by hand;
* closed forms: g = 0 (orbital energies), on-site-only g with diagonal h;
* an independent dense Jordan-Wigner construction of the same operator;
* LAPACK eigh vs the matrix-free product, hermiticity, 8-fold symmetry.
"""
from itertools import combinations

import numpy as np
import pytest

import synth
from oracle import fci
from tests import jw


def test_integral_symmetry_bitwise():
    h, g = synth.make_integrals(7, 123)
    assert np.array_equal(h, h.T)
    for perm in ["jikl", "ijlk", "klij", "jilk", "lkij", "klji", "lkji"]:
        assert np.array_equal(g, np.einsum("ijkl->" + perm, g)), perm
    # g is a Gram matrix over pairs, so positive semidefinite as (ij) x (kl)
    w = np.linalg.eigvalsh(g.reshape(49, 49))
    assert w.min() > -1e-12


def test_integrals_reproducible():
    a = synth.make_integrals(6, 5)
    b = synth.make_integrals(6, 5)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_two_orbital_hand_matrix():
    h, g = synth.make_integrals(2, 99)
    H = fci.FCIHamiltonian(h, g, 1, 1).dense()
    # determinants sorted by bit string: |0a 0b>, |0b 1a>, |0a 1b>, |1a 1b>
    U0, U1 = g[0, 0, 0, 0], g[1, 1, 1, 1]
    J, Kx = g[0, 0, 1, 1], g[0, 1, 0, 1]
    a, b = g[0, 0, 0, 1], g[1, 1, 0, 1]
    h00, h11, h01 = h[0, 0], h[1, 1], h[0, 1]
    ref = np.array([
        [2 * h00 + U0, -(h01 + a), h01 + a, Kx],
        [-(h01 + a), h00 + h11 + J, -Kx, -(h01 + b)],
        [h01 + a, -Kx, h00 + h11 + J, h01 + b],
        [Kx, -(h01 + b), h01 + b, 2 * h11 + U1],
    ])
    assert np.allclose(H, ref, atol=1e-14, rtol=0)


@pytest.mark.parametrize("K,na,nb", [(4, 2, 2), (5, 3, 1), (6, 2, 3)])
def test_noninteracting_closed_form(K, na, nb):
    h, g = synth.make_integrals(K, 17 + K)
    E = fci.fci_ground_energy(h, 0.0 * g, na, nb)
    w = np.linalg.eigvalsh(h)
    assert abs(E - (w[:na].sum() + w[:nb].sum())) < 1e-12


def test_onsite_only_brute_force():
    K, na, nb = 5, 3, 2
    rng = np.random.default_rng(4)
    h = np.diag(rng.normal(size=K))
    g = np.zeros((K,) * 4)
    U = rng.uniform(0.5, 2.0, K)
    for i in range(K):
        g[i, i, i, i] = U[i]
    E = fci.fci_ground_energy(h, g, na, nb)
    best = np.inf
    for oa in combinations(range(K), na):
        for ob in combinations(range(K), nb):
            e = sum(h[i, i] for i in oa) + sum(h[i, i] for i in ob) + sum(U[i] for i in oa if i in ob)
            best = min(best, e)
    assert abs(E - best) < 1e-12


@pytest.mark.parametrize("K,na,nb", [(3, 2, 1), (3, 1, 1), (4, 2, 2)])
def test_matches_jordan_wigner(K, na, nb):
    h, g = synth.make_integrals(K, 31 + K)
    t, v = fci.spin_integrals(h, g)
    Hjw = jw.hamiltonian(t, v)
    idx = jw.sector_indices(2 * K, na, nb)
    Hs = Hjw[np.ix_(idx, idx)]
    dets = fci.determinants(K, na, nb)
    assert np.array_equal(np.sort(idx), dets)      # same basis, same order
    H = fci.FCIHamiltonian(h, g, na, nb).dense()
    assert np.allclose(H, Hs, atol=1e-13, rtol=0)


def test_matvec_hermitian_and_eigh():
    h, g = synth.make_integrals(5, 8)
    H = fci.FCIHamiltonian(h, g, 3, 2)
    Hd = H.dense()
    assert np.abs(Hd - Hd.T).max() < 1e-13
    x = np.random.default_rng(1).standard_normal(H.dim)
    assert np.allclose(H.matvec(x), Hd @ x, atol=1e-12)
    w = np.linalg.eigvalsh(Hd)
    assert abs(w[0] - fci.fci_ground_energy(h, g, 3, 2)) < 1e-12
