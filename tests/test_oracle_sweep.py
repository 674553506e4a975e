"""Pins of O4 (decimation and two-site sweeps).

* the weights of a decimation are the squared singular values of the
  two-site wavefunction written out as one dense matrix (LAPACK SVD), on
  either side, and its isometry acts on the side asked for;
* the truncation error equals the projection error ||Psi - U U^T Psi||^2
  and the sum of the discarded squared singular values (Eckart-Young: the
  kept states are the heaviest ones);
* the kept set completes degenerate multiplets and drops weightless states
  (hand-made density matrices);
* sweeps without truncation give the FCI energy at every step (LAPACK on
  the determinant-space Hamiltonian of O1); truncated sweeps stay above it
  (variational bound) and approach it as M grows.
"""
import numpy as np
import pytest

import synth
from oracle import blockops as bo
from oracle import fci
from oracle import sweep as osw


def _dense(H, psi):
    """Psi as one dense matrix: rows enlarged-left states, columns enlarged-right
    states, sectors in sorted order."""
    lo, ro = {}, {}
    n = 0
    for q in sorted(H.enl_L.dims):
        lo[q] = n
        n += H.enl_L.dims[q]
    m = 0
    for q in sorted(H.enl_R.dims):
        ro[q] = m
        m += H.enl_R.dims[q]
    D = np.zeros((n, m))
    for (QL, QR), X in H.to_matrix(psi).items():
        D[lo[QL]:lo[QL] + X.shape[0], ro[QR]:ro[QR] + X.shape[1]] = X
    return D, lo, ro


def _same_spectrum(w, s2):
    """Equal up to zeros (sectors without wavefunction weight have no rows)."""
    r = min(len(w), len(s2))
    np.testing.assert_allclose(w[:r], s2[:r], rtol=0, atol=1e-13)
    assert np.all(np.abs(w[r:]) < 1e-13) and np.all(np.abs(s2[r:]) < 1e-13)


@pytest.fixture(scope="module")
def middle():
    p = synth.make_problem(8, 8, 0, 12, 7100)
    return p, bo.MiddleHeff(p, "NC")


@pytest.mark.parametrize("side", ["left", "right"])
def test_weights_are_squared_singular_values(middle, side):
    p, H = middle
    D, lo, ro = _dense(H, p.psi)
    s = np.linalg.svd(D, compute_uv=False)
    d = osw.decimate(H, [p.psi], side, None)
    _same_spectrum(d.all_weights, s ** 2)
    # the isometry acts on the side asked for
    enl = H.enl_L.dims if side == "left" else H.enl_R.dims
    for q, U in d.U.items():
        assert U.shape[0] == enl[q]
        np.testing.assert_allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-12)
    # untruncated: the kept states reproduce Psi exactly
    for (QL, QR), X in H.to_matrix(p.psi).items():
        if side == "left":
            Y = d.U[QL] @ (d.U[QL].T @ X) if QL in d.U else 0 * X
        else:
            Y = (X @ d.U[QR]) @ d.U[QR].T if QR in d.U else 0 * X
        np.testing.assert_allclose(Y, X, atol=1e-12)


@pytest.mark.parametrize("M", [5, 20, 33])
def test_truncation_error_is_eckart_young(middle, M):
    p, H = middle
    D, lo, ro = _dense(H, p.psi)
    s2 = np.linalg.svd(D, compute_uv=False) ** 2
    d = osw.decimate(H, [p.psi], "left", M)
    assert d.kept == M                        # random Psi: no degenerate weights
    proj = 0.0
    for (QL, QR), X in H.to_matrix(p.psi).items():
        Y = d.U[QL] @ (d.U[QL].T @ X) if QL in d.U else 0 * X
        proj += float(np.sum((X - Y) ** 2))
    tot = float(np.sum(s2))
    assert abs(d.trunc_err - proj / tot) < 1e-12
    assert abs(d.trunc_err - float(np.sum(s2[M:])) / tot) < 1e-12


def test_two_roots_average_density_matrix(middle):
    p, H = middle
    rng = np.random.default_rng(5)
    x = rng.standard_normal(H.dim)
    x /= np.linalg.norm(x)
    D1, _, _ = _dense(H, p.psi)
    D2, _, _ = _dense(H, x)
    s = np.linalg.svd(np.hstack([D1, D2]) / np.sqrt(2.0), compute_uv=False)
    d = osw.decimate(H, [p.psi, x], "left", None)
    _same_spectrum(d.all_weights, s ** 2)


def test_noise_adds_the_perturbation_density_matrix(middle):
    p, H = middle
    rng = np.random.default_rng(6)
    xi = rng.standard_normal(H.dim)
    D, _, _ = _dense(H, p.psi)
    X, _, _ = _dense(H, xi)
    s = np.linalg.svd(np.hstack([D, np.sqrt(1e-3) * X]), compute_uv=False)
    d = osw.decimate(H, [p.psi], "left", None, noise=1e-3, xis=[xi])
    _same_spectrum(d.all_weights, s ** 2)
    # independent of the sign of the root
    d2 = osw.decimate(H, [-p.psi], "left", None, noise=1e-3, xis=[xi])
    np.testing.assert_allclose(d2.all_weights, d.all_weights, atol=1e-15)


def test_kept_set_completes_multiplets_and_drops_weightless_states():
    rho = {(1, 0): np.diag([0.5, 0.2, 0.1]), (0, 1): np.diag([0.2, 0.0]), (1, 1): np.diag([0.2 + 1e-10])}
    d = osw.select_states(rho, 2)
    assert d.kept == 4 and d.dims == {(1, 0): 2, (0, 1): 1, (1, 1): 1}
    d = osw.select_states(rho, None)
    assert d.kept == 5 and d.dims == {(1, 0): 3, (0, 1): 1, (1, 1): 1}
    d = osw.select_states(rho, 1)
    assert d.kept == 1 and d.dims == {(1, 0): 1}
    assert abs(d.trunc_err - (0.7 + 1e-10) / (1.2 + 1e-10)) < 1e-14


def _run(inp, n_sweeps, M):
    return osw.sweeps(inp, n_sweeps, lambda dim, seed, n: synth.random_vectors(dim, n, seed), M=M,
                      seed_of=lambda sw, b, KL: synth.sweep_seed(inp, sw, b, KL))


def test_untruncated_sweep_gives_fci_at_every_step():
    inp = synth.make_sweep_inputs(6, 6, 0, None, 7200)
    e_fci = fci.fci_ground_energy(inp.h1e, inp.g2e, 3, 3)
    steps = _run(inp, 1, None)
    assert len(steps) == 6
    for st in steps:
        assert abs(st.energies[0] - e_fci) < 1e-10, (st.KL, st.backward, st.energies[0], e_fci)


def test_untruncated_sweep_odd_electrons():
    inp = synth.make_sweep_inputs(6, 5, 1, None, 7300)
    e_fci = fci.fci_ground_energy(inp.h1e, inp.g2e, 3, 2)
    steps = _run(inp, 1, None)
    for st in steps:
        assert abs(st.energies[0] - e_fci) < 1e-10


def test_truncated_sweeps_are_variational_and_improve_with_m():
    inp = synth.make_sweep_inputs(7, 6, 0, 8, 7400)
    e_fci = fci.fci_ground_energy(inp.h1e, inp.g2e, 3, 3)
    finals = []
    for M in (4, 12):
        steps = _run(inp, 2, M)
        for st in steps:
            assert st.energies[0] >= e_fci - 1e-10
            if st.kept:
                assert st.kept <= M + 2          # ties only add a multiplet's partners
        finals.append(steps[-1].energies[0])
    assert finals[1] <= finals[0] + 1e-12
    assert finals[1] - e_fci < finals[0] - e_fci


def test_schedule_of_bond_dimensions():
    """A schedule (M = 4, then 12): the first sweep keeps at most M = 4 states
    (plus multiplet partners), the second grows past them from the blocks the
    first left, and its last energy lies above FCI and below the first
    sweep's."""
    inp = synth.make_sweep_inputs(7, 6, 0, 8, 7400)
    e_fci = fci.fci_ground_energy(inp.h1e, inp.g2e, 3, 3)
    steps = osw.sweeps(inp, 0, lambda dim, seed, n: synth.random_vectors(dim, n, seed),
                       seed_of=lambda sw, b, KL: synth.sweep_seed(inp, sw, b, KL), schedule=[(4, 0.0), (12, 0.0)])
    assert len(steps) == 16
    assert all(st.kept <= 4 + 2 for st in steps[:8])
    assert max(st.kept for st in steps[8:]) > 4
    assert e_fci - 1e-10 <= steps[-1].energies[0] < steps[7].energies[0]
