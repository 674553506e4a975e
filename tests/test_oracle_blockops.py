"""Pins of O2 (renormalized-operator algebra).

* every renormalized block operator equals its definition W_b^T O W_b, with
  O built from dense Jordan-Wigner matrices on the block's own modes and W_b
  the block basis written out as Fock-space vectors (so a wrong sign, a
  dropped term or a transposed index in any blocking formula shows up);
* H_eff psi equals W^T H W psi of O1 on truncated and untruncated bases,
  odd and even N, S_z in {0, 1/2, 1}, for the CN+transform and NC schemes;
* the lowest eigenvalue at full bond dimension equals the FCI one (LAPACK);
  truncated bases give an upper bound;
* index symmetry of the two-index operators, hermiticity of H_eff;
* sum of sub-Hamiltonians: sum_p H^(p)_eff psi = H_eff psi for P in {2,3,16}.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as sla

import synth
from oracle import blockops as bo
from oracle import fci, share
from tests import jw


def _block_W(states, nmodes):
    W = {}
    for q, d in states.items():
        m = len(next(iter(d.values())))
        M = np.zeros((1 << nmodes, m))
        for bits, vec in d.items():
            M[bits] += vec
        W[q] = M
    return W


def _fock_ops(prob, orbs0, nsite):
    """JW creation ops on the block's modes and the block-restricted t, v."""
    cs = jw.creation_ops(2 * nsite)
    t, v = fci.spin_integrals(prob.h1e, prob.g2e)
    return cs, t, v


def _check(op, O, W, tol=1e-12):
    for q, blk in op.blocks.items():
        qb = (q[0] + op.dq[0], q[1] + op.dq[1])
        ref = W[qb].T @ O @ W[q]
        assert np.allclose(blk, ref, atol=tol, rtol=0), (q, np.abs(blk - ref).max())
    # blocks absent from op must vanish in the definition
    for q in W:
        qb = (q[0] + op.dq[0], q[1] + op.dq[1])
        if q not in op.blocks and qb in W:
            assert np.abs(W[qb].T @ O @ W[q]).max() < tol


def test_left_block_operators_match_definition():
    prob = synth.make_problem(8, 8, 0, 12, 41)
    ints = bo.Integrals(prob.h1e, prob.g2e)
    n = 3
    blk = bo.build_left(prob, ints, n)
    states = fci._block_states(prob.left_dims[: n + 1], prob.left_iso[:n], True)
    W = _block_W(states, 2 * n)
    cs = jw.creation_ops(2 * n)
    ds = [c.T for c in cs]
    t, v = fci.spin_integrals(prob.h1e, prob.g2e)
    modes = list(range(2 * n))
    _check(blk.ops[("H",)], jw.hamiltonian(t[:2 * n, :2 * n], v[:2 * n, :2 * n, :2 * n, :2 * n], cs), W)
    for p in modes:
        _check(blk.C(p), cs[p], W)
        for q in modes:
            _check(blk.B(p, q), cs[p] @ ds[q], W)
            if p < q:
                _check(blk.A(p, q), cs[p] @ cs[q], W)
    for p in range(2 * n, 2 * prob.K, 3):
        R = sum(0.5 * t[p, q] * ds[q] for q in modes)
        for q in modes:
            for r in modes:
                for s in modes:
                    if v[p, q, r, s]:
                        R = R + v[p, q, r, s] * cs[r] @ ds[s] @ ds[q]
        _check(blk.ops[("R", p)], R, W)


@pytest.mark.parametrize("scheme", ["CN", "NC"])
def test_right_block_operators_match_definition(scheme):
    prob = synth.make_problem(8, 8, 0, 12, 43)
    ints = bo.Integrals(prob.h1e, prob.g2e)
    n = 3
    K = prob.K
    blk = bo.build_right(prob, ints, n, scheme)
    states = fci._block_states(prob.right_dims[: n + 1], prob.right_iso[:n], False)
    W = _block_W(states, 2 * n)
    cs = jw.creation_ops(2 * n)
    ds = [c.T for c in cs]
    t, v = fci.spin_integrals(prob.h1e, prob.g2e)
    o0 = 2 * (K - n)                       # first spin-orbital of the block
    modes = list(range(2 * n))
    tb = t[o0:, o0:]
    vb = v[o0:, o0:, o0:, o0:]
    _check(blk.ops[("H",)], jw.hamiltonian(tb, vb, cs), W)
    for p in modes:
        _check(blk.C(o0 + p), cs[p], W)
    outside = list(range(0, o0, 3))
    for p in outside:
        R = sum(0.5 * t[p, o0 + q] * ds[q] for q in modes)
        for q in modes:
            for r in modes:
                for s in modes:
                    c = v[p, o0 + q, o0 + r, o0 + s]
                    if c:
                        R = R + c * cs[r] @ ds[s] @ ds[q]
        _check(blk.ops[("R", p)], R, W)
    if scheme == "CN":
        for p in modes:
            for q in modes:
                _check(blk.B(o0 + p, o0 + q), cs[p] @ ds[q], W)
                if p < q:
                    _check(blk.A(o0 + p, o0 + q), cs[p] @ cs[q], W)
        blk = bo.to_complementary(blk, ints, list(range(o0)))
    for p in outside:
        for r in range(o0):
            Qpr = 0
            for a in modes:
                for b in modes:
                    c = v[p, r, o0 + a, o0 + b] - v[p, o0 + b, o0 + a, r]
                    if c:
                        Qpr = Qpr + c * cs[a] @ ds[b]
            _check(blk.ops[("Q", p, r)], Qpr, W)
            if p < r:
                Ppr = 0
                for a in modes:
                    for b in modes:
                        c = v[p, o0 + a, r, o0 + b]
                        if c:
                            Ppr = Ppr + c * ds[b] @ ds[a]
                _check(blk.ops[("P", p, r)], Ppr, W)


CASES = [
    (4, 4, 0, None, 11),     # untruncated
    (6, 6, 0, 8, 12),        # truncated
    (6, 5, 1, 6, 13),        # odd N, S_z = 1/2
    (6, 6, 2, 7, 14),        # S_z = 1
    (8, 7, 1, 14, 15),
]


@pytest.mark.parametrize("K,N,tsz,M,seed", CASES)
@pytest.mark.parametrize("scheme", ["CN", "NC"])
def test_heff_equals_definition(K, N, tsz, M, seed, scheme):
    p = synth.make_problem(K, N, tsz, M, seed)
    Hm = bo.MiddleHeff(p, scheme)
    W, _ = fci.embedding(p)
    H = fci.FCIHamiltonian(p.h1e, p.g2e, *p.target)
    for x in [p.psi, synth.random_vectors(p.psi.size, 1, seed + 7)[0]]:
        s2 = Hm.apply(x)
        s1 = fci.heff_apply_definition(p, x, W, H)
        assert np.linalg.norm(s2 - s1) <= 1e-13 * np.linalg.norm(s1)


def test_c1_full_energy_equals_fci():
    p = synth.config_problem("C1")
    Hm = bo.MiddleHeff(p, "CN")
    n = p.psi.size
    op = sla.LinearOperator((n, n), matvec=Hm.apply, dtype=float)
    e_dmrg = sla.eigsh(op, k=1, which="SA", tol=1e-13, v0=p.psi)[0][0]
    e_fci = np.linalg.eigvalsh(fci.FCIHamiltonian(p.h1e, p.g2e, *p.target).dense())[0]
    assert abs(e_dmrg - e_fci) < 1e-10


def test_truncated_energy_is_upper_bound():
    p = synth.make_problem(8, 8, 0, 10, 55)
    Hm = bo.MiddleHeff(p, "CN")
    n = p.psi.size
    op = sla.LinearOperator((n, n), matvec=Hm.apply, dtype=float)
    e_dmrg = sla.eigsh(op, k=1, which="SA", tol=1e-12, v0=p.psi)[0][0]
    e_fci = fci.fci_ground_energy(p.h1e, p.g2e, *p.target)
    assert e_dmrg > e_fci + 1e-6


def test_heff_hermitian_and_index_symmetry():
    p = synth.make_problem(8, 8, 0, 16, 61)
    Hm = bo.MiddleHeff(p, "CN")
    xs = synth.random_vectors(p.psi.size, 2, 3)
    a = xs[0] @ Hm.apply(xs[1])
    b = Hm.apply(xs[0]) @ xs[1]
    assert abs(a - b) < 1e-12 * max(1.0, abs(a))
    Rb = Hm.Rb
    before = list(range(0, 2 * (p.KL + 2)))
    for pp in before[::3]:
        for qq in before[::2]:
            Qpq, Qqp = Rb.ops[("Q", pp, qq)], Rb.ops[("Q", qq, pp)]
            for q, blk in Qpq.T.blocks.items():
                assert np.allclose(blk, Qqp.blocks.get(q, 0 * blk), atol=1e-13)
    Lb = Hm.Lb
    for pp in Lb.orbs[::3]:
        for qq in Lb.orbs[::2]:
            for q, blk in Lb.B(pp, qq).T.blocks.items():
                assert np.allclose(blk, Lb.B(qq, pp).blocks.get(q, 0 * blk), atol=1e-13)


@pytest.mark.parametrize("P", [2, 3, 16])
def test_sub_hamiltonian_sum(P):
    p = synth.make_problem(6, 6, 0, 8, 21)
    full = bo.MiddleHeff(p, "NC").apply(p.psi)
    acc = np.zeros_like(full)
    for q in range(1, P + 1):
        hp, gp = share.masked_integrals(p.h1e, p.g2e, P, q)
        s_nc = bo.MiddleHeff(p, "NC", hp, gp).apply(p.psi)
        s_cn = bo.MiddleHeff(p, "CN", hp, gp).apply(p.psi)
        assert np.linalg.norm(s_nc - s_cn) <= 1e-13 * np.linalg.norm(full)
        acc += s_nc
    assert np.linalg.norm(acc - full) <= 1e-13 * np.linalg.norm(full)


def test_share_assignment_is_a_partition():
    K, P = 7, 5
    for i in range(1, K + 1):
        for j in range(1, K + 1):
            owners = [p for p in range(1, P + 1) if share.proc2(p, i, j, P)]
            assert len(owners) == 1
            assert share.proc2(owners[0], j, i, P)
    g = np.ones((K,) * 4)
    tot = sum(share.masked_integrals(np.ones((K, K)), g, P, p)[1] for p in range(1, P + 1))
    assert np.array_equal(tot, g)
    # the benzene-shaped share: 93 owned spatial pairs among 54 (1-based p = 1 of 16)
    own = share.owned_pairs(1, 16, 54)
    assert len(own) == 93 and sum(1 for (i, j) in own if i == j) == 3


def test_renormalized_left_block_matches_definition():
    prob = synth.make_problem(8, 8, 0, 12, 47)
    Hm = bo.MiddleHeff(prob, "CN")
    nxt = Hm.renormalize_left()
    n = prob.KL + 1
    states = fci._block_states(prob.left_dims[: prob.KL + 1] + [prob.next_dims],
                               prob.left_iso + [prob.next_iso], True)
    W = _block_W(states, 2 * n)
    cs = jw.creation_ops(2 * n)
    ds = [c.T for c in cs]
    t, v = fci.spin_integrals(prob.h1e, prob.g2e)
    m = 2 * n
    _check(nxt.ops[("H",)], jw.hamiltonian(t[:m, :m], v[:m, :m, :m, :m], cs), W)
    for pp in range(m):
        _check(nxt.C(pp), cs[pp], W)
        _check(nxt.B(pp, (pp + 3) % m), cs[pp] @ ds[(pp + 3) % m], W)
