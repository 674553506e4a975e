"""Pins of the sub-Hamiltonian assignment (Section II.B: eq. sum-h, sub-h,
proc-def, proc-def-nc) in the oracle's ``share`` module.

The expected owners below were worked out by hand from the printed
definitions, with 1-based orbital indices and p = 1..P (residue 0 is p = P):

  proc(p, i)    = 1 iff p = i (mod P)
  proc(p, i, j) = 1 iff p = (j-1) j / 2 + i (mod P) for i <= j (symmetric)
  NC rule on the sorted tuple i <= j <= k <= l:
                  owner = proc(., j) if j = k, else proc(., i, j)
  one-body weight of t_ij in H^(p): [proc(p, i) + proc(p, j)] / 2

Each case is chosen so that a plausible slip gives a different answer: the
j = k case sent to proc(p, i, j), the CN rule (k, l) used instead of (i, j),
residue 0 mapped to p = 0, t_ij given wholly to proc(p, i), an index made
0-based.
"""
import numpy as np
import pytest

import synth
from oracle import blockops as bo
from oracle import share


def owner(fn, P, *idx):
    owners = [p for p in range(1, P + 1) if fn(p, *idx, P)]
    assert len(owners) == 1, (idx, owners)
    return owners[0]


# (i, j) 1-based -> owner for P = 16, worked by hand:
#   (1,1): 0+1=1; (1,2): 1+1=2; (2,2): 1+2=3; (1,3): 3+1=4; (2,3): 3+2=5;
#   (3,3): 3+3=6; (5,6): 15+5=20=4 (mod 16); (1,6): 15+1=16 -> p=16;
#   (16,16): 120+16=136=8; (10,54): 1431+10=1441=1; (54,54): 1431+54=1485=13;
#   (100,108): 5778+100=5878=6.
PAIR16 = [((1, 1), 1), ((1, 2), 2), ((2, 2), 3), ((1, 3), 4), ((2, 3), 5), ((3, 3), 6),
          ((5, 6), 4), ((6, 5), 4), ((1, 6), 16), ((16, 16), 8), ((10, 54), 1), ((54, 10), 1),
          ((54, 54), 13), ((100, 108), 6)]


@pytest.mark.parametrize("ij,p", PAIR16)
def test_pair_owner_p16(ij, p):
    assert owner(share.proc2, 16, *ij) == p


def test_pair_owner_p3():
    # (1,1): 1; (1,2): 2; (2,2): 3 -> residue 0 -> p = 3; (2,3): 5 = 2 (mod 3)
    assert [owner(share.proc2, 3, *ij) for ij in [(1, 1), (1, 2), (2, 2), (2, 3)]] == [1, 2, 3, 2]


def test_single_owner():
    # P = 16: 1 -> 1, 16 -> 16 (residue 0), 17 -> 1, 32 -> 16, 33 -> 1
    assert [owner(share.proc1, 16, i) for i in [1, 16, 17, 32, 33]] == [1, 16, 1, 16, 1]


# sorted-tuple NC rule, P = 16 (1-based indices):
#   (1,3,3,5): j = k = 3 -> proc(3) = 3      (proc(1,3) would give 4)
#   (2,2,2,2): j = k = 2 -> proc(2) = 2      (proc(2,2) would give 3)
#   (1,2,5,7): j != k -> proc(1,2) = 2       (the CN rule proc(5,7) = 26 -> 10)
#   (3,3,4,9): j != k -> proc(3,3) = 6
#   (1,4,4,4): j = k = 4 -> proc(4) = 4      (proc(1,4) = 6+1 = 7)
#   (5,6,7,7): j != k -> proc(5,6) = 4       (the CN rule proc(7,7) = 28 -> 12)
#   (17,17,20,20): proc(17,17) = 136+17 = 153 = 9
QUAD16 = [((1, 3, 3, 5), 3), ((3, 5, 1, 3), 3), ((2, 2, 2, 2), 2), ((1, 2, 5, 7), 2), ((7, 5, 2, 1), 2),
          ((3, 3, 4, 9), 6), ((1, 4, 4, 4), 4), ((4, 1, 4, 4), 4), ((5, 6, 7, 7), 4), ((17, 17, 20, 20), 9)]


@pytest.mark.parametrize("idx,p", QUAD16)
def test_nc_tuple_owner_p16(idx, p):
    owners = [q for q in range(1, 17) if share.proc4_nc(q, idx, 16)]
    assert owners == [p]


def test_one_body_weights():
    # P = 4, p = 1 owns single indices 1, 5, 9 (1-based).  0-based entries:
    #   h[0,0] -> (1,1): 1;  h[0,1] -> (1,2): 1/2;  h[1,2] -> (2,3): 0;
    #   h[0,4] -> (1,5): 1;  h[4,6] -> (5,7): 1/2;  h[3,3] -> (4,4): 0;  h[8,1] -> (9,2): 1/2
    K = 10
    h = np.arange(1.0, K * K + 1).reshape(K, K)
    h = h + h.T
    hp, _ = share.masked_integrals(h, np.zeros((K,) * 4), 4, 1)
    expect = {(0, 0): 1.0, (0, 1): 0.5, (1, 2): 0.0, (0, 4): 1.0, (4, 6): 0.5, (3, 3): 0.0, (8, 1): 0.5}
    for (i, j), w in expect.items():
        assert hp[i, j] == w * h[i, j], (i, j)
        assert hp[j, i] == w * h[j, i], (i, j)
    # the weights of one entry over the four shares add to one
    tot = sum(share.masked_integrals(h, np.zeros((K,) * 4), 4, q)[0] for q in range(1, 5))
    assert np.array_equal(tot, h)


def test_two_body_mask_entries():
    # P = 16; 0-based g[i,j,k,l] with the 1-based tuple in the comment
    K = 8
    g = np.ones((K,) * 4)
    m3 = share.masked_integrals(np.zeros((K, K)), g, 16, 3)[1]
    m2 = share.masked_integrals(np.zeros((K, K)), g, 16, 2)[1]
    assert m3[0, 2, 2, 4] == 1.0     # (1,3,3,5) -> 3
    assert m3[2, 4, 0, 2] == 1.0     # same tuple, chemists' pair swap
    assert m3[0, 1, 4, 6] == 0.0     # (1,2,5,7) -> 2
    assert m2[0, 1, 4, 6] == 1.0
    assert m2[1, 1, 1, 1] == 1.0     # (2,2,2,2) -> 2
    assert m3[1, 1, 1, 1] == 0.0
    assert m3[2, 2, 3, 7] == 0.0     # (3,3,4,8) -> proc(3,3) = 6
    assert share.masked_integrals(np.zeros((K, K)), g, 16, 6)[1][2, 2, 3, 7] == 1.0


def test_nc_share_keeps_only_owned_two_index_pairs():
    """With the NC rule, the two-index complementary operators of the right
    block vanish unless the spatial pair of their left indices is owned
    (Section II.B: the NC sums run over the small indices i, j)."""
    P, pid = 5, 2
    p = synth.make_problem(8, 8, 0, 12, 31, n_proc=P, proc_id=pid)
    hp, gp = share.masked_integrals(p.h1e, p.g2e, P, pid)
    Hm = bo.MiddleHeff(p, "NC", hp, gp)
    seen_owned = seen_free = 0
    for key, op in Hm.Rb.ops.items():
        if key[0] not in ("P", "Q"):
            continue
        i, j = key[1] // 2 + 1, key[2] // 2 + 1
        nrm = sum(float(np.abs(b).sum()) for b in op.blocks.values())
        if share.proc2(pid, i, j, P):
            seen_owned += nrm > 0
        else:
            seen_free += 1
            assert nrm == 0.0, key
    assert seen_owned > 0 and seen_free > 0
