"""GPU parity of decimation and two-site sweeps (through the C ABI) against
the CPU oracle (oracle.sweep).

Bar: kept states per sector bit-exact (an integer decision taken from FP64
weights on both sides, with the same multiplet window); weights within 1e-13
(absolute, unit-norm wavefunctions); per-sector projectors U U^T within
1e-10 (the eigenvectors themselves are fixed only up to sign and rotations
inside degenerate multiplets); truncation errors within 1e-12; sweep
energies within 1e-8 E_h of the oracle's step by step (Davidson converged to
residual 1e-10), and within 1e-9 of FCI when nothing is truncated.
"""
import numpy as np
import pytest

import synth
from oracle import blockops, fci
from oracle import sweep as osw

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2103_09976_amd import dmrg
    return dmrg


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def _check_decimation(iso, ref):
    w = iso.weights()
    dims = iso.dims
    assert dims == ref.dims
    got = {}
    o = 0
    for q in sorted(dims):
        got[q] = w[o:o + dims[q]]
        o += dims[q]
    for q in ref.dims:
        np.testing.assert_allclose(got[q], ref.weights[q], rtol=0, atol=1e-13)
    U = iso.to_host()
    for q, Ur in ref.U.items():
        assert U[q].shape == Ur.shape
        np.testing.assert_allclose(U[q].T @ U[q], np.eye(Ur.shape[1]), atol=1e-12)
        np.testing.assert_allclose(U[q] @ U[q].T, Ur @ Ur.T, atol=1e-10)
    assert abs(iso.info["trunc_err"] - ref.trunc_err) < 1e-12
    assert iso.info["kept"] == ref.kept


@pytest.fixture(scope="module")
def nc_middle():
    d = _lib()
    p = synth.make_problem(10, 10, 0, 30, 7500)
    print(f"[gpu] decimation setup K={p.K} M={p.M}", flush=True)
    ctx, L, R, H, holders = d.middle_step(p, 1 << 30, "NC", n_roots=2, precision=d.DMRG_PREC_F64)
    ref = blockops.MiddleHeff(p, "NC")
    yield d, p, ctx, H, ref
    H.free()
    L.free()
    R.free()
    ctx.close()


@pytest.mark.parametrize("side", ["left", "right"])
@pytest.mark.parametrize("M", [None, 7, 40])
def test_decimation_matches_oracle(nc_middle, side, M):
    d, p, ctx, H, ref = nc_middle
    print(f"[gpu] decimate side={side} M={M}", flush=True)
    iso = H.decimate(_dev(p.psi), d.DMRG_LEFT if side == "left" else d.DMRG_RIGHT, M or 0)
    try:
        _check_decimation(iso, osw.decimate(ref, [p.psi], side, M))
    finally:
        iso.free()


def test_decimation_two_roots_and_noise(nc_middle):
    d, p, ctx, H, ref = nc_middle
    x = synth.random_vectors(H.dim, 2, 77)
    xi = synth.random_vectors(H.dim, 2, 78)
    psis = np.stack([p.psi, x[0]])
    print("[gpu] decimate two roots with noise", flush=True)
    iso = H.decimate(_dev(psis), d.DMRG_LEFT, 25, n_vec=2, noise=1e-3, xi=_dev(xi))
    try:
        _check_decimation(iso, osw.decimate(ref, list(psis), "left", 25, noise=1e-3, xis=list(xi)))
    finally:
        iso.free()


def test_decimated_basis_renormalizes_like_the_oracle(nc_middle):
    """The left block renormalized through the decimated basis: its block
    Hamiltonian has the oracle's spectrum per sector (a gauge-invariant
    check of the transformation through the GPU's own isometry)."""
    d, p, ctx, H, ref = nc_middle
    iso = H.decimate(_dev(p.psi), d.DMRG_LEFT, 40)
    new = H.renormalize(iso)
    try:
        dec = osw.decimate(ref, [p.psi], "left", 40)
        blk = blockops.renorm_block(ref.Lp, dec.U, dec.dims)
        basis = new.basis()
        assert basis == dec.dims
        for q, m in basis.items():
            h = new.block("H", -1, -1, q, (m, m))
            hr = blk.ops[("H",)].blocks[q]
            np.testing.assert_allclose(np.linalg.eigvalsh(0.5 * (h + h.T)), np.linalg.eigvalsh(hr), atol=1e-10)
    finally:
        new.free()
        iso.free()


def _sweep_pair(K, N, tsz, M, seed, n_sweeps, n_roots=1, noise=0.0):
    d = _lib()
    from paper_2103_09976_amd import sweep as gsw
    inp = synth.make_sweep_inputs(K, N, tsz, M, seed)
    start = lambda dim, s, n: synth.random_vectors(dim, n, s)  # noqa: E731
    seed_of = lambda sw, b, KL: synth.sweep_seed(inp, sw, b, KL)  # noqa: E731
    nvec = lambda dim, s: synth.random_vectors(dim, 1, s)[0]  # noqa: E731
    ctx = d.Context(1 << 30)
    try:
        print(f"[gpu] sweeps K={K} N={N} M={M} roots={n_roots} noise={noise}", flush=True)
        got = gsw.run_sweeps(ctx, inp, n_sweeps, M, start, seed_of, n_roots=n_roots, tol=1e-10,
                             noise=noise, noise_vec=nvec)
    finally:
        ctx.close()
    ref = osw.sweeps(inp, n_sweeps, start, M=M, n_roots=n_roots, noise=noise, noise_vec=nvec, seed_of=seed_of)
    assert len(got) == len(ref)
    for g, r in zip(got, ref):
        assert (g.KL, g.backward, g.dim) == (r.KL, r.backward, r.dim)
        np.testing.assert_allclose(g.energies, r.energies, rtol=0, atol=1e-8)
        assert g.kept == r.kept and g.dims == r.dims
        assert abs(g.trunc_err - r.trunc_err) < 1e-9
    return inp, got


@pytest.mark.parametrize("K,N,tsz,seed", [(6, 6, 0, 7200), (6, 5, 1, 7300)])
def test_untruncated_sweep_gives_fci(K, N, tsz, seed):
    inp, got = _sweep_pair(K, N, tsz, None, seed, 1)
    e_fci = fci.fci_ground_energy(inp.h1e, inp.g2e, *inp.target)
    for st in got:
        assert abs(st.energies[0] - e_fci) < 1e-9


@pytest.mark.parametrize("M", [4, 12])
def test_truncated_sweeps_match_oracle(M):
    _sweep_pair(7, 6, 0, M, 7400, 2)


@pytest.mark.parametrize("K,N,tsz,M,seed,n_sweeps", [(10, 10, 0, 40, 7800, 2), (10, 9, 1, 30, 7900, 1)])
def test_ten_orbital_sweeps_match_oracle(K, N, tsz, M, seed, n_sweeps):
    """Ten orbitals, M = 40 and 30: blocks of up to 40 rows span three 16-row
    tiles with a ragged tail, and H_eff reaches a few thousand states; even and
    odd electron counts."""
    _sweep_pair(K, N, tsz, M, seed, n_sweeps)


def test_two_root_sweep_matches_oracle():
    _sweep_pair(6, 6, 0, 10, 7600, 1, n_roots=2)


def test_noisy_sweep_stays_variational():
    """With noise the kept bases depend on the perturbation as written in each
    side's own basis (the decimated bases agree only up to the signs of their
    vectors), so a noisy sweep is checked by its properties: every energy at
    or above FCI, and the final energy within 1e-3 of the noiseless sweep's
    (the single-step noisy decimation is compared with the oracle above)."""
    d = _lib()
    from paper_2103_09976_amd import sweep as gsw
    inp = synth.make_sweep_inputs(7, 6, 0, 12, 7400)
    e_fci = fci.fci_ground_energy(inp.h1e, inp.g2e, *inp.target)
    start = lambda dim, s, n: synth.random_vectors(dim, n, s)  # noqa: E731
    seed_of = lambda sw, b, KL: synth.sweep_seed(inp, sw, b, KL)  # noqa: E731
    nvec = lambda dim, s: synth.random_vectors(dim, 1, s)[0]  # noqa: E731
    finals = []
    for noise in (0.0, 1e-4):
        ctx = d.Context(1 << 30)
        try:
            print(f"[gpu] noisy sweep noise={noise}", flush=True)
            got = gsw.run_sweeps(ctx, inp, 2, 12, start, seed_of, tol=1e-10, noise=noise, noise_vec=nvec)
        finally:
            ctx.close()
        for st in got:
            assert st.energies[0] >= e_fci - 1e-9
        finals.append(got[-1].energies[0])
    assert abs(finals[1] - finals[0]) < 1e-3


def test_mixed_precision_sweep_matches_oracle():
    """The FP32-mixed policy (FP32 products while the residual is large, FP64
    to finish) inside a sweep: the same energies and kept dimensions as the
    oracle's exact solves."""
    d = _lib()
    from paper_2103_09976_amd import sweep as gsw
    inp = synth.make_sweep_inputs(7, 6, 0, 8, 7700)
    start = lambda dim, s, n: synth.random_vectors(dim, n, s)  # noqa: E731
    seed_of = lambda sw, b, KL: synth.sweep_seed(inp, sw, b, KL)  # noqa: E731
    ctx = d.Context(1 << 30)
    try:
        print("[gpu] mixed-precision sweep K=7 M=8", flush=True)
        got = gsw.run_sweeps(ctx, inp, 1, 8, start, seed_of, tol=1e-10, precision=d.DMRG_PREC_F32)
    finally:
        ctx.close()
    ref = osw.sweeps(inp, 1, start, M=8, seed_of=seed_of)
    for g, r in zip(got, ref):
        np.testing.assert_allclose(g.energies, r.energies, rtol=0, atol=1e-8)
        assert g.kept == r.kept and g.dims == r.dims
    assert any(g.davidson.get("matvecs_f32", 0) > 0 for g in got)


def test_bond_dimension_schedule_matches_oracle():
    d = _lib()
    from paper_2103_09976_amd import sweep as gsw
    inp = synth.make_sweep_inputs(7, 6, 0, 8, 7400)
    start = lambda dim, s, n: synth.random_vectors(dim, n, s)  # noqa: E731
    seed_of = lambda sw, b, KL: synth.sweep_seed(inp, sw, b, KL)  # noqa: E731
    sched = [(4, 0.0), (12, 0.0)]
    ctx = d.Context(1 << 30)
    try:
        print("[gpu] schedule sweep K=7 M=4,12", flush=True)
        got = gsw.run_sweeps(ctx, inp, 0, None, start, seed_of, tol=1e-10, schedule=sched)
    finally:
        ctx.close()
    ref = osw.sweeps(inp, 0, start, seed_of=seed_of, schedule=sched)
    assert len(got) == len(ref) == 16
    for g, r in zip(got, ref):
        np.testing.assert_allclose(g.energies, r.energies, rtol=0, atol=1e-8)
        assert g.kept == r.kept and g.dims == r.dims
