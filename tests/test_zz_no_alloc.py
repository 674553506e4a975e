"""dmrg_heff_apply_static -- the entry point that allocates nothing (the
partial tiles of split tasks live in the library's static 256 MiB device
array) -- against dmrg_heff_apply on the same H_eff, through the C ABI:
bitwise equal, FP64 and FP32, on two calls in a row, the second with a
smaller input; an H_eff whose partial tiles exceed the array is refused with
DMRG_E_WORKSPACE before any device work."""
import ctypes as C

import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

SCRATCH = 256 << 20


def _static(d):
    f = d.load().dmrg_heff_apply_static
    f.restype = C.c_int32
    f.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
    return f


def _call(d, H, x, y, prec, n_vec):
    return _static(d)(H.ptr, prec, n_vec, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                      C.c_void_p(torch.cuda.current_stream().cuda_stream))


def test_static_scratch_product_matches_arena_product():
    from paper_2103_09976_amd import dmrg as d
    lib = d.load()
    # problems whose split tiles fit the array, the larger first (the second call's input is smaller)
    shapes = [(12, 12, 0, 60, 28), (10, 10, 0, 30, 23), (10, 9, 1, 30, 24), (8, 8, 0, 14, 47)]
    used = []
    for (K, N, tsz, M, seed) in shapes:
        if len(used) == 2:
            break
        p = synth.make_problem(K, N, tsz, M, seed)
        ctx, L, R, H, keep = d.middle_step(p, 4 << 30, n_roots=2)
        info = H.info()
        fits = 0 < info["partial_elems"] * 8 <= SCRATCH
        print(f"[gpu] static scratch K={K} M={M}: reductions {info['reductions']} "
              f"partial {info['partial_elems'] * 8} B fits={fits}", flush=True)
        if fits:
            nv = 2 if not used else 1
            X = torch.from_numpy(synth.random_vectors(H.dim, nv, 40 + len(used)).ravel().copy()).cuda()
            for prec, dt in ((d.DMRG_PREC_F64, torch.float64), (d.DMRG_PREC_F32, torch.float32)):
                x = X.to(dt)
                ref = torch.empty_like(x)
                got = torch.full_like(x, float("nan"))
                H.apply(x, ref, prec, nv)
                st = _call(d, H, x, got, prec, nv)
                torch.cuda.synchronize()
                assert st == 0, lib.dmrg_last_error()
                assert torch.equal(ref, got), (K, M, prec)
            used.append((K, M, H.dim))
        for o in (H, L, R):
            o.free()
        ctx.close()
    assert len(used) == 2 and used[1][2] < used[0][2], used


def test_static_scratch_refuses_oversized_partials():
    from paper_2103_09976_amd import dmrg as d
    p = synth.make_problem(14, 14, 0, 1000, 82)
    ctx, L, R, H, keep = d.middle_step(p, 8 << 30)
    assert H.info()["partial_elems"] * 8 > SCRATCH
    x = torch.from_numpy(p.psi.copy()).cuda()
    y = torch.empty_like(x)
    st = _call(d, H, x, y, d.DMRG_PREC_F64, 1)
    msg = d.load().dmrg_last_error()
    for o in (H, L, R):
        o.free()
    ctx.close()
    assert st == -3 and b"static scratch" in msg, (st, msg)
