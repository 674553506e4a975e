"""Thin ctypes binding of libdmrg_hip.so (the C ABI declared in include/dmrg.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch provides device memory (the context arena and the
caller's psi / sigma / isometry tensors) and the current stream.  The
binding fails loudly when the library is missing; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdmrg_hip.so")

DMRG_OK = 0
DMRG_LEFT, DMRG_RIGHT = 0, 1
DMRG_SCHEME_NC, DMRG_SCHEME_CN = 0, 1
DMRG_F64, DMRG_F32 = 0, 1
DMRG_PREC_F64, DMRG_PREC_F32 = 0, 1
DMRG_HEFF_LAUNCHES = 23   # kernel launches of one H_eff product (dmrg_heff_profile)

SITE_Q = ((0, 0), (1, 0), (0, 1), (1, 1))


class DmrgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"dmrg status {status}: {msg}")
        self.status = status


class Bsm(C.Structure):
    _fields_ = [("n_blocks", C.c_int32), ("qn_row", C.POINTER(C.c_int32)),
                ("qn_col", C.POINTER(C.c_int32)), ("rows", C.POINTER(C.c_int64)),
                ("cols", C.POINTER(C.c_int64)), ("offset", C.POINTER(C.c_int64)),
                ("dtype", C.c_int32), ("data", C.c_void_p)]


class DavOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("max_subspace", C.c_int32), ("tol", C.c_double),
                ("precision", C.c_int32), ("switch_tol", C.c_double), ("fixed_iters", C.c_int32),
                ("precond_clamp", C.c_double)]


class DavStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("matvecs", C.c_int32), ("matvecs_f32", C.c_int32),
                ("converged", C.c_int32), ("max_residual", C.c_double), ("ms_total", C.c_double),
                ("ms_matvec", C.c_double)]


class PsiLayout(C.Structure):
    _fields_ = [("n_blocks", C.c_int32), ("qn_left", C.POINTER(C.c_int32)), ("site1", C.POINTER(C.c_int32)),
                ("site2", C.POINTER(C.c_int32)), ("offset", C.POINTER(C.c_int64))]


DMRG_WS_BLOCK, DMRG_WS_TRANSFORM, DMRG_WS_HEFF, DMRG_WS_DAVIDSON, DMRG_WS_RENORMALIZE = 0, 1, 2, 3, 4
DMRG_HEFF_GRAPH, DMRG_HEFF_AUTOTUNE = 1, 2


class HeffInfo(C.Structure):
    _fields_ = [("flags", C.c_int32), ("balance_target", C.c_int32), ("tall_min_rows", C.c_int32),
                ("tuned", C.c_int32), ("n_candidates", C.c_int32), ("candidate_ms", C.c_float * 8),
                ("candidate_balance", C.c_int32 * 8), ("candidate_tall_min", C.c_int32 * 8),
                ("graphs", C.c_int32), ("graph_launches", C.c_int64), ("tasks", C.c_int64),
                ("reductions", C.c_int32), ("partial_elems", C.c_int64)]


class DecimInfo(C.Structure):
    _fields_ = [("kept", C.c_int64), ("n_blocks", C.c_int32), ("trunc_err", C.c_double),
                ("weight_total", C.c_double)]


class WsBlock(C.Structure):
    _fields_ = [("K", C.c_int32), ("n_elec", C.c_int32), ("two_sz", C.c_int32), ("n_proc", C.c_int32),
                ("proc_id", C.c_int32), ("side", C.c_int32), ("n_sites", C.c_int32), ("scheme", C.c_int32),
                ("isometries", C.POINTER(Bsm))]


class WsTransform(C.Structure):
    _fields_ = [("right", C.c_void_p)]


class WsHeff(C.Structure):
    _fields_ = [("left", C.c_void_p), ("right", C.c_void_p), ("n_roots", C.c_int32), ("precision", C.c_int32)]


class WsDavidson(C.Structure):
    _fields_ = [("dim", C.c_int64), ("n_roots", C.c_int32), ("opts", DavOpts)]


class WsRenorm(C.Structure):
    _fields_ = [("inp", C.c_void_p), ("isometry", C.POINTER(Bsm))]


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "dmrg_status_string": (C.c_char_p, [C.c_int32]),
    "dmrg_last_error": (C.c_char_p, []),
    "dmrg_create": (C.c_int32, [C.POINTER(C.c_void_p), C.c_int32, C.c_void_p, C.c_int64]),
    "dmrg_destroy": (None, [C.c_void_p]),
    "dmrg_arena_used": (C.c_int64, [C.c_void_p]),
    "dmrg_arena_peak": (C.c_int64, [C.c_void_p]),
    "dmrg_set_integrals": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                       C.c_void_p, C.c_void_p, C.c_double, C.c_int32, C.c_int32]),
    "dmrg_build_block": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(Bsm), C.c_int32,
                                     C.POINTER(C.c_void_p), C.c_void_p]),
    "dmrg_normal_to_complementary": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "dmrg_heff_create": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(PsiLayout), C.c_int32,
                                     C.c_int32, C.c_int32, C.POINTER(C.c_void_p), C.c_void_p]),
    "dmrg_heff_get_info": (C.c_int32, [C.c_void_p, C.POINTER(HeffInfo)]),
    "dmrg_heff_dim": (C.c_int64, [C.c_void_p]),
    "dmrg_heff_psi_layout": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_void_p, C.c_void_p, C.c_void_p]),
    "dmrg_davidson_start": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(DavOpts),
                                        C.POINTER(C.c_void_p), C.c_void_p]),
    "dmrg_davidson_step": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                       C.POINTER(C.c_double)]),
    "dmrg_davidson_finish": (C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(C.c_double), C.POINTER(DavStats)]),
    "dmrg_davidson_free": (None, [C.c_void_p]),
    "dmrg_heff_renormalize": (C.c_int32, [C.c_void_p, C.POINTER(Bsm), C.POINTER(C.c_void_p), C.c_void_p]),
    "dmrg_query_workspace": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(C.c_int64)]),
    "dmrg_heff_apply": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                    C.c_void_p]),
    "dmrg_heff_diag": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "dmrg_davidson": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(C.c_double),
                                  C.POINTER(DavOpts), C.POINTER(DavStats), C.c_void_p]),
    "dmrg_renormalize": (C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(Bsm), C.POINTER(C.c_void_p),
                                     C.c_void_p]),
    "dmrg_heff_flops": (C.c_int64, [C.c_void_p]),
    "dmrg_heff_bytes": (C.c_int64, [C.c_void_p, C.c_int32]),
    "dmrg_heff_terms": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int32)]),
    "dmrg_heff_profile": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32,
                                      C.POINTER(C.c_float), C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                      C.c_void_p]),
    "dmrg_opset_basis": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "dmrg_opset_block": (C.c_int32, [C.c_void_p, C.c_char, C.c_int32, C.c_int32, C.c_void_p,
                                     C.c_void_p, C.c_int64]),
    "dmrg_decimate": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_double, C.c_void_p,
                                  C.c_int32, C.POINTER(C.c_void_p), C.POINTER(DecimInfo), C.c_void_p]),
    "dmrg_iso_bsm": (C.c_int32, [C.c_void_p, C.POINTER(Bsm)]),
    "dmrg_iso_weights": (C.c_int64, [C.c_void_p, C.c_int64, C.c_void_p]),
    "dmrg_iso_free": (None, [C.c_void_p]),
    "dmrg_opset_free": (None, [C.c_void_p]),
    "dmrg_heff_free": (None, [C.c_void_p]),
}


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with python -m paper_2103_09976_amd.build_lib")
    lib = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(st: int):
    if st != DMRG_OK:
        lib = load()
        raise DmrgError(st, f"{lib.dmrg_status_string(st).decode()}: {lib.dmrg_last_error().decode()}")


def _stream(torch):
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Isometry:
    """Device copy of one site isometry {q: U_q (d_q x m_q)} as a dmrg_bsm.
    With device=None only the metadata is kept (data = NULL), which is what
    the workspace queries read."""

    def __init__(self, iso: Dict[Tuple[int, int], np.ndarray], device):
        qs = sorted(iso)
        offs, rows, cols = [], [], []
        o = 0
        for q in qs:
            d, m = iso[q].shape
            offs.append(o)
            rows.append(d)
            cols.append(m)
            o += d * m
        if device is None:
            self.data = None
            ptr = None
        else:
            import torch
            host = np.concatenate([np.ascontiguousarray(iso[q], dtype=np.float64).ravel() for q in qs])
            self.data = torch.from_numpy(host).to(device)
            ptr = self.data.data_ptr()
        qn = np.array([x for q in qs for x in q], dtype=np.int32)
        self._qn = qn
        self._rows = np.array(rows, dtype=np.int64)
        self._cols = np.array(cols, dtype=np.int64)
        self._offs = np.array(offs, dtype=np.int64)
        self.bsm = Bsm(len(qs), self._qn.ctypes.data_as(C.POINTER(C.c_int32)),
                       self._qn.ctypes.data_as(C.POINTER(C.c_int32)),
                       self._rows.ctypes.data_as(C.POINTER(C.c_int64)),
                       self._cols.ctypes.data_as(C.POINTER(C.c_int64)),
                       self._offs.ctypes.data_as(C.POINTER(C.c_int64)), DMRG_F64, C.c_void_p(ptr))


class DecimatedIsometry:
    """An isometry made by dmrg_decimate, held in the context arena; usable
    wherever an Isometry is (its .bsm)."""

    def __init__(self, ctx: "Context", ptr: C.c_void_p, info: DecimInfo):
        self.ctx = ctx
        self.ptr = ptr
        self.info = {f: getattr(info, f) for f, _ in DecimInfo._fields_}
        self.bsm = Bsm()
        _check(load().dmrg_iso_bsm(self.ptr, C.byref(self.bsm)))

    @property
    def dims(self) -> Dict[Tuple[int, int], int]:
        b = self.bsm
        return {(b.qn_col[2 * i], b.qn_col[2 * i + 1]): int(b.cols[i]) for i in range(b.n_blocks)}

    def weights(self) -> np.ndarray:
        lib = load()
        n = lib.dmrg_iso_weights(self.ptr, 0, None)
        w = np.zeros(n)
        lib.dmrg_iso_weights(self.ptr, n, w.ctypes.data_as(C.c_void_p))
        return w

    def to_host(self) -> Dict[Tuple[int, int], np.ndarray]:
        """{q: U_q} copied to the host (device bytes read through the arena tensor)."""
        import torch
        b = self.bsm
        base = self.ctx.arena.data_ptr()
        off0 = b.data - base
        n = sum(int(b.rows[i]) * int(b.cols[i]) for i in range(b.n_blocks))
        flat = self.ctx.arena[off0:off0 + 8 * n].view(torch.float64).cpu().numpy()
        out = {}
        for i in range(b.n_blocks):
            o, r, c = int(b.offset[i]), int(b.rows[i]), int(b.cols[i])
            out[(b.qn_col[2 * i], b.qn_col[2 * i + 1])] = flat[o:o + r * c].reshape(r, c).copy()
        return out

    def free(self):
        if self.ptr:
            load().dmrg_iso_free(self.ptr)
            self.ptr = None


class OpSet:
    def __init__(self, ctx: "Context", ptr: C.c_void_p):
        self.ctx = ctx
        self.ptr = ptr

    def basis(self) -> Dict[Tuple[int, int], int]:
        lib = load()
        n = lib.dmrg_opset_basis(self.ptr, 0, None, None)
        qn = np.zeros(2 * n, dtype=np.int32)
        dims = np.zeros(n, dtype=np.int64)
        lib.dmrg_opset_basis(self.ptr, n, qn.ctypes.data_as(C.c_void_p), dims.ctypes.data_as(C.c_void_p))
        return {(int(qn[2 * i]), int(qn[2 * i + 1])): int(dims[i]) for i in range(n)}

    def block(self, kind: str, p: int, q: int, qket: Tuple[int, int], shape) -> np.ndarray:
        out = np.zeros(shape, dtype=np.float64)
        qk = np.array(qket, dtype=np.int32)
        _check(load().dmrg_opset_block(self.ptr, kind.encode(), p, q, qk.ctypes.data_as(C.c_void_p),
                                       out.ctypes.data_as(C.c_void_p), out.size))
        return out

    def free(self):
        if self.ptr:
            load().dmrg_opset_free(self.ptr)
            self.ptr = None


class Heff:
    def __init__(self, ctx: "Context", ptr: C.c_void_p):
        self.ctx = ctx
        self.ptr = ptr

    @property
    def dim(self) -> int:
        return int(load().dmrg_heff_dim(self.ptr))

    @property
    def flops(self) -> int:
        return int(load().dmrg_heff_flops(self.ptr))

    def bytes(self, precision: int) -> int:
        return int(load().dmrg_heff_bytes(self.ptr, precision))

    def terms(self) -> Tuple[int, int, int]:
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        load().dmrg_heff_terms(self.ptr, C.byref(a), C.byref(b), C.byref(c))
        return a.value, b.value, c.value

    def profile(self, psi, sigma, precision: int = DMRG_PREC_F64):
        """One product with every kernel launch timed (HIP events on the current
        stream): list of (kind, ms, useful_flops) per launch, in launch-slot order."""
        import torch
        want = torch.float64 if precision == DMRG_PREC_F64 else torch.float32
        assert psi.dtype == want and sigma.dtype == want and psi.is_cuda and sigma.is_cuda
        assert psi.numel() >= self.dim and sigma.numel() >= self.dim
        n = DMRG_HEFF_LAUNCHES
        ms, fl, kd = (C.c_float * n)(), (C.c_double * n)(), (C.c_int32 * n)()
        r = load().dmrg_heff_profile(self.ptr, precision, C.c_void_p(psi.data_ptr()),
                                     C.c_void_p(sigma.data_ptr()), n, ms, fl, kd, _stream(torch))
        if r < 0:
            _check(r)
        return [(int(kd[i]), float(ms[i]), float(fl[i])) for i in range(r)]

    def apply(self, psi, sigma, precision: int = DMRG_PREC_F64, n_vec: int = 1):
        import torch
        want = torch.float64 if precision == DMRG_PREC_F64 else torch.float32
        assert psi.dtype == want and sigma.dtype == want and psi.is_cuda and sigma.is_cuda
        assert psi.numel() >= n_vec * self.dim and sigma.numel() >= n_vec * self.dim
        _check(load().dmrg_heff_apply(self.ptr, precision, n_vec, C.c_void_p(psi.data_ptr()),
                                      C.c_void_p(sigma.data_ptr()), _stream(torch)))

    def diag(self, out):
        import torch
        assert out.dtype == torch.float64 and out.numel() >= self.dim
        _check(load().dmrg_heff_diag(self.ptr, C.c_void_p(out.data_ptr()), _stream(torch)))

    def davidson(self, psi, n_roots: int = 1, tol: float = 1e-6, max_iter: int = 300,
                 max_subspace: int = 24, precision: int = DMRG_PREC_F64, switch_tol: float = 1e-4,
                 fixed_iters: int = 0, precond_clamp: float = 0.0):
        import torch
        assert psi.dtype == torch.float64 and psi.numel() >= n_roots * self.dim
        e = (C.c_double * n_roots)()
        opts = DavOpts(max_iter, max_subspace, tol, precision, switch_tol, fixed_iters, precond_clamp)
        st = DavStats()
        _check(load().dmrg_davidson(self.ptr, n_roots, C.c_void_p(psi.data_ptr()), e, C.byref(opts),
                                    C.byref(st), _stream(torch)))
        stats = {f: getattr(st, f) for f, _ in DavStats._fields_}
        return np.array(list(e)), stats

    def davidson_start(self, psi0, n_roots: int = 1, tol: float = 1e-6, max_iter: int = 300,
                       max_subspace: int = 24, precision: int = DMRG_PREC_F64, switch_tol: float = 1e-4,
                       fixed_iters: int = 0, precond_clamp: float = 0.0) -> "DavidsonSolve":
        import torch
        assert psi0.dtype == torch.float64 and psi0.numel() >= n_roots * self.dim
        opts = DavOpts(max_iter, max_subspace, tol, precision, switch_tol, fixed_iters, precond_clamp)
        out = C.c_void_p()
        _check(load().dmrg_davidson_start(self.ptr, n_roots, C.c_void_p(psi0.data_ptr()), C.byref(opts),
                                          C.byref(out), _stream(torch)))
        return DavidsonSolve(out, n_roots)

    def info(self) -> dict:
        """Work-list parameters (tuned or default), tuning record and graph use."""
        x = HeffInfo()
        _check(load().dmrg_heff_get_info(self.ptr, C.byref(x)))
        n = x.n_candidates
        return {"flags": x.flags, "balance_target": x.balance_target, "tall_min_rows": x.tall_min_rows,
                "tuned": {0: "default", 1: "timed", 2: "cached"}[x.tuned],
                "candidates": [{"balance_target": x.candidate_balance[i], "tall_min_rows": x.candidate_tall_min[i],
                                "ms_f32": round(float(x.candidate_ms[i]), 3)} for i in range(n)],
                "graphs": x.graphs, "graph_launches": x.graph_launches, "tasks": x.tasks,
                "reductions": x.reductions, "partial_elems": x.partial_elems}

    def psi_layout(self):
        """[(qn_left, s1, s2, qn_right, rows, cols, offset)] of the layout in use."""
        lib = load()
        n = lib.dmrg_heff_psi_layout(self.ptr, 0, None, None, None, None, None, None, None)
        ql, qr = np.zeros(2 * n, np.int32), np.zeros(2 * n, np.int32)
        s1, s2 = np.zeros(n, np.int32), np.zeros(n, np.int32)
        rows, cols, off = np.zeros(n, np.int64), np.zeros(n, np.int64), np.zeros(n, np.int64)
        ptr = lambda a: a.ctypes.data_as(C.c_void_p)  # noqa: E731
        lib.dmrg_heff_psi_layout(self.ptr, n, ptr(ql), ptr(s1), ptr(s2), ptr(qr), ptr(rows), ptr(cols), ptr(off))
        return [((int(ql[2 * i]), int(ql[2 * i + 1])), int(s1[i]), int(s2[i]), (int(qr[2 * i]), int(qr[2 * i + 1])),
                 int(rows[i]), int(cols[i]), int(off[i])) for i in range(n)]

    def decimate(self, psi, side: int = DMRG_LEFT, max_states: int = 0, n_vec: int = 1, noise: float = 0.0,
                 xi=None) -> DecimatedIsometry:
        """dmrg_decimate: the new basis of the block that moves on (side)."""
        import torch
        assert psi.dtype == torch.float64 and psi.is_cuda
        out = C.c_void_p()
        info = DecimInfo()
        xp = C.c_void_p(xi.data_ptr()) if xi is not None else None
        _check(load().dmrg_decimate(self.ptr, side, n_vec, C.c_void_p(psi.data_ptr()), float(noise), xp,
                                    int(max_states), C.byref(out), C.byref(info), _stream(torch)))
        return DecimatedIsometry(self.ctx, out, info)

    def renormalize(self, iso: Isometry) -> OpSet:
        """The blocked L' operators transformed through the isometry adding d1."""
        import torch
        out = C.c_void_p()
        _check(load().dmrg_heff_renormalize(self.ptr, C.byref(iso.bsm), C.byref(out), _stream(torch)))
        return OpSet(self.ctx, out)

    def free(self):
        if self.ptr:
            load().dmrg_heff_free(self.ptr)
            self.ptr = None


class DavidsonSolve:
    """A block Davidson solve driven one iteration at a time."""

    def __init__(self, ptr: C.c_void_p, n_roots: int):
        self.ptr = ptr
        self.n_roots = n_roots

    def step(self):
        """One iteration; returns (done, Ritz values, largest residual norm)."""
        done = C.c_int32()
        e = (C.c_double * self.n_roots)()
        r = C.c_double()
        _check(load().dmrg_davidson_step(self.ptr, C.byref(done), e, C.byref(r)))
        return bool(done.value), np.array(list(e)), r.value

    def finish(self, psi_out):
        import torch
        assert psi_out.dtype == torch.float64
        e = (C.c_double * self.n_roots)()
        st = DavStats()
        _check(load().dmrg_davidson_finish(self.ptr, C.c_void_p(psi_out.data_ptr()), e, C.byref(st)))
        return np.array(list(e)), {f: getattr(st, f) for f, _ in DavStats._fields_}

    def free(self):
        if self.ptr:
            load().dmrg_davidson_free(self.ptr)
            self.ptr = None


def query_workspace(ctx, what: int, args) -> int:
    """Arena bytes a call needs (dmrg_query_workspace); ctx may be None for the
    block build and Davidson queries."""
    b = C.c_int64()
    _check(load().dmrg_query_workspace(ctx.ptr if ctx is not None else None, what, C.byref(args), C.byref(b)))
    return int(b.value)


def block_workspace(prob, side: int, scheme: int, ctx=None) -> int:
    """Arena bytes of dmrg_build_block for one block of a synthetic problem,
    from the isometries' metadata (no device memory needed)."""
    isos = prob.left_iso if side == DMRG_LEFT else prob.right_iso
    holders = [Isometry(u, None) for u in isos]
    arr = (Bsm * len(holders))(*[h.bsm for h in holders])
    n_elec = prob.target[0] + prob.target[1]
    a = WsBlock(prob.K, n_elec, prob.target[0] - prob.target[1], prob.n_proc, prob.proc_id, side, len(holders),
                scheme, arr)
    return query_workspace(ctx, DMRG_WS_BLOCK, a)


class Context:
    """A library context on one GPU with a PyTorch-allocated device arena."""

    def __init__(self, arena_bytes: int, device: int = 0):
        import torch
        lib = load()
        self.device = torch.device("cuda", device)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.device)
        self.ptr = C.c_void_p()
        _check(lib.dmrg_create(C.byref(self.ptr), device, C.c_void_p(self.arena.data_ptr()),
                               int(arena_bytes)))

    def set_integrals(self, h1e: np.ndarray, g2e: np.ndarray, n_elec: int, two_sz: int,
                      e_core: float = 0.0, n_proc: int = 1, proc_id: int = 1):
        K = h1e.shape[0]
        self._h = np.ascontiguousarray(h1e, dtype=np.float64)
        self._g = np.ascontiguousarray(g2e, dtype=np.float64)
        _check(load().dmrg_set_integrals(self.ptr, K, n_elec, two_sz, self._h.ctypes.data_as(C.c_void_p),
                                         self._g.ctypes.data_as(C.c_void_p), e_core, n_proc, proc_id))

    def build_block(self, side: int, isos: Sequence[Isometry], scheme: int) -> OpSet:
        import torch
        arr = (Bsm * len(isos))(*[i.bsm for i in isos])
        out = C.c_void_p()
        _check(load().dmrg_build_block(self.ptr, side, len(isos), arr, scheme, C.byref(out), _stream(torch)))
        return OpSet(self, out)

    def normal_to_complementary(self, right: OpSet):
        import torch
        _check(load().dmrg_normal_to_complementary(self.ptr, right.ptr, _stream(torch)))

    def heff_create(self, left: OpSet, right: OpSet, n_roots: int = 1, precision: int = DMRG_PREC_F32,
                    layout=None, flags: int = 0) -> Heff:
        """layout: None (default order) or a list of (qn_left, s1, s2, offset)."""
        import torch
        out = C.c_void_p()
        lay = None
        if layout is not None:
            n = len(layout)
            self._lay = (np.array([x for l in layout for x in l[0]], np.int32), np.array([l[1] for l in layout], np.int32),
                         np.array([l[2] for l in layout], np.int32), np.array([l[3] for l in layout], np.int64))
            p = [a.ctypes.data_as(C.POINTER(t)) for a, t in zip(self._lay, (C.c_int32, C.c_int32, C.c_int32, C.c_int64))]
            lay = C.byref(PsiLayout(n, *p))
        _check(load().dmrg_heff_create(self.ptr, left.ptr, right.ptr, lay, n_roots, precision, flags, C.byref(out),
                                       _stream(torch)))
        return Heff(self, out)

    def renormalize(self, block: OpSet, iso: Isometry) -> OpSet:
        """`block` grown by its next site and transformed through `iso`."""
        import torch
        out = C.c_void_p()
        _check(load().dmrg_renormalize(self.ptr, block.ptr, C.byref(iso.bsm), C.byref(out), _stream(torch)))
        return OpSet(self, out)

    @property
    def arena_used(self) -> int:
        return int(load().dmrg_arena_used(self.ptr))

    @property
    def arena_peak(self) -> int:
        return int(load().dmrg_arena_peak(self.ptr))

    def close(self):
        if self.ptr:
            load().dmrg_destroy(self.ptr)
            self.ptr = None


def middle_step(prob, arena_bytes: int, scheme: Optional[str] = None, n_roots: int = 1,
                device: int = 0, precision: int = DMRG_PREC_F32, flags: int = 0):
    """Set up one middle-site step of a synthetic problem on the GPU.

    Builds both blocks through the problem's isometries, applies the
    normal -> complementary transform (CN scheme) and creates H_eff.
    Returns (context, left opset, right opset, heff, isometry holders).
    """
    if scheme is None:
        scheme = "NC" if prob.n_proc > 1 else "CN"
    ctx = Context(arena_bytes, device)
    n_elec = prob.target[0] + prob.target[1]
    two_sz = prob.target[0] - prob.target[1]
    ctx.set_integrals(prob.h1e, prob.g2e, n_elec, two_sz, prob.e_core, prob.n_proc, prob.proc_id)
    li = [Isometry(u, ctx.device) for u in prob.left_iso]
    ri = [Isometry(u, ctx.device) for u in prob.right_iso]
    L = ctx.build_block(DMRG_LEFT, li, DMRG_SCHEME_NC)
    R = ctx.build_block(DMRG_RIGHT, ri, DMRG_SCHEME_CN if scheme == "CN" else DMRG_SCHEME_NC)
    if scheme == "CN":
        ctx.normal_to_complementary(R)
    H = ctx.heff_create(L, R, n_roots, precision, flags=flags)
    return ctx, L, R, H, (li, ri)
