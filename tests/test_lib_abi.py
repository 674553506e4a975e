"""CPU checks of the C-ABI library: it loads and exports every symbol that
include/dmrg.h declares; host-only argument checks (no device work)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dmrg.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(dmrg_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2103_09976_amd import build_lib, dmrg
    if not os.path.exists(dmrg.LIB_PATH):
        build_lib.build()
    return dmrg.load()


def test_header_declares_the_calls():
    names = _declared()
    for n in ["dmrg_create", "dmrg_set_integrals", "dmrg_build_block", "dmrg_normal_to_complementary",
              "dmrg_heff_create", "dmrg_heff_apply", "dmrg_heff_diag", "dmrg_davidson",
              "dmrg_renormalize", "dmrg_heff_flops", "dmrg_heff_bytes"]:
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings(lib):
    for s in range(0, -8, -1):
        assert lib.dmrg_status_string(s)
    assert lib.dmrg_status_string(-99) == b"unknown status"


def test_null_arguments_are_rejected(lib):
    from paper_2103_09976_amd import dmrg
    assert lib.dmrg_create(None, 0, None, 0) == -1
    out = ctypes.c_void_p()
    assert lib.dmrg_create(ctypes.byref(out), 0, None, 0) == -1
    assert b"arena" in lib.dmrg_last_error()
    assert lib.dmrg_heff_apply(None, 0, 1, None, None, None) == -1
    assert lib.dmrg_set_integrals(None, 8, 8, 0, None, None, 0.0, 1, 1) == -1
    assert lib.dmrg_heff_flops(None) == -1
    assert lib.dmrg_davidson(None, 1, None, None, None, None, None) == -1
    assert lib.dmrg_heff_profile(None, 0, None, None, 0, None, None, None, None) == -1
    iso = ctypes.c_void_p()
    assert lib.dmrg_decimate(None, 0, 1, None, 0.0, None, 0, ctypes.byref(iso), None, None) == -1
    assert lib.dmrg_iso_bsm(None, None) == -1
    assert lib.dmrg_iso_weights(None, 0, None) == -1
    lib.dmrg_iso_free(None)
    assert dmrg.DMRG_OK == 0


def test_launch_count_matches_header():
    from paper_2103_09976_amd import dmrg
    m = re.search(r"#define\s+DMRG_HEFF_LAUNCHES\s+(\d+)", open(HEADER).read())
    assert m and int(m.group(1)) == dmrg.DMRG_HEFF_LAUNCHES


def test_workspace_queries_without_device(lib):
    """dmrg_query_workspace runs the build's own allocation sequence on the host
    (no device work): it answers without a GPU and without a context for the
    block build and the Davidson workspace."""
    import synth
    from paper_2103_09976_amd import dmrg
    p = synth.make_problem(10, 10, 0, 30, 61)
    left = dmrg.block_workspace(p, dmrg.DMRG_LEFT, dmrg.DMRG_SCHEME_NC)
    right_cn = dmrg.block_workspace(p, dmrg.DMRG_RIGHT, dmrg.DMRG_SCHEME_CN)
    assert left > 0 and right_cn > 0
    # fewer sites need no more memory
    short = synth.make_problem(10, 10, 0, 30, 61)
    short.left_iso = short.left_iso[:2]
    assert dmrg.block_workspace(short, dmrg.DMRG_LEFT, dmrg.DMRG_SCHEME_NC) <= left
    # a sub-Hamiltonian share keeps fewer complementary operators than the full NC block
    ps = synth.make_problem(10, 10, 0, 30, 61, n_proc=4, proc_id=2)
    full_nc = dmrg.block_workspace(p, dmrg.DMRG_RIGHT, dmrg.DMRG_SCHEME_NC)
    share_nc = dmrg.block_workspace(ps, dmrg.DMRG_RIGHT, dmrg.DMRG_SCHEME_NC)
    assert share_nc < full_nc
    # Davidson: at least the V and W blocks of max_subspace vectors
    dim, k = 123457, 2
    opts = dmrg.DavOpts(300, 24, 1e-6, dmrg.DMRG_PREC_F32, 1e-4, 0, 0.0)
    b = dmrg.query_workspace(None, dmrg.DMRG_WS_DAVIDSON, dmrg.WsDavidson(dim, k, opts))
    assert 2 * 24 * dim * 8 <= b <= 2 * (2 * 24 + 3 * k + 2 * 16 + 1) * dim * 8
    # queries that need an operator set reject a missing context
    bad = dmrg.WsHeff(None, None, 1, 0)
    with pytest.raises(dmrg.DmrgError):
        dmrg.query_workspace(None, dmrg.DMRG_WS_HEFF, bad)


def test_operand_span_guard_on_host(lib, tmp_path):
    """The host check that keeps every kernel operand below 2^32 bytes (the
    kernels' 32-bit in-block offsets): a work list whose B operand spans 2^32
    bytes is refused with DMRG_E_UNSUPPORTED, one element less passes.  The
    check is compiled into a small host program that calls the library's
    validate_work directly (no device work)."""
    import shutil
    import subprocess
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    src = tmp_path / "span.cpp"
    src.write_text(r"""
#include <cstdio>
#include "core.hpp"
using namespace dmrg;
static int run(int64_t extra) {
    WorkList w;
    dmrgk::Group g{};
    g.xid_coef = 1.0; g.mu = 1; g.c0 = 0; g.c1 = 1;
    w.groups.push_back(g);
    dmrgk::Contrib c{};
    const int64_t ldb = 1 << 20;
    c.lda = 4; c.k = 4; c.alpha = 1.0; c.flags = 0 | (1 << 3);
    c.b_off = 0; c.ldb = (int32_t)ldb;
    w.contribs.push_back(c);
    // B spans (k-1)*ldb + n - 1 elements: choose n so the span is 2^29 - 1 + extra
    const int64_t n = (int64_t(1) << 29) - 3 * ldb + extra;
    dmrgk::Task t{};
    t.c_off = 0; t.ldc = (int32_t)n; t.m = 1; t.n = (int32_t)n; t.col0 = 0; t.ncol = 16; t.g0 = 0; t.g1 = 1; t.cbuf = 3;
    w.task[dmrgk::task_class(1, 16)].push_back(t);
    int64_t size[dmrgk::kMaxBuf] = {0};
    size[0] = 4; size[1] = int64_t(1) << 31; size[3] = n;
    return validate_work(w, size);
}
int main() { std::printf("%d %d\n", run(0), run(1)); return 0; }
""")
    here = os.path.join(ROOT, "paper_2103_09976_amd")
    exe = tmp_path / "span"
    cmd = [gxx, "-std=c++17", "-O1", "-I", os.path.join(here, "csrc"), "-I", os.path.join(ROOT, "include"),
           str(src), "-o", str(exe), "-L", here, "-ldmrg_hip", f"-Wl,-rpath,{here}"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stderr
    ok, over = (int(x) for x in out.stdout.split())
    assert ok == 0            # span 2^29 - 1 elements of 8 bytes: below 2^32 bytes
    assert over == -7         # DMRG_E_UNSUPPORTED
