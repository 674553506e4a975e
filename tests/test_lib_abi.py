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
    assert dmrg.DMRG_OK == 0


def test_launch_count_matches_header():
    from paper_2103_09976_amd import dmrg
    m = re.search(r"#define\s+DMRG_HEFF_LAUNCHES\s+(\d+)", open(HEADER).read())
    assert m and int(m.group(1)) == dmrg.DMRG_HEFF_LAUNCHES
