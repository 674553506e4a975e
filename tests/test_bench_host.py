"""CPU checks of bench.py's host logic: the counted HBM traffic of the roofline
is taken from the committed counter summary only when that summary was made on
the same kernel source and the same work list (chunk count, tall threshold)."""
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

KERNEL = "tall_kernel<float, 6, true>"


def _profiled_list():
    text = open(os.path.join(ROOT, "profiles", "hbm_traffic_C5.txt")).read()
    m = re.search(r"DMRG_BALANCE=(\d+), tall from (\d+) rows", text)
    assert m, "the summary states the work list it was taken on"
    return int(m.group(1)), int(m.group(2))


def test_traffic_for_the_profiled_list():
    bal, tall = _profiled_list()
    t = bench.counted_traffic("C5", KERNEL, {"balance_target": bal, "tall_min_rows": tall})
    assert t is not None and t > 0


def test_no_traffic_for_another_list():
    bal, tall = _profiled_list()
    assert bench.counted_traffic("C5", KERNEL, {"balance_target": bal // 2, "tall_min_rows": tall}) is None
    assert bench.counted_traffic("C5", KERNEL, {"balance_target": bal, "tall_min_rows": tall - 16}) is None


def test_no_traffic_for_another_kernel_source(monkeypatch, tmp_path):
    src = tmp_path / "kernels.hip"
    src.write_text(open(bench.KERNEL_SRC).read() + "\n// changed\n")
    monkeypatch.setattr(bench, "KERNEL_SRC", str(src))
    bal, tall = _profiled_list()
    assert bench.counted_traffic("C5", KERNEL, {"balance_target": bal, "tall_min_rows": tall}) is None


def test_no_traffic_without_a_summary():
    assert bench.counted_traffic("C1", KERNEL) is None
