"""The rocprofv3 summary helper (host logic only): counters per kernel and dispatch, and the ratios read from them."""

import csv
import importlib.util
from pathlib import Path

ROOT = Path(__file__).resolve().parents[1]
_spec = importlib.util.spec_from_file_location("_glop_profiling", ROOT / "paper_1704_02278_amd" / "profiling.py")
profiling = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(profiling)

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
SCAN = "void glop::detail::glop_scan_kernel<1, true, 3, true, 8, false>(glop::detail::ScanParams)"
EMIT = "void glop::detail::glop_emit_kernel<1, true, 3, true, 8, false>(glop::detail::ScanParams, glop::detail::EmitParams)"


def _csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(FIELDS, r)))
    return path


def test_counter_table_sums_instances_and_averages_dispatches(tmp_path):
    a = _csv(tmp_path / "a.csv", [(1, SCAN, "SQ_INSTS_VALU", 100), (1, SCAN, "SQ_INSTS_VALU", 50),
                                  (2, SCAN, "SQ_INSTS_VALU", 250), (3, EMIT, "SQ_INSTS_VALU", 7)])
    b = _csv(tmp_path / "b.csv", [(5, SCAN, "TCC_HIT_sum", 30), (5, SCAN, "TCC_MISS_sum", 10)])
    tab = profiling.counter_table([a, b])
    assert tab["glop_scan_kernel<1, true, 3, true, 8, false>"] == {"SQ_INSTS_VALU": 200.0, "TCC_HIT_sum": 30.0,
                                                                   "TCC_MISS_sum": 10.0}
    assert tab["glop_emit_kernel<1, true, 3, true, 8, false>"] == {"SQ_INSTS_VALU": 7.0}


def test_counters_report_ratios(tmp_path):
    a = _csv(tmp_path / "a.csv", [(1, SCAN, "SQ_INSTS_VALU", 8192 * 10), (1, SCAN, "SQ_INSTS_LDS", 400),
                                  (1, SCAN, "SQ_LDS_BANK_CONFLICT", 100), (1, SCAN, "TCC_HIT_sum", 3),
                                  (1, SCAN, "TCC_MISS_sum", 1)])
    rep = profiling.counters_report([a], "glop_scan_kernel", text_bytes=8192 * 4, kernel_us=1.0, cus=4,
                                    clock_ghz=1.0)
    assert "| VALU wave instructions per 8 KiB of text | 20,480 |" in rep
    assert "| VALU lane operations per text byte | 160.00 |" in rep
    # 81,920 wave instructions over 4 CUs x 1,000 cycles
    assert "| VALU issue rate (wave instructions per CU per cycle; 1 is the CU's limit) | 20.480 |" in rep
    assert "| LDS bank-conflict cycles per LDS instruction | 0.250 |" in rep
    assert "| L2 (TCC) hit rate | 0.7500 |" in rep
