"""rocprofv3 summaries for the matching kernels (run by path; reads CSV only).

    python paper_1704_02278_amd/profiling.py stats <..._kernel_stats.csv>
    python paper_1704_02278_amd/profiling.py counters --text-bytes N [--kernel-us T] <..._counter_collection.csv> ...
    python paper_1704_02278_amd/profiling.py traffic --workload medium \\
        --fetch <fetch ..._counter_collection.csv> --write <write ..._counter_collection.csv> \\
        --out profiles/glop_scan_kernel_medium_traffic.json

``stats`` prints a markdown table of a ``--kernel-trace --stats`` run.
``counters`` prints one kernel's counters from ``--pmc`` runs (SQ, TCC) with
the ratios read from them: VALU instructions per tile and per byte, the VALU
issue rate, LDS bank-conflict cycles per LDS instruction, the L2 hit rate.
``traffic`` turns two ``--pmc`` runs (FETCH_SIZE, then WRITE_SIZE) of a
program that also made one device copy of ``--copy-bytes`` bytes into HBM
bytes per scan launch: each counter is scaled by what it reads for that copy.
The record carries the hash of the kernel sources it was measured on, so a
later change to the kernels makes it stale.
"""

from __future__ import annotations

import argparse
import csv
import hashlib
import json
import statistics
import sys
from pathlib import Path

ROOT = Path(__file__).resolve().parents[1]
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def kernel_sources_sha256(root: Path = ROOT) -> str:
    """Hash of every source the device kernels are built from."""
    csrc = root / "paper_1704_02278_amd" / "csrc"
    files = sorted(csrc.glob("glop_kernels*")) + [csrc / "glop_layout.hpp"]
    h = hashlib.sha256()
    for f in files:
        h.update(f.name.encode())
        h.update(f.read_bytes())
    return h.hexdigest()


def short_name(name: str) -> str:
    """Kernel name without namespaces, return type and parameter list."""
    n = name.replace("(anonymous namespace)::", "").split("(")[0]
    for prefix in ("void ", "glop::detail::", "glop::"):
        n = n.replace(prefix, "")
    return n.strip()


def stats_table(path) -> str:
    rows = list(csv.DictReader(open(path)))
    out = ["| kernel | calls | avg us | min us | max us |", "|---|---|---|---|---|"]
    for r in rows:
        out.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} |")
    return "\n".join(out)


def counter_values(path):
    """{kernel short name: [counter value per dispatch]} from a --pmc CSV."""
    agg = {}
    for r in csv.DictReader(open(path)):
        agg.setdefault(short_name(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    return agg


def traffic(fetch_csv, write_csv, copy_bytes: int, kernel_prefix: str = "glop_scan_kernel"):
    """HBM bytes per launch of the scan kernel, calibrated on the device copy."""
    F, W = counter_values(fetch_csv), counter_values(write_csv)
    copies_f = [v for k, vs in F.items() if k.startswith(COPY_KERNEL) for v in vs]
    copies_w = [v for k, vs in W.items() if k.startswith(COPY_KERNEL) for v in vs]
    if not copies_f or not copies_w:
        raise ValueError("no device copy in the counter runs (run the program with its copy probe)")
    cal_f, cal_w = max(copies_f), max(copies_w)  # the probe is the largest copy
    f_factor = copy_bytes / (cal_f * 1024.0)
    w_factor = copy_bytes / (cal_w * 1024.0)
    scans = [k for k in F if k.startswith(kernel_prefix)]
    if len(scans) != 1:
        raise ValueError(f"expected one scan kernel in the counter run, found {scans}")
    k = scans[0]
    fetch_kib = statistics.mean(F[k])
    write_kib = statistics.mean(W.get(k, [0.0]))
    rec = {
        "kernel": k,
        "kernel_sources_sha256": kernel_sources_sha256(),
        "fetch_size_kib": round(fetch_kib, 1),
        "write_size_kib": round(write_kib, 1),
        "dispatches": len(F[k]),
        "copy_calibration": {"bytes_read": copy_bytes, "bytes_written": copy_bytes,
                             "fetch_size_kib": round(cal_f, 1), "write_size_kib": round(cal_w, 1),
                             "fetch_factor": round(f_factor, 4), "write_factor": round(w_factor, 4)},
        "traffic_bytes_per_launch": int(round(fetch_kib * 1024 * f_factor + write_kib * 1024 * w_factor)),
    }
    others = {}
    for name in sorted(F):
        others[name] = {"fetch_size_kib": round(statistics.mean(F[name]), 1),
                        "write_size_kib": round(statistics.mean(W.get(name, [0.0])), 1),
                        "dispatches": len(F[name])}
    rec["all_kernels"] = others
    return rec


def counter_table(paths):
    """{kernel short name: {counter: mean value per dispatch}} from --pmc CSVs."""
    vals = {}
    for path in paths:
        for r in csv.DictReader(open(path)):
            k = short_name(r["Kernel_Name"])
            vals.setdefault(k, {}).setdefault(r["Counter_Name"], {}).setdefault(r["Dispatch_Id"], 0.0)
            # A counter collected per block instance sums over the instances of one dispatch.
            vals[k][r["Counter_Name"]][r["Dispatch_Id"]] += float(r["Counter_Value"])
    return {k: {c: statistics.mean(d.values()) for c, d in cs.items()} for k, cs in vals.items()}


def counters_report(paths, kernel_prefix, text_bytes, kernel_us=None, cus=256, clock_ghz=2.4):
    """Markdown rows of raw counters and the ratios read from them for one kernel."""
    tab = counter_table(paths)
    ks = [k for k in tab if k.startswith(kernel_prefix)]
    if len(ks) != 1:
        raise ValueError(f"expected one {kernel_prefix} kernel in the counter runs, found {ks}")
    c = tab[ks[0]]
    out = [f"Kernel `{ks[0]}`, mean per dispatch:", "", "| counter | value |", "|---|---|"]
    for name in sorted(c):
        out.append(f"| {name} | {c[name]:,.0f} |")
    out += ["", "| ratio | value |", "|---|---|"]
    tiles = text_bytes / 8192.0
    if "SQ_INSTS_VALU" in c:
        out.append(f"| VALU wave instructions per 8 KiB of text | {c['SQ_INSTS_VALU'] / tiles:,.0f} |")
        out.append(f"| VALU lane operations per text byte | {c['SQ_INSTS_VALU'] * 64 / text_bytes:.2f} |")
        if kernel_us:
            issue = c["SQ_INSTS_VALU"] / (cus * kernel_us * 1e-6 * clock_ghz * 1e9)
            out.append(f"| VALU issue rate (wave instructions per CU per cycle; 1 is the CU's limit) | {issue:.3f} |")
    if "SQ_INSTS_LDS" in c:
        out.append(f"| LDS wave instructions per 8 KiB of text | {c['SQ_INSTS_LDS'] / tiles:,.0f} |")
    if "SQ_LDS_BANK_CONFLICT" in c and c.get("SQ_INSTS_LDS"):
        out.append(f"| LDS bank-conflict cycles per LDS instruction | "
                   f"{c['SQ_LDS_BANK_CONFLICT'] / c['SQ_INSTS_LDS']:.3f} |")
    if "TCC_HIT_sum" in c and "TCC_MISS_sum" in c:
        tot = c["TCC_HIT_sum"] + c["TCC_MISS_sum"]
        if tot:
            out.append(f"| L2 (TCC) hit rate | {c['TCC_HIT_sum'] / tot:.4f} |")
    if "SQ_INSTS_SALU" in c:
        out.append(f"| SALU wave instructions per 8 KiB of text | {c['SQ_INSTS_SALU'] / tiles:,.0f} |")
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    t = sub.add_parser("traffic")
    t.add_argument("--workload", required=True)
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-bytes", type=int, default=1 << 30)
    t.add_argument("--out")
    c = sub.add_parser("counters")
    c.add_argument("csvs", nargs="+")
    c.add_argument("--kernel", default="glop_scan_kernel")
    c.add_argument("--text-bytes", type=int, required=True)
    c.add_argument("--kernel-us", type=float, help="the kernel's average duration (for the issue rate)")
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        print(stats_table(a.csv))
        return 0
    if a.cmd == "counters":
        print(counters_report(a.csvs, a.kernel, a.text_bytes, a.kernel_us))
        return 0
    rec = traffic(a.fetch, a.write, a.copy_bytes)
    rec = {"workload": a.workload, **rec}
    text = json.dumps(rec, indent=1)
    if a.out:
        Path(a.out).write_text(text + "\n")
    print(text)
    return 0


if __name__ == "__main__":
    sys.exit(main())
