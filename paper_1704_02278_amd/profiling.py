"""rocprofv3 summaries for the matching kernels (run by path; reads CSV only).

    python paper_1704_02278_amd/profiling.py stats <..._kernel_stats.csv>
    python paper_1704_02278_amd/profiling.py traffic --workload medium \\
        --fetch <fetch ..._counter_collection.csv> --write <write ..._counter_collection.csv> \\
        --out profiles/glop_scan_kernel_medium_traffic.json

``stats`` prints a markdown table of a ``--kernel-trace --stats`` run.
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
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        print(stats_table(a.csv))
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
