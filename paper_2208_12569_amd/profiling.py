"""Summaries of rocprofv3 runs of bench.py (CSV output), for the record kept with
the library: per-kernel duration statistics, and HBM traffic of the tracer kernel
from the FETCH_SIZE / WRITE_SIZE counters, calibrated on a 1 GiB device copy run in
the same process.

  python -m paper_2208_12569_amd.profiling stats <kernel_stats.csv> <out.md> "<command>"
  python -m paper_2208_12569_amd.profiling traffic <fetch counter csv> <write counter csv>
        <out.json> <key> "<command>" [kernel]
  python -m paper_2208_12569_amd.profiling l2 <tcc counter csv> <tcp counter csv> <out.md>
        "<command>" [kernel]
"""

from __future__ import annotations

import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 1 << 30
TRACER = "trace_kernel<float, float, 1, true, false, 0, false>"


def kernel_source_sha() -> str:
    """Hash of the tracer's sources: traffic figures are valid for this code only."""
    h = hashlib.sha256()
    for f in ("trace.hip", "trace_core.h"):
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _short(name: str) -> str:
    name = name.replace("fq::(anonymous namespace)::", "").replace("(anonymous namespace)::", "")
    if name.startswith("void "):
        name = name[5:]
    return name.split("(")[0] if "(" in name and "<" not in name.split("(")[0] else name[:110]


def stats_md(path: str, command: str) -> str:
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = [f"Command: `{command}`", "",
           "| kernel | calls | total ms | avg us | min us | max us | % |",
           "|---|---|---|---|---|---|---|"]
    for r in rows[:15]:
        out.append(f"| {_short(r['Name'])} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                   f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                   f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out) + "\n"


def _counter_rows(path: str, counter: str):
    """(kernel name, value) per dispatch of one counter."""
    per = {}
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name") != counter:
            continue
        key = (r["Dispatch_Id"], r["Kernel_Name"])
        per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    return [(k[1], v) for k, v in sorted(per.items(), key=lambda kv: int(kv[0][0]))]


def _copy_value(rows):
    """The counter of the calibration copy: the last copy-like dispatch."""
    for name, v in reversed(rows):
        if "copy" in name.lower() or "elementwise" in name.lower():
            return v
    raise ValueError("no calibration copy found in the counter run")


def traffic(fetch_csv: str, write_csv: str, kernel: str = TRACER) -> dict:
    f_rows = _counter_rows(fetch_csv, "FETCH_SIZE")
    w_rows = _counter_rows(write_csv, "WRITE_SIZE")
    f_scale = COPY_BYTES / (_copy_value(f_rows) * 1024.0)
    w_scale = COPY_BYTES / (_copy_value(w_rows) * 1024.0)
    fk = [v for n, v in f_rows if kernel in n.replace("fq::(anonymous namespace)::", "")]
    wk = [v for n, v in w_rows if kernel in n.replace("fq::(anonymous namespace)::", "")]
    if not fk or not wk:
        raise ValueError(f"kernel {kernel} not found in the counter runs")
    fetch = sum(fk) / len(fk) * 1024.0 * f_scale
    write = sum(wk) / len(wk) * 1024.0 * w_scale
    return {"kernel": kernel, "kernel_source_sha": kernel_source_sha(),
            "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
            "traffic_bytes_per_launch": fetch + write, "launches": len(fk),
            "fetch_calibration": f_scale, "write_calibration": w_scale}


def _mean_counter(path: str, counter: str, kernel: str) -> float:
    vals = [v for n, v in _counter_rows(path, counter)
            if kernel in n.replace("fq::(anonymous namespace)::", "")]
    if not vals:
        raise ValueError(f"{counter} of {kernel} not found in {path}")
    return sum(vals) / len(vals)


def l2_md(tcc_csv: str, tcp_csv: str, command: str, kernel: str = TRACER,
          kernel_ms: float = None) -> str:
    """L2 (TCC) hits, misses and requests of one kernel per launch, the bytes the L2
    returned (32-byte read sectors) and, with the kernel's duration, the L2 read
    rate; beside the L1 (TCP) accesses and the requests the L1 sent to the L2."""
    hit = _mean_counter(tcc_csv, "TCC_HIT_sum", kernel)
    miss = _mean_counter(tcc_csv, "TCC_MISS_sum", kernel)
    req = _mean_counter(tcc_csv, "TCC_REQ_sum", kernel)
    sect = _mean_counter(tcc_csv, "TCC_READ_SECTORS_sum", kernel)
    tcp_req = _mean_counter(tcp_csv, "TCP_TCC_READ_REQ_sum", kernel)
    tcp_acc = _mean_counter(tcp_csv, "TCP_TOTAL_CACHE_ACCESSES_sum", kernel)
    rows = [f"Command: `{command}` (one `--pmc` pass per counter group: "
            "TCC_HIT_sum TCC_MISS_sum TCC_REQ_sum TCC_READ_SECTORS_sum, then "
            "TCP_TCC_READ_REQ_sum TCP_TOTAL_CACHE_ACCESSES_sum)", "",
            f"Kernel: `{kernel}`, per launch (mean over launches):", "",
            "| counter | value |", "|---|---|",
            f"| L1 (TCP) cache accesses | {tcp_acc:.4g} |",
            f"| L1 -> L2 read requests | {tcp_req:.4g} |",
            f"| L2 (TCC) requests | {req:.4g} |",
            f"| L2 hits | {hit:.4g} |", f"| L2 misses | {miss:.4g} |",
            f"| L2 hit rate | {hit / max(hit + miss, 1):.3f} |",
            f"| L2 read sectors (32 B) | {sect:.4g} |",
            f"| bytes read from L2 | {sect * 32 / 1e9:.3f} GB |"]
    if kernel_ms:
        rows.append(f"| L2 read rate at {kernel_ms:.3f} ms per launch | "
                    f"{sect * 32 / (kernel_ms * 1e-3) / 1e12:.2f} TB/s |")
    return "\n".join(rows) + "\n"


def main(argv):
    if argv[0] == "stats":
        open(argv[2], "w").write(stats_md(argv[1], argv[3]))
    elif argv[0] == "traffic":
        d = {}
        if os.path.exists(argv[3]):
            d = json.load(open(argv[3]))
        e = traffic(argv[1], argv[2], *(argv[6:7] or [TRACER]))
        e["command"] = argv[5]
        d[argv[4]] = e
        json.dump(d, open(argv[3], "w"), indent=1)
    elif argv[0] == "l2":
        kernel = argv[5] if len(argv) > 5 else TRACER
        ms = float(argv[6]) if len(argv) > 6 else None
        open(argv[3], "w").write(l2_md(argv[1], argv[2], argv[4], kernel, ms))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
