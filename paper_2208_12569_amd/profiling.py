"""Summaries of rocprofv3 runs of bench.py (CSV output), for the record kept with
the library: per-kernel duration statistics, and HBM traffic of the tracer kernel
from the FETCH_SIZE / WRITE_SIZE counters, calibrated on a 1 GiB device copy run in
the same process.

  python -m paper_2208_12569_amd.profiling stats <kernel_stats.csv> <out.md> "<command>"
  python -m paper_2208_12569_amd.profiling traffic <fetch counter csv> <write counter csv>
        <out.json> <key> "<command>" [kernel]
  python -m paper_2208_12569_amd.profiling l2 <tcc counter csv> <tcp counter csv> <out.md>
        "<command>" [kernel] [kernel ms]
  python -m paper_2208_12569_amd.profiling valu <SQ pass A csv> <SQ pass B csv> <out.md>
        "<command A>" "<command B>" <kernel ms> <trial steps> <cell fetches>
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


VALU_A = ("SQ_THREAD_CYCLES_VALU", "SQ_ACTIVE_INST_VALU", "SQ_INSTS_VALU", "SQ_INSTS_VALU_FMA_F32",
          "SQ_INSTS_VALU_TRANS_F32", "SQ_INSTS_VALU_MUL_F32", "SQ_INSTS_VALU_ADD_F32",
          "SQ_INSTS_VALU_FLOPS_FP32")
VALU_B = ("SQ_INSTS_VALU_CVT", "SQ_INSTS_VALU_INT32", "SQ_INSTS_VALU_INT64",
          "SQ_INSTS_VALU_FLOPS_FP32_TRANS", "SQ_INSTS_SALU", "SQ_INSTS_VMEM_RD", "SQ_INSTS_BRANCH",
          "SQ_WAVES")


def valu_md(a_csv: str, b_csv: str, command_a: str, command_b: str, kernel_ms: float,
            trials: float, fetches: float, kernel: str = TRACER) -> str:
    """The instruction mix of one kernel per launch from two SQ counter passes, with
    lanes per instruction, VALU busy (4 cycles per wave instruction on 1024 SIMDs at
    2.4 GHz) and VALU instructions per lane trial step."""
    v = {c: _mean_counter(a_csv, c, kernel) for c in VALU_A}
    v.update({c: _mean_counter(b_csv, c, kernel) for c in VALU_B})
    valu = v["SQ_INSTS_VALU"]
    share = ("SQ_INSTS_VALU_ADD_F32", "SQ_INSTS_VALU_CVT", "SQ_INSTS_VALU_FMA_F32",
             "SQ_INSTS_VALU_INT32", "SQ_INSTS_VALU_INT64", "SQ_INSTS_VALU_MUL_F32",
             "SQ_INSTS_VALU_TRANS_F32")
    rows = [f"# Instruction mix of `{kernel}`, per launch", "",
            "Commands (two counter passes, each its own run):", "", f"`{command_a}`", "",
            f"`{command_b}`", "",
            f"Mean over launches; whole-chip totals. Per launch: {trials:.5g} trial steps, "
            f"{fetches:.5g} cell fetches, {kernel_ms:.2f} ms (kernel trace of the same build).", "",
            "| counter | value | share of VALU instructions |", "|---|---|---|"]
    for c in sorted(v):
        sh = f"{100 * v[c] / valu:.1f}%" if c in share else ""
        rows.append(f"| {c} | {v[c]:.4e} | {sh} |")
    other = valu - sum(v[c] for c in share)
    busy = valu * 4 / (1024 * kernel_ms * 1e-3 * 2.4e9)
    rows += ["", "Derived:", "",
             f"* active lanes per VALU instruction: SQ_THREAD_CYCLES_VALU / SQ_ACTIVE_INST_VALU = "
             f"{v['SQ_THREAD_CYCLES_VALU'] / v['SQ_ACTIVE_INST_VALU']:.1f} of 64",
             f"* VALU instructions other than FP32 FMA/MUL/ADD/transcendental, integer and "
             f"conversions (moves, selects, compares, min/max, bit operations): {other:.4g}, "
             f"{100 * other / valu:.0f}%",
             f"* VALU busy: SQ_INSTS_VALU x 4 cycles / (1024 SIMDs x {kernel_ms:.2f} ms x 2.4 GHz) "
             f"= {100 * busy:.0f}%",
             f"* VALU instructions per lane trial step: SQ_INSTS_VALU x 64 / trial steps = "
             f"{valu * 64 / trials:.0f}",
             f"* vector memory reads per wave-level cell fetch: "
             f"{v['SQ_INSTS_VMEM_RD'] * 64 / fetches:.1f} (16 loads per fetch)"]
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
    elif argv[0] == "valu":
        open(argv[3], "w").write(valu_md(argv[1], argv[2], argv[4], argv[5], float(argv[6]),
                                         float(argv[7]), float(argv[8])))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
