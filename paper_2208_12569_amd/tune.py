"""Autotuner for the tracer's launch shape and step-control tolerance.

The tracer keeps one half line per lane and refills idle lanes with one atomic per
wave, so its launch has two free knobs: the block size and the resident waves per
CU the persistent grid is sized for (fewer waves trade latency hiding for cache
footprint). The step-control tolerance tol_perp trades accuracy for steps. The
tuner times the candidates on the caller's own jobs with HIP events and, for the
tolerance, accepts only values whose maps stay within a fraction of the accuracy
bar (relative 1e-4 on log10 Q where Q < 1e8, 1e-5 on Tw, 1e-6 box units on
footpoints, growing as sqrt(Q/1e4) above Q = 1e4) against the all-FP64 form run at
a much tighter tolerance on the same GPU.
"""

from __future__ import annotations

import dataclasses
import json
import math
import os
from typing import Optional, Sequence

from . import (FQ_PREC_F64, ST_EDGE, ST_FATAL, ST_MIXEDFACE, Params, _torch,
               alloc_q2d_outputs, q2d_batch_into, q2d_workspace_size)

BAR_LOGQ = 1e-4
BAR_TW = 1e-5
BAR_FOOT = 1e-6

_CACHE: dict = {}


class NoToleranceMeetsBar(RuntimeError):
    """No candidate tol_perp kept the maps within the accuracy bar; `report` holds
    the errors and times of every candidate."""

    def __init__(self, report: dict):
        super().__init__("no candidate tolerance keeps the maps within the accuracy bar: "
                         + ", ".join(f"{t:g}: logq {r['logq']:.2e} tw {r['tw']:.2e} "
                                     f"foot {r['foot']:.2e}" for t, r in report.items()))
        self.report = report


def _key(jobs, params: Params):
    """Launch shapes are timed per job shapes, precision and Tw flag."""
    return (tuple((tuple(B.shape), str(B.dtype), pl.nu, pl.nv) for B, _, pl in jobs),
            params.precision, params.want_tw)


def size_class(jobs) -> str:
    """The class a launch shape is stored under on disk: single job or batch, the
    base-2 logarithms of the total seed count and of the largest cube edge, and the
    grid dtype (the best block size and residency depend on these, not on the exact
    shapes)."""
    seeds = sum(int(pl.nu) * int(pl.nv) for _, _, pl in jobs)
    edge = max(max(int(n) for n in B.shape[-3:]) for B, _, _ in jobs)
    dtypes = sorted({str(B.dtype).replace("torch.", "") for B, _, _ in jobs})
    return (f"{'batch' if len(jobs) > 1 else 'single'}-seeds2^{int(math.log2(max(seeds, 1)))}"
            f"-edge2^{int(math.log2(max(edge, 1)))}-{'+'.join(dtypes)}")


def _arch(device) -> str:
    torch = _torch()
    name = getattr(torch.cuda.get_device_properties(device), "gcnArchName", "") or "unknown"
    return name.split(":")[0]


def _disk_key(jobs, params: Params) -> str:
    return f"{_arch(jobs[0][0].device)}|{size_class(jobs)}|prec{params.precision}|tw{int(params.want_tw)}"


def _load(path: str) -> dict:
    try:
        with open(path) as fh:
            d = json.load(fh)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def _store(path: str, key: str, fields: dict) -> None:
    d = _load(path)
    d[key] = fields
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as fh:
        json.dump(d, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _field_key(jobs):
    """A fingerprint of the field values and seed planes: an accepted tolerance holds
    for the fields it was checked on, not for every field of the same shape."""
    torch = _torch()
    out = []
    for B, grid, pl in jobs:
        x = B.to(torch.float64)
        out.append((float(x.sum()), float((x * x).sum()), float(x.abs().amax()),
                    tuple(float(v) for v in grid.origin), tuple(float(v) for v in grid.spacing),
                    tuple(float(v) for v in pl.origin), float(pl.du), float(pl.dv)))
    return tuple(out)


def _timed(jobs, params: Params, outs, ws, reps: int) -> float:
    """Median device time (ms) of `reps` calls on the current stream."""
    torch = _torch()
    q2d_batch_into(jobs, outs, ws, params)  # warm
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        q2d_batch_into(jobs, outs, ws, params)
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    times.sort()
    return times[len(times) // 2]


def tune_launch(jobs: Sequence, params: Optional[Params] = None, blocks=(64, 128, 256),
                waves=(0, 4, 8, 12), reps: int = 3) -> tuple:
    """Pick (block, waves_per_cu) by timing; returns (Params, {(block, waves): ms})."""
    torch = _torch()
    params = params or Params()
    jobs = list(jobs)
    base = dataclasses.replace(params, stats=None, events=None)
    need = q2d_workspace_size(jobs, base)
    ws = torch.empty(max(need, 256), dtype=torch.uint8, device=jobs[0][0].device)
    outs = alloc_q2d_outputs(jobs)
    table = {}
    for b in blocks:
        for w in waves:
            cand = dataclasses.replace(base, block=b, waves_per_cu=w)
            table[(b, w)] = _timed(jobs, cand, outs, ws, reps)
    best = min(table, key=table.get)
    return dataclasses.replace(params, block=best[0], waves_per_cu=best[1]), table


def map_errors(test: dict, ref: dict) -> dict:
    """Errors of one q2d map (with lines) against a reference map, on the points
    where both succeed, no stencil line ends near a box edge and Q < 1e8."""
    torch = _torch()
    st_t = test["status"].to(torch.int32)
    st_r = ref["status"].to(torch.int32)
    bad = ST_FATAL | ST_MIXEDFACE | ST_EDGE
    qr, qt = ref["q"], test["q"]
    mask = (((st_t | st_r) & bad) == 0) & torch.isfinite(qr) & torch.isfinite(qt) & (qr < 1e8)
    out = {"points": int(mask.sum()), "status_mismatch": int(((st_t != st_r) & (((st_t | st_r) & ST_EDGE) == 0)).sum())}
    if out["points"] == 0:
        return dict(out, logq=math.inf, tw=math.inf, foot=math.inf)
    lr = torch.log10(qr[mask])
    lt = torch.log10(qt[mask])
    out["logq"] = float((torch.abs(lt - lr) / torch.clamp(torch.abs(lr), min=math.log10(2.0))).max())
    out["tw"] = float(torch.abs(test["tw"][mask] - ref["tw"][mask]).max())
    foot = 0.0
    if "lines" in test and "lines" in ref:
        scale = torch.clamp(torch.sqrt(qr / 1e4), min=1.0)[mask]
        for k in ("end_b", "end_f"):
            d = torch.abs(test["lines"][k] - ref["lines"][k]).amax(dim=-1).reshape(qr.shape)
            foot = max(foot, float((d[mask] / scale).max()))
    out["foot"] = foot
    return out


def tune_tol(jobs: Sequence, params: Optional[Params] = None,
             tols=(1e-5, 3e-6, 1e-6), ref_tol: float = 1e-9, margin: float = 0.5,
             reps: int = 3) -> tuple:
    """Loosest-and-fastest tol_perp whose maps stay within margin x the bar against
    the all-FP64 form at ref_tol; returns (Params, report). Raises
    NoToleranceMeetsBar (with the report) when no candidate does."""
    torch = _torch()
    params = params or Params()
    jobs = list(jobs)
    base = dataclasses.replace(params, stats=None, events=None)
    ref_p = dataclasses.replace(base, precision=FQ_PREC_F64, tol_perp=ref_tol)
    need = max(q2d_workspace_size(jobs, base), q2d_workspace_size(jobs, ref_p))
    ws = torch.empty(max(need, 256), dtype=torch.uint8, device=jobs[0][0].device)
    ref = alloc_q2d_outputs(jobs, want_lines=True)
    q2d_batch_into(jobs, ref, ws, ref_p)
    test = alloc_q2d_outputs(jobs, want_lines=True)
    report = {}
    for t in tols:
        cand = dataclasses.replace(base, tol_perp=t)
        ms = _timed(jobs, cand, test, ws, reps)
        errs = [map_errors(a, b) for a, b in zip(test, ref)]
        worst = {k: max(e[k] for e in errs) for k in ("logq", "tw", "foot", "status_mismatch")}
        ok = (worst["logq"] <= margin * BAR_LOGQ and worst["tw"] <= margin * BAR_TW
              and worst["foot"] <= margin * BAR_FOOT)
        report[t] = dict(worst, ms=ms, ok=ok)
    good = [t for t in tols if report[t]["ok"]]
    if not good:
        raise NoToleranceMeetsBar(report)
    best = min(good, key=lambda t: report[t]["ms"])
    return dataclasses.replace(params, tol_perp=best), report


def autotune(jobs: Sequence, params: Optional[Params] = None, tune_tolerance: bool = False,
             cache_file: Optional[str] = None, **kw) -> Params:
    """Tuned Params for these jobs. The launch shape is cached in memory per job
    shapes, precision and Tw flag, and, with cache_file, on disk per GPU
    architecture, size class (size_class()), precision and Tw flag, so that later
    processes reuse it for jobs of the same class without timing them. A tuned
    tolerance is cached in memory only, per field values and seed planes (it was
    checked against the bar on those fields only). A tolerance search that finds no
    candidate within the bar raises NoToleranceMeetsBar and caches nothing."""
    params = params or Params()
    jobs = list(jobs)
    key = _key(jobs, params) + ((_field_key(jobs),) if tune_tolerance else ())
    if key in _CACHE:
        return dataclasses.replace(params, **_CACHE[key])
    fields = None
    if cache_file:
        fields = _load(cache_file).get(_disk_key(jobs, params))
        if fields is not None:
            fields = {"block": int(fields["block"]), "waves_per_cu": int(fields["waves_per_cu"])}
    if fields is None:
        p, _ = tune_launch(jobs, params, **{k: v for k, v in kw.items() if k in ("blocks", "waves", "reps")})
        fields = {"block": p.block, "waves_per_cu": p.waves_per_cu}
        if cache_file:
            _store(cache_file, _disk_key(jobs, params), fields)
    p = dataclasses.replace(params, **fields)
    if tune_tolerance:
        p, _ = tune_tol(jobs, p, **{k: v for k, v in kw.items() if k in ("tols", "ref_tol", "margin")})
        fields["tol_perp"] = p.tol_perp
    _CACHE[key] = fields
    return p
