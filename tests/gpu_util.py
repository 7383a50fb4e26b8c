"""Helpers for the GPU parity tests: run the HIP path through the C-ABI and compare
it with the oracle on the same seeded inputs."""

from __future__ import annotations

import numpy as np

import oracle

# Tolerances: relative 1e-4 on log10 Q where Q < 1e8, 1e-5 absolute on Tw, and
# 1e-6 box units on footpoints where Q < 1e4, growing as sqrt(Q / 1e4) above it
# (footpoint errors are amplified by the squashing of the map itself).
TOL_LOGQ = 1e-4
TOL_TW = 1e-5
TOL_FOOT = 1e-6
QMAX = 1e8
LOG10_2 = float(np.log10(2.0))

EXCLUDE = oracle.FATAL | oracle.ORC_MIXEDFACE | oracle.ORC_EDGE


def to_np(t):
    return t.detach().cpu().numpy()


def compare_maps(g: dict, o: dict, label: str = "", foot: bool = True, raw: bool = False) -> dict:
    """Compare a GPU map (dict of tensors, with lines) against an oracle map.

    Returns statistics; raises AssertionError when a tolerance is broken on the
    parity mask or the two sides disagree on statuses or faces outside it."""
    cv = (lambda x: np.asarray(x)) if raw else to_np
    qg = cv(g["q"]).ravel()
    qo = o["q"].ravel()
    sg = cv(g["status"]).astype(np.uint16).ravel()
    so = o["status"].astype(np.uint16).ravel()
    twg = cv(g["tw"]).ravel()
    two = o["tw"].ravel()
    n = qo.size
    edge = ((sg | so) & oracle.ORC_EDGE) != 0
    # statuses agree wherever no line of the stencil is near a box edge
    ne = ~edge
    bad_st = ne & ((sg & ~np.uint16(oracle.ORC_EDGE)) != (so & ~np.uint16(oracle.ORC_EDGE)))
    assert not bad_st.any(), (label, "status mismatch", np.flatnonzero(bad_st)[:10],
                              sg[bad_st][:10], so[bad_st][:10])
    mask = ((sg | so) & EXCLUDE) == 0
    mask &= np.isfinite(qo) & (qo < QMAX)
    stats = {"n": n, "masked": int(mask.sum()), "excluded_frac": float(1 - mask.mean())}
    # Q: relative error of log10 Q, on the scale max(|log10 Q|, log10 2): Q >= 2 in
    # theory, and the relative measure degenerates where discretisation puts Q near 1
    lq_o = np.log10(qo[mask])
    lq_g = np.log10(qg[mask])
    rel = np.abs(lq_g - lq_o) / np.maximum(np.abs(lq_o), LOG10_2)
    stats["logq_rel_max"] = float(rel.max()) if rel.size else 0.0
    stats["logq_rel_p999"] = float(np.quantile(rel, 0.999)) if rel.size else 0.0
    worst = np.argmax(rel) if rel.size else None
    assert stats["logq_rel_max"] <= TOL_LOGQ, (label, stats,
                                               None if worst is None else (qo[mask][worst], qg[mask][worst]))
    # Tw on every line that is not fatal on either side
    tmask = (((sg | so) & oracle.FATAL) == 0) & np.isfinite(two)
    dtw = np.abs(twg[tmask] - two[tmask])
    stats["tw_abs_max"] = float(dtw.max()) if dtw.size else 0.0
    assert stats["tw_abs_max"] <= TOL_TW, (label, stats)
    if foot and "lines" in g and "lines" in o:
        L = g["lines"]
        for key in ("end_b", "end_f"):
            eg = cv(L[key])
            eo = o["lines"][key]
            fg = cv(L["face_" + key[-1]]).astype(np.int8)
            fo = o["lines"]["face_" + key[-1]]
            lm = (((sg | so) & (oracle.FATAL | oracle.ORC_EDGE)) == 0)
            assert np.array_equal(fg[lm], fo[lm]), (label, key, "face mismatch")
            d = np.max(np.abs(eg - eo), axis=1)
            qq = np.where(np.isfinite(qo), qo, 1e12)
            bound = TOL_FOOT * np.maximum(1.0, np.sqrt(qq / 1e4))
            fm = lm & (qq < QMAX)
            stats[key + "_max"] = float(d[fm].max()) if fm.any() else 0.0
            over = fm & (d > bound)
            assert not over.any(), (label, key, int(over.sum()), d[over][:5], qq[over][:5])
    return stats


def compare_points(g: dict, idx, o: dict, label: str = "") -> dict:
    """Compare a full GPU map (tensors, with lines) at flat indices idx with oracle
    values computed at those points only (oracle.q2d_points / q3d_points)."""
    sub = {"q": to_np(g["q"]).ravel()[idx], "status": to_np(g["status"]).ravel()[idx],
           "tw": to_np(g["tw"]).ravel()[idx],
           "lines": {k: to_np(v)[idx] for k, v in g["lines"].items()}}
    return compare_maps(sub, o, label, raw=True)
