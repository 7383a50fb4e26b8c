"""The accuracy figures bench.py reports, on hand-made maps (no GPU needed): which
points count, the log10 Q error scale and the Q-conditioned footpoint bound."""

import numpy as np
import pytest

import bench
import paper_2208_12569_amd as fq


def test_logq_error_counts_only_comparable_points():
    qo = np.array([2.0, 10.0, 1e3, 1e9, np.nan, 50.0, 1e4])
    # relative errors of log10 Q: 2e-5 on Q = 10 (scale |log10 Q| = 1), 5e-5 on
    # Q = 1e3 (scale 3), 2e-4 on Q = 1e4 (scale 4); Q = 2 is scaled by log10 2
    lo = np.log10(np.where(np.isfinite(qo), qo, 1.0))
    lg = lo + np.array([1e-6, 2e-5, 1.5e-4, 0.0, 0.0, 0.3, 8e-4])
    qg = 10.0 ** lg
    qg[4] = 5.0
    so = np.zeros(7, np.uint16)
    sg = np.zeros(7, np.uint16)
    sg[5] = fq.ST_EDGE  # a stencil line ends near a box edge: not compared
    two = np.array([0.1, 0.2, 0.3, 0.4, 0.5, 0.6, np.nan])
    twg = two + np.array([1e-7, -3e-6, 0.0, 0.0, 0.0, 0.0, 0.0])
    e = bench.err_stats(qg, twg, sg, qo, two, so)
    assert e["points"] == 4  # Q = 1e9 (over 1e8), NaN and the edge point are out
    assert e["logq_rel_max"] == pytest.approx(8e-4 / 4.0)
    assert e["points_over_1e-4"] == 1
    assert e["tw_abs_max"] == pytest.approx(3e-6)
    assert 1e-6 / np.log10(2.0) <= e["logq_rel_p999"] <= 2e-4


def test_footpoint_bound_grows_with_sqrt_q_and_skips_the_rim():
    side = 4
    n = side * side
    ends_o = {k: np.zeros((n, 3)) for k in ("end_b", "end_f")}
    ends_g = {k: np.zeros((n, 3)) for k in ("end_b", "end_f")}
    q = np.full((side, side), 2.0)
    st = np.zeros((side, side), np.uint16)
    q.ravel()[6] = 1e6                    # bound 1e-6 * sqrt(100) = 1e-5
    ends_g["end_f"][5, 1] = 5e-7          # within the plain bound
    ends_g["end_b"][6, 2] = 8e-6          # within the stretched bound
    ends_g["end_f"][9, 0] = 3e-6          # over the plain bound
    ends_g["end_f"][10, 0] = 1.0          # its line failed: not compared
    st.ravel()[10] = fq.ST_NULLB
    ends_g["end_f"][0, 0] = 1.0           # map rim: not compared
    orc = {"lines": ends_o, "q": q, "status": st}
    f = bench.foot_stats(ends_g, orc, side)
    assert f["foot_max"] == pytest.approx(8e-6)
    assert f["foot_over_bound"] == 1
    assert f["foot_max_over_bound"] == pytest.approx(3.0)
