"""The tuner's disk cache of launch shapes (per GPU architecture and size class),
with the timing replaced by a stand-in: host logic only."""

import json

import torch

import paper_2208_12569_amd as fq
from paper_2208_12569_amd import tune
from synth import Plane, cubic_grid


def _jobs(nu, nv, edge=8):
    g = cubic_grid(edge, edge, edge)
    B = torch.zeros((3, edge, edge, edge), dtype=torch.float32)
    return [(B, g, Plane((0.0, 0.0, 0.0), (1, 0, 0), (0, 1, 0), nu, nv, 0.01, 0.01))]


def test_launch_shape_is_reused_per_arch_and_size_class(tmp_path, monkeypatch):
    calls = []

    def fake_tune_launch(jobs, params=None, **kw):
        calls.append(len(jobs))
        return fq.Params(block=128, waves_per_cu=8), {}

    monkeypatch.setattr(tune, "tune_launch", fake_tune_launch)
    monkeypatch.setattr(tune, "_arch", lambda device: "gfx950")
    monkeypatch.setattr(tune, "_CACHE", {})
    path = str(tmp_path / "sub" / "tune.json")
    p = tune.autotune(_jobs(64, 64), fq.Params(), cache_file=path)
    assert (p.block, p.waves_per_cu) == (128, 8) and len(calls) == 1
    d = json.load(open(path))
    assert d == {"gfx950|single-seeds2^12-edge2^3-float32|prec0|tw1": {"block": 128, "waves_per_cu": 8}}
    # another process (empty memory cache), other shapes of the same class: no timing
    monkeypatch.setattr(tune, "_CACHE", {})
    p = tune.autotune(_jobs(70, 60), fq.Params(), cache_file=path)
    assert (p.block, p.waves_per_cu) == (128, 8) and len(calls) == 1
    # another class (more seeds), and another architecture: timed and stored beside it
    tune.autotune(_jobs(256, 256), fq.Params(), cache_file=path)
    monkeypatch.setattr(tune, "_arch", lambda device: "gfx942")
    tune.autotune(_jobs(64, 64), fq.Params(), cache_file=path)
    assert len(calls) == 3
    assert sorted(json.load(open(path))) == [
        "gfx942|single-seeds2^12-edge2^3-float32|prec0|tw1",
        "gfx950|single-seeds2^12-edge2^3-float32|prec0|tw1",
        "gfx950|single-seeds2^16-edge2^3-float32|prec0|tw1"]


def test_size_class():
    assert tune.size_class(_jobs(1024, 1024, 16)) == "single-seeds2^20-edge2^4-float32"
    assert tune.size_class(_jobs(8, 8) + _jobs(8, 8)) == "batch-seeds2^7-edge2^3-float32"
