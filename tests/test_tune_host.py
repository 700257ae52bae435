"""Host logic of the launch autotuner (paper_2511_19633_amd/tune.py) with a
stand-in for the library's timing call: the fastest runnable shape wins, the
hand-picked default is always among the candidates, shapes the kernels cannot
run are skipped, and the choice is stored per key and reused."""
import json

import pytest

torch = pytest.importorskip("torch")


class FakeEvents:
    def __init__(self, cap, max_slots):
        self.cap, self.max_slots = cap, max_slots


class FakeGaps:
    """Times a shape as a made-up function of it; the three-wave shapes are 'not runnable'."""

    def __init__(self):
        self.calls = 0

    def tune(self, batches, seed, points, repeats=3, stream=None, **params):
        self.calls += 1
        out = []
        for p in points:
            ms = -1.0 if p["waves_per_simd"] == 3 else 10.0 + abs(p["compact_every"] - 16) + 5 * (1 - p["fill"]) + \
                (0.5 if p["block"] == 512 else 0.0)
            out.append(dict(p, grid=int(256 * p["fill"]), ms=ms))
        return out


def test_autotune_picks_fastest_and_caches(tmp_path, monkeypatch):
    from paper_2511_19633_amd import tune
    monkeypatch.setenv("GAPS_TUNE_CACHE", str(tmp_path / "tune.json"))
    monkeypatch.setattr(torch.cuda, "get_device_name", lambda *_: "testdev")
    monkeypatch.setattr(torch.cuda, "current_device", lambda: 0)
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *_: None)
    G = FakeGaps()
    batches = [(FakeEvents(1000, 8), FakeEvents(1000, 128), 1000)]
    rec = tune.autotune(G, batches, 1, "nlo", 1, True)
    assert rec["chosen"] == dict(block=256, compact_every=16, waves_per_simd=2, fill=1.0, grid=256, ms=10.0)
    assert rec["params"] == dict(block=256, grid=256, compact_every=16, waves_per_simd=2)
    assert rec["default"]["block"] == 512 and rec["default"]["compact_every"] == 8
    assert rec["chosen"]["ms"] <= rec["default"]["ms"]
    assert not rec["cached"] and G.calls == 1
    stored = json.load(open(tmp_path / "tune.json"))
    assert list(stored) == [tune.tuning_key("testdev", "nlo", 1, True, 128)]
    again = tune.autotune(G, batches, 1, "nlo", 1, True)
    assert again["cached"] and G.calls == 1 and again["params"] == rec["params"]
    other = tune.autotune(G, batches, 1, "nlo", 0, True)  # another mode: timed again
    assert not other["cached"] and G.calls == 2


def test_default_space_contains_the_default():
    from paper_2511_19633_amd import tune
    for retain in (False, True):
        sp = tune.default_space(retain)
        assert any(all(p[k] == v for k, v in tune.DEFAULT.items()) for p in sp)
        assert all(p["block"] % 64 == 0 and 0 < p["fill"] <= 1 for p in sp)
        assert any(p["waves_per_simd"] == 3 for p in sp) == retain
