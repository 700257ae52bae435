"""The launch autotuner (gaps_tune, paper_2511_19633_amd/tune.py) and streams
of in-place event ranges on the GPU: every candidate shape runs, the chosen
one is no slower than the hand-picked default on the calibration batch, and
the tuned shape, like any other, gives bitwise the same events; uneven
batches made of views of the records give the events of the even batches."""
import sys

import numpy as np
import pytest

from gapsinputs import workloads

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def G(cfgs):
    import torch
    from paper_2511_19633_amd import binding
    assert torch.cuda.is_available()
    return binding.Gaps(cfgs["nlo"])


def test_autotune_runs_every_shape_and_keeps_events(G, tmp_path, monkeypatch):
    import torch
    from paper_2511_19633_amd import binding, tune
    monkeypatch.setenv("GAPS_TUNE_CACHE", str(tmp_path / "tune.json"))
    n = 200_000
    gin = G.hard_events(0, n, 1, max_slots=8)
    out = binding.DeviceEvents(n, workloads.MAX_SLOTS)
    rec = tune.autotune(G, [(gin, out, n)], 1, "pp_nlo_test", binding.MODE_PLAIN, True, repeats=2)
    for p in rec["points"]:
        say(f"  {p}")
        assert p["ms"] > 0.0 and p["grid"] >= 1
    assert rec["chosen"]["ms"] <= rec["default"]["ms"]
    assert tune.autotune(G, [(gin, out, n)], 1, "pp_nlo_test", binding.MODE_PLAIN, True)["cached"]
    ref = G.shower(gin, 1, retain=True).to_host()
    tuned = G.shower(gin, 1, retain=True, **rec["params"]).to_host()
    torch.cuda.synchronize()
    for name in ref.fields():
        assert np.array_equal(getattr(ref, name), getattr(tuned, name)), name
    with pytest.raises(binding.GapsError):
        G.tune([(gin, out, n)], 1, [dict(block=128, compact_every=8, waves_per_simd=2, fill=1.0)], repeats=0)
    bad = G.tune([(gin, out, n)], 1, [dict(block=1024, compact_every=8, waves_per_simd=2, fill=1.0)], repeats=1)
    assert bad[0]["ms"] == -1.0


def test_stream_of_views_equals_even_batches(G):
    import torch
    from paper_2511_19633_amd import binding
    n = 300_000
    ins = [G.hard_events(k * n, n, 2, max_slots=8) for k in range(2)]
    outs = [binding.DeviceEvents(n, workloads.MAX_SLOTS) for _ in range(2)]
    G.shower_stream([(ins[k], outs[k], n) for k in range(2)], 5, retain=True)
    torch.cuda.synchronize()
    ref = [o.to_host() for o in outs]
    for o in outs:
        o.n.fill_(-1)
        o.E.fill_(0.0)
    # uneven pieces, one crossing the records' boundary split in two
    cuts = [0, 12_345, 250_000, 300_000 + 7, 480_000, 600_000]
    pieces = []
    for a, b in zip(cuts[:-1], cuts[1:]):
        while a < b:
            k, off = divmod(a, n)
            take = min(b - a, n - off)
            pieces.append((ins[k].view(off, take), outs[k].view(off, take), take))
            a += take
    stream = torch.cuda.Stream()
    g = G.capture(pieces, 5, stream, retain=True)
    g.launch(stream)
    stream.synchronize()
    g.close()
    for k in range(2):
        h = outs[k].to_host()
        for name in h.fields():
            assert np.array_equal(getattr(h, name), getattr(ref[k], name)), (k, name)
