"""The matching variants on the GPU (libgaps through the C-ABI) against the
oracle: MC@NLO with the start scale mu_Q^2 and POWHEG-like Born events (hard
events to 1e-11, showers event by event in every form of the competition and
in learned mode: integer and colour data bit-exact, >= 99.9 % identical,
momenta within 1e-9 of the event's scale), the trial log without corrected
trials, and the rejected configurations."""
import sys

import numpy as np
import pytest

from gapsinputs import records, workloads
from tests.test_gpu_parity import compare_events

pytestmark = pytest.mark.gpu

SCALE = 13000.0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu(cfgs):
    import torch
    from paper_2511_19633_amd import binding
    assert torch.cuda.is_available()
    out = {k: binding.Gaps(cfgs[k]) for k in ("muq", "powheg")}
    out["lo_mec"] = binding.Gaps(dict(cfgs["lo"], matching=2))
    out["lo_muq"] = binding.Gaps(dict(cfgs["lo"], matching=1, mu_q2=400.0))
    return out


@pytest.fixture(scope="module")
def orc(cfgs, oracles):
    from oracle.pyoracle import Oracle
    return {"muq": oracles["muq"], "powheg": oracles["powheg"],
            "lo_mec": Oracle(dict(cfgs["lo"], matching=2)),
            "lo_muq": Oracle(dict(cfgs["lo"], matching=1, mu_q2=400.0))}


@pytest.mark.parametrize("key", ["muq", "powheg", "lo_mec", "lo_muq"])
def test_hard_events(gpu, orc, key):
    n = 20000
    say(f"hard events {key} n={n}")
    g = gpu[key].hard_events(0, n, 1).to_host()
    o = orc[key].hard_events(0, n, 1)
    assert np.array_equal(g.n, o.n) and np.array_equal(g.flags, o.flags) and np.array_equal(g.id, o.id)
    for name in ("pid", "col", "acol", "status"):
        assert np.array_equal(getattr(g, name), getattr(o, name))
    for name in ("E", "px", "py", "pz"):
        assert np.max(np.abs(getattr(g, name) - getattr(o, name))) < 1e-11 * SCALE
    assert np.allclose(g.w, o.w, rtol=1e-11, atol=0)
    assert np.array_equal(g.t_start, o.t_start)
    if key in ("powheg", "lo_mec"):
        assert np.all(g.flags == records.FLAG_MEC)


# the GPU parameters and the oracle's of each form of the competition
FORMS = pytest.mark.parametrize("form", [(dict(retain=True), dict(retain=True)),
                                         (dict(retain=False), dict(retain=False)),
                                         (dict(variant=1, gen_select=True), dict(gen_select=True)),
                                         (dict(variant=1, veto_max=True), dict(veto_max=True))],
                                ids=["retain", "regenerate", "gen_select", "veto_max"])


@FORMS
@pytest.mark.parametrize("key", ["powheg", "muq", "lo_mec"])
def test_shower_parity(gpu, orc, key, form):
    gk, ok = form
    n = 3000
    say(f"shower {key} {list(ok)[0]}={list(ok.values())[0]} n={n}")
    G, O = gpu[key], orc[key]
    gout = G.shower(G.hard_events(0, n, 1), 7, **gk).to_host()
    oout = O.shower(O.hard_events(0, n, 1), 7, nthreads=8, **ok)
    frac, worst, _ = compare_events(oout, gout, SCALE)
    say(f"  identical {frac:.5f}  worst rel diff {worst:.2e}")
    assert frac >= 0.999 and worst < 1e-9
    assert int(gout.n_viol.sum()) == 0
    assert np.array_equal(oout.t1, gout.t1) or np.max(np.abs(oout.t1 - gout.t1) / SCALE ** 2) < 1e-9


@pytest.mark.parametrize("retain", [True, False])
def test_learned_shower_parity(gpu, orc, retain):
    """Learned mode on POWHEG-like events with an oracle-made table (the
    analytic bound cut to an eighth in every third eta bin of cells 2-4):
    corrected first emissions, nulls, refreshed cells and fallbacks."""
    from paper_2511_19633_amd import binding
    G, O = gpu["powheg"], orc["powheg"]
    tab = np.ascontiguousarray(np.broadcast_to(O.bounds()[8:72, :, None], (64, 48, 8))).copy()
    tab[:, ::3, 2:5] *= 0.125
    G.learned_set_table(tab)
    n = 3000
    gout = G.shower(G.hard_events(0, n, 2), 6, mode=binding.MODE_LEARNED, retain=retain).to_host()
    oout = O.shower_learned(O.hard_events(0, n, 2), 6, tab, nthreads=8, retain=retain)
    fb = (oout.flags & records.FLAG_FALLBACK) != 0
    frac, worst, _ = compare_events(oout, gout, SCALE)
    say(f"  retain={retain}: identical {frac:.5f}, worst rel diff {worst:.3g}, fallbacks {fb.mean():.4f}")
    assert frac >= 0.999 and worst < 1e-9


def test_trial_log_leaves_out_corrected_trials(gpu, orc):
    """The trial log of POWHEG-like events has the oracle's rows (corrected
    first-emission trials are not logged), as a multiset."""
    import torch
    G, O = gpu["powheg"], orc["powheg"]
    n = 2000
    _, grows, gcnt = G.shower_log(G.hard_events(0, n, 3), 3, 2_000_000)
    _, orows, ocnt = O.shower_log(O.hard_events(0, n, 3), 3, 2_000_000, nthreads=8)
    say(f"  rows: gpu {gcnt}, oracle {ocnt}")
    assert gcnt == ocnt
    g = grows[:gcnt].cpu().numpy() if isinstance(grows, torch.Tensor) else np.asarray(grows[:gcnt])
    o = np.asarray(orows[:ocnt])
    key = lambda a: a[np.lexsort(a.T[::-1])]
    assert np.allclose(key(g), key(o), rtol=1e-5, atol=1e-6)


def test_rejected_configurations(cfgs):
    from paper_2511_19633_amd import binding
    for bad in (dict(cfgs["ee"], matching=2), dict(cfgs["dy"], matching=1, mu_q2=100.0),
                dict(cfgs["nlo"], matching=1, mu_q2=0.0), dict(cfgs["nlo"], matching=3)):
        with pytest.raises(binding.GapsError):
            binding.Gaps(bad)


def test_powheg_full_size_streamed_sampled(gpu, orc):
    """POWHEG-like events at the benchmark's batch size and launch: two
    batches of 10^6 events (ids 0 .. 2 * 10^6 - 1) streamed through one
    graph-captured persistent launch with retained trials; 300 sampled events
    against the oracle one by one."""
    import torch
    from paper_2511_19633_amd import binding
    G, O = gpu["powheg"], orc["powheg"]
    NPB, SEED = 1_000_000, 1
    ins = [G.hard_events(k * NPB, NPB, SEED, max_slots=8) for k in range(2)]
    outs = [binding.DeviceEvents(NPB, workloads.MAX_SLOTS) for _ in range(2)]
    say("powheg full size: 2 x 10^6 events streamed")
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    graph = G.capture([(i, o, NPB) for i, o in zip(ins, outs)], SEED, stream, mode=binding.MODE_PLAIN, retain=True)
    try:
        graph.launch(stream)
        stream.synchronize()
    finally:
        graph.close()
    ids = np.sort(np.random.default_rng(11).choice(2 * NPB, size=300, replace=False))
    g = records.Events(len(ids), workloads.MAX_SLOTS)
    o_in = records.Events(len(ids), 8)
    for s, i in enumerate(ids):
        d = outs[int(i) // NPB]
        j = int(i) % NPB
        for name in g.fields():
            t = getattr(d, name)
            a = getattr(g, name)
            if a.ndim == 1:
                a[s] = t[j].item()
            else:
                a[:, s] = t[:, j].cpu().numpy()
        one = O.hard_events(int(i), 1, SEED, max_slots=8)
        for name in o_in.fields():
            a = getattr(o_in, name)
            if a.ndim == 1:
                a[s] = getattr(one, name)[0]
            else:
                a[:, s] = getattr(one, name)[:, 0]
    oout = O.shower(o_in, SEED, nthreads=8, max_slots=workloads.MAX_SLOTS, retain=True)
    frac, worst, _ = compare_events(oout, g, SCALE)
    say(f"  identical {frac:.5f}, worst rel diff {worst:.2e}")
    assert np.array_equal(oout.id, g.id)
    assert frac >= 0.999 and worst < 1e-9
    assert np.all(g.flags == records.FLAG_MEC)
