"""At the benchmark's full size and in its launch configuration: 10 batches of
10^6 NLO events (ids 0 .. 10^7 - 1, seed 1) streamed through one graph-captured
persistent launch with retained trials, plain and learned; sampled events
across all batches against the oracle, one by one (integer and colour data
bit-exact, >= 99.9 % identical, weights within 1e-9, every parton's momentum
within 1e-9 of its own energy)."""
import sys

import numpy as np
import pytest

from gapsinputs import records, workloads
from tests.test_gpu_parity import SCALE, compare_events

pytestmark = pytest.mark.gpu

# 2000 sampled events: at the 99.9 % bar up to two may differ (300 would
# allow none, a resolution of 0.33 %)
NB, NPB, SEED, NSAMPLE = 10, 1_000_000, 1, 2000


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def full(cfgs):
    import torch
    from paper_2511_19633_amd import binding
    assert torch.cuda.is_available()
    G = binding.Gaps(cfgs["nlo"])
    ins = [G.hard_events(k * NPB, NPB, SEED, max_slots=8) for k in range(NB)]
    outs = [binding.DeviceEvents(NPB, workloads.MAX_SLOTS) for _ in range(NB)]
    ids = np.sort(np.random.default_rng(7).choice(NB * NPB, size=NSAMPLE, replace=False))
    return G, ins, outs, ids


def _run(G, ins, outs, mode):
    """The benchmark's launch: the ten batches in one captured persistent stream."""
    import torch
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    graph = G.capture([(i, o, NPB) for i, o in zip(ins, outs)], SEED, stream, mode=mode, retain=True)
    try:
        graph.launch(stream)
        stream.synchronize()
    finally:
        graph.close()


def _gather(outs, ids, npb=NPB):
    """The sampled events (ids over the concatenated batches of npb events)
    of the device outputs, as one host record."""
    import torch
    h = records.Events(len(ids), workloads.MAX_SLOTS)
    for k in range(len(outs)):
        sel = np.nonzero(ids // npb == k)[0]
        if not len(sel):
            continue
        idx = torch.from_numpy((ids[sel] % npb).astype(np.int64)).cuda()
        d = outs[k]
        for name in d.fields():
            t = getattr(d, name)
            g = (t.index_select(0, idx) if t.dim() == 1 else t.index_select(1, idx)).cpu().numpy()
            if t.dim() == 1:
                getattr(h, name)[sel] = g
            else:
                getattr(h, name)[:, sel] = g
    return h


def _oracle_inputs(O, ids):
    """The sampled events' hard events from the oracle's own generator (keyed by id)."""
    h = records.Events(len(ids), 8)
    for s, i in enumerate(ids):
        one = O.hard_events(int(i), 1, SEED, max_slots=8)
        for name in h.fields():
            a = getattr(h, name)
            if a.ndim == 1:
                a[s] = getattr(one, name)[0]
            else:
                a[:, s] = getattr(one, name)[:, 0]
    return h


def _check(oout, gout, what):
    frac, worst, _ = compare_events(oout, gout, SCALE["nlo"])
    say(f"  {what}: identical {frac:.5f}, worst rel diff {worst:.2e}")
    assert np.array_equal(oout.id, gout.id)
    assert frac >= 0.999 and worst < 1e-9
    assert not np.any(gout.flags & records.FLAG_OVERFLOW)


def test_full_size_plain_sampled(full, oracles):
    from paper_2511_19633_amd import binding
    G, ins, outs, ids = full
    O = oracles["nlo"]
    say(f"full size plain: {NB} x {NPB} events, {NSAMPLE} sampled")
    _run(G, ins, outs, binding.MODE_PLAIN)
    gout = _gather(outs, ids)
    oout = O.shower(_oracle_inputs(O, ids), SEED, nthreads=8, max_slots=workloads.MAX_SLOTS, retain=True)
    _check(oout, gout, "plain")


def test_full_size_learned_sampled(full, oracles):
    """Learned mode with an oracle-made table (the analytic bound cut to an
    eighth in every third eta bin of cells 2-4: nulls, refreshed cells and
    fallbacks all occur)."""
    from paper_2511_19633_amd import binding
    G, ins, outs, ids = full
    O = oracles["nlo"]
    tab = np.ascontiguousarray(np.broadcast_to(O.bounds()[8:72, :, None], (64, 48, 8))).copy()
    tab[:, ::3, 2:5] *= 0.125
    G.learned_set_table(tab)
    say(f"full size learned: {NB} x {NPB} events, {NSAMPLE} sampled")
    _run(G, ins, outs, binding.MODE_LEARNED)
    gout = _gather(outs, ids)
    oout = O.shower_learned(_oracle_inputs(O, ids), SEED, tab, nthreads=8, max_slots=workloads.MAX_SLOTS,
                            retain=True)
    fb = (gout.flags & records.FLAG_FALLBACK) != 0
    say(f"  fallbacks among the sampled events: {int(fb.sum())}")
    _check(oout, gout, "learned")
