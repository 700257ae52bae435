"""NLO pp -> Z/photon -> e+e- events (process 4) on the GPU beyond the parity
cases of test_gpu_parity: the other forms of the competition, learned mode,
and the benchmark's batch size and streamed launch, against the oracle event
by event (integer and colour data bit-exact, >= 99.9 % identical, momenta
within 1e-9 of the event's scale)."""
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
def G(cfgs):
    import torch
    from paper_2511_19633_amd import binding
    assert torch.cuda.is_available()
    return binding.Gaps(cfgs["dynlo"])


@pytest.mark.parametrize("form", [(dict(variant=1, gen_select=True), dict(gen_select=True)),
                                  (dict(variant=1, veto_max=True), dict(veto_max=True)),
                                  (dict(variant=1), dict())],
                         ids=["gen_select", "veto_max", "max_veto_lanes"])
def test_forms(G, oracles, form):
    gk, ok = form
    O = oracles["dynlo"]
    n = 3000
    say(f"dynlo form {gk}")
    gout = G.shower(G.hard_events(0, n, 4), 9, **gk).to_host()
    oout = O.shower(O.hard_events(0, n, 4), 9, nthreads=8, **ok)
    frac, worst, _ = compare_events(oout, gout, SCALE)
    say(f"  identical {frac:.5f}  worst rel diff {worst:.2e}")
    assert frac >= 0.999 and worst < 1e-9
    assert int(gout.n_viol.sum()) == 0


@pytest.mark.parametrize("retain", [True, False])
def test_learned(G, oracles, retain):
    """Learned mode with an oracle-made table (the analytic bound cut to an
    eighth in every third eta bin of cells 2-4: nulls, refreshed cells and
    fallbacks all occur)."""
    from paper_2511_19633_amd import binding
    O = oracles["dynlo"]
    tab = np.ascontiguousarray(np.broadcast_to(O.bounds()[8:72, :, None], (64, 48, 8))).copy()
    tab[:, ::3, 2:5] *= 0.125
    G.learned_set_table(tab)
    n = 3000
    gout = G.shower(G.hard_events(0, n, 5), 6, mode=binding.MODE_LEARNED, retain=retain).to_host()
    oout = O.shower_learned(O.hard_events(0, n, 5), 6, tab, nthreads=8, retain=retain)
    fb = (oout.flags & records.FLAG_FALLBACK) != 0
    frac, worst, _ = compare_events(oout, gout, SCALE)
    say(f"  retain={retain}: identical {frac:.5f}, worst rel diff {worst:.3g}, fallbacks {fb.mean():.4f}")
    assert frac >= 0.999 and worst < 1e-9


def test_full_size_streamed_sampled(G, oracles):
    """Two batches of 10^6 events streamed through one graph-captured
    persistent launch with retained trials (the benchmark's batch size and
    launch); 2000 sampled events against the oracle one by one."""
    import torch
    from paper_2511_19633_amd import binding
    O = oracles["dynlo"]
    NPB, SEED = 1_000_000, 1
    ins = [G.hard_events(k * NPB, NPB, SEED, max_slots=8) for k in range(2)]
    outs = [binding.DeviceEvents(NPB, workloads.MAX_SLOTS) for _ in range(2)]
    say("dynlo full size: 2 x 10^6 events streamed")
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    graph = G.capture([(i, o, NPB) for i, o in zip(ins, outs)], SEED, stream, mode=binding.MODE_PLAIN, retain=True)
    try:
        graph.launch(stream)
        stream.synchronize()
    finally:
        graph.close()
    from tests.test_gpu_fullsize import _gather
    ids = np.sort(np.random.default_rng(13).choice(2 * NPB, size=2000, replace=False))
    g = _gather(outs, ids, NPB)
    o_in = records.Events(len(ids), 8)
    for s, i in enumerate(ids):
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
    assert not np.any(g.flags & records.FLAG_OVERFLOW)
