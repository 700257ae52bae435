"""The generate-select and veto-max forms of the competition on the GPU
(libgaps through the C-ABI, the one event per lane kernels) against the
oracle's same forms, event by event (integer and colour data bit-exact,
>= 99.9 % identical, momenta within 1e-9 of the event's scale); then against
the max-veto competition in distribution."""
import sys

import numpy as np
import pytest

from gapsinputs import records, workloads
from tests.test_gpu_parity import SCALE, compare_events

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu(cfgs):
    import torch
    from paper_2511_19633_amd import binding
    assert torch.cuda.is_available()
    return {k: binding.Gaps(v) for k, v in cfgs.items()}


GS = dict(variant=1, gen_select=True)
# the GPU parameters and the oracle's of each form
FORMS = pytest.mark.parametrize("form", [(dict(variant=1, gen_select=True), dict(gen_select=True)),
                                         (dict(variant=1, veto_max=True), dict(veto_max=True))],
                                ids=["gen_select", "veto_max"])


@FORMS
@pytest.mark.parametrize("key,n", [("ee", 5000), ("lo", 3000), ("nlo", 3000)])
def test_form_parity(gpu, oracles, key, n, form):
    gk, ok = form
    say(f"{list(ok)[0]} parity {key} n={n}")
    G, O = gpu[key], oracles[key]
    gout = G.shower(G.hard_events(0, n, 1), 7, **gk).to_host()
    oout = O.shower(O.hard_events(0, n, 1), 7, nthreads=8, **ok)
    frac, worst, _ = compare_events(oout, gout, SCALE[key])
    say(f"  identical {frac:.5f}  worst rel diff {worst:.2e}  draws/event {gout.n_trials.mean():.1f}"
        f"  cycles/event {gout.n_cycles.mean():.1f}")
    assert frac >= 0.999 and worst < 1e-9
    assert int(gout.n_viol.sum()) == 0
    assert np.all((gout.flags & ~np.uint32(records.FLAG_HEVENT)) == 0)
    if "gen_select" in ok:
        assert np.all(gout.n_trials <= gout.n_cycles)
    else:
        assert np.array_equal(gout.n_cycles, gout.n_accept)


@FORMS
def test_form_ragged_overflow_and_scheduling(gpu, oracles, form):
    gk, ok = form
    G, O = gpu["nlo"], oracles["nlo"]
    for n in (1, 63, 65, 257):
        gout = G.shower(G.hard_events(100, n, 3), 9, block=64, **gk).to_host()
        oout = O.shower(O.hard_events(100, n, 3), 9, **ok)
        frac, _, _ = compare_events(oout, gout, SCALE["nlo"])
        assert frac == 1.0, n
    gout = G.shower(G.hard_events(0, 500, 5), 3, max_slots=8, **gk).to_host()
    oout = O.shower(O.hard_events(0, 500, 5), 3, max_slots=8, **ok)
    assert np.any(oout.flags & records.FLAG_OVERFLOW)
    assert np.array_equal(gout.flags & records.FLAG_OVERFLOW, oout.flags & records.FLAG_OVERFLOW)
    frac, _, _ = compare_events(oout, gout, SCALE["nlo"])
    assert frac >= 0.99
    gin = G.hard_events(0, 2000, 11)
    a = G.shower(gin, 5, **gk).to_host()
    for kw in (dict(block=64, grid=7), dict(block=128)):
        b = G.shower(gin, 5, **gk, **kw).to_host()
        for name in a.fields():
            assert np.array_equal(getattr(a, name), getattr(b, name)), (kw, name)


def test_forms_reject_other_settings(gpu):
    from paper_2511_19633_amd import binding
    G = gpu["nlo"]
    gin = G.hard_events(0, 64, 1)
    for kw in (dict(gen_select=True), dict(variant=1, gen_select=True, retain=True),
               dict(variant=1, gen_select=True, mode=binding.MODE_LEARNED), dict(veto_max=True),
               dict(variant=1, veto_max=True, gen_select=True), dict(variant=1, veto_max=True, retain=True),
               dict(variant=1, veto_max=True, mode=binding.MODE_LEARNED)):
        with pytest.raises(binding.GapsError):
            G.shower(gin, 1, **kw)
    outs = [binding.DeviceEvents(64, workloads.MAX_SLOTS)]
    with pytest.raises(binding.GapsError):
        G.shower_stream([(gin, outs[0], 64)], 1, **GS)


@FORMS
def test_form_matches_max_veto_in_distribution(gpu, form):
    """2 * 10^5 NLO events in the form and in max-veto (retained trials) on
    the GPU: the same distributions of emissions, Z pT, jets and partons."""
    from tests.histcheck import chi2_compare
    gk, _ = form
    G = gpu["nlo"]
    n = 200_000
    gin = G.hard_events(0, n, 1, max_slots=8)
    a = G.shower(gin, 2, max_slots=workloads.MAX_SLOTS, retain=True)
    b = G.shower(gin, 3, max_slots=workloads.MAX_SLOTS, **gk)
    na, nb = a.n_accept.cpu().numpy(), b.n_accept.cpu().numpy()
    one = np.ones(n)
    chi, ndf, p = chi2_compare(na, nb, one, one, np.arange(-0.5, 40.0))
    say(f"  emissions chi2/ndf {chi / ndf:.3f} (p {p:.3g}); draws/event {b.n_trials.double().mean().item():.1f}")
    assert p > 1e-3
    w = gin.w.cpu().numpy()
    oa, ob = G.observables(a).cpu().numpy(), G.observables(b).cpu().numpy()
    for col, edges in ((0, np.linspace(0.0, 60.0, 31)), (4, np.arange(-0.5, 7.0)), (9, np.arange(3.5, 31.0))):
        chi, ndf, p = chi2_compare(oa[:, col], ob[:, col], w, w, edges)
        say(f"  column {col}: chi2/ndf {chi / ndf:.3f} (p {p:.3g})")
        assert p > 1e-3
