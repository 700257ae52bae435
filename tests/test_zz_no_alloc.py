"""The allocation-free shower entry point (gaps_shower_noalloc) through the
C-ABI against gaps_shower: two calls in a row, the second with a smaller
input, every event bitwise equal (plain and learned, both forms)."""
import sys

import numpy as np
import pytest

from gapsinputs import records, workloads

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _equal(a, b, what):
    for name in a.fields():
        assert np.array_equal(getattr(a, name), getattr(b, name)), (what, name)


@pytest.mark.parametrize("retain", [False, True], ids=["regenerate", "retain"])
def test_noalloc_matches_shower(cfgs, oracles, retain):
    import torch
    from paper_2511_19633_amd import binding
    assert torch.cuda.is_available()
    G = binding.Gaps(cfgs["nlo"])
    for mode in (binding.MODE_PLAIN, binding.MODE_LEARNED):
        if mode == binding.MODE_LEARNED:
            # a bound that fails often: the weighted veto's weight factors too
            B = oracles["nlo"].bounds()
            G.learned_set_table(np.ascontiguousarray(np.broadcast_to(B[8:72, :, None] * 2.0 ** -3, (64, 48, 8))))
        for n, first in ((50000, 0), (7001, 123456)):
            say(f"noalloc retain={retain} mode={mode} n={n}")
            gin = G.hard_events(first, n, 3)
            ref = G.shower(gin, 17, mode=mode, retain=retain).to_host()
            out = binding.DeviceEvents(n, workloads.MAX_SLOTS)
            out.n.fill_(-1)
            G.shower_noalloc(gin, 17, out, mode=mode, retain=retain)
            torch.cuda.synchronize()
            _equal(ref, out.to_host(), (mode, n))
    G.close()


def test_noalloc_rejects_bad_arguments(cfgs):
    import torch
    from paper_2511_19633_amd import binding
    G = binding.Gaps(cfgs["nlo"])
    gin = G.hard_events(0, 100, 3)
    out = binding.DeviceEvents(100, workloads.MAX_SLOTS)
    with pytest.raises(binding.GapsError):
        G.shower_noalloc(gin, 1, out, block=96)  # not a multiple of 64
    with pytest.raises(binding.GapsError):
        G.shower_noalloc(gin, 1, gin)  # output aliases input
    torch.cuda.synchronize()
    G.close()
