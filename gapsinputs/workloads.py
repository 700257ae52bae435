"""Workload definitions shared by the oracle tests and the GPU library.

Each workload is the physics configuration plus the sizes the shower is run
at.  Nothing here computes any part of the shower; the values are inputs:
collider energy, couplings, masses, the cutoff and the toy PDF grid.

Processes (the ``process`` field):
  0  e+e- -> Z/gamma* -> q qbar at sqrt(s) = 91.2 GeV, final-state shower only
  1  pp -> Z -> e+e- LO Born at 13 TeV, initial + final-state shower
  2  pp -> Z (-> e+e-) NLO, MC@NLO-style S and H events, power shower
  3  pp -> gamma*/Z -> e+e- LO Born with the photon and the interference,
     m_ee in [mll_min, mll_max], at 13 TeV, initial + final-state shower
"""
from __future__ import annotations

import numpy as np

from . import toypdf

# Stream ids for the counter-based generator (the key's second word).
STREAM_PLAIN = 0
STREAM_LEARNED = 1
STREAM_HARD = 2

COMMON = dict(
    t_cut=1.0,            # shower cutoff in GeV^2
    alphas_mz=0.118,      # alpha_s(mZ^2), one-loop running, nf = 5
    mz=91.1876, gz=2.4952,
    sw2=0.23122, gf=1.1663788e-5,
    mc=1.3, mb=4.75,
    mll_min=66.0, mll_max=116.0,
    p_s=0.75,             # probability to generate an S event (NLO)
)

EE = dict(COMMON, process=0, sqrt_s=91.2)
PP_LO = dict(COMMON, process=1, sqrt_s=13000.0)
PP_NLO = dict(COMMON, process=2, sqrt_s=13000.0)
PP_DY = dict(COMMON, process=3, sqrt_s=13000.0)
# the matching variants of the NLO workload: MC@NLO with every event starting
# at mZ^2 instead of the hadronic S, and POWHEG-like Born events whose first
# emission the shower corrects to the real matrix element
PP_NLO_MUQ = dict(PP_NLO, matching=1, mu_q2=91.1876 ** 2)
PP_NLO_POWHEG = dict(PP_NLO, matching=2)
# the second workload at NLO: pp -> Z/photon -> e+e- with the interference,
# MC@NLO S/H events, the real emission by the Kleiss trick
PP_DY_NLO = dict(COMMON, process=4, sqrt_s=13000.0)

MAX_SLOTS = 128

WORKLOADS = {
    # small case: the oracle finishes it in seconds
    "ee_fs_10k": dict(cfg=EE, n_events=10_000, seed=1),
    "pp_lo_1m": dict(cfg=PP_LO, n_events=1_000_000, seed=1),
    "pp_nlo_1m": dict(cfg=PP_NLO, n_events=1_000_000, seed=1),
    "pp_nlo_batched_10m": dict(cfg=PP_NLO, n_events=10_000_000, seed=1),
    "pp_nlo_learned_10m": dict(cfg=PP_NLO, n_events=10_000_000, seed=1),
}


def config_dict(cfg: dict) -> dict:
    """Physics config plus the toy PDF grid, ready to hand to either side."""
    out = dict(cfg)
    out.update(toypdf.grid_config())
    out["pdf"] = toypdf.make_grid()
    return out


def batch_sizes(n_total: int, seed: int = 1, lo: int = 10_000, hi: int = 500_000):
    """Uneven batch sizes, uniform integers in [lo, hi], last one truncated.

    Drawn with numpy's Philox bit generator (an input-side generator only)."""
    rng = np.random.Generator(np.random.Philox(seed))
    sizes = []
    done = 0
    while done < n_total:
        b = int(rng.integers(lo, hi + 1))
        b = min(b, n_total - done)
        sizes.append(b)
        done += b
    return sizes
