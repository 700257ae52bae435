"""Mutation tests of the oracle's pins: each plants one plausible mistake in a
copy of the oracle's sources (a wrong colour factor, a dropped factor of a
kernel, the heavy-quark measure or factor left out, the weighted veto of a
violated learned bound replaced by plain acceptance), builds that copy into a
temporary library, and checks that the pin meant to catch it fails.  The
in-tree oracle is untouched; the pins themselves pass on it (the tests of
test_oracle_kernels.py and test_oracle_learned.py)."""
import os
import shutil
import subprocess

import pytest

from gapsinputs import workloads
from oracle.pyoracle import Oracle
from tests import sudakov_pins as P

ORACLE_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")

# name, [(text in shower.c, which occurrence, replacement)], pin
MUTANTS = [
    ("ff_g_to_gg_colour_factor",
     [("P = 0.5 * OR_CA * (2.0 / den1 - 2.0 + z * omz);", 0, "P = OR_CA * (2.0 / den1 - 2.0 + z * omz);")], "ff"),
    ("ff_g_to_qq_normalisation",
     [("P = 0.5 * OR_TR * (1.0 - 2.0 * z * omz);", 0, "P = OR_TR * (1.0 - 2.0 * z * omz);")], "ff"),
    ("fi_q_to_qg_soft_term",
     [("P = OR_CF * (2.0 / den1 - (1.0 + z));", 1, "P = OR_CF * (1.0 / den1 - (1.0 + z));")], "h_fi"),
    ("if_family_c_colour_factor",
     [("case K_C: P = OR_CA * (1.0 / (omx + uv)", 0, "case K_C: P = OR_CF * (1.0 / (omx + uv)")], "h_is"),
    ("ii_family_d_factor",
     [("default: P = OR_CF * (x + 2.0 * omx / x); break;", 1, "default: P = OR_CF * (x + omx / x); break;")], "h_is"),
    ("heavy_factor_dropped",
     [("double hf = ch->heavy ? (t - ch->m2) / t : 1.0;", 0, "double hf = 1.0;")], "charm"),
    ("heavy_measure_massless",
     [("else key = log(C->m2 + (Tch - C->m2) * exp(lu * invc));", 0, "else key = lnTch + lu * invc;")], "charm"),
    ("learned_violation_accepted_unweighted",
     [("st.acc = u[3] < v->w / g;", 0, "st.acc = 1;"), ("r->wfac *= st.acc ? g : -g;", 0, "(void)g;")],
     "learned"),
]


def _replace_nth(text, old, k, new):
    pos = -1
    for _ in range(k + 1):
        pos = text.index(old, pos + 1)
    return text[:pos] + new + text[pos + len(old):]


def build_mutant(tmp, edits):
    src = os.path.join(tmp, "src")
    os.makedirs(src)
    for f in os.listdir(ORACLE_DIR):
        if f.endswith((".c", ".h")):
            shutil.copy(os.path.join(ORACLE_DIR, f), src)
    path = os.path.join(src, "shower.c")
    text = open(path).read()
    for old, k, new in edits:
        assert text.count(old) > k, old
        text = _replace_nth(text, old, k, new)
    open(path, "w").write(text)
    lib = os.path.join(tmp, "liboracle_mutant.so")
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off", "-w", "-o", lib,
                           *[os.path.join(src, f) for f in ("core.c", "shower.c", "hard.c", "observables.c")],
                           "-lm", "-lpthread"])
    return lib


def run_pin(pin, lib):
    if pin == "ff":
        return P.check_ff_qqg(Oracle(workloads.config_dict(workloads.EE), lib_path=lib), "paper")
    if pin in ("h_fi", "h_is"):
        cfg = workloads.config_dict(workloads.PP_NLO)
        return P.check_h_gluon(Oracle(cfg, lib_path=lib), P.PDF(cfg["pdf"]), "paper", pin[2:])
    if pin == "charm":
        cfg = workloads.config_dict(workloads.PP_LO)
        return P.check_heavy_born(Oracle(cfg, lib_path=lib), P.PDF(cfg["pdf"]), "paper", 4)
    cfg = workloads.config_dict(workloads.PP_LO)
    return P.check_learned_planted(Oracle(cfg, lib_path=lib), P.PDF(cfg["pdf"]), False)


@pytest.mark.slow
@pytest.mark.parametrize("name,edits,pin", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_its_pin(tmp_path, name, edits, pin):
    lib = build_mutant(str(tmp_path), edits)
    with pytest.raises(AssertionError):
        run_pin(pin, lib)
