"""ctypes binding of the CPU oracle.  TEST INFRASTRUCTURE ONLY: loaded by the
tests, the smoke check and the CPU-baseline leg of the benchmark, never by the
GPU library or its binding."""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

from gapsinputs import records

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")


MODE_PLAIN, MODE_LEARNED, MODE_LOG = 0, 1, 2


class OrOpts(C.Structure):
    _fields_ = [("mode", C.c_int), ("log", C.POINTER(C.c_float)), ("log_cap", C.c_int64),
                ("log_count", C.POINTER(C.c_int64)), ("learned", C.POINTER(C.c_double)),
                ("retain", C.c_int), ("gen_select", C.c_int), ("veto_max", C.c_int)]


def build():
    subprocess.check_call(["sh", os.path.join(_HERE, "build.sh")])


class OrConfig(C.Structure):
    _fields_ = [
        ("process", C.c_int), ("nf", C.c_int),
        ("sqrt_s", C.c_double), ("t_cut", C.c_double), ("alphas_mz", C.c_double),
        ("mz", C.c_double), ("gz", C.c_double), ("sw2", C.c_double), ("gf", C.c_double),
        ("mc", C.c_double), ("mb", C.c_double),
        ("mll_min", C.c_double), ("mll_max", C.c_double), ("p_s", C.c_double),
        ("pdf", C.POINTER(C.c_float)), ("nx", C.c_int), ("nq", C.c_int), ("ntab", C.c_int),
        ("lnx0", C.c_double), ("lnx1", C.c_double), ("lnq0", C.c_double), ("lnq1", C.c_double),
        ("over_scale", C.c_double), ("matching", C.c_int), ("mu_q2", C.c_double),
    ]


class OrEvents(C.Structure):
    _fields_ = [
        ("id", C.c_void_p), ("w", C.c_void_p), ("t_start", C.c_void_p), ("n", C.c_void_p),
        ("flags", C.c_void_p),
        ("E", C.c_void_p), ("px", C.c_void_p), ("py", C.c_void_p), ("pz", C.c_void_p),
        ("pid", C.c_void_p), ("col", C.c_void_p), ("acol", C.c_void_p), ("status", C.c_void_p),
        ("n_cycles", C.c_void_p), ("n_trials", C.c_void_p), ("n_accept", C.c_void_p),
        ("n_viol", C.c_void_p), ("t1", C.c_void_p),
        ("max_slots", C.c_int32), ("cap", C.c_int64),
    ]


def _lib(path=None):
    if path is None:
        path = _LIB
        if not os.path.exists(path):
            build()
    lib = C.CDLL(path)
    lib.or_init.restype = C.c_void_p
    lib.or_init.argtypes = [C.POINTER(OrConfig)]
    lib.or_free.argtypes = [C.c_void_p]
    lib.or_philox4x32.argtypes = [C.POINTER(C.c_uint32)] * 3
    lib.or_alphas.restype = C.c_double
    lib.or_alphas.argtypes = [C.c_void_p, C.c_double]
    lib.or_alphas_ln.restype = C.c_double
    lib.or_alphas_ln.argtypes = [C.c_void_p, C.c_double]
    lib.or_pdf_f_lq.restype = C.c_double
    lib.or_pdf_f_lq.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_double, C.c_double]
    lib.or_pdf_xf.restype = C.c_double
    lib.or_pdf_xf.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_double]
    lib.or_bounds_shape.argtypes = [C.POINTER(C.c_int), C.POINTER(C.c_int)]
    lib.or_bounds.argtypes = [C.c_void_p, C.c_void_p]
    lib.or_lo_wmax.restype = C.c_double
    lib.or_lo_wmax.argtypes = [C.c_void_p]
    lib.or_hard_events.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_uint64, C.POINTER(OrEvents)]
    lib.or_shower.argtypes = [C.c_void_p, C.POINTER(OrEvents), C.c_int64, C.c_uint64,
                              C.POINTER(OrEvents), C.c_int]
    lib.or_shower_ex.argtypes = [C.c_void_p, C.POINTER(OrEvents), C.c_int64, C.c_uint64,
                                 C.POINTER(OrEvents), C.c_int, C.POINTER(OrOpts)]
    lib.or_cell_edges.argtypes = [C.c_void_p, C.c_void_p]
    lib.or_map.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_double,
                           C.c_void_p, C.c_void_p, C.c_int]
    lib.or_is_vars.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double,
                               C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.or_n_obs.restype = C.c_int
    lib.or_observables.argtypes = [C.c_void_p, C.POINTER(OrEvents), C.c_int64, C.c_void_p]
    for name in ("or_li2",):
        getattr(lib, name).restype = C.c_double
        getattr(lib, name).argtypes = [C.c_double]
    for name in ("or_nlo_bvi_factor", "or_nlo_aqq"):
        getattr(lib, name).restype = C.c_double
        getattr(lib, name).argtypes = [C.c_void_p]
    for name in ("or_nlo_bqq", "or_nlo_gqq"):
        getattr(lib, name).restype = C.c_double
        getattr(lib, name).argtypes = [C.c_void_p, C.c_double]
    lib.or_nlo_rs.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double,
                              C.POINTER(C.c_double)]
    lib.or_nlo_sub.restype = C.c_double
    lib.or_nlo_sub.argtypes = [C.c_int, C.c_double, C.c_double]
    lib.or_mec_ratio.restype = C.c_double
    lib.or_mec_ratio.argtypes = [C.c_int, C.c_double, C.c_double]
    lib.or_mec_bound.restype = C.c_double
    lib.or_mec_bound.argtypes = []
    lib.or_dy_real.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int] + [C.c_double] * 7 + [C.c_void_p]
    return lib


LIB = None
_OTHER = {}


def lib(path=None):
    """The oracle library (path: another build of the oracle's sources, as the
    mutation tests make; default the in-tree one)."""
    global LIB
    if path is not None:
        if path not in _OTHER:
            _OTHER[path] = _lib(path)
        return _OTHER[path]
    if LIB is None:
        LIB = _lib()
    return LIB


def philox4x32(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().or_philox4x32(c, k, o)
    return list(o)


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def events_struct(ev: records.Events) -> OrEvents:
    s = OrEvents()
    for name in ev.fields():
        setattr(s, name, _ptr(getattr(ev, name)))
    s.max_slots = ev.max_slots
    s.cap = ev.cap
    return s


class Oracle:
    """One configured oracle instance (keeps the config arrays alive)."""

    def __init__(self, cfg: dict, over_scale: float = 1.0, lib_path=None):
        self._pdf = np.ascontiguousarray(cfg["pdf"], dtype=np.float32)
        c = OrConfig()
        for name, _ in OrConfig._fields_:
            if name in ("pdf",):
                continue
            if name in cfg:
                setattr(c, name, cfg[name])
        c.nf = cfg.get("nf", 5)
        c.pdf = self._pdf.ctypes.data_as(C.POINTER(C.c_float))
        c.over_scale = over_scale
        self.cfg = cfg
        self._c = c
        self.L = lib(lib_path)
        self.h = self.L.or_init(C.byref(c))

    def __del__(self):
        if getattr(self, "h", None) and getattr(self, "L", None) is not None:
            self.L.or_free(self.h)
            self.h = None

    def alphas(self, t):
        return self.L.or_alphas(self.h, t)

    def alphas_ln(self, lnt):
        """The coupling at ln t (the veto weight's form: the trial's ln t)."""
        return self.L.or_alphas_ln(self.h, lnt)

    def pdf_f_lq(self, tab, x, q2, lq):
        """f (not x f) at ln Q^2 = lq given with Q^2."""
        return self.L.or_pdf_f_lq(self.h, tab, x, q2, lq)

    def pdf_xf(self, tab, x, q2):
        return self.L.or_pdf_xf(self.h, tab, x, q2)

    def bounds(self):
        ne, nb = C.c_int(), C.c_int()
        self.L.or_bounds_shape(C.byref(ne), C.byref(nb))
        out = np.zeros((ne.value, nb.value), dtype=np.float64)
        self.L.or_bounds(self.h, _ptr(out))
        return out

    def lo_wmax(self):
        return self.L.or_lo_wmax(self.h)

    def hard_events(self, first_id, n, seed, max_slots=128):
        ev = records.Events(n, max_slots)
        s = events_struct(ev)
        if self.L.or_hard_events(self.h, first_id, n, seed, C.byref(s)) != 0:
            raise ValueError("or_hard_events: invalid matching for this process")
        return ev

    def shower(self, ev_in: records.Events, seed, nthreads=1, max_slots=None, retain=False, gen_select=False,
               veto_max=False):
        """Plain shower; retain=True: the retained-trial form of the competition;
        gen_select=True: the generate-select form (one trial per cycle from the
        sum of the overestimates, the channel chosen by its share);
        veto_max=True: the veto-max form (every channel's own first accepted
        trial, the largest wins)."""
        out = records.Events(ev_in.cap, max_slots or ev_in.max_slots)
        si, so = events_struct(ev_in), events_struct(out)
        if not retain and not gen_select and not veto_max:
            self.L.or_shower(self.h, C.byref(si), ev_in.cap, seed, C.byref(so), nthreads)
            return out
        o = OrOpts(MODE_PLAIN, None, 0, None, None, int(retain), int(gen_select), int(veto_max))
        rc = self.L.or_shower_ex(self.h, C.byref(si), ev_in.cap, seed, C.byref(so), nthreads, C.byref(o))
        if rc != 0:
            raise RuntimeError("or_shower_ex failed")
        return out

    def shower_log(self, ev_in: records.Events, seed, log_cap, nthreads=1, max_slots=None, retain=False):
        """LOG mode: the plain shower plus its initial-state trial log
        (rows: ln t, ln eta, z, table entry, ln weight).  Returns (events, rows,
        total rows seen)."""
        out = records.Events(ev_in.cap, max_slots or ev_in.max_slots)
        si, so = events_struct(ev_in), events_struct(out)
        log = np.zeros((max(int(log_cap), 1), 5), dtype=np.float32)
        cnt = C.c_int64(0)
        o = OrOpts(MODE_LOG, log.ctypes.data_as(C.POINTER(C.c_float)), int(log_cap), C.pointer(cnt), None,
                   int(retain))
        rc = self.L.or_shower_ex(self.h, C.byref(si), ev_in.cap, seed, C.byref(so), nthreads, C.byref(o))
        if rc != 0:
            raise RuntimeError("or_shower_ex failed")
        return out, log[:min(cnt.value, int(log_cap))], cnt.value

    def shower_learned(self, ev_in: records.Events, seed, table, nthreads=1, max_slots=None, retain=False):
        """LEARNED mode with the bound table [64][48][8] (doubles).  A trial
        above its learned bound goes through the weighted veto and its event
        continues on the analytic bound (flag FALLBACK, weight multiplied by
        +-(2w - 1))."""
        out = records.Events(ev_in.cap, max_slots or ev_in.max_slots)
        si, so = events_struct(ev_in), events_struct(out)
        tab = np.ascontiguousarray(table, dtype=np.float64)
        assert tab.shape == (64, 48, 8)
        o = OrOpts(MODE_LEARNED, None, 0, None, tab.ctypes.data_as(C.POINTER(C.c_double)), int(retain))
        rc = self.L.or_shower_ex(self.h, C.byref(si), ev_in.cap, seed, C.byref(so), nthreads, C.byref(o))
        if rc != 0:
            raise RuntimeError("or_shower_ex failed")
        return out

    def cell_edges(self):
        out = np.zeros(9, dtype=np.float64)
        self.L.or_cell_edges(self.h, out.ctypes.data_as(C.c_void_p))
        return out

    def observables(self, ev: records.Events):
        nobs = self.L.or_n_obs()
        obs = np.zeros((ev.cap, nobs), dtype=np.float64)
        s = events_struct(ev)
        self.L.or_observables(self.h, C.byref(s), ev.cap, _ptr(obs))
        return obs

    # NLO pieces
    def li2(self, x):
        return self.L.or_li2(x)

    def bvi_factor(self):
        return self.L.or_nlo_bvi_factor(self.h)

    def aqq(self):
        return self.L.or_nlo_aqq(self.h)

    def bqq(self, eta):
        return self.L.or_nlo_bqq(self.h, eta)

    def gqq(self, x):
        return self.L.or_nlo_gqq(self.h, x)

    def rs(self, kind, sbar, tbar, ubar, mborn2):
        r = C.c_double()
        self.L.or_nlo_rs(self.h, kind, sbar, tbar, ubar, mborn2, C.byref(r))
        return r.value

    @staticmethod
    def nlo_sub(kind, x, va):
        return lib().or_nlo_sub(kind, x, va)

    @staticmethod
    def mec_ratio(family_b, x, v):
        return lib().or_mec_ratio(int(family_b), x, v)

    @staticmethod
    def mec_bound():
        return lib().or_mec_bound()

    def dy_real(self, f, kind, o2, m2, x, y, v, phi, c, uphi):
        out = np.zeros(4)
        self.L.or_dy_real(self.h, f, kind, o2, m2, x, y, v, phi, c, uphi, out.ctypes.data_as(C.c_void_p))
        return out


def kin_map(typ, pe, ps, v1, v2, phi, rest=None):
    pe = np.ascontiguousarray(pe, dtype=np.float64)
    ps = np.ascontiguousarray(ps, dtype=np.float64)
    out = np.zeros(12)
    nrest = 0
    if rest is not None:
        rest = np.ascontiguousarray(rest, dtype=np.float64).copy()
        nrest = rest.shape[0]
    lib().or_map(typ, _ptr(pe), _ptr(ps), v1, v2, phi, _ptr(out), _ptr(rest), nrest)
    return out.reshape(3, 4), rest


def is_vars(typ, z, t, s):
    x, uv = C.c_double(), C.c_double()
    lib().or_is_vars(typ, z, t, s, C.byref(x), C.byref(uv))
    return x.value, uv.value
