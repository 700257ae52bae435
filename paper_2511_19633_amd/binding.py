"""ctypes binding of libgaps (include/gaps.h).

Argument marshalling only: torch tensors provide device memory and streams;
every step of the shower runs in the library's HIP kernels.  Importing this
module never falls back to anything else: if libgaps.so is missing or no GPU
is visible, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

from gapsinputs import records

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgaps.so")

MODE_PLAIN, MODE_LEARNED, MODE_LOG = 0, 1, 2
NSTATS = 8
ST_CYCLES, ST_TRIALS, ST_ACCEPT, ST_VIOL, ST_LANE_ITERS, ST_LANE_ACTIVE, ST_FALLBACK, ST_NULL = range(8)
NOBS = 12
# per-event flags (GAPS_F_* of include/gaps.h)
F_OVERFLOW, F_COLOUR, F_NAN, F_FALLBACK, F_VIOL, F_HARDFAIL, F_HEVENT, F_MAXCYC = (1 << k for k in range(8))


class GapsError(RuntimeError):
    pass


class GapsConfig(C.Structure):
    _fields_ = [
        ("process", C.c_int), ("nf", C.c_int),
        ("sqrt_s", C.c_double), ("t_cut", C.c_double), ("alphas_mz", C.c_double),
        ("mz", C.c_double), ("gz", C.c_double), ("sw2", C.c_double), ("gf", C.c_double),
        ("mc", C.c_double), ("mb", C.c_double),
        ("mll_min", C.c_double), ("mll_max", C.c_double), ("p_s", C.c_double),
        ("pdf_xf", C.POINTER(C.c_float)), ("nx", C.c_int), ("nq", C.c_int), ("ntab", C.c_int),
        ("lnx0", C.c_double), ("lnx1", C.c_double), ("lnq0", C.c_double), ("lnq1", C.c_double),
        ("over_scale", C.c_double), ("matching", C.c_int), ("mu_q2", C.c_double),
    ]


class GapsEvents(C.Structure):
    _fields_ = [(name, C.c_void_p) for name in
                ("id", "w", "t_start", "n", "flags", "E", "px", "py", "pz", "pid", "col", "acol",
                 "status", "n_cycles", "n_trials", "n_accept", "n_viol", "t1")] + [
        ("max_slots", C.c_int32), ("cap", C.c_int64)]


class GapsParams(C.Structure):
    _fields_ = [("mode", C.c_int), ("block", C.c_int), ("grid", C.c_int), ("compact_every", C.c_int),
                ("trial_log", C.c_void_p), ("log_cap", C.c_int64), ("log_count", C.c_void_p),
                ("stats", C.c_void_p), ("variant", C.c_int), ("waves_per_simd", C.c_int),
                ("tail_every", C.c_int), ("retain", C.c_int), ("gen_select", C.c_int), ("veto_max", C.c_int)]


class GapsBatch(C.Structure):
    _fields_ = [("in_", GapsEvents), ("out", GapsEvents), ("n", C.c_int64)]


MAX_BATCHES = 4096
MLP_PARAMS = 4545
LEARN_SHAPE = (64, 48, 8)


class GapsTunePoint(C.Structure):
    _fields_ = [("block", C.c_int), ("compact_every", C.c_int), ("waves_per_simd", C.c_int), ("fill", C.c_float),
                ("grid", C.c_int), ("ms", C.c_float)]


class GapsTrainParams(C.Structure):
    _fields_ = [("steps", C.c_int64), ("batch", C.c_int64), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("tau", C.c_float), ("seed", C.c_uint64)]

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise GapsError(f"{LIB_PATH} is not built (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp, i64, u64 = C.c_void_p, C.c_int64, C.c_uint64
        L.gaps_init.argtypes = [C.POINTER(GapsConfig), C.POINTER(vp)]
        L.gaps_destroy.argtypes = [vp]
        L.gaps_strerror.restype = C.c_char_p
        L.gaps_strerror.argtypes = [C.c_int]
        L.gaps_hard_events.argtypes = [vp, i64, i64, u64, C.POINTER(GapsEvents), vp]
        L.gaps_shower.argtypes = [vp, C.POINTER(GapsEvents), i64, C.POINTER(GapsParams), u64,
                                  C.POINTER(GapsEvents), vp]
        L.gaps_shower_noalloc.argtypes = [vp, C.POINTER(GapsEvents), i64, C.POINTER(GapsParams), u64,
                                          C.POINTER(GapsEvents), vp]
        L.gaps_shower_stream.argtypes = [vp, C.POINTER(GapsBatch), C.c_int, C.POINTER(GapsParams), u64, vp]
        L.gaps_graph_capture.argtypes = [vp, C.POINTER(GapsBatch), C.c_int, C.POINTER(GapsParams), u64, vp,
                                         C.POINTER(vp)]
        L.gaps_tune.argtypes = [vp, C.POINTER(GapsBatch), C.c_int, C.POINTER(GapsParams), u64,
                                C.POINTER(GapsTunePoint), C.c_int, C.c_int, vp]
        L.gaps_graph_launch.argtypes = [vp, vp]
        L.gaps_graph_destroy.argtypes = [vp]
        L.gaps_observables.argtypes = [vp, C.POINTER(GapsEvents), i64, vp, vp]
        L.gaps_mlp_init.argtypes = [vp, u64]
        L.gaps_mlp_set.argtypes = [vp, vp]
        L.gaps_mlp_get.argtypes = [vp, vp]
        L.gaps_mlp_features.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp]
        L.gaps_mlp_forward.argtypes = [vp, vp, i64, vp, vp]
        L.gaps_mlp_grad.argtypes = [vp, vp, vp, i64, C.c_float, vp, vp, vp]
        L.gaps_mlp_train.argtypes = [vp, vp, vp, i64, C.POINTER(GapsTrainParams), vp, vp]
        L.gaps_mlp_adam_step.argtypes = [vp, vp, C.c_float, C.c_float, C.c_float, C.c_float, vp]
        L.gaps_mlp_calibrate.argtypes = [vp, vp, vp, vp, i64, vp]
        L.gaps_mlp_set_delta.argtypes = [vp, vp]
        L.gaps_cellmax_table.argtypes = [vp, vp, i64, i64, vp]
        L.gaps_cellmax_table_adaptive.argtypes = [vp, vp, i64, i64, vp]
        L.gaps_mlp_get_delta.argtypes = [vp, vp]
        L.gaps_mlp_tabulate.argtypes = [vp, vp]
        L.gaps_learned_table.argtypes = [vp, vp]
        L.gaps_learned_set_table.argtypes = [vp, vp]
        L.gaps_histogram.argtypes = [vp, vp, vp, i64, C.c_int, C.c_double, C.c_double, C.c_int, vp, vp, vp]
        L.gaps_bounds.argtypes = [vp, vp]
        L.gaps_pdf_eval.argtypes = [vp, vp, vp, vp, i64, vp, vp]
        L.gaps_rng_blocks.argtypes = [u64, C.c_uint32, vp, vp, vp, i64, vp, vp]
        _lib = L
    return _lib


def _check(status):
    if status != 0:
        raise GapsError(f"libgaps: {lib().gaps_strerror(status).decode()} ({status})")


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


_TORCH = {np.int64: torch.int64, np.float64: torch.float64, np.int32: torch.int32,
          np.uint32: torch.uint32, np.int8: torch.int8}


class DeviceEvents:
    """Event record in device memory (same layout as gapsinputs.records)."""

    def __init__(self, cap: int, max_slots: int, device="cuda"):
        self.cap, self.max_slots = int(cap), int(max_slots)
        for name, dt in records.PER_EVENT + records.COUNTERS:
            setattr(self, name, torch.zeros(self.cap, dtype=_TORCH[dt], device=device))
        for name, dt in records.PER_SLOT:
            setattr(self, name, torch.zeros((self.max_slots, self.cap), dtype=_TORCH[dt], device=device))

    def fields(self):
        return [n for n, _ in records.PER_EVENT + records.PER_SLOT + records.COUNTERS]

    def struct(self) -> GapsEvents:
        s = GapsEvents()
        for name in self.fields():
            setattr(s, name, getattr(self, name).data_ptr())
        s.max_slots, s.cap = self.max_slots, self.cap
        return s

    @classmethod
    def from_host(cls, ev: records.Events) -> "DeviceEvents":
        d = cls(ev.cap, ev.max_slots)
        for name in d.fields():
            getattr(d, name).copy_(torch.from_numpy(np.ascontiguousarray(getattr(ev, name))))
        return d

    def to_host(self) -> records.Events:
        ev = records.Events(self.cap, self.max_slots)
        for name in self.fields():
            getattr(ev, name)[...] = getattr(self, name).cpu().numpy()
        return ev

    def view(self, start: int, n: int) -> "EventsView":
        """Events start .. start+n-1 of this record, without a copy."""
        return EventsView(self, start, n)


class EventsView:
    """A contiguous range of events of a DeviceEvents record, in place: its
    fields are torch views, and its C-ABI description points at the range's
    first event with the parent's stride (cap), so the library reads and
    writes the parent's storage.  Pass its length `n` explicitly to the
    library calls."""

    def __init__(self, parent: DeviceEvents, start: int, n: int):
        if start < 0 or n < 0 or start + n > parent.cap:
            raise ValueError("view outside the record")
        self.parent, self.start, self.n_events = parent, int(start), int(n)
        self.cap, self.max_slots = parent.cap, parent.max_slots
        for name in parent.fields():
            t = getattr(parent, name)
            setattr(self, name, t[start:start + n] if t.dim() == 1 else t[:, start:start + n])

    def fields(self):
        return self.parent.fields()

    def struct(self) -> GapsEvents:
        s = GapsEvents()
        for name in self.fields():
            t = getattr(self.parent, name)
            setattr(s, name, t.data_ptr() + self.start * t.element_size())
        s.max_slots, s.cap = self.max_slots, self.cap
        return s


class Gaps:
    """A configured libgaps context on the current device."""

    def __init__(self, cfg: dict, over_scale: float = 1.0):
        if not torch.cuda.is_available():
            raise GapsError("libgaps needs a GPU; none is visible")
        self._pdf = np.ascontiguousarray(cfg["pdf"], dtype=np.float32)
        c = GapsConfig()
        for name, _ in GapsConfig._fields_:
            if name == "pdf_xf":
                continue
            if name in cfg:
                setattr(c, name, cfg[name])
        c.nf = cfg.get("nf", 5)
        c.pdf_xf = self._pdf.ctypes.data_as(C.POINTER(C.c_float))
        c.over_scale = over_scale
        self.cfg = cfg
        h = C.c_void_p()
        torch.cuda.init()
        _check(lib().gaps_init(C.byref(c), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().gaps_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def bounds(self) -> np.ndarray:
        out = np.zeros((72, 48), dtype=np.float64)
        _check(lib().gaps_bounds(self.h, out.ctypes.data_as(C.c_void_p)))
        return out

    def hard_events(self, first_id: int, n: int, seed: int, max_slots: int = 128, out=None,
                    stream=None) -> DeviceEvents:
        ev = out if out is not None else DeviceEvents(n, max_slots)
        s = ev.struct()
        _check(lib().gaps_hard_events(self.h, first_id, n, seed, C.byref(s), _stream(stream)))
        return ev

    @staticmethod
    def _params(mode=MODE_PLAIN, block=0, grid=0, compact_every=0, stats=None, trial_log=None,
                log_count=None, variant=0, waves_per_simd=0, tail_every=0, retain=False,
                gen_select=False, veto_max=False) -> GapsParams:
        p = GapsParams()
        p.mode, p.block, p.grid, p.compact_every = mode, block, grid, compact_every
        p.variant = variant
        p.waves_per_simd = waves_per_simd
        p.tail_every = tail_every
        p.retain = int(bool(retain))
        p.gen_select = int(bool(gen_select))
        p.veto_max = int(bool(veto_max))
        p.stats = stats.data_ptr() if stats is not None else None
        if trial_log is not None:
            p.trial_log = trial_log.data_ptr()
            p.log_cap = trial_log.shape[0]
            p.log_count = log_count.data_ptr()
        return p

    def shower(self, ev_in: DeviceEvents, seed: int, n: int | None = None, out=None, max_slots=None,
               stream=None, **params) -> DeviceEvents:
        n = ev_in.cap if n is None else n
        ev_out = out if out is not None else DeviceEvents(n, max_slots or ev_in.max_slots)
        p = self._params(**params)
        si, so = ev_in.struct(), ev_out.struct()
        _check(lib().gaps_shower(self.h, C.byref(si), n, C.byref(p), seed, C.byref(so), _stream(stream)))
        return ev_out

    def shower_noalloc(self, ev_in: DeviceEvents, seed: int, out: DeviceEvents, n: int | None = None,
                       stream=None, **params) -> DeviceEvents:
        """gaps_shower_noalloc: the shower with the library's static working
        storage (no device allocation in the call); the caller passes the
        output record."""
        n = ev_in.cap if n is None else n
        p = self._params(**params)
        si, so = ev_in.struct(), out.struct()
        _check(lib().gaps_shower_noalloc(self.h, C.byref(si), n, C.byref(p), seed, C.byref(so), _stream(stream)))
        return out

    @staticmethod
    def _batches(batches):
        """[(ev_in, ev_out[, n]), ...] -> ctypes array of GapsBatch."""
        arr = (GapsBatch * max(len(batches), 1))()
        for k, b in enumerate(batches):
            ev_in, ev_out = b[0], b[1]
            arr[k].in_ = ev_in.struct()
            arr[k].out = ev_out.struct()
            arr[k].n = b[2] if len(b) > 2 else ev_in.cap
        return arr

    def shower_stream(self, batches, seed: int, stream=None, **params):
        """Shower a list of (ev_in, ev_out[, n]) batches in one persistent launch."""
        arr = self._batches(batches)
        p = self._params(**params)
        _check(lib().gaps_shower_stream(self.h, arr, len(batches), C.byref(p), seed, _stream(stream)))

    def tune(self, batches, seed: int, points, repeats: int = 3, stream=None, **params):
        """gaps_tune: time the streamed launch over `batches` for each point
        (dicts with block, compact_every, waves_per_simd, fill); returns the
        points with their resolved grid and median ms (-1: not runnable)."""
        arr = self._batches(batches)
        pts = (GapsTunePoint * len(points))()
        for k, q in enumerate(points):
            pts[k].block, pts[k].compact_every = int(q["block"]), int(q["compact_every"])
            pts[k].waves_per_simd, pts[k].fill = int(q["waves_per_simd"]), float(q["fill"])
        p = self._params(**params)
        _check(lib().gaps_tune(self.h, arr, len(batches), C.byref(p), seed, pts, len(points), repeats,
                               _stream(stream)))
        return [dict(block=q.block, compact_every=q.compact_every, waves_per_simd=q.waves_per_simd,
                     fill=round(float(q.fill), 4), grid=q.grid, ms=float(q.ms)) for q in pts]

    def capture(self, batches, seed: int, stream, **params) -> "Graph":
        """HIP graph of one shower_stream call, captured on `stream` (a side stream)."""
        arr = self._batches(batches)
        p = self._params(**params)
        g = C.c_void_p()
        _check(lib().gaps_graph_capture(self.h, arr, len(batches), C.byref(p), seed, _stream(stream),
                                        C.byref(g)))
        return Graph(g, batches)

    # ---- trial log and the learned bound
    def shower_log(self, ev_in: DeviceEvents, seed: int, log_cap: int, stream=None, **params):
        """LOG mode: returns (events, rows [min(count, cap)][5] device tensor, count)."""
        log = torch.zeros((max(int(log_cap), 1), 5), dtype=torch.float32, device="cuda")
        cnt = torch.zeros(1, dtype=torch.uint64, device="cuda")
        out = self.shower(ev_in, seed, mode=MODE_LOG, trial_log=log, log_count=cnt, stream=stream, **params)
        torch.cuda.synchronize()
        count = int(cnt.item())
        return out, log[:min(count, int(log_cap))], count

    def mlp_init(self, seed: int):
        _check(lib().gaps_mlp_init(self.h, seed))

    def mlp_set(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float32)
        assert th.shape == (MLP_PARAMS,)
        _check(lib().gaps_mlp_set(self.h, th.ctypes.data_as(C.c_void_p)))

    def mlp_get(self) -> np.ndarray:
        th = np.zeros(MLP_PARAMS, dtype=np.float32)
        _check(lib().gaps_mlp_get(self.h, th.ctypes.data_as(C.c_void_p)))
        return th

    def mlp_features(self, rows: torch.Tensor, stream=None):
        n = rows.shape[0]
        x = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
        y = torch.zeros(n, dtype=torch.float32, device="cuda")
        ent = torch.zeros(n, dtype=torch.int32, device="cuda")
        cell = torch.zeros(n, dtype=torch.int32, device="cuda")
        _check(lib().gaps_mlp_features(self.h, _ptr(rows.contiguous()), n, _ptr(x), _ptr(y), _ptr(ent), _ptr(cell),
                                       _stream(stream)))
        return x, y, ent, cell

    def mlp_forward(self, x: torch.Tensor, stream=None) -> torch.Tensor:
        f = torch.zeros(x.shape[0], dtype=torch.float32, device="cuda")
        _check(lib().gaps_mlp_forward(self.h, _ptr(x.contiguous()), x.shape[0], _ptr(f), _stream(stream)))
        return f

    def mlp_grad(self, x: torch.Tensor, y: torch.Tensor, tau: float, stream=None):
        g = torch.zeros(MLP_PARAMS, dtype=torch.float32, device="cuda")
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        _check(lib().gaps_mlp_grad(self.h, _ptr(x.contiguous()), _ptr(y.contiguous()), x.shape[0], tau, _ptr(g),
                                   _ptr(loss), _stream(stream)))
        return g, loss

    def mlp_adam_step(self, grad: torch.Tensor, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        """One Adam step of the weights with a device gradient (cleared afterwards)."""
        if grad.dtype != torch.float32 or grad.numel() != MLP_PARAMS or not grad.is_contiguous():
            raise ValueError("grad must be a contiguous float32 tensor of MLP_PARAMS elements")
        _check(lib().gaps_mlp_adam_step(self.h, _ptr(grad), lr, beta1, beta2, eps, _stream(stream)))

    def mlp_train(self, x: torch.Tensor, y: torch.Tensor, steps: int, batch: int = 65536, lr: float = 3e-3,
                  tau: float = 0.999, beta1=0.9, beta2=0.999, eps=1e-8, seed=0, stream=None) -> torch.Tensor:
        p = GapsTrainParams(steps, batch, lr, beta1, beta2, eps, tau, seed)
        loss = torch.zeros(max(steps, 1), dtype=torch.float32, device="cuda")
        _check(lib().gaps_mlp_train(self.h, _ptr(x.contiguous()), _ptr(y.contiguous()), x.shape[0], C.byref(p),
                                    _ptr(loss), _stream(stream)))
        return loss

    def mlp_calibrate(self, x, y, cell, stream=None):
        """Margins per cell from held-out rows (cell: as mlp_features gives it)."""
        _check(lib().gaps_mlp_calibrate(self.h, _ptr(x.contiguous()), _ptr(y.contiguous()), _ptr(cell.contiguous()),
                                        x.shape[0], _stream(stream)))

    def mlp_set_delta(self, delta):
        d = np.ascontiguousarray(np.broadcast_to(np.asarray(delta, dtype=np.float64).reshape(
            (64, 1, 1) if np.size(delta) == 64 else LEARN_SHAPE), LEARN_SHAPE))
        _check(lib().gaps_mlp_set_delta(self.h, d.ctypes.data_as(C.c_void_p)))

    def mlp_get_delta(self) -> np.ndarray:
        d = np.zeros(LEARN_SHAPE, dtype=np.float64)
        _check(lib().gaps_mlp_get_delta(self.h, d.ctypes.data_as(C.c_void_p)))
        return d

    def mlp_tabulate(self, stream=None):
        _check(lib().gaps_mlp_tabulate(self.h, _stream(stream)))

    def cellmax_table(self, rows, n_fit, stream=None, adaptive=False):
        """Cell-maximum bound from LOG rows (device [n][5] float32): the first
        n_fit rows fit the cells, the rest calibrate; becomes the learned table.
        adaptive: each cell from the finest block around it with enough rows."""
        assert rows.dtype == torch.float32 and rows.is_cuda and rows.dim() == 2 and rows.shape[1] == 5
        rows = rows.contiguous()
        fn = lib().gaps_cellmax_table_adaptive if adaptive else lib().gaps_cellmax_table
        _check(fn(self.h, _ptr(rows), int(n_fit), int(rows.shape[0] - n_fit), _stream(stream)))

    def learned_table(self) -> np.ndarray:
        t = np.zeros(LEARN_SHAPE, dtype=np.float64)
        _check(lib().gaps_learned_table(self.h, t.ctypes.data_as(C.c_void_p)))
        return t

    def learned_set_table(self, table):
        t = np.ascontiguousarray(table, dtype=np.float64)
        assert t.shape == LEARN_SHAPE
        _check(lib().gaps_learned_set_table(self.h, t.ctypes.data_as(C.c_void_p)))

    def observables(self, ev: DeviceEvents, n: int | None = None, stream=None) -> torch.Tensor:
        n = ev.cap if n is None else n
        obs = torch.zeros((n, NOBS), dtype=torch.float64, device="cuda")
        s = ev.struct()
        _check(lib().gaps_observables(self.h, C.byref(s), n, _ptr(obs), _stream(stream)))
        return obs

    def histogram(self, obs: torch.Tensor, w, col: int, lo: float, hi: float, nbins: int, stream=None):
        sw = torch.zeros(nbins, dtype=torch.float64, device="cuda")
        sw2 = torch.zeros(nbins, dtype=torch.float64, device="cuda")
        _check(lib().gaps_histogram(self.h, _ptr(obs), _ptr(w), obs.shape[0], col, lo, hi, nbins,
                                    _ptr(sw), _ptr(sw2), _stream(stream)))
        return sw, sw2

    def pdf_eval(self, tab: torch.Tensor, x: torch.Tensor, q2: torch.Tensor, stream=None) -> torch.Tensor:
        out = torch.zeros_like(x)
        _check(lib().gaps_pdf_eval(self.h, _ptr(tab), _ptr(x), _ptr(q2), x.numel(), _ptr(out), _stream(stream)))
        return out


class Graph:
    """A captured shower stream; holds the batch records it points to."""

    def __init__(self, handle, batches):
        self.h = handle
        self._keep = batches

    def launch(self, stream=None):
        _check(lib().gaps_graph_launch(self.h, _stream(stream)))

    def close(self):
        if getattr(self, "h", None):
            lib().gaps_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rng_blocks(seed: int, stream_id: int, ids: torch.Tensor, c2: torch.Tensor, c3: torch.Tensor,
               stream=None) -> torch.Tensor:
    out = torch.zeros((ids.numel(), 4), dtype=torch.uint32, device="cuda")
    _check(lib().gaps_rng_blocks(seed, stream_id, _ptr(ids), _ptr(c2), _ptr(c3), ids.numel(), _ptr(out),
                                 _stream(stream)))
    return out
