"""The C-ABI library loads and exports every entry point include/gaps.h declares;
argument validation that happens before any device work is checked on CPU."""
import ctypes as C
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    text = open(os.path.join(ROOT, "include", "gaps.h")).read()
    return sorted(set(re.findall(r"\b(gaps_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    from paper_2511_19633_amd import binding
    lib = C.CDLL(binding.LIB_PATH)
    names = declared()
    assert "gaps_shower" in names and "gaps_init" in names and "gaps_observables" in names
    for name in names:
        assert hasattr(lib, name), name


def test_argument_errors_without_device_work():
    from paper_2511_19633_amd import binding
    lib = binding.lib()
    assert lib.gaps_init(None, None) == -1
    cfg = binding.GapsConfig()
    h = C.c_void_p()
    assert lib.gaps_init(C.byref(cfg), C.byref(h)) == -1  # no PDF grid
    assert lib.gaps_shower(None, None, 0, None, 0, None, None) == -1
    assert lib.gaps_hard_events(None, 0, 0, 0, None, None) == -1
    assert lib.gaps_destroy(None) == -1
    assert lib.gaps_strerror(-4) == b"size exceeds capacity"


def test_stream_and_graph_argument_errors():
    from paper_2511_19633_amd import binding
    lib = binding.lib()
    assert lib.gaps_shower_stream(None, None, 0, None, 0, None) == -1
    assert lib.gaps_graph_capture(None, None, 0, None, 0, None, None) == -1
    assert lib.gaps_graph_launch(None, None) == -1
    assert lib.gaps_graph_destroy(None) == -1
    assert C.sizeof(binding.GapsBatch) == 2 * C.sizeof(binding.GapsEvents) + 8


def test_config_and_cellmax_argument_errors():
    """Matching and process combinations gaps_init rejects before any device
    work, and the cell-maximum entry points' argument checks."""
    import numpy as np
    from gapsinputs import workloads
    from paper_2511_19633_amd import binding
    lib = binding.lib()
    base = workloads.config_dict(workloads.PP_NLO)
    pdf = np.ascontiguousarray(base["pdf"], dtype=np.float32)

    def init(**over):
        cfg = dict(base, **over)
        c = binding.GapsConfig()
        for name, _ in binding.GapsConfig._fields_:
            if name != "pdf_xf" and name in cfg:
                setattr(c, name, cfg[name])
        c.nf = 5
        c.pdf_xf = pdf.ctypes.data_as(C.POINTER(C.c_float))
        h = C.c_void_p()
        return lib.gaps_init(C.byref(c), C.byref(h))

    assert init(matching=3) == -1
    assert init(matching=-1) == -1
    assert init(matching=1, mu_q2=0.0) == -1
    assert init(process=3, matching=2) == -1
    assert init(process=0, matching=1, mu_q2=100.0) == -1
    assert init(process=4, p_s=0.0) == -1
    assert init(process=4, mll_min=120.0, mll_max=100.0) == -1
    assert init(process=5) == -1
    assert lib.gaps_mlp_adam_step(None, None, 1e-3, 0.9, 0.999, 1e-8, None) == -1
    for fn in (lib.gaps_cellmax_table, lib.gaps_cellmax_table_adaptive):
        fn.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_void_p]
        assert fn(None, None, 10, 0, None) == -1


def test_noalloc_and_tune_argument_errors():
    from paper_2511_19633_amd import binding
    lib = binding.lib()
    assert lib.gaps_shower_noalloc(None, None, 0, None, 0, None, None) == -1
    pts = (binding.GapsTunePoint * 1)()
    assert lib.gaps_tune(None, None, 0, None, 0, pts, 1, 3, None) == -1
    assert C.sizeof(binding.GapsTunePoint) == 24
