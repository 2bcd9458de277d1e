"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad plan parameters before touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "t3pcf.h")
LIB = os.path.join(ROOT, "paper_2309_08601_amd", "libt3pcf.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(t3_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    return ctypes.CDLL(LIB)


def test_header_declares_entry_points():
    names = _declared()
    for n in ["t3_plan_create", "t3_plan_destroy", "t3_forward", "t3_forward_tomo",
              "t3_harmonics", "t3_normalise_resum", "t3_backward", "t3_error_string",
              "t3_last_error_message", "t3_version"]:
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for n in _declared():
        assert hasattr(lib, n), n


def test_binding_covers_header():
    src = open(os.path.join(ROOT, "paper_2309_08601_amd", "t3.py")).read()
    for n in _declared():
        assert n in src, n


def _params(**kw):
    from paper_2309_08601_amd.t3 import t3_params
    edges = np.asarray(kw.pop("edges", [1.0, 2.0, 4.0]), dtype=np.float64)
    p = t3_params(len(edges) - 1, edges.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                  kw.pop("n_max", 4), kw.pop("precision", 0), kw.pop("flags", 0), 0.0, 0, 0,
                  kw.pop("box_size", 1 << 20), 0.0, 0, 0, kw.pop("max_workspace_bytes", 0))
    for k, v in kw.items():
        setattr(p, k, v)
    return p, edges


@pytest.mark.parametrize("kw,code", [
    (dict(edges=[0.0, 1.0]), -1),
    (dict(edges=[1.0, 1.0]), -1),
    (dict(edges=[2.0, 1.0]), -1),
    (dict(edges=[1.0, 600.0]), -2),
    (dict(edges=list(np.geomspace(1.0, 100.0, 66))), -2),  # 65 bins: above the 64 a plan holds
    (dict(n_max=65), -2),
    (dict(n_max=-1), -2),
    (dict(precision=7), -1),
    (dict(flags=128), -1),
    (dict(max_workspace_bytes=-1), -1),
    (dict(box_size=0), -1),
    (dict(box_size=1 << 40), -2),
    (dict(lane_neighbours=-1.0), -1),
    (dict(lane_neighbours=129.0), -1),
    (dict(lane_neighbours=float("nan")), -1),
    (dict(tile_mode=2), -1),
])
def test_plan_create_rejects(lib, kw, code):
    pytest.importorskip("torch")
    from paper_2309_08601_amd import t3
    p, edges = _params(**kw)
    h = ctypes.c_void_p()
    rc = t3._lib.t3_plan_create(ctypes.byref(p), ctypes.byref(h))
    assert rc == code
    assert not h.value
    assert len(t3._lib.t3_last_error_message()) > 0


@pytest.mark.parametrize("flags", [0, 1 | 16, 32, 64, 1 | 2 | 4 | 8 | 16 | 32 | 64])
def test_plan_create_and_destroy_ok(lib, flags):
    """Every defined flag bit, alone and together (keep j = k, timing, no
    graph, edge correction, no lane kernel, keep planes, deterministic)."""
    pytest.importorskip("torch")
    from paper_2309_08601_amd import t3
    p, edges = _params(flags=flags)
    h = ctypes.c_void_p()
    assert t3._lib.t3_plan_create(ctypes.byref(p), ctypes.byref(h)) == 0
    assert h.value
    t3._lib.t3_plan_destroy(h)
    assert t3._lib.t3_error_string(-5) == b"position outside the lattice box"


def test_plan_settings_reports_parameters(lib):
    """The tunables a plan is created with are what t3_plan_settings reports
    (lane threshold 0 means the automatic 128)."""
    pytest.importorskip("torch")
    from paper_2309_08601_amd import t3
    for kw, lane in [(dict(), 128.0), (dict(lane_neighbours=64.0, tile_mode=1, scan_mode=1, chunk_centres=512), 64.0)]:
        p, edges = _params(**kw)
        h = ctypes.c_void_p()
        assert t3._lib.t3_plan_create(ctypes.byref(p), ctypes.byref(h)) == 0
        cell, mode, ln, tile, chunk = (ctypes.c_double(), ctypes.c_int32(), ctypes.c_double(), ctypes.c_int32(),
                                       ctypes.c_int32())
        assert t3._lib.t3_plan_settings(h, ctypes.byref(cell), ctypes.byref(mode), ctypes.byref(ln),
                                        ctypes.byref(tile), ctypes.byref(chunk)) == 0
        assert ln.value == lane
        assert tile.value == kw.get("tile_mode", 0) and mode.value == kw.get("scan_mode", 0)
        assert chunk.value == kw.get("chunk_centres", 0)
        t3._lib.t3_plan_destroy(h)
    assert t3._lib.t3_plan_settings(None, None, None, None, None, None) == -1


def test_edge_correct_plan_rejects_adjoint_and_bad_theta(lib):
    """Argument errors of the edge-correction and centroid entry points are
    caught before any launch (no GPU needed)."""
    pytest.importorskip("torch")
    from paper_2309_08601_amd import t3
    p, edges = _params(flags=8)
    h = ctypes.c_void_p()
    assert t3._lib.t3_plan_create(ctypes.byref(p), ctypes.byref(h)) == 0
    try:
        dummy = ctypes.c_void_p(16)
        assert t3._lib.t3_normalise_backward(h, dummy, 1, dummy, dummy, None) == -1
        assert b"edge" in t3._lib.t3_last_error_message()
        bad = (ctypes.c_double * 2)(1.0, -1.0)
        assert t3._lib.t3_x_to_centroid(h, dummy, 1, 8, bad, dummy, None) == -1
        assert t3._lib.t3_x_to_centroid(h, dummy, 1, 0, None, dummy, None) == -2
    finally:
        t3._lib.t3_plan_destroy(h)


def test_aperture_stats_argument_errors(lib):
    pytest.importorskip("torch")
    from paper_2309_08601_amd import t3
    p, edges = _params()
    h = ctypes.c_void_p()
    assert t3._lib.t3_plan_create(ctypes.byref(p), ctypes.byref(h)) == 0
    try:
        dummy = ctypes.c_void_p(16)
        good = (ctypes.c_double * 3)(1.0, 2.0, 3.0)
        bad = (ctypes.c_double * 3)(1.0, 0.0, 3.0)
        assert t3._lib.t3_aperture_stats(h, dummy, 1, 8, None, 1, dummy, None, None) == -1
        assert t3._lib.t3_aperture_stats(h, dummy, 1, 8, bad, 1, dummy, None, None) == -1
        assert t3._lib.t3_aperture_stats(h, dummy, 1, 0, good, 1, dummy, None, None) == -2
        assert t3._lib.t3_aperture_stats(h, dummy, 1, 8, good, 0, dummy, None, None) == -1
    finally:
        t3._lib.t3_plan_destroy(h)


def test_forward_sphere_argument_errors(lib):
    pytest.importorskip("torch")
    from paper_2309_08601_amd import t3
    p, edges = _params()  # edges 1', 2', 4'
    h = ctypes.c_void_p()
    assert t3._lib.t3_plan_create(ctypes.byref(p), ctypes.byref(h)) == 0
    try:
        cat = t3.t3_sphere_catalog(0, None, None, None, None, None)
        ok = (t3.t3_patch * 1)(t3.t3_patch(10.0, 12.0, 0.0, 2.0))
        bad = (t3.t3_patch * 1)(t3.t3_patch(10.0, 50.0, 0.0, 2.0))
        out = ctypes.c_void_p(16)
        npairs = ctypes.c_int64(0)
        assert t3._lib.t3_forward_sphere(h, ctypes.byref(cat), bad, 1, 10.0, out, ctypes.byref(npairs), None) == -1
        assert t3._lib.t3_forward_sphere(h, ctypes.byref(cat), ok, 1, 2.0, out, ctypes.byref(npairs), None) == -1
        assert t3._lib.t3_forward_sphere(h, ctypes.byref(cat), ok, 0, 10.0, out, ctypes.byref(npairs), None) == -1
    finally:
        t3._lib.t3_plan_destroy(h)


def test_forward_grid_argument_errors(lib):
    pytest.importorskip("torch")
    from paper_2309_08601_amd import t3
    p, edges = _params()  # 2 bins, box 2^20 steps
    h = ctypes.c_void_p()
    assert t3._lib.t3_plan_create(ctypes.byref(p), ctypes.byref(h)) == 0
    try:
        cat = t3.t3_catalog(0, None, None, None, None, None)
        out = ctypes.c_void_p(16)
        lv = lambda *v: (ctypes.c_int32 * 2)(*v)  # noqa: E731
        call = lambda delta, levels, m=0: t3._lib.t3_forward_grid(h, ctypes.byref(cat), delta, levels, m,  # noqa: E731
                                                                   out, None, None)
        assert call(1 << 14, None) == -1                 # no levels
        assert call(0, lv(0, 1)) == -1                   # delta < 1
        assert call(1 << 21, lv(0, 1)) == -1             # delta above the box
        assert call(1 << 14, lv(1, 0)) == -1             # decreasing levels
        assert call(1 << 14, lv(0, 9)) == -1             # level above 8
        assert call(1 << 14, lv(-1, 0)) == -1            # negative level
        assert call(1 << 14, lv(0, 8)) == -2             # pixel side 2^21 > box
        assert call(64, lv(0, 1)) == -2                  # 16384 pixels along the box
        assert call(1 << 14, lv(0, 1), 3) == -1          # unknown method
        assert t3._lib.t3_forward_grid(h, ctypes.byref(cat), 1 << 14, lv(0, 1), 0, None, None, None) == -1
    finally:
        t3._lib.t3_plan_destroy(h)


def test_workspace_limit_refuses_before_allocating(lib):
    """A plan whose max_workspace_bytes is below what a call needs returns
    T3_ENOMEM from the limit check itself, before any device allocation or
    launch (so this runs without a GPU), and holds no memory afterwards."""
    pytest.importorskip("torch")
    from paper_2309_08601_amd import t3
    p, edges = _params(max_workspace_bytes=64)
    h = ctypes.c_void_p()
    assert t3._lib.t3_plan_create(ctypes.byref(p), ctypes.byref(h)) == 0
    try:
        cat = t3.t3_catalog(0, None, None, None, None, None)
        out = ctypes.c_void_p(16)
        npairs = ctypes.c_int64(0)
        assert t3._lib.t3_forward(h, ctypes.byref(cat), None, -1, out, ctypes.byref(npairs), None) == t3.T3_ENOMEM
        assert b"max_workspace_bytes" in t3._lib.t3_last_error_message()
        g = ctypes.c_void_p(16)
        assert t3._lib.t3_backward(h, ctypes.byref(cat), None, -1, g, g, g, g, None) == t3.T3_ENOMEM
        assert b"max_workspace_bytes" in t3._lib.t3_last_error_message()
        used, peak = ctypes.c_int64(-1), ctypes.c_int64(-1)
        assert t3._lib.t3_workspace_bytes(h, ctypes.byref(used), ctypes.byref(peak)) == 0
        assert used.value == 0 and peak.value == 0
    finally:
        t3._lib.t3_plan_destroy(h)
    assert t3._lib.t3_workspace_bytes(None, None, None) == t3.T3_EINVAL


def test_backward_centre_argument_errors(lib):
    pytest.importorskip("torch")
    from paper_2309_08601_amd import t3
    p, edges = _params()
    h = ctypes.c_void_p()
    assert t3._lib.t3_plan_create(ctypes.byref(p), ctypes.byref(h)) == 0
    try:
        cat = t3.t3_catalog(0, None, None, None, None, None)
        g = ctypes.c_void_p(16)
        assert t3._lib.t3_backward(h, ctypes.byref(cat), g, -1, g, g, g, g, None) == t3.T3_EINVAL
        assert t3._lib.t3_backward(h, ctypes.byref(cat), None, 5, g, g, g, g, None) == t3.T3_EINVAL
        assert t3._lib.t3_backward(h, ctypes.byref(cat), g, 1 << 31, g, g, g, g, None) == t3.T3_EINVAL
    finally:
        t3._lib.t3_plan_destroy(h)
