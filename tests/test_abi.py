"""The C ABI library loads, exports what include/eles.h declares, and rejects
invalid arguments before touching the device (runs without a GPU)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "eles.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    src = re.sub(r"#[^\n]*", "", src)
    names = []
    for stmt in src.split(";"):
        stmt = " ".join(stmt.split())
        if "typedef" in stmt or "{" in stmt or "}" in stmt:
            stmt = stmt.split("}")[-1]
            if "typedef" in stmt:
                continue
        m = re.match(r"^(?:const\s+)?[A-Za-z_]\w*[\s\*]+([A-Za-z_]\w*)\s*\(", stmt.strip())
        if m:
            names.append(m.group(1))
    return names


@pytest.fixture(scope="module")
def eles():
    from paper_1902_02508_amd import eles as E
    return E


def test_header_declares_the_boundary():
    names = set(declared_functions())
    for must in ("filter_setup", "filter_fields", "sgs_stress", "filter_state_bytes",
                 "filter_workspace_bytes", "sgs_workspace_bytes", "filter_destroy",
                 "eles_status_string", "filter_state_layout", "filter_set_ygemm"):
        assert must in names


def test_library_exports_every_declared_symbol(eles):
    for name in declared_functions():
        assert hasattr(eles.lib, name), name
        assert name in eles.EXPORTS, name


def _desc(eles, **over):
    y = np.cos(np.pi * np.arange(17)[::-1] / 16) * 1.0
    y[0], y[-1] = -1.0, 1.0
    kw = dict(nx=16, ny=17, nz=12, lx=2.0, lz=1.0, y=y, delta_x=0.3, delta_y=0.2, delta_z=0.2)
    kw.update(over)
    return eles.make_desc(**kw)


def test_valid_descriptor_sizes(eles):
    d, y = _desc(eles)
    assert eles.filter_state_bytes(d) > 17 * 17 * 16


@pytest.mark.parametrize("over,status", [
    (dict(nx=0), 1), (dict(ny=2, y=np.array([-1.0, 1.0])), 1), (dict(lx=-1.0), 1),
    (dict(lz=float("nan")), 1), (dict(delta_y=0.0), 1), (dict(delta_x=float("inf")), 1),
    (dict(tail_tol=0.5), 1), (dict(ygemm=7), 1),
    (dict(y=np.linspace(-1, 1, 17)[::-1].copy()), 1),             # decreasing
    (dict(y=np.linspace(-1, 0.9, 17)), 1),                          # wall not at +1
    (dict(y=np.concatenate([[-1.0], np.full(15, 0.0), [1.0]])), 1),  # repeated nodes
    (dict(delta_y=1e-300), 4),                                     # width underflows
    (dict(delta_x=50.0), 5),                                       # stencil too wide
])
def test_invalid_descriptors_rejected(eles, over, status):
    d, y = _desc(eles, **over)
    assert eles.filter_state_bytes(d) == 0
    h = ctypes.c_void_p()
    buf = ctypes.create_string_buffer(1 << 20)
    aligned = (ctypes.addressof(buf) + 255) & ~255
    st = eles.lib.filter_setup(ctypes.byref(d), aligned, 1 << 19, None, ctypes.byref(h))
    assert st == status
    assert not h.value


def test_setup_rejects_bad_buffers_before_any_launch(eles):
    d, y = _desc(eles)
    n = eles.filter_state_bytes(d)
    h = ctypes.c_void_p()
    assert eles.lib.filter_setup(ctypes.byref(d), None, n, None, ctypes.byref(h)) == eles.ELES_EINVAL
    assert eles.lib.filter_setup(ctypes.byref(d), 0x1003, n, None, ctypes.byref(h)) == eles.ELES_EINVAL
    assert eles.lib.filter_setup(ctypes.byref(d), 0x1000, n - 1, None, ctypes.byref(h)) == eles.ELES_ENOSPACE
    assert eles.lib.filter_setup(ctypes.byref(d), 0x1000, n, None, None) == eles.ELES_EINVAL


def test_calls_on_null_handle_rejected(eles):
    assert eles.lib.sgs_stress(None, 16, 16, 16, None, 16, 1 << 20, None) == eles.ELES_EINVAL
    assert eles.lib.filter_fields(None, 16, 1, 16, 16, 16, 1 << 20, None) == eles.ELES_EINVAL
    assert eles.lib.filter_workspace_bytes(None, 3) == 0
    assert eles.lib.sgs_workspace_bytes(None) == 0
    assert eles.lib.filter_set_ygemm(None, 0) == eles.ELES_EINVAL
    for s in range(7):
        assert eles.eles_status_string(s)


def test_closure_validation_without_device(eles):
    import ctypes as C
    h = C.c_void_p()
    p = np.zeros(eles.NPARAM, dtype=np.float32)
    n = np.ones(32)
    assert eles.closure_state_bytes() > 9414 * 12
    assert eles.lib.closure_create(None, 1 << 20, p.ctypes.data, n.ctypes.data, None, None, C.byref(h)) == eles.ELES_EINVAL
    assert eles.lib.closure_create(0x1000, 16, p.ctypes.data, n.ctypes.data, None, None, C.byref(h)) == eles.ELES_ENOSPACE
    bad = p.copy()
    bad[5] = np.nan
    big = eles.closure_state_bytes()
    assert eles.lib.closure_create(0x1000, big, bad.ctypes.data, n.ctypes.data, None, None, C.byref(h)) == eles.ELES_ENUMERIC
    n0 = n.copy()
    n0[12] = 0.0            # a feature with zero spread
    assert eles.lib.closure_create(0x1000, big, p.ctypes.data, n0.ctypes.data, None, None, C.byref(h)) == eles.ELES_ENUMERIC
    assert eles.closure_train_workspace_bytes(33) == 0
    assert eles.closure_train_workspace_bytes(0) == 0
    assert eles.closure_train_workspace_bytes(65536) > 65536 * 64
    assert eles.lib.closure_sample_indices(1, 0, 0, 10, 0x1000, None) == eles.ELES_EINVAL
    fell = C.c_int32(7)
    for mode in (eles.INFER_UNCHECKED, eles.INFER_CHECK, eles.INFER_FALLBACK, 2, -2):
        assert eles.lib.closure_infer(None, None, 16, 16, None, mode, 16, C.byref(fell), 16, 1 << 20,
                                      None) == eles.ELES_EINVAL
        assert fell.value == 0
    assert eles.closure_infer_workspace_bytes(None, 1) == 0
    blob = C.create_string_buffer(eles.closure_blob_bytes())
    assert eles.lib.closure_get_params(None, blob, len(blob), None) == eles.ELES_EINVAL
    assert eles.lib.closure_set_params(None, blob, len(blob), None) == eles.ELES_EINVAL
    assert eles.lib.closure_step(None) == -1
    neg = np.array([0.1, -1e-3, 0.2])
    assert eles.lib.closure_create(0x1000, big, p.ctypes.data, n.ctypes.data, neg.ctypes.data, None,
                                   C.byref(h)) == eles.ELES_ENUMERIC
    assert eles.closure_blob_bytes() == 3 * 9414 * 4 + 32 * 8 + 8 + 3 * 8


def _ddesc(eles, nx=16, ny=17, nz=12, lx=2.0, lz=1.0, y=None, a=0.1):
    if y is None:
        y = np.cos(np.pi * np.arange(ny)[::-1] / (ny - 1))
        y[0], y[-1] = -1.0, 1.0
    y = np.ascontiguousarray(y, dtype=np.float64)
    d = eles.DFilterDesc(nx, ny, nz, lx, lz, y.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), a)
    return d, y


def test_dfilter_state_size_and_validation(eles):
    d, y = _ddesc(eles)
    n = eles.dfilter_state_bytes(d)
    # at least the factor tables: 2 (hx+1)(hz+1) ny pivots and inverses in FP32
    assert n > 2 * 2 * 9 * 7 * 17 * 4
    h = ctypes.c_void_p()
    assert eles.lib.dfilter_setup(ctypes.byref(d), None, n, None, ctypes.byref(h)) == eles.ELES_EINVAL
    assert eles.lib.dfilter_setup(ctypes.byref(d), 0x1003, n, None, ctypes.byref(h)) == eles.ELES_EINVAL
    assert eles.lib.dfilter_setup(ctypes.byref(d), 0x1000, n - 1, None, ctypes.byref(h)) == eles.ELES_ENOSPACE
    assert eles.lib.dfilter_setup(ctypes.byref(d), 0x1000, n, None, None) == eles.ELES_EINVAL
    assert not h.value


@pytest.mark.parametrize("over", [
    dict(nx=1), dict(nz=1), dict(nx=7), dict(nz=5), dict(ny=3, y=np.array([-1.0, 0.0, 1.0])), dict(lx=0.0),
    dict(lz=float("nan")), dict(a=0.0), dict(a=-0.1), dict(a=float("inf")),
    dict(y=np.linspace(-1, 0.9, 17)), dict(y=np.linspace(1, -1, 17)),
    dict(y=np.concatenate([[-1.0], np.full(15, 0.0), [1.0]])),
])
def test_dfilter_invalid_descriptors_rejected(eles, over):
    d, y = _ddesc(eles, **over)
    assert eles.dfilter_state_bytes(d) == 0
    h = ctypes.c_void_p()
    buf = ctypes.create_string_buffer(1 << 20)
    aligned = (ctypes.addressof(buf) + 255) & ~255
    assert eles.lib.dfilter_setup(ctypes.byref(d), aligned, 1 << 19, None, ctypes.byref(h)) == eles.ELES_EINVAL
    assert not h.value


def test_dfilter_calls_on_null_handle_rejected(eles):
    par = (ctypes.c_int8 * 1)(1)
    assert eles.lib.dfilter_fields(None, 16, 1, ctypes.cast(par, ctypes.c_void_p), 16, 16, 1 << 20,
                                   None) == eles.ELES_EINVAL
    assert eles.lib.dfilter_sgs_stress(None, 16, 16, 16, None, 16, 1 << 20, None) == eles.ELES_EINVAL
    assert eles.lib.dfilter_workspace_bytes(None, 3) == 0
    assert eles.lib.dfilter_sgs_workspace_bytes(None) == 0


def _ldesc(eles, ny=9, nyl=5, y=None, yl=None, **over):
    y = np.linspace(-1, 1, ny) if y is None else y
    yl = np.linspace(-1, 1, nyl) if yl is None else yl
    y = np.ascontiguousarray(y, dtype=np.float64)
    yl = np.ascontiguousarray(yl, dtype=np.float64)
    kw = dict(nx=8, nz=6, nxl=4, nzl=3)
    kw.update(over)
    dp = ctypes.POINTER(ctypes.c_double)
    d = eles.LesDesc(kw["nx"], len(y), kw["nz"], y.ctypes.data_as(dp), kw["nxl"], len(yl), kw["nzl"],
                     yl.ctypes.data_as(dp))
    return d, (y, yl)


def test_les_descriptor_validation(eles):
    d, keep = _ldesc(eles)
    assert eles.les_state_bytes(d) > 0
    for bad in (dict(nx=0), dict(nxl=0), dict(nzl=-1)):
        d, keep = _ldesc(eles, **bad)
        assert eles.les_state_bytes(d) == 0
    for y, yl in ((np.linspace(-1, 0.9, 9), None), (np.linspace(-1, 1, 2), None),
                  (None, np.linspace(-1.1, 1, 5)), (None, np.array([-1.0, 0.5, 0.2, 1.0])),
                  (None, np.linspace(-1, 1, 2))):
        d, keep = _ldesc(eles, y=y, yl=yl)
        assert eles.les_state_bytes(d) == 0
    d, keep = _ldesc(eles)
    n = eles.les_state_bytes(d)
    h = ctypes.c_void_p()
    assert eles.lib.les_setup(ctypes.byref(d), None, n, None, ctypes.byref(h)) == eles.ELES_EINVAL
    assert eles.lib.les_setup(ctypes.byref(d), 0x1000, n - 1, None, ctypes.byref(h)) == eles.ELES_ENOSPACE
    assert eles.lib.les_stress(None, 16, 16, 16, 16, None) == eles.ELES_EINVAL
    assert eles.lib.les_commutation(None, 16, 16, 16, 1 << 20, None) == eles.ELES_EINVAL
    assert eles.lib.les_commutation_workspace_bytes(None) == 0
