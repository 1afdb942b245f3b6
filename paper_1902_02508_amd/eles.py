"""ctypes binding of the C ABI in include/eles.h (argument marshalling only).

The functions keep the C names. ``Filter`` is a small convenience wrapper
that allocates the caller-owned state and workspace as torch tensors on the
current device and passes torch's current stream; every step of the
computation runs in the HIP library. If ``libeles.so`` is missing the import
of this module fails: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch  # load torch's HIP runtime first so the library binds to the same one

_HERE = os.path.dirname(os.path.abspath(__file__))
# ELES_LIB selects another build of the same library (the host-sanitized one
# of the CPU sanitizer test)
LIB_PATH = os.environ.get("ELES_LIB") or os.path.join(_HERE, "libeles.so")

ELES_OK, ELES_EINVAL, ELES_ENOSPACE, ELES_EHIP, ELES_ENUMERIC, ELES_ENOTSUP = range(6)
YGEMM = {"fp32": 0, "bf16": 1, "bf16x3": 2}


class FilterDesc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("lx", ctypes.c_double), ("lz", ctypes.c_double),
        ("y", ctypes.POINTER(ctypes.c_double)),
        ("delta_x", ctypes.c_double), ("delta_y", ctypes.c_double), ("delta_z", ctypes.c_double),
        ("tail_tol", ctypes.c_double),
        ("ygemm", ctypes.c_int32),
    ]


class DFilterDesc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("lx", ctypes.c_double), ("lz", ctypes.c_double),
        ("y", ctypes.POINTER(ctypes.c_double)),
        ("a", ctypes.c_double),
    ]


class LesDesc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("y", ctypes.POINTER(ctypes.c_double)),
        ("nx_les", ctypes.c_int32), ("ny_les", ctypes.c_int32), ("nz_les", ctypes.c_int32),
        ("y_les", ctypes.POINTER(ctypes.c_double)),
    ]


class StateLayout(ctypes.Structure):
    _fields_ = [
        ("mx", ctypes.c_int32), ("mz", ctypes.c_int32),
        ("ny_pad_m", ctypes.c_int32), ("ny_pad_k", ctypes.c_int32),
        ("off_wp64", ctypes.c_size_t), ("off_wm64", ctypes.c_size_t),
        ("off_wx64", ctypes.c_size_t), ("off_wz64", ctypes.c_size_t),
        ("off_y64", ctypes.c_size_t), ("off_shift", ctypes.c_size_t),
        ("state_bytes", ctypes.c_size_t),
        ("y_groups", ctypes.c_int32), ("y_blocks", ctypes.c_int32),
        ("xz_waves", ctypes.c_int32), ("xz_wide", ctypes.c_int32),
    ]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run python -m paper_1902_02508_amd.build")
lib = ctypes.CDLL(LIB_PATH)

_P = ctypes.c_void_p
_S = ctypes.c_size_t
_I = ctypes.c_int32
_SIG = {
    "eles_status_string": (ctypes.c_char_p, [_I]),
    "filter_state_bytes": (_S, [ctypes.POINTER(FilterDesc)]),
    "filter_setup": (_I, [ctypes.POINTER(FilterDesc), _P, _S, _P, ctypes.POINTER(_P)]),
    "filter_set_ygemm": (_I, [_P, _I]),
    "filter_set_xz": (_I, [_P, _I]),
    "filter_state_layout": (_I, [_P, ctypes.POINTER(StateLayout)]),
    "filter_workspace_bytes": (_S, [_P, _I]),
    "sgs_workspace_bytes": (_S, [_P]),
    "filter_fields": (_I, [_P, _P, _I, _P, _P, _P, _S, _P]),
    "sgs_stress": (_I, [_P, _P, _P, _P, _P, _P, _S, _P]),
    "filter_profile_begin": (_I, [_P, _I, ctypes.c_uint32]),
    "filter_profile_end": (_I, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I)]),
    "filter_destroy": (None, [_P]),
    "dfilter_state_bytes": (_S, [ctypes.POINTER(DFilterDesc)]),
    "dfilter_setup": (_I, [ctypes.POINTER(DFilterDesc), _P, _S, _P, ctypes.POINTER(_P)]),
    "dfilter_workspace_bytes": (_S, [_P, _I]),
    "dfilter_sgs_workspace_bytes": (_S, [_P]),
    "dfilter_fields": (_I, [_P, _P, _I, _P, _P, _P, _S, _P]),
    "dfilter_sgs_stress": (_I, [_P, _P, _P, _P, _P, _P, _S, _P]),
    "dfilter_destroy": (None, [_P]),
    "dfilter_inverse": (_I, [_P, _P, _I, _P, _P, _P, _S, _P]),
    "dfilter_errors_workspace_bytes": (_S, [_P]),
    "dfilter_errors": (_I, [_P, _P, _P, ctypes.c_double, ctypes.c_double, _P, _P, _S, _P]),
    "les_state_bytes": (_S, [ctypes.POINTER(LesDesc)]),
    "les_setup": (_I, [ctypes.POINTER(LesDesc), _P, _S, _P, ctypes.POINTER(_P)]),
    "les_stress": (_I, [_P, _P, _P, _P, _P, _P]),
    "les_commutation_workspace_bytes": (_S, [_P]),
    "les_commutation": (_I, [_P, _P, _P, _P, _S, _P]),
    "les_destroy": (None, [_P]),
    "dfilter_profile_begin": (_I, [_P, _I, ctypes.c_uint32]),
    "dfilter_profile_end": (_I, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I)]),
    "closure_state_bytes": (_S, []),
    "closure_create": (_I, [_P, _S, _P, _P, _P, _P, ctypes.POINTER(_P)]),
    "closure_step": (ctypes.c_int64, [_P]),
    "closure_blob_bytes": (_S, []),
    "closure_get_params": (_I, [_P, _P, _S, _P]),
    "closure_set_params": (_I, [_P, _P, _S, _P]),
    "closure_features": (_I, [_P, _P, _P, _P]),
    "closure_moments_workspace_bytes": (_S, [_I]),
    "closure_moments": (_I, [_P, _I, _I, ctypes.c_int64, _P, _P, _S, _P]),
    "closure_moments_noalloc": (_I, [_P, _I, _I, ctypes.c_int64, _P, _P]),
    "closure_train_workspace_bytes": (_S, [_I]),
    "closure_train": (_I, [_P, _P, _P, _I, ctypes.c_int64, _P, _P, _P, _S, _P]),
    "closure_infer_workspace_bytes": (_S, [_P, _I]),
    "closure_infer": (_I, [_P, _P, _P, _P, _P, _I, _P, ctypes.POINTER(_I), _P, _S, _P]),
    "closure_sample_indices": (_I, [ctypes.c_uint64, ctypes.c_int64, _I, ctypes.c_uint64, _P, _P]),
    "closure_destroy": (None, [_P]),
}
for _name, (_res, _args) in _SIG.items():
    _fn = getattr(lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTS = tuple(_SIG)


NPARAM = 9414


class TrainDesc(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("steps", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float)]


class ElesError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {lib.eles_status_string(status).decode()} ({status})")


def _check(status: int, where: str):
    if status != ELES_OK:
        raise ElesError(status, where)


# ---- the C functions under their own names -----------------------------

def eles_status_string(status: int) -> str:
    return lib.eles_status_string(status).decode()


def filter_state_bytes(desc: FilterDesc) -> int:
    return lib.filter_state_bytes(ctypes.byref(desc))


def filter_setup(desc, state_ptr, state_bytes, stream) -> _P:
    h = _P()
    _check(lib.filter_setup(ctypes.byref(desc), state_ptr, state_bytes, stream, ctypes.byref(h)), "filter_setup")
    return h


def filter_set_ygemm(h, ygemm: int):
    _check(lib.filter_set_ygemm(h, ygemm), "filter_set_ygemm")


def filter_set_xz(h, matrix_cores: int):
    _check(lib.filter_set_xz(h, matrix_cores), "filter_set_xz")


def filter_state_layout(h) -> StateLayout:
    out = StateLayout()
    _check(lib.filter_state_layout(h, ctypes.byref(out)), "filter_state_layout")
    return out


def filter_workspace_bytes(h, nfields: int) -> int:
    return lib.filter_workspace_bytes(h, nfields)


def sgs_workspace_bytes(h) -> int:
    return lib.sgs_workspace_bytes(h)


def filter_fields(h, in_ptr, nfields, parity_ptr, out_ptr, ws_ptr, ws_bytes, stream):
    _check(lib.filter_fields(h, in_ptr, nfields, parity_ptr, out_ptr, ws_ptr, ws_bytes, stream), "filter_fields")


def sgs_stress(h, u_ptr, ubar_ptr, tau_ptr, stats_ptr, ws_ptr, ws_bytes, stream):
    _check(lib.sgs_stress(h, u_ptr, ubar_ptr, tau_ptr, stats_ptr, ws_ptr, ws_bytes, stream), "sgs_stress")


NPASS = 4
PASS_NAMES = ("shift", "xz", "y", "stats")


def _pass_mask(passes, npass):
    return (1 << npass) - 1 if passes is None else sum(1 << int(p) for p in set(passes))


def filter_profile_begin(h, max_calls: int, passes=None):
    """Time the passes listed (indices into PASS_NAMES; all when None) of
    the next max_calls calls."""
    _check(lib.filter_profile_begin(h, max_calls, _pass_mask(passes, NPASS)), "filter_profile_begin")


def filter_profile_end(h):
    """{pass name: (total ms, launches)} of the calls timed since begin."""
    ms = (ctypes.c_double * NPASS)()
    n = (_I * NPASS)()
    _check(lib.filter_profile_end(h, ms, n), "filter_profile_end")
    return {PASS_NAMES[p]: (ms[p], n[p]) for p in range(NPASS)}


def filter_destroy(h):
    lib.filter_destroy(h)


# ---- convenience wrapper -------------------------------------------------

def make_desc(nx, ny, nz, lx, lz, y, delta_x, delta_y, delta_z, tail_tol=0.0, ygemm="fp32"):
    """FilterDesc plus the host y array it points to (keep both alive)."""
    yarr = np.ascontiguousarray(np.asarray(y, dtype=np.float64))
    d = FilterDesc(int(nx), int(ny), int(nz), float(lx), float(lz),
                   yarr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                   float(delta_x), float(delta_y), float(delta_z), float(tail_tol),
                   YGEMM[ygemm] if isinstance(ygemm, str) else int(ygemm))
    return d, yarr


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


class Filter:
    """A filter handle with its state allocated on the current CUDA (HIP) device."""

    def __init__(self, nx, ny, nz, lx, lz, y, delta_x, delta_y, delta_z,
                 tail_tol=0.0, ygemm="fp32", device="cuda"):
        self.shape = (int(nx), int(ny), int(nz))
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        desc, self._y = make_desc(nx, ny, nz, lx, lz, y, delta_x, delta_y, delta_z, tail_tol, ygemm)
        nbytes = filter_state_bytes(desc)
        if nbytes == 0:
            raise ElesError(ELES_EINVAL, "filter_state_bytes")
        self.state = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.h = filter_setup(desc, _ptr(self.state), nbytes, _stream())
        self.layout = filter_state_layout(self.h)
        self._ws = torch.empty(0, dtype=torch.uint8, device=self.device)

    @classmethod
    def from_config(cls, cfg, tail_tol=0.0, ygemm="fp32", y=None, device="cuda"):
        from .synth import ygrid
        if y is None:
            y = ygrid(cfg.ny, cfg.ykind, cfg.stretch)
        return cls(cfg.nx, cfg.ny, cfg.nz, cfg.lx, cfg.lz, y,
                   cfg.delta_x, cfg.delta_y, cfg.delta_z, tail_tol, ygemm, device)

    # bound at class creation: module globals may already be gone when an
    # object is collected at interpreter exit
    def __del__(self, _destroy=lib.filter_destroy):
        h = getattr(self, "h", None)
        if h:
            _destroy(h)
            self.h = None

    def set_ygemm(self, ygemm):
        filter_set_ygemm(self.h, YGEMM[ygemm] if isinstance(ygemm, str) else int(ygemm))

    def set_xz(self, matrix_cores: bool):
        filter_set_xz(self.h, 1 if matrix_cores else 0)

    def _workspace(self, nbytes):
        if self._ws.numel() < nbytes:
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self._ws

    def _field_check(self, t, n):
        if t.dtype != torch.float32 or not t.is_contiguous() or t.device != self.device:
            raise ValueError("fields must be contiguous float32 tensors on the filter's device")
        if tuple(t.shape) != (n,) + self.shape:
            raise ValueError(f"expected shape {(n,) + self.shape}, got {tuple(t.shape)}")

    def filter_fields(self, fields: torch.Tensor, parity: Sequence[int], out: Optional[torch.Tensor] = None):
        nf = fields.shape[0]
        self._field_check(fields, nf)
        if out is None:
            out = torch.empty_like(fields)
        self._field_check(out, nf)
        par = (ctypes.c_int8 * nf)(*[int(p) for p in parity])
        nb = filter_workspace_bytes(self.h, nf)
        ws = self._workspace(nb)
        filter_fields(self.h, _ptr(fields), nf, ctypes.cast(par, ctypes.c_void_p), _ptr(out),
                      _ptr(ws), ws.numel(), _stream())
        return out

    def inverse(self, fields: torch.Tensor, parity: Sequence[int], out: Optional[torch.Tensor] = None):
        """u = (1 - a^2 lap) ubar, field by field."""
        nf = fields.shape[0]
        self._field_check(fields, nf)
        if out is None:
            out = torch.empty_like(fields)
        self._field_check(out, nf)
        if len(parity) != nf or any(int(p) not in (1, -1) for p in parity):
            raise ValueError("one parity (+1 even, -1 odd) per field")
        par = (ctypes.c_int8 * nf)(*[int(p) for p in parity])
        ws = self._workspace(dfilter_workspace_bytes(self.h, nf))
        dfilter_inverse(self.h, _ptr(fields), nf, ctypes.cast(par, ctypes.c_void_p), _ptr(out),
                        _ptr(ws), ws.numel(), _stream())
        return out

    def errors(self, les: torch.Tensor, dns: torch.Tensor, utau_les: float, utau_dns: float):
        """Device FP64 [5]: eq. (13) volume error of u1, eq. (14) <u1> profile
        error, eq. (15) rms profile errors of u1, u2, u3."""
        self._field_check(les, 3)
        self._field_check(dns, 3)
        out = torch.empty(5, dtype=torch.float64, device=self.device)
        ws = self._workspace(dfilter_errors_workspace_bytes(self.h))
        dfilter_errors(self.h, _ptr(les), _ptr(dns), utau_les, utau_dns, _ptr(out), _ptr(ws), ws.numel(),
                       _stream())
        return out

    def sgs_stress(self, u: torch.Tensor, ubar=None, tau=None, stats=True):
        self._field_check(u, 3)
        if ubar is None:
            ubar = torch.empty((3,) + self.shape, dtype=torch.float32, device=self.device)
        if tau is None:
            tau = torch.empty((6,) + self.shape, dtype=torch.float32, device=self.device)
        self._field_check(ubar, 3)
        self._field_check(tau, 6)
        st = None
        if stats is True:
            st = torch.empty((9, self.shape[1]), dtype=torch.float64, device=self.device)
        elif isinstance(stats, torch.Tensor):
            st = stats
        nb = sgs_workspace_bytes(self.h)
        ws = self._workspace(nb)
        sgs_stress(self.h, _ptr(u), _ptr(ubar), _ptr(tau), _ptr(st) if st is not None else None,
                   _ptr(ws), ws.numel(), _stream())
        return ubar, tau, st

    def operators(self):
        """FP64 operators copied back from the device state (for inspection)."""
        L = self.layout
        nx, ny, nz = self.shape
        raw = self.state.cpu().numpy()

        def f64(off, n):
            return raw[off:off + 8 * n].view(np.float64).copy()
        return {
            "wp": f64(L.off_wp64, ny * ny).reshape(ny, ny),
            "wm": f64(L.off_wm64, ny * ny).reshape(ny, ny),
            "wx": f64(L.off_wx64, 2 * L.mx + 1),
            "wz": f64(L.off_wz64, 2 * L.mz + 1),
            "y": f64(L.off_y64, ny),
            "shift": f64(L.off_shift, 3 * ny).reshape(3, ny),
            "mx": L.mx, "mz": L.mz,
        }


# ---- the learned closure ----------------------------------------------------

def closure_state_bytes() -> int:
    return lib.closure_state_bytes()


def closure_create(state_ptr, state_bytes, params_host, norms_host, coef_host, stream):
    h = _P()
    _check(lib.closure_create(state_ptr, state_bytes, params_host, norms_host, coef_host, stream, ctypes.byref(h)),
           "closure_create")
    return h


def closure_step(h) -> int:
    return lib.closure_step(h)


def closure_blob_bytes() -> int:
    return lib.closure_blob_bytes()


def closure_get_params(h, stream) -> bytes:
    n = lib.closure_blob_bytes()
    buf = ctypes.create_string_buffer(n)
    _check(lib.closure_get_params(h, buf, n, stream), "closure_get_params")
    return buf.raw


def closure_set_params(h, blob: bytes, stream):
    buf = ctypes.create_string_buffer(blob, len(blob))
    _check(lib.closure_set_params(h, buf, len(blob), stream), "closure_set_params")


def closure_features(fh, ubar_ptr, feat_ptr, stream):
    _check(lib.closure_features(fh, ubar_ptr, feat_ptr, stream), "closure_features")


def closure_moments_workspace_bytes(nchan: int) -> int:
    return lib.closure_moments_workspace_bytes(nchan)


def closure_moments(data_ptr, nchan, nsnap, npts, out_ptr, ws_ptr, ws_bytes, stream):
    _check(lib.closure_moments(data_ptr, nchan, nsnap, npts, out_ptr, ws_ptr, ws_bytes, stream), "closure_moments")


MOMENTS_NOALLOC_MAX_CHAN = 64


def closure_moments_noalloc(data_ptr, nchan, nsnap, npts, out_ptr, stream):
    _check(lib.closure_moments_noalloc(data_ptr, nchan, nsnap, npts, out_ptr, stream), "closure_moments_noalloc")


def closure_train_workspace_bytes(batch: int) -> int:
    return lib.closure_train_workspace_bytes(batch)


def closure_train(h, feat_ptr, tau_ptr, nsnap, npts, desc, loss_ptr, ws_ptr, ws_bytes, stream):
    _check(lib.closure_train(h, feat_ptr, tau_ptr, nsnap, npts, ctypes.byref(desc), loss_ptr, ws_ptr, ws_bytes,
                             stream), "closure_train")


INFER_UNCHECKED, INFER_CHECK, INFER_FALLBACK = -1, 0, 1


def closure_infer_workspace_bytes(fh, with_fallback: int = 0) -> int:
    return lib.closure_infer_workspace_bytes(fh, with_fallback)


def closure_infer(h, fh, ubar_ptr, tau_ptr, stats_ptr, fallback, u_ptr, ws_ptr, ws_bytes, stream) -> int:
    """Returns 1 when the exact stress replaced a non-finite prediction."""
    fell = _I(0)
    _check(lib.closure_infer(h, fh, ubar_ptr, tau_ptr, stats_ptr, fallback, u_ptr, ctypes.byref(fell), ws_ptr,
                             ws_bytes, stream), "closure_infer")
    return fell.value


def closure_sample_indices(seed, step, batch, count, out_ptr, stream):
    _check(lib.closure_sample_indices(seed, step, batch, count, out_ptr, stream), "closure_sample_indices")


def closure_destroy(h):
    lib.closure_destroy(h)


def features(f: "Filter", ubar: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """closure_features for a Filter's grid: [10][nx][ny][nz] FP32."""
    f._field_check(ubar, 3)
    if out is None:
        out = torch.empty((10,) + f.shape, dtype=torch.float32, device=f.device)
    f._field_check(out, 10)
    closure_features(f.h, _ptr(ubar), _ptr(out), _stream())
    return out


def moments(data: torch.Tensor) -> torch.Tensor:
    """FP64 [2][C] mean and standard deviation per channel of [S][C][...] data."""
    if data.dtype != torch.float32 or not data.is_contiguous():
        raise ValueError("data must be contiguous float32")
    S, C = data.shape[0], data.shape[1]
    npts = data[0, 0].numel()
    out = torch.empty((2, C), dtype=torch.float64, device=data.device)
    ws = torch.empty(closure_moments_workspace_bytes(C), dtype=torch.uint8, device=data.device)
    closure_moments(_ptr(data), C, S, npts, _ptr(out), _ptr(ws), ws.numel(), _stream())
    return out


def moments_noalloc(data: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """moments() through the entry point that takes no workspace; out, if
    given, is the caller's [2][C] FP64 result buffer."""
    if data.dtype != torch.float32 or not data.is_contiguous():
        raise ValueError("data must be contiguous float32")
    S, C = data.shape[0], data.shape[1]
    npts = data[0, 0].numel()
    if out is None:
        out = torch.empty((2, C), dtype=torch.float64, device=data.device)
    closure_moments_noalloc(_ptr(data), C, S, npts, _ptr(out), _stream())
    return out


class Closure:
    """A closure handle; state, workspace and norms live on the current device."""

    def __init__(self, params: np.ndarray, norms: np.ndarray, device="cuda", gm_coef=None):
        """gm_coef: the gradient-model coefficients c_k = Delta_k^2 / 12 (three
        values), or None for the plain network."""
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        p = np.ascontiguousarray(params, dtype=np.float32)
        n = np.ascontiguousarray(norms, dtype=np.float64)
        if p.size != NPARAM or n.size != 32:
            raise ValueError("params must hold 9414 values and norms 32")
        c = None
        if gm_coef is not None:
            c = np.ascontiguousarray(gm_coef, dtype=np.float64)
            if c.size != 3:
                raise ValueError("gm_coef must hold 3 values")
        self._coef = c
        self.state = torch.empty(closure_state_bytes(), dtype=torch.uint8, device=dev)
        self.h = closure_create(_ptr(self.state), self.state.numel(), p.ctypes.data_as(_P),
                                n.ctypes.data_as(_P), c.ctypes.data_as(_P) if c is not None else None, _stream())
        self._ws = torch.empty(0, dtype=torch.uint8, device=dev)
        self.fell_back = 0

    # bound at class creation: module globals may already be gone when an
    # object is collected at interpreter exit
    def __del__(self, _destroy=lib.closure_destroy):
        h = getattr(self, "h", None)
        if h:
            _destroy(h)
            self.h = None

    def _workspace(self, nbytes):
        if self._ws.numel() < nbytes:
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self._ws

    @property
    def step(self) -> int:
        return closure_step(self.h)

    def get_params(self) -> bytes:
        return closure_get_params(self.h, _stream())

    def set_params(self, blob: bytes):
        closure_set_params(self.h, blob, _stream())

    def theta(self) -> np.ndarray:
        return np.frombuffer(self.get_params(), dtype=np.float32, count=NPARAM).copy()

    def train(self, feat: torch.Tensor, tau: torch.Tensor, steps: int, batch: int = 65536, seed: int = 1,
              lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
              loss_hist: Optional[torch.Tensor] = None):
        """feat [S][10][...], tau [S][6][...] on the device."""
        S = feat.shape[0]
        npts = feat[0, 0].numel()
        if tuple(tau.shape[:2]) != (S, 6) or feat.shape[1] != 10 or tau[0, 0].numel() != npts:
            raise ValueError("feat must be [S][10][...] and tau [S][6][...] over the same points")
        d = TrainDesc(batch, steps, seed, lr, beta1, beta2, eps)
        nb = closure_train_workspace_bytes(batch)
        if nb == 0:
            raise ValueError("batch must be a positive multiple of 32")
        ws = self._workspace(nb)
        if loss_hist is None and steps > 0:
            loss_hist = torch.empty(steps, dtype=torch.float32, device=self.device)
        closure_train(self.h, _ptr(feat), _ptr(tau), S, npts, d, _ptr(loss_hist) if steps > 0 else None,
                      _ptr(ws), ws.numel(), _stream())
        return loss_hist

    def infer(self, f: "Filter", ubar: torch.Tensor, tau: Optional[torch.Tensor] = None, stats=True,
              fallback: int = INFER_UNCHECKED, u: Optional[torch.Tensor] = None):
        """tau_pred [6][...] and its plane means [6][ny] (or None). With
        fallback=INFER_FALLBACK and the unfiltered velocity u, a non-finite
        prediction is replaced by the exact stress; self.fell_back reports
        it. INFER_CHECK raises ElesError (ENUMERIC) instead."""
        f._field_check(ubar, 3)
        if u is not None:
            f._field_check(u, 3)
        if tau is None:
            tau = torch.empty((6,) + f.shape, dtype=torch.float32, device=f.device)
        st = torch.empty((6, f.shape[1]), dtype=torch.float64, device=f.device) if stats is True else stats
        nb = closure_infer_workspace_bytes(f.h, int(fallback == INFER_FALLBACK))
        ws = self._workspace(nb)
        self.fell_back = closure_infer(self.h, f.h, _ptr(ubar), _ptr(tau), _ptr(st) if st is not None else None,
                                       fallback, _ptr(u) if u is not None else None, _ptr(ws), ws.numel(),
                                       _stream())
        return tau, st


def sample_indices(seed: int, step: int, batch: int, count: int, device="cuda") -> torch.Tensor:
    out = torch.empty(batch, dtype=torch.int64, device=device)
    closure_sample_indices(seed, step, batch, count, _ptr(out), _stream())
    return out


# ---- the paper's differential filter -------------------------------------

def dfilter_state_bytes(desc: DFilterDesc) -> int:
    return lib.dfilter_state_bytes(ctypes.byref(desc))


def dfilter_setup(desc, state_ptr, state_bytes, stream) -> _P:
    h = _P()
    _check(lib.dfilter_setup(ctypes.byref(desc), state_ptr, state_bytes, stream, ctypes.byref(h)), "dfilter_setup")
    return h


def dfilter_workspace_bytes(h, nfields: int) -> int:
    return lib.dfilter_workspace_bytes(h, nfields)


def dfilter_sgs_workspace_bytes(h) -> int:
    return lib.dfilter_sgs_workspace_bytes(h)


def dfilter_fields(h, in_ptr, nfields, parity_ptr, out_ptr, ws_ptr, ws_bytes, stream):
    _check(lib.dfilter_fields(h, in_ptr, nfields, parity_ptr, out_ptr, ws_ptr, ws_bytes, stream), "dfilter_fields")


def dfilter_sgs_stress(h, u_ptr, ubar_ptr, tau_ptr, stats_ptr, ws_ptr, ws_bytes, stream):
    _check(lib.dfilter_sgs_stress(h, u_ptr, ubar_ptr, tau_ptr, stats_ptr, ws_ptr, ws_bytes, stream),
           "dfilter_sgs_stress")


def dfilter_destroy(h):
    lib.dfilter_destroy(h)


def dfilter_inverse(h, in_ptr, nfields, parity_ptr, out_ptr, ws_ptr, ws_bytes, stream):
    _check(lib.dfilter_inverse(h, in_ptr, nfields, parity_ptr, out_ptr, ws_ptr, ws_bytes, stream), "dfilter_inverse")


def dfilter_errors_workspace_bytes(h) -> int:
    return lib.dfilter_errors_workspace_bytes(h)


def dfilter_errors(h, les_ptr, dns_ptr, utau_les, utau_dns, out_ptr, ws_ptr, ws_bytes, stream):
    _check(lib.dfilter_errors(h, les_ptr, dns_ptr, float(utau_les), float(utau_dns), out_ptr, ws_ptr, ws_bytes,
                              stream), "dfilter_errors")


DNPASS = 7
DPASS_NAMES = ("shift", "x_fwd", "z_fwd", "y_solve", "z_inv", "x_inv", "epilogue")


def dfilter_profile_begin(h, max_calls: int, passes=None):
    """Time the passes listed (indices into DPASS_NAMES; all when None) of
    the next max_calls calls."""
    _check(lib.dfilter_profile_begin(h, max_calls, _pass_mask(passes, DNPASS)), "dfilter_profile_begin")


def dfilter_profile_end(h):
    """{pass name: (summed ms, timed launches)}."""
    ms = (ctypes.c_double * DNPASS)()
    n = (_I * DNPASS)()
    _check(lib.dfilter_profile_end(h, ms, n), "dfilter_profile_end")
    return {DPASS_NAMES[p]: (ms[p], n[p]) for p in range(DNPASS)}


class DFilter:
    """A differential-filter handle with its state on the current device."""

    def __init__(self, nx, ny, nz, lx, lz, y, a=0.1, device="cuda"):
        self.shape = (int(nx), int(ny), int(nz))
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self._y = np.ascontiguousarray(np.asarray(y, dtype=np.float64))
        desc = DFilterDesc(int(nx), int(ny), int(nz), float(lx), float(lz),
                           self._y.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(a))
        nbytes = dfilter_state_bytes(desc)
        if nbytes == 0:
            raise ElesError(ELES_EINVAL, "dfilter_state_bytes")
        self.state = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.h = dfilter_setup(desc, _ptr(self.state), nbytes, _stream())
        self._ws = torch.empty(0, dtype=torch.uint8, device=self.device)

    @classmethod
    def from_config(cls, cfg, a=0.1, y=None, device="cuda"):
        from .synth import ygrid
        if y is None:
            y = ygrid(cfg.ny, cfg.ykind, cfg.stretch)
        return cls(cfg.nx, cfg.ny, cfg.nz, cfg.lx, cfg.lz, y, a, device)

    # bound at class creation: module globals may already be gone when an
    # object is collected at interpreter exit
    def __del__(self, _destroy=lib.dfilter_destroy):
        h = getattr(self, "h", None)
        if h:
            _destroy(h)
            self.h = None

    def _workspace(self, nbytes):
        if self._ws.numel() < nbytes:
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self._ws

    def _field_check(self, t, n):
        if t.dtype != torch.float32 or not t.is_contiguous() or t.device != self.device:
            raise ValueError("fields must be contiguous float32 tensors on the filter's device")
        if tuple(t.shape) != (n,) + self.shape:
            raise ValueError(f"expected shape {(n,) + self.shape}, got {tuple(t.shape)}")

    def filter_fields(self, fields: torch.Tensor, parity: Sequence[int], out: Optional[torch.Tensor] = None):
        nf = fields.shape[0]
        self._field_check(fields, nf)
        if out is None:
            out = torch.empty_like(fields)
        self._field_check(out, nf)
        if len(parity) != nf or any(int(p) not in (1, -1) for p in parity):
            raise ValueError("one parity (+1 even, -1 odd) per field")
        par = (ctypes.c_int8 * nf)(*[int(p) for p in parity])
        ws = self._workspace(dfilter_workspace_bytes(self.h, nf))
        dfilter_fields(self.h, _ptr(fields), nf, ctypes.cast(par, ctypes.c_void_p), _ptr(out),
                       _ptr(ws), ws.numel(), _stream())
        return out

    def inverse(self, fields: torch.Tensor, parity: Sequence[int], out: Optional[torch.Tensor] = None):
        """u = (1 - a^2 lap) ubar, field by field."""
        nf = fields.shape[0]
        self._field_check(fields, nf)
        if out is None:
            out = torch.empty_like(fields)
        self._field_check(out, nf)
        if len(parity) != nf or any(int(p) not in (1, -1) for p in parity):
            raise ValueError("one parity (+1 even, -1 odd) per field")
        par = (ctypes.c_int8 * nf)(*[int(p) for p in parity])
        ws = self._workspace(dfilter_workspace_bytes(self.h, nf))
        dfilter_inverse(self.h, _ptr(fields), nf, ctypes.cast(par, ctypes.c_void_p), _ptr(out),
                        _ptr(ws), ws.numel(), _stream())
        return out

    def errors(self, les: torch.Tensor, dns: torch.Tensor, utau_les: float, utau_dns: float):
        """Device FP64 [5]: eq. (13) volume error of u1, eq. (14) <u1> profile
        error, eq. (15) rms profile errors of u1, u2, u3."""
        self._field_check(les, 3)
        self._field_check(dns, 3)
        out = torch.empty(5, dtype=torch.float64, device=self.device)
        ws = self._workspace(dfilter_errors_workspace_bytes(self.h))
        dfilter_errors(self.h, _ptr(les), _ptr(dns), utau_les, utau_dns, _ptr(out), _ptr(ws), ws.numel(),
                       _stream())
        return out

    def sgs_stress(self, u: torch.Tensor, ubar=None, tau=None, stats=True):
        self._field_check(u, 3)
        if ubar is None:
            ubar = torch.empty((3,) + self.shape, dtype=torch.float32, device=self.device)
        if tau is None:
            tau = torch.empty((6,) + self.shape, dtype=torch.float32, device=self.device)
        self._field_check(ubar, 3)
        self._field_check(tau, 6)
        st = None
        if stats is True:
            st = torch.empty((9, self.shape[1]), dtype=torch.float64, device=self.device)
        elif isinstance(stats, torch.Tensor):
            if (stats.dtype != torch.float64 or not stats.is_contiguous() or stats.device != self.device
                    or tuple(stats.shape) != (9, self.shape[1])):
                raise ValueError("stats must be a contiguous float64 [9, ny] tensor on the filter's device")
            st = stats
        ws = self._workspace(dfilter_sgs_workspace_bytes(self.h))
        dfilter_sgs_stress(self.h, _ptr(u), _ptr(ubar), _ptr(tau), _ptr(st) if st is not None else None,
                           _ptr(ws), ws.numel(), _stream())
        return ubar, tau, st


# ---- the stress on an LES grid -----------------------------------------------

def les_state_bytes(desc: LesDesc) -> int:
    return lib.les_state_bytes(ctypes.byref(desc))


def les_setup(desc, state_ptr, state_bytes, stream) -> _P:
    h = _P()
    _check(lib.les_setup(ctypes.byref(desc), state_ptr, state_bytes, stream, ctypes.byref(h)), "les_setup")
    return h


def les_stress(h, ubar_ptr, tau_ptr, ubar_les_ptr, T_ptr, stream):
    _check(lib.les_stress(h, ubar_ptr, tau_ptr, ubar_les_ptr, T_ptr, stream), "les_stress")


def les_commutation_workspace_bytes(h) -> int:
    return lib.les_commutation_workspace_bytes(h)


def les_commutation(h, g_ptr, out_ptr, ws_ptr, ws_bytes, stream):
    _check(lib.les_commutation(h, g_ptr, out_ptr, ws_ptr, ws_bytes, stream), "les_commutation")


def les_destroy(h):
    lib.les_destroy(h)


class LesGrid:
    """The discretization operator from a DNS grid to an LES grid, with its
    state on the current device."""

    def __init__(self, nx, ny, nz, y, nx_les, ny_les, nz_les, y_les, device="cuda"):
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.shape = (int(nx), int(ny), int(nz))
        self.les_shape = (int(nx_les), int(ny_les), int(nz_les))
        self._y = np.ascontiguousarray(np.asarray(y, dtype=np.float64))
        self._yl = np.ascontiguousarray(np.asarray(y_les, dtype=np.float64))
        dp = ctypes.POINTER(ctypes.c_double)
        desc = LesDesc(int(nx), int(ny), int(nz), self._y.ctypes.data_as(dp),
                       int(nx_les), int(ny_les), int(nz_les), self._yl.ctypes.data_as(dp))
        nbytes = les_state_bytes(desc)
        if nbytes == 0:
            raise ElesError(ELES_EINVAL, "les_state_bytes")
        self.state = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.h = les_setup(desc, _ptr(self.state), nbytes, _stream())
        self._ws = torch.empty(0, dtype=torch.uint8, device=dev)

    @classmethod
    def coarsened(cls, cfg, ratio, device="cuda"):
        """The LES grid coarser by `ratio` in every direction (LES2, LES4), its
        y nodes from the same stretching."""
        from .synth import ygrid
        y = ygrid(cfg.ny, cfg.ykind, cfg.stretch)
        yl = ygrid((cfg.ny - 1) // ratio + 1, cfg.ykind, cfg.stretch)
        return cls(cfg.nx, cfg.ny, cfg.nz, y, cfg.nx // ratio, len(yl), cfg.nz // ratio, yl, device)

    # bound at class creation: module globals may already be gone when an
    # object is collected at interpreter exit
    def __del__(self, _destroy=lib.les_destroy):
        h = getattr(self, "h", None)
        if h:
            _destroy(h)
            self.h = None

    def _check(self, t, n, shape):
        if t.dtype != torch.float32 or not t.is_contiguous() or t.device != self.device:
            raise ValueError("fields must be contiguous float32 tensors on the grid's device")
        if tuple(t.shape) != (n,) + shape:
            raise ValueError(f"expected shape {(n,) + shape}, got {tuple(t.shape)}")

    def stress(self, ubar: torch.Tensor, tau: torch.Tensor, ubar_les=None, T=None):
        self._check(ubar, 3, self.shape)
        self._check(tau, 6, self.shape)
        if ubar_les is None:
            ubar_les = torch.empty((3,) + self.les_shape, dtype=torch.float32, device=self.device)
        if T is None:
            T = torch.empty((6,) + self.les_shape, dtype=torch.float32, device=self.device)
        self._check(ubar_les, 3, self.les_shape)
        self._check(T, 6, self.les_shape)
        les_stress(self.h, _ptr(ubar), _ptr(tau), _ptr(ubar_les), _ptr(T), _stream())
        return ubar_les, T

    def commutation(self, g: torch.Tensor) -> torch.Tensor:
        """Device FP64 [1]: the commutation error of the DNS field g."""
        if g.dim() == 4 and g.shape[0] == 1:
            g = g[0]
        if g.dtype != torch.float32 or not g.is_contiguous() or tuple(g.shape) != self.shape:
            raise ValueError(f"g must be a contiguous float32 {self.shape} tensor")
        out = torch.empty(1, dtype=torch.float64, device=self.device)
        nb = les_commutation_workspace_bytes(self.h)
        if self._ws.numel() < nb:
            self._ws = torch.empty(nb, dtype=torch.uint8, device=self.device)
        les_commutation(self.h, _ptr(g), _ptr(out), _ptr(self._ws), self._ws.numel(), _stream())
        return out

