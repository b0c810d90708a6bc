"""ctypes binding of libsph.so (include/sph.h): argument marshalling only.

Every step of the path runs in the HIP kernels of the library; PyTorch is used
for device memory (tensors) and streams. If the library is missing the
binding raises: there is no other implementation to fall back on.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsph.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "sph.h")

F32_FIELDS = ("x", "y", "z", "vx", "vy", "vz", "rho", "vxp", "vyp", "vzp", "rhop")
SOA_FIELDS = F32_FIELDS + ("type", "id")

SPH_OK = 0
STATUS_NONFINITE, STATUS_DT, STATUS_RUN_OVERFLOW, STATUS_EXCLUDED = 1, 2, 4, 8
STATUS_NN_RANGE, STATUS_NN_LIST = 16, 32
NN_SLOTS, NN_IN, NN_OUT, NN_LAYERS = 64, 544, 4, 4
NN_RESIDUAL, NN_CARRY_PREV = 1, 2


class SphError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libsph error {code}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("dp", C.c_double), ("h", C.c_double), ("rho0", C.c_double),
                ("gamma", C.c_double), ("c0", C.c_double), ("alpha", C.c_double),
                ("eta_over_h", C.c_double), ("cfl", C.c_double), ("mass", C.c_double),
                ("g", C.c_double * 3), ("origin", C.c_double * 3), ("ncell", C.c_int32 * 3),
                ("euler_every", C.c_int32), ("slab_mode", C.c_int32), ("options", C.c_int32),
                ("slab_xlo", C.c_double), ("slab_xhi", C.c_double),
                ("capacity", C.c_uint32), ("features", C.c_uint32)]

FEATURE_CELL, FEATURE_FP64, FEATURE_SURROGATE = 1, 2, 4
OPTION_CUBIC, OPTION_RHO_FLOOR, OPTION_SYMPLECTIC = 1, 2, 4
CSTATE_FIELDS = ("cell", "ox", "oy", "oz", "vx", "vy", "vz", "rho", "vxp", "vyp", "vzp", "rhop",
                 "type", "id")
DSTATE_F64 = ("x", "y", "z", "vx", "vy", "vz", "rho", "vxp", "vyp", "vzp", "rhop")


class SoA(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in SOA_FIELDS]


RATE_FIELDS = ("ax", "ay", "az", "arho", "press", "nu", "npair")


class Rates(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in RATE_FIELDS]


class CState(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in CSTATE_FIELDS]


class DState(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in DSTATE_F64 + ("type", "id")]


class DRates(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("ax", "ay", "az", "arho")]


class Counts(C.Structure):
    _fields_ = [("n_label", C.c_uint32 * 4), ("halo_lo", C.c_uint32 * 2),
                ("edge_lo", C.c_uint32 * 2), ("edge_hi", C.c_uint32 * 2),
                ("halo_hi", C.c_uint32 * 2), ("out_lo", C.c_uint32 * 2),
                ("out_hi", C.c_uint32 * 2), ("excluded", C.c_uint32 * 2)]

    def as_dict(self) -> dict:
        return {k: list(getattr(self, k)) for k, _ in self._fields_}


class NnScales(C.Structure):
    _fields_ = [("inv_len", C.c_float), ("inv_vel", C.c_float), ("rho_ref", C.c_float),
                ("inv_rho", C.c_float), ("r2f", C.c_float), ("inv_acc", C.c_float),
                ("inv_drho", C.c_float), ("inv_dt", C.c_float)]


_P4 = C.c_void_p * 4


class MlpStruct(C.Structure):
    _fields_ = [("width", C.c_int32), ("capacity", C.c_uint32),
                ("w", _P4), ("b", _P4), ("wb", _P4), ("gw", _P4), ("gb", _P4),
                ("mw", _P4), ("vw", _P4), ("mb", _P4), ("vb", _P4), ("z", _P4),
                ("a", C.c_void_p * 3), ("da", C.c_void_p), ("dz", C.c_void_p),
                ("dy", C.c_void_p), ("work", C.c_void_p), ("loss", C.c_void_p)]


_lib = None


def lib() -> C.CDLL:
    """Load libsph.so (built by ``paper_1210_1017_amd.build``); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1210_1017_amd.build` (no fallback exists)")
        L = C.CDLL(LIB_PATH)
        vp, i32, u32, u64 = C.c_void_p, C.c_int, C.c_uint32, C.c_uint64
        P = C.POINTER
        L.sph_abi_version.restype = i32
        L.sph_error_string.argtypes = [i32]
        L.sph_error_string.restype = C.c_char_p
        L.sph_last_error.argtypes = [vp]
        L.sph_last_error.restype = C.c_char_p
        L.sph_create.argtypes = [P(Params), P(vp)]
        L.sph_destroy.argtypes = [vp]
        L.sph_destroy.restype = None
        L.sph_cell_bits.argtypes = [vp]
        L.sph_sort_kv.argtypes = [vp, vp, vp, vp, vp, u32, i32, vp]
        L.sph_sort_kv_noalloc.argtypes = [vp, vp, vp, vp, u32, i32, vp]
        L.sph_sort.argtypes = [vp, P(SoA), P(SoA), u32, vp]
        L.sph_interact.argtypes = [vp, P(SoA), u32, P(Rates), vp]
        L.sph_update.argtypes = [vp, P(SoA), P(Rates), u32, u64, vp]
        L.sph_step.argtypes = [vp, P(SoA), P(SoA), u32, u64, vp]
        L.sph_get_counts.argtypes = [vp, P(Counts), vp]
        L.sph_get_dt.argtypes = [vp, P(C.c_float), vp]
        L.sph_get_pairs.argtypes = [vp, P(C.c_uint64), vp]
        L.sph_get_sort_stats.argtypes = [vp, P(C.c_uint32), P(C.c_uint32), vp]
        L.sph_get_status.argtypes = [vp, P(C.c_uint32), vp]
        L.sph_clear_status.argtypes = [vp, vp]
        L.sph_get_pair_total.argtypes = [vp, P(C.c_uint64), vp]
        L.sph_get_candidate_total.argtypes = [vp, P(C.c_uint64), vp]
        L.sph_timing_begin.argtypes = [vp, u32]
        L.sph_timing_read.argtypes = [vp, P(C.c_float), u32, P(C.c_uint32)]
        L.sph_copy_keys.argtypes = [vp, vp, u32, vp]
        L.sph_cstate_from_positions.argtypes = [vp, vp, vp, vp, P(CState), u32, vp]
        L.sph_cstate_positions.argtypes = [vp, P(CState), vp, vp, vp, u32, vp]
        L.sph_csort.argtypes = [vp, P(CState), P(CState), u32, vp]
        L.sph_cinteract.argtypes = [vp, P(CState), u32, P(Rates), vp]
        L.sph_cstep.argtypes = [vp, P(CState), P(CState), u32, u64, vp]
        L.sph_ctotals.argtypes = [vp, P(CState), u32, P(C.c_double), vp]
        L.sph_dsort.argtypes = [vp, P(DState), P(DState), u32, vp]
        L.sph_dinteract.argtypes = [vp, P(DState), u32, P(DRates), vp]
        L.sph_dstep.argtypes = [vp, P(DState), P(DState), u32, u64, vp]
        L.sph_dtotals.argtypes = [vp, P(DState), u32, P(C.c_double), vp]
        L.sph_get_dt64.argtypes = [vp, P(C.c_double), vp]
        L.sph_copy_cell_tables.argtypes = [vp, vp, vp, vp]
        f32 = C.c_float
        L.sph_mlp_work_floats.argtypes = [C.c_int32, u32]
        L.sph_mlp_work_floats.restype = u64
        L.sph_mlp_sync.argtypes = [vp, P(MlpStruct), vp]
        L.sph_nn_features.argtypes = [vp, P(SoA), vp, u32, P(NnScales), vp, vp, vp]
        L.sph_nn_index.argtypes = [vp, vp, u32, vp, vp]
        L.sph_nn_targets.argtypes = [vp, P(SoA), P(SoA), vp, vp, u32, vp, f32, f32, f32, vp, vp]
        L.sph_mlp_forward.argtypes = [vp, P(MlpStruct), vp, u32, vp, vp]
        L.sph_mlp_backward.argtypes = [vp, P(MlpStruct), vp, u32, vp, P(f32), vp]
        L.sph_mlp_adam.argtypes = [vp, P(MlpStruct), f32, f32, f32, f32, u32, vp]
        L.sph_nn_apply.argtypes = [vp, P(SoA), vp, vp, u32, f32, f32, f32, f32, i32, vp]
        L.sph_nn_advance.argtypes = [vp, P(MlpStruct), P(SoA), P(SoA), u32, P(NnScales), f32,
                                     f32, f32, f32, i32, vp]
        L.sph_nn_perturb.argtypes = [vp, P(SoA), u32, u32, f32, f32, vp]
        L.sph_nn_judge.argtypes = [vp, P(SoA), P(SoA), P(SoA), vp, vp, u32, P(C.c_double), vp]
        L.sph_probe_fma.argtypes = [vp, u32, C.c_int32, vp]
        L.sph_probe_copy.argtypes = [vp, vp, u64, u32, vp]
        _lib = L
    return _lib


def _probe_check(rc: int):
    if rc != 0:
        L = lib()
        raise SphError(rc, f"{L.sph_error_string(rc).decode()}: {L.sph_last_error(None).decode()}")


def probe_fma(out, blocks: int, iters: int, stream=None):
    """sph_probe_fma: 16 * iters FP32 FLOP per lane over blocks x 256 lanes;
    ``out`` is a float32 device tensor of at least blocks * 256 elements."""
    if out.dtype.itemsize != 4 or out.numel() < blocks * 256 or not out.is_cuda:
        raise ValueError("out must be a float32 device tensor of blocks * 256 elements")
    _probe_check(lib().sph_probe_fma(_addr(out), blocks, iters, _stream_ptr(stream)))


SORT_NOALLOC_MAX = 1 << 21


def sort_kv_noalloc(keys, vals, keys_out, vals_out, n: int, key_bits: int, stream=None):
    """sph_sort_kv_noalloc: the stable key-value sort without a context and
    without allocation (scratch in a fixed device array; n <= SORT_NOALLOC_MAX)."""
    _probe_check(lib().sph_sort_kv_noalloc(_addr(keys), _addr(vals), _addr(keys_out),
                                           _addr(vals_out), n, key_bits, _stream_ptr(stream)))


def probe_copy(src, dst, blocks: int, stream=None):
    """sph_probe_copy of all of ``src`` (a device tensor) into ``dst``."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nbytes or not (src.is_cuda and dst.is_cuda):
        raise ValueError("dst must be a device tensor at least as large as src")
    _probe_check(lib().sph_probe_copy(_addr(src), _addr(dst), nbytes, blocks,
                                      _stream_ptr(stream)))


def header_functions() -> list[str]:
    """Names of the functions that include/sph.h declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sph_[a-z0-9_]+)\s*\(", txt)))


def make_params(p: dict, capacity: int, features: int = 0) -> Params:
    s = Params()
    for k in ("dp", "h", "rho0", "gamma", "c0", "alpha", "eta_over_h", "cfl", "mass"):
        setattr(s, k, float(p[k]))
    for a in range(3):
        s.g[a] = float(p["g"][a])
        s.origin[a] = float(p["origin"][a])
        s.ncell[a] = int(p["ncell"][a])
    s.euler_every = int(p["euler_every"])
    s.slab_mode = int(p.get("slab_mode", 0))
    s.options = int(p.get("options", 0))
    s.slab_xlo = float(p.get("slab_xlo", 0.0))
    s.slab_xhi = float(p.get("slab_xhi", 0.0))
    s.capacity = int(capacity)
    s.features = int(features)
    return s


def _stream_ptr(stream) -> C.c_void_p:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _addr(t) -> C.c_void_p:
    return C.c_void_p(t.data_ptr())


class DeviceState:
    """A particle state as torch tensors on the GPU (SoA, one tensor per field)."""

    def __init__(self, tensors: dict):
        self.t = tensors

    @classmethod
    def empty(cls, capacity: int, device="cuda") -> "DeviceState":
        import torch
        t = {k: torch.empty(capacity, dtype=torch.float32, device=device) for k in F32_FIELDS}
        t["type"] = torch.empty(capacity, dtype=torch.uint8, device=device)
        t["id"] = torch.empty(capacity, dtype=torch.int32, device=device)
        return cls(t)

    @classmethod
    def from_numpy(cls, st: dict, capacity: int | None = None, device="cuda") -> "DeviceState":
        import torch
        n = st["x"].shape[0]
        cap = n if capacity is None else capacity
        ds = cls.empty(max(cap, 1), device)
        for k in SOA_FIELDS:
            ds.t[k][:n].copy_(torch.from_numpy(np.ascontiguousarray(st[k])))
        return ds

    def to_numpy(self, n: int) -> dict:
        return {k: self.t[k][:n].cpu().numpy().copy() for k in SOA_FIELDS}

    def soa(self) -> SoA:
        return SoA(*[self.t[k].data_ptr() for k in SOA_FIELDS])


class CellState:
    """Cell + offset particle state on the GPU (int32 cell, FP32 offsets)."""

    def __init__(self, tensors: dict):
        self.t = tensors

    @classmethod
    def empty(cls, capacity: int, device="cuda") -> "CellState":
        import torch
        t = {k: torch.empty(capacity, dtype=torch.float32, device=device)
             for k in CSTATE_FIELDS if k not in ("cell", "type", "id")}
        t["cell"] = torch.empty(capacity, dtype=torch.int32, device=device)
        t["type"] = torch.empty(capacity, dtype=torch.uint8, device=device)
        t["id"] = torch.empty(capacity, dtype=torch.int32, device=device)
        return cls(t)

    def soa(self) -> CState:
        return CState(*[self.t[k].data_ptr() for k in CSTATE_FIELDS])

    def to_numpy(self, n: int) -> dict:
        return {k: self.t[k][:n].cpu().numpy().copy() for k in CSTATE_FIELDS}


class F64State:
    """FP64 particle state on the GPU (SoA)."""

    def __init__(self, tensors: dict):
        self.t = tensors

    @classmethod
    def empty(cls, capacity: int, device="cuda") -> "F64State":
        import torch
        t = {k: torch.empty(capacity, dtype=torch.float64, device=device) for k in DSTATE_F64}
        t["type"] = torch.empty(capacity, dtype=torch.uint8, device=device)
        t["id"] = torch.empty(capacity, dtype=torch.int32, device=device)
        return cls(t)

    @classmethod
    def from_numpy(cls, st: dict, capacity: int | None = None, device="cuda") -> "F64State":
        import torch
        n = st["x"].shape[0]
        ds = cls.empty(max(n if capacity is None else capacity, 1), device)
        for k in DSTATE_F64:
            ds.t[k][:n].copy_(torch.from_numpy(np.ascontiguousarray(st[k], dtype=np.float64)))
        ds.t["type"][:n].copy_(torch.from_numpy(np.ascontiguousarray(st["type"])))
        ds.t["id"][:n].copy_(torch.from_numpy(np.ascontiguousarray(st["id"])))
        return ds

    def soa(self) -> DState:
        return DState(*[self.t[k].data_ptr() for k in DSTATE_F64 + ("type", "id")])

    def to_numpy(self, n: int) -> dict:
        return {k: self.t[k][:n].cpu().numpy().copy() for k in DSTATE_F64 + ("type", "id")}


def make_rates(capacity: int, with_aux: bool = True, device="cuda") -> dict:
    import torch
    keys = ("ax", "ay", "az", "arho") + (("press", "nu") if with_aux else ())
    r = {k: torch.zeros(max(capacity, 1), dtype=torch.float32, device=device) for k in keys}
    if with_aux:
        r["npair"] = torch.zeros(max(capacity, 1), dtype=torch.int32, device=device)
    return r


def _rates_struct(r: dict) -> Rates:
    return Rates(*[(r[k].data_ptr() if k in r and r[k] is not None else None)
                   for k in RATE_FIELDS])


class Context:
    """One libsph context (scratch for ``capacity`` particles on the current GPU)."""

    def __init__(self, params: dict, capacity: int, features: int = 0):
        self.L = lib()
        self.params = dict(params)
        self.capacity = int(capacity)
        self._p = make_params(params, capacity, features)
        h = C.c_void_p()
        rc = self.L.sph_create(C.byref(self._p), C.byref(h))
        if rc != SPH_OK:
            raise SphError(rc, self.L.sph_last_error(None).decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.L.sph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int):
        if rc != SPH_OK:
            raise SphError(rc, self.L.sph_last_error(self.h).decode())

    @property
    def cell_bits(self) -> int:
        return int(self.L.sph_cell_bits(self.h))

    def sort_kv(self, keys, vals, keys_out, vals_out, n: int, key_bits: int, stream=None):
        self._check(self.L.sph_sort_kv(self.h, _addr(keys), _addr(vals), _addr(keys_out),
                                       _addr(vals_out), n, key_bits, _stream_ptr(stream)))

    def sort(self, cur: DeviceState, out: DeviceState, n: int, stream=None):
        a, b = cur.soa(), out.soa()
        self._check(self.L.sph_sort(self.h, C.byref(a), C.byref(b), n, _stream_ptr(stream)))

    def interact(self, srt: DeviceState, n: int, rates: dict, stream=None):
        a, r = srt.soa(), _rates_struct(rates)
        self._check(self.L.sph_interact(self.h, C.byref(a), n, C.byref(r), _stream_ptr(stream)))

    def update(self, srt: DeviceState, rates: dict, n: int, step: int, stream=None):
        a, r = srt.soa(), _rates_struct(rates)
        self._check(self.L.sph_update(self.h, C.byref(a), C.byref(r), n, step,
                                      _stream_ptr(stream)))

    def step(self, cur: DeviceState, nxt: DeviceState, n: int, step: int, stream=None):
        a, b = cur.soa(), nxt.soa()
        self._check(self.L.sph_step(self.h, C.byref(a), C.byref(b), n, step, _stream_ptr(stream)))

    # ---- cell + offset path
    def cstate_from_positions(self, x, y, z, out: CellState, n: int, stream=None):
        o = out.soa()
        self._check(self.L.sph_cstate_from_positions(self.h, _addr(x), _addr(y), _addr(z),
                                                     C.byref(o), n, _stream_ptr(stream)))

    def cstate_positions(self, st: CellState, n: int, stream=None):
        import torch
        out = [torch.empty(max(n, 1), dtype=torch.float64, device="cuda") for _ in range(3)]
        a = st.soa()
        self._check(self.L.sph_cstate_positions(self.h, C.byref(a), *[_addr(t) for t in out], n,
                                                _stream_ptr(stream)))
        return [t[:n] for t in out]

    def csort(self, cur: CellState, out: CellState, n: int, stream=None):
        a, b = cur.soa(), out.soa()
        self._check(self.L.sph_csort(self.h, C.byref(a), C.byref(b), n, _stream_ptr(stream)))

    def cinteract(self, srt: CellState, n: int, rates: dict, stream=None):
        a, r = srt.soa(), _rates_struct(rates)
        self._check(self.L.sph_cinteract(self.h, C.byref(a), n, C.byref(r), _stream_ptr(stream)))

    def cstep(self, cur: CellState, nxt: CellState, n: int, step: int, stream=None):
        a, b = cur.soa(), nxt.soa()
        self._check(self.L.sph_cstep(self.h, C.byref(a), C.byref(b), n, step, _stream_ptr(stream)))

    def ctotals(self, st: CellState, n: int, stream=None) -> np.ndarray:
        out = (C.c_double * 8)()
        a = st.soa()
        self._check(self.L.sph_ctotals(self.h, C.byref(a), n, out, _stream_ptr(stream)))
        return np.array(out[:])

    # ---- FP64 reference path
    def dsort(self, cur: F64State, out: F64State, n: int, stream=None):
        a, b = cur.soa(), out.soa()
        self._check(self.L.sph_dsort(self.h, C.byref(a), C.byref(b), n, _stream_ptr(stream)))

    def dinteract(self, srt: F64State, n: int, rates: dict, stream=None):
        a = srt.soa()
        r = DRates(*[rates[k].data_ptr() for k in ("ax", "ay", "az", "arho")])
        self._check(self.L.sph_dinteract(self.h, C.byref(a), n, C.byref(r), _stream_ptr(stream)))

    def dstep(self, cur: F64State, nxt: F64State, n: int, step: int, stream=None):
        a, b = cur.soa(), nxt.soa()
        self._check(self.L.sph_dstep(self.h, C.byref(a), C.byref(b), n, step, _stream_ptr(stream)))

    def dtotals(self, st: F64State, n: int, stream=None) -> np.ndarray:
        out = (C.c_double * 8)()
        a = st.soa()
        self._check(self.L.sph_dtotals(self.h, C.byref(a), n, out, _stream_ptr(stream)))
        return np.array(out[:])

    def dt64(self, stream=None) -> float:
        v = C.c_double()
        self._check(self.L.sph_get_dt64(self.h, C.byref(v), _stream_ptr(stream)))
        return float(v.value)

    def counts(self, stream=None) -> dict:
        c = Counts()
        self._check(self.L.sph_get_counts(self.h, C.byref(c), _stream_ptr(stream)))
        return c.as_dict()

    def dt(self, stream=None) -> float:
        v = C.c_float()
        self._check(self.L.sph_get_dt(self.h, C.byref(v), _stream_ptr(stream)))
        return float(v.value)

    def pairs(self, stream=None) -> int:
        v = C.c_uint64()
        self._check(self.L.sph_get_pairs(self.h, C.byref(v), _stream_ptr(stream)))
        return int(v.value)

    def sort_stats(self, stream=None) -> tuple:
        """(movers, path) of the last plain sort: path 0 when the radix sort
        of all keys ran, 1 when one block sorted the movers for the merge, 2
        when the movers' own radix passes did (truthy: merged)."""
        m, g = C.c_uint32(), C.c_uint32()
        self._check(self.L.sph_get_sort_stats(self.h, C.byref(m), C.byref(g),
                                               _stream_ptr(stream)))
        return int(m.value), int(g.value)

    def pair_total(self, stream=None) -> int:
        v = C.c_uint64()
        self._check(self.L.sph_get_pair_total(self.h, C.byref(v), _stream_ptr(stream)))
        return int(v.value)

    def candidate_total(self, stream=None) -> int:
        v = C.c_uint64()
        self._check(self.L.sph_get_candidate_total(self.h, C.byref(v), _stream_ptr(stream)))
        return int(v.value)

    def timing_begin(self, max_steps: int):
        self._check(self.L.sph_timing_begin(self.h, max_steps))

    def timing_read(self, max_steps: int) -> np.ndarray:
        """Per timed step: [sort ms, interaction-kernel ms, dt+update ms]."""
        buf = (C.c_float * (3 * max(max_steps, 1)))()
        cnt = C.c_uint32()
        self._check(self.L.sph_timing_read(self.h, buf, max_steps, C.byref(cnt)))
        return np.frombuffer(buf, dtype=np.float32, count=3 * cnt.value).reshape(-1, 3).copy()

    def status(self, stream=None) -> int:
        v = C.c_uint32()
        self._check(self.L.sph_get_status(self.h, C.byref(v), _stream_ptr(stream)))
        return int(v.value)

    def clear_status(self, stream=None):
        self._check(self.L.sph_clear_status(self.h, _stream_ptr(stream)))

    def sorted_keys(self, n: int, stream=None):
        import torch
        out = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
        self._check(self.L.sph_copy_keys(self.h, _addr(out), n, _stream_ptr(stream)))
        return out[:n]

    def cell_tables(self, stream=None):
        import torch
        nc = int(np.prod(self.params["ncell"]))
        b = torch.empty(nc, dtype=torch.int32, device="cuda")
        e = torch.empty(nc, dtype=torch.int32, device="cuda")
        self._check(self.L.sph_copy_cell_tables(self.h, _addr(b), _addr(e), _stream_ptr(stream)))
        return b, e


    # ------------------------------------------------------------ surrogate
    def mlp_sync(self, net: "Mlp", stream=None):
        self._check(self.L.sph_mlp_sync(self.h, C.byref(net.struct()), _stream_ptr(stream)))

    def nn_features(self, srt: DeviceState, rows, nrows: int, scales, X, rates=None,
                    stream=None):
        sc = NnScales(*[float(v) for v in scales[:8]])
        self._check(self.L.sph_nn_features(self.h, C.byref(srt.soa()),
                                           None if rows is None else _addr(rows), nrows,
                                           C.byref(sc), _addr(X),
                                           None if rates is None else _addr(rates),
                                           _stream_ptr(stream)))

    def nn_index(self, ids, n: int, where, stream=None):
        self._check(self.L.sph_nn_index(self.h, _addr(ids), n, _addr(where), _stream_ptr(stream)))

    def nn_targets(self, a: DeviceState, b: DeviceState, where_b, rows, nrows: int,
                   inv_dv: float, inv_dr: float, T, rates=None, span: float = 0.0, stream=None):
        self._check(self.L.sph_nn_targets(self.h, C.byref(a.soa()), C.byref(b.soa()),
                                          _addr(where_b), None if rows is None else _addr(rows),
                                          nrows, None if rates is None else _addr(rates), span,
                                          inv_dv, inv_dr, _addr(T), _stream_ptr(stream)))

    def mlp_forward(self, net: "Mlp", X, rows: int, Y, stream=None):
        self._check(self.L.sph_mlp_forward(self.h, C.byref(net.struct()), _addr(X), rows,
                                           _addr(Y), _stream_ptr(stream)))

    def mlp_backward(self, net: "Mlp", X, rows: int, T, wcol, stream=None):
        w = (C.c_float * 4)(*[float(v) for v in wcol])
        self._check(self.L.sph_mlp_backward(self.h, C.byref(net.struct()), _addr(X), rows,
                                            _addr(T), w, _stream_ptr(stream)))

    def mlp_adam(self, net: "Mlp", lr: float, beta1: float = 0.9, beta2: float = 0.999,
                 eps: float = 1e-8, t: int | None = None, stream=None):
        if t is None:
            net.t += 1
            t = net.t
        self._check(self.L.sph_mlp_adam(self.h, C.byref(net.struct()), lr, beta1, beta2, eps,
                                        int(t), _stream_ptr(stream)))

    def nn_apply(self, srt: DeviceState, Y, nrows: int, dv_scale: float, dr_scale: float,
                 dt4: float, rho_tol: float, rates=None, carry_prev: bool = False, stream=None):
        self._check(self.L.sph_nn_apply(self.h, C.byref(srt.soa()), _addr(Y),
                                        None if rates is None else _addr(rates), nrows,
                                        dv_scale, dr_scale, dt4, rho_tol,
                                        NN_CARRY_PREV if carry_prev else 0,
                                        _stream_ptr(stream)))

    def nn_advance(self, net: "Mlp", cur: DeviceState, nxt: DeviceState, n: int, scales,
                   dv_scale: float, dr_scale: float, dt4: float, rho_tol: float,
                   residual: bool = False, carry_prev: bool = False, stream=None):
        sc = NnScales(*[float(v) for v in scales[:8]])
        self._check(self.L.sph_nn_advance(self.h, C.byref(net.struct()), C.byref(cur.soa()),
                                          C.byref(nxt.soa()), n, C.byref(sc), dv_scale, dr_scale,
                                          dt4, rho_tol,
                                          (NN_RESIDUAL if residual else 0)
                                          | (NN_CARRY_PREV if carry_prev else 0),
                                          _stream_ptr(stream)))

    def nn_perturb(self, st: DeviceState, n: int, seed: int, sigma_u: float, sigma_rho: float,
                   stream=None):
        self._check(self.L.sph_nn_perturb(self.h, C.byref(st.soa()), n, int(seed) & 0xffffffff,
                                          sigma_u, sigma_rho, _stream_ptr(stream)))

    def nn_judge(self, s: DeviceState, r: DeviceState, b: DeviceState, where_r, where_b, n: int,
                 stream=None) -> np.ndarray:
        out = (C.c_double * 8)()
        self._check(self.L.sph_nn_judge(self.h, C.byref(s.soa()), C.byref(r.soa()),
                                        C.byref(b.soa()), _addr(where_r), _addr(where_b), n, out,
                                        _stream_ptr(stream)))
        return np.array(list(out))


def layer_dims(width: int) -> list[tuple[int, int]]:
    """(in, out) of the four layers of the surrogate network."""
    return [(NN_IN, width), (width, width), (width, width), (width, NN_OUT)]


class Mlp:
    """The surrogate network and its training workspace as device tensors
    (the buffers of ``sph_mlp``). ``train=False`` allocates the weights only
    (enough for ``nn_advance``)."""

    def __init__(self, width: int = 128, capacity: int = 32768, train: bool = True,
                 device="cuda"):
        import torch
        f32, bf = torch.float32, torch.bfloat16
        self.width, self.capacity, self.train_mode = int(width), int(capacity), train
        dims = layer_dims(self.width)
        z = lambda *s, dt=f32: torch.zeros(*s, dtype=dt, device=device)
        self.w = [z(o, i) for i, o in dims]
        self.b = [z(o) for _, o in dims]
        self.wb = [z(o, i, dt=bf) for i, o in dims]
        self.t = 0
        if train:
            cap = self.capacity
            self.gw = [z(o, i) for i, o in dims]
            self.gb = [z(o) for _, o in dims]
            self.mw = [z(o, i) for i, o in dims]
            self.vw = [z(o, i) for i, o in dims]
            self.mb = [z(o) for _, o in dims]
            self.vb = [z(o) for _, o in dims]
            self.z = [z(cap, o) for _, o in dims]
            self.a = [z(cap, self.width, dt=bf) for _ in range(3)]
            self.da = z(cap, self.width)
            self.dz = z(cap, self.width, dt=bf)
            self.dy = z(cap, NN_OUT)
            self.work = z(int(lib().sph_mlp_work_floats(self.width, cap)))
            self.loss = z(1)

    def struct(self) -> MlpStruct:
        s = MlpStruct()
        s.width, s.capacity = self.width, (self.capacity if self.train_mode else 0)
        for l in range(NN_LAYERS):
            s.w[l], s.b[l], s.wb[l] = (self.w[l].data_ptr(), self.b[l].data_ptr(),
                                       self.wb[l].data_ptr())
            if self.train_mode:
                for name in ("gw", "gb", "mw", "vw", "mb", "vb", "z"):
                    getattr(s, name)[l] = getattr(self, name)[l].data_ptr()
        if self.train_mode:
            for l in range(3):
                s.a[l] = self.a[l].data_ptr()
            s.da, s.dz, s.dy = self.da.data_ptr(), self.dz.data_ptr(), self.dy.data_ptr()
            s.work, s.loss = self.work.data_ptr(), self.loss.data_ptr()
        return s

    def init(self, seed: int):
        """Seeded initial weights: N(0, 1/in) for the hidden layers (variance
        preserving for unit-scale inputs), N(0, 0.01^2/in) for the output
        layer (start near the zero prediction), zero biases."""
        rng = np.random.Generator(np.random.PCG64(seed))
        arrays = {}
        for l, (i, o) in enumerate(layer_dims(self.width)):
            sd = (1.0 if l < NN_LAYERS - 1 else 0.01) / np.sqrt(i)
            arrays[f"w{l}"] = (rng.standard_normal((o, i)) * sd).astype(np.float32)
            arrays[f"b{l}"] = np.zeros(o, dtype=np.float32)
        self.load(arrays)

    def load(self, arrays: dict):
        """Set the FP32 masters (w0..w3, b0..b3) and zero the Adam state;
        the caller then runs Context.mlp_sync for the bfloat16 copies."""
        import torch
        for l in range(NN_LAYERS):
            self.w[l].copy_(torch.from_numpy(np.ascontiguousarray(arrays[f"w{l}"], np.float32)))
            self.b[l].copy_(torch.from_numpy(np.ascontiguousarray(arrays[f"b{l}"], np.float32)))
            if self.train_mode:
                for name in ("mw", "vw", "mb", "vb"):
                    getattr(self, name)[l].zero_()
        self.t = 0

    def arrays(self) -> dict:
        out = {}
        for l in range(NN_LAYERS):
            out[f"w{l}"] = self.w[l].cpu().numpy().copy()
            out[f"b{l}"] = self.b[l].cpu().numpy().copy()
        return out


def u32(t) -> np.ndarray:
    """View a device int32 tensor (holding uint32 bits) as a host uint32 array."""
    return t.cpu().numpy().view(np.uint32)
