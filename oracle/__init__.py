"""Python entry points of the FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package. It shares no code with the HIP path: the C library
``liboracle.so`` is built from ``sph_oracle.c`` alone, and this module only
marshals numpy arrays into it. The one composite routine, ``step``, strings
the oracle's own pieces together in the order of the method (keys, stable
sort, reorder, cell tables, interaction, dt, Verlet).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sph_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

F32_FIELDS = ("x", "y", "z", "vx", "vy", "vz", "rho", "vxp", "vyp", "vzp", "rhop")
FLUID, BOUNDARY, GHOST = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile liboracle.so (gcc, -O2, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("dp", C.c_double), ("h", C.c_double), ("rho0", C.c_double),
                ("gamma", C.c_double), ("c0", C.c_double), ("alpha", C.c_double),
                ("eta_over_h", C.c_double), ("cfl", C.c_double), ("mass", C.c_double),
                ("g", C.c_double * 3), ("origin", C.c_double * 3), ("ncell", C.c_int32 * 3),
                ("euler_every", C.c_int32), ("slab_mode", C.c_int32), ("options", C.c_int32),
                ("slab_xlo", C.c_double), ("slab_xhi", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        P = C.POINTER
        d, u8, u32, i32, i64 = (P(C.c_double), P(C.c_uint8), P(C.c_uint32), P(C.c_int32),
                                P(C.c_int64))
        pp = P(_Params)
        L.orc_cell_bits.argtypes = [pp]
        L.orc_keys.argtypes = [pp, C.c_int64, d, d, d, u8, u32]
        L.orc_stable_sort.argtypes = [C.c_int64, u32, u32, i32]
        L.orc_stable_sort_kv.argtypes = [C.c_int64, u32, i32, u32, i32]
        L.orc_cell_tables.argtypes = [pp, C.c_int64, u32, u32, u32, u32]
        L.orc_ranges.argtypes = [pp, u32, u32, u32, u32]
        L.orc_kernel_w.argtypes = [C.c_double, C.c_double]
        L.orc_kernel_w.restype = C.c_double
        L.orc_kernel_f.argtypes = [C.c_double, C.c_double]
        L.orc_kernel_f.restype = C.c_double
        L.orc_symplectic_half.argtypes = [pp, C.c_int64, C.c_double, u8] + [d] * 18
        L.orc_symplectic_full.argtypes = [pp, C.c_int64, C.c_double, u8] + [d] * 16
        for f in ("orc_cubic_w", "orc_cubic_f"):
            getattr(L, f).argtypes = [C.c_double, C.c_double]
            getattr(L, f).restype = C.c_double
        L.orc_eos.argtypes = [pp, C.c_double, d, d]
        L.orc_interact.argtypes = [pp, C.c_int64, d, d, d, d, d, d, d, u8, u32, u32, u32,
                                   C.c_int64, C.c_int64, i64, d, d, d, d, d, d, d, i64]
        L.orc_interact_brute.argtypes = [pp, C.c_int64, d, d, d, d, d, d, d, u8, d,
                                         d, d, d, d, d, i64]
        L.orc_neighbours_brute.argtypes = [pp, C.c_int64, d, d, d, i64, i32, C.c_int64]
        L.orc_neighbours_brute.restype = C.c_int64
        L.orc_neighbours_cells.argtypes = [pp, C.c_int64, d, d, d, u32, u32, u32, i64, i32,
                                           C.c_int64]
        L.orc_neighbours_cells.restype = C.c_int64
        L.orc_dt.argtypes = [pp, C.c_int64, u8, d, d, d, d, d]
        L.orc_dt.restype = C.c_double
        L.orc_verlet.argtypes = [pp, C.c_int64, C.c_int64, C.c_double, u8] + [d] * 15
        L.orc_threads.restype = C.c_int
        L.orc_internal_energy.argtypes = [pp, C.c_double]
        L.orc_internal_energy.restype = C.c_double
        L.orc_totals.argtypes = [pp, C.c_int64, d, d, d, d, d, d, d, u8, d]
        L.orc_nn_rows.argtypes = [pp, d, d, d, u32, u32, u32, C.c_int64, i64, C.c_float,
                                  C.c_int32, i32, i32]
        L.orc_nn_sums.argtypes = [pp, d, d, d, d, d, d, d, C.c_int64, i64, i32, C.c_int32, d]
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ct):
    assert a.flags["C_CONTIGUOUS"], "arrays passed to the oracle must be contiguous"
    return a.ctypes.data_as(C.POINTER(ct))


def _d(a):
    return _ptr(a, C.c_double)


def make_params(p: dict) -> _Params:
    s = _Params()
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
    return s


def threads() -> int:
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's loops from now on (timing only)."""
    L = lib()
    L.orc_set_threads.argtypes = [C.c_int]
    L.orc_set_threads(int(n))


def to_f64(state: dict) -> dict:
    """Exact upcast of an FP32 state to the oracle's FP64 state."""
    out = {k: np.ascontiguousarray(state[k], dtype=np.float64) for k in F32_FIELDS}
    out["type"] = np.ascontiguousarray(state["type"], dtype=np.uint8)
    out["id"] = np.ascontiguousarray(state["id"], dtype=np.int32)
    return out


def to_f32(state: dict) -> dict:
    out = {k: np.ascontiguousarray(state[k], dtype=np.float32) for k in F32_FIELDS}
    out["type"] = state["type"].copy()
    out["id"] = state["id"].copy()
    return out


def cell_bits(p: dict) -> int:
    return int(lib().orc_cell_bits(C.byref(make_params(p))))


def ncells(p: dict) -> int:
    return int(p["ncell"][0]) * int(p["ncell"][1]) * int(p["ncell"][2])


def keys(p: dict, st: dict) -> np.ndarray:
    s = to_f64(st) if st["x"].dtype != np.float64 else st
    n = s["x"].shape[0]
    k = np.empty(n, dtype=np.uint32)
    lib().orc_keys(C.byref(make_params(p)), n, _d(s["x"]), _d(s["y"]), _d(s["z"]),
                   _ptr(s["type"], C.c_uint8), _ptr(k, C.c_uint32))
    return k


def stable_sort(k: np.ndarray):
    k = np.ascontiguousarray(k, dtype=np.uint32)
    n = k.shape[0]
    ko = np.empty(n, dtype=np.uint32)
    perm = np.empty(n, dtype=np.int32)
    lib().orc_stable_sort(n, _ptr(k, C.c_uint32), _ptr(ko, C.c_uint32), _ptr(perm, C.c_int32))
    return ko, perm


def stable_sort_kv(k: np.ndarray, v: np.ndarray):
    k = np.ascontiguousarray(k, dtype=np.uint32)
    v = np.ascontiguousarray(v, dtype=np.int32)
    n = k.shape[0]
    ko = np.empty(n, dtype=np.uint32)
    vo = np.empty(n, dtype=np.int32)
    lib().orc_stable_sort_kv(n, _ptr(k, C.c_uint32), _ptr(v, C.c_int32), _ptr(ko, C.c_uint32),
                             _ptr(vo, C.c_int32))
    return ko, vo


def cell_tables(p: dict, skey: np.ndarray):
    nc = ncells(p)
    b = np.empty(nc, dtype=np.uint32)
    e = np.empty(nc, dtype=np.uint32)
    cnt = np.zeros(4, dtype=np.uint32)
    skey = np.ascontiguousarray(skey, dtype=np.uint32)
    lib().orc_cell_tables(C.byref(make_params(p)), skey.shape[0], _ptr(skey, C.c_uint32),
                          _ptr(b, C.c_uint32), _ptr(e, C.c_uint32), _ptr(cnt, C.c_uint32))
    return b, e, cnt


def ranges(p: dict, begin, end, counts) -> np.ndarray:
    out = np.zeros(14, dtype=np.uint32)
    lib().orc_ranges(C.byref(make_params(p)), _ptr(begin, C.c_uint32), _ptr(end, C.c_uint32),
                     _ptr(np.ascontiguousarray(counts, dtype=np.uint32), C.c_uint32),
                     _ptr(out, C.c_uint32))
    return out


def gather(st: dict, perm: np.ndarray) -> dict:
    return {k: np.ascontiguousarray(v[perm]) for k, v in st.items()}


def sort_state(p: dict, st: dict):
    """Keys (a1), stable sort (a2), reorder (a3), cell tables and counts (a4),
    packing ranges (a5). Returns a dict with the sorted FP64 state and tables."""
    s = to_f64(st) if st["x"].dtype != np.float64 else st
    k = keys(p, s)
    sk, perm = stable_sort(k)
    ss = gather(s, perm)
    b, e, cnt = cell_tables(p, sk)
    return dict(state=ss, keys=sk, perm=perm, begin=b, end=e, counts=cnt,
                ranges=ranges(p, b, e, cnt), unsorted_keys=k)


def kernel_w(r: float, h: float) -> float:
    return float(lib().orc_kernel_w(r, h))


def kernel_f(r: float, h: float) -> float:
    return float(lib().orc_kernel_f(r, h))


def cubic_w(r: float, h: float) -> float:
    """Cubic spline kernel W(r) of Sec. 2.2 (3-D, support 2h)."""
    return float(lib().orc_cubic_w(r, h))


def cubic_f(r: float, h: float) -> float:
    """F(r) of the cubic spline: grad_i W_ij = F(r) (r_i - r_j)."""
    return float(lib().orc_cubic_f(r, h))


def eos(p: dict, rho: float):
    pr, c = C.c_double(), C.c_double()
    lib().orc_eos(C.byref(make_params(p)), float(rho), C.byref(pr), C.byref(c))
    return pr.value, c.value


def internal_energy(p: dict, rho: float) -> float:
    return float(lib().orc_internal_energy(C.byref(make_params(p)), float(rho)))


def totals(p: dict, st: dict) -> np.ndarray:
    """[mass, px, py, pz, E_kin, E_pot, E_int, count] over non-ghost particles."""
    s = to_f64(st) if st["x"].dtype != np.float64 else st
    out = np.zeros(8)
    lib().orc_totals(C.byref(make_params(p)), s["x"].shape[0], _d(s["x"]), _d(s["y"]), _d(s["z"]),
                     _d(s["vx"]), _d(s["vy"]), _d(s["vz"]), _d(s["rho"]),
                     _ptr(s["type"], C.c_uint8), _d(out))
    return out


def interact(p: dict, srt: dict, sel: np.ndarray | None = None) -> dict:
    """Interaction sums over the sorted state of ``sort_state`` (optionally only
    for the sorted indices in ``sel``)."""
    s = srt["state"]
    n = s["x"].shape[0]
    n0 = int(srt["counts"][0])
    if sel is None:
        m, selp = n0, None
    else:
        sel = np.ascontiguousarray(sel, dtype=np.int64)
        m, selp = sel.shape[0], _ptr(sel, C.c_int64)
    out = {k: np.zeros(m) for k in ("ax", "ay", "az", "drho", "nu", "p", "c")}
    out["npair"] = np.zeros(m, dtype=np.int64)
    lib().orc_interact(C.byref(make_params(p)), n, _d(s["x"]), _d(s["y"]), _d(s["z"]),
                       _d(s["vx"]), _d(s["vy"]), _d(s["vz"]), _d(s["rho"]),
                       _ptr(s["type"], C.c_uint8), _ptr(srt["keys"], C.c_uint32),
                       _ptr(srt["begin"], C.c_uint32), _ptr(srt["end"], C.c_uint32), n0, m,
                       selp, _d(out["ax"]), _d(out["ay"]), _d(out["az"]), _d(out["drho"]),
                       _d(out["nu"]), _d(out["p"]), _d(out["c"]), _ptr(out["npair"], C.c_int64))
    return out


def interact_brute(p: dict, st: dict, box=None) -> dict:
    s = to_f64(st) if st["x"].dtype != np.float64 else st
    n = s["x"].shape[0]
    out = {k: np.zeros(n) for k in ("ax", "ay", "az", "drho", "nu")}
    out["npair"] = np.zeros(n, dtype=np.int64)
    boxa = None if box is None else np.ascontiguousarray(box, dtype=np.float64)
    lib().orc_interact_brute(C.byref(make_params(p)), n, _d(s["x"]), _d(s["y"]), _d(s["z"]),
                             _d(s["vx"]), _d(s["vy"]), _d(s["vz"]), _d(s["rho"]),
                             _ptr(s["type"], C.c_uint8), None if boxa is None else _d(boxa),
                             _d(out["ax"]), _d(out["ay"]), _d(out["az"]), _d(out["drho"]),
                             _d(out["nu"]), _ptr(out["npair"], C.c_int64))
    return out


def neighbours_brute(p: dict, st: dict, cap: int = 1 << 24):
    s = to_f64(st) if st["x"].dtype != np.float64 else st
    n = s["x"].shape[0]
    row = np.zeros(n + 1, dtype=np.int64)
    cols = np.zeros(cap, dtype=np.int32)
    m = lib().orc_neighbours_brute(C.byref(make_params(p)), n, _d(s["x"]), _d(s["y"]),
                                   _d(s["z"]), _ptr(row, C.c_int64), _ptr(cols, C.c_int32), cap)
    assert m <= cap
    return row, cols[:m].copy()


def neighbours_cells(p: dict, srt: dict, cap: int = 1 << 24):
    s = srt["state"]
    n0 = int(srt["counts"][0])
    row = np.zeros(n0 + 1, dtype=np.int64)
    cols = np.zeros(cap, dtype=np.int32)
    m = lib().orc_neighbours_cells(C.byref(make_params(p)), n0, _d(s["x"]), _d(s["y"]),
                                   _d(s["z"]), _ptr(srt["keys"], C.c_uint32),
                                   _ptr(srt["begin"], C.c_uint32), _ptr(srt["end"], C.c_uint32),
                                   _ptr(row, C.c_int64), _ptr(cols, C.c_int32), cap)
    assert m <= cap
    return row, cols[:m].copy()


def nn_rows(p: dict, srt: dict, sel, r2f: float, k: int = 64):
    """Neighbours of the sorted particles ``sel`` with FP32 squared distance
    below the FP32 number ``r2f``, in increasing sorted index: (nbr
    [len(sel), k] int32 with -1 padding, number found per particle)."""
    s = srt["state"]
    sel = np.ascontiguousarray(sel, dtype=np.int64)
    m = sel.shape[0]
    nbr = np.full((m, k), -1, dtype=np.int32)
    cnt = np.zeros(m, dtype=np.int32)
    lib().orc_nn_rows(C.byref(make_params(p)), _d(s["x"]), _d(s["y"]), _d(s["z"]),
                      _ptr(srt["keys"], C.c_uint32), _ptr(srt["begin"], C.c_uint32),
                      _ptr(srt["end"], C.c_uint32), m, _ptr(sel, C.c_int64), float(r2f), k,
                      _ptr(nbr, C.c_int32), _ptr(cnt, C.c_int32))
    return nbr, cnt


def nn_sums(p: dict, srt: dict, sel, nbr) -> np.ndarray:
    """FP64 pressure acceleration and continuity rate of the sorted particles
    ``sel`` over their listed neighbours ``nbr`` (-1 = none): [len(sel), 4]."""
    s = srt["state"]
    sel = np.ascontiguousarray(sel, dtype=np.int64)
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    out = np.zeros((sel.shape[0], 4))
    lib().orc_nn_sums(C.byref(make_params(p)), _d(s["x"]), _d(s["y"]), _d(s["z"]), _d(s["vx"]),
                      _d(s["vy"]), _d(s["vz"]), _d(s["rho"]), sel.shape[0], _ptr(sel, C.c_int64),
                      _ptr(nbr, C.c_int32), nbr.shape[1], _d(out))
    return out


def dt(p: dict, srt: dict, acc: dict) -> float:
    s = srt["state"]
    n0 = int(srt["counts"][0])
    return float(lib().orc_dt(C.byref(make_params(p)), n0, _ptr(s["type"], C.c_uint8),
                              _d(acc["ax"]), _d(acc["ay"]), _d(acc["az"]), _d(s["rho"]),
                              _d(acc["nu"])))


def verlet(p: dict, st: dict, n0: int, step: int, dtv: float, acc: dict) -> dict:
    """Verlet update (in place on a copy of ``st``, an FP64 sorted state)."""
    s = {k: v.copy() for k, v in st.items()}
    a = {k: np.ascontiguousarray(acc[k], dtype=np.float64) for k in ("ax", "ay", "az", "drho")}
    lib().orc_verlet(C.byref(make_params(p)), int(n0), int(step), float(dtv),
                     _ptr(s["type"], C.c_uint8), *[_d(s[k]) for k in F32_FIELDS],
                     _d(a["ax"]), _d(a["ay"]), _d(a["az"]), _d(a["drho"]))
    return s


OPTION_SYMPLECTIC = 4


def symplectic_half(p: dict, st: dict, n0: int, dtv: float, acc: dict) -> dict:
    """Half step of the symplectic variant: a copy of the FP64 sorted state
    with (r, v, rho) at n + 1/2 (see orc_symplectic_half)."""
    s = {k: v.copy() for k, v in st.items()}
    a = {k: np.ascontiguousarray(acc[k], dtype=np.float64) for k in ("ax", "ay", "az", "drho")}
    lib().orc_symplectic_half(C.byref(make_params(p)), int(n0), float(dtv),
                              _ptr(st["type"], C.c_uint8),
                              *[_d(st[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "rho")],
                              _d(a["ax"]), _d(a["ay"]), _d(a["az"]), _d(a["drho"]),
                              *[_d(s[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "rho")])
    return s


def symplectic_full(p: dict, st: dict, half: dict, n0: int, dtv: float, acc_h: dict) -> dict:
    """Full step of the symplectic variant from the state at n and the rates
    of the half state (in place on a copy of ``st``)."""
    s = {k: v.copy() for k, v in st.items()}
    a = {k: np.ascontiguousarray(acc_h[k], dtype=np.float64) for k in ("ax", "ay", "az", "drho")}
    lib().orc_symplectic_full(C.byref(make_params(p)), int(n0), float(dtv),
                              _ptr(s["type"], C.c_uint8), *[_d(s[k]) for k in F32_FIELDS],
                              _d(np.ascontiguousarray(half["rho"], dtype=np.float64)),
                              _d(a["ax"]), _d(a["ay"]), _d(a["az"]), _d(a["drho"]))
    return s


def step(p: dict, st: dict, step_index: int, dt_override: float | None = None) -> dict:
    """One full time step: sort (a1-a5), interaction (b1-b3), dt (c1), Verlet (c2);
    with the symplectic option, a half step, the interaction of the half state
    (same cell tables) and the full step in place of the Verlet update.

    Returns dict(state=new sorted FP64 state, srt=sort products, acc=rates,
    dt=dt used, dt_cfl=CFL dt, pairs=total neighbour pairs) and, for the
    symplectic option, half (the half state) and acc_half (its rates)."""
    srt = sort_state(p, st)
    acc = interact(p, srt)
    dtc = dt(p, srt, acc)
    dtv = dtc if dt_override is None else float(dt_override)
    n0 = int(srt["counts"][0])
    if int(p.get("options", 0)) & OPTION_SYMPLECTIC:
        half = symplectic_half(p, srt["state"], n0, dtv, acc)
        acc_h = interact(p, dict(srt, state=half))
        new = symplectic_full(p, srt["state"], half, n0, dtv, acc_h)
        return dict(state=new, srt=srt, acc=acc, dt=dtv, dt_cfl=dtc, half=half, acc_half=acc_h,
                    pairs=int(acc_h["npair"].sum()))
    new = verlet(p, srt["state"], n0, step_index, dtv, acc)
    return dict(state=new, srt=srt, acc=acc, dt=dtv, dt_cfl=dtc, pairs=int(acc["npair"].sum()))
