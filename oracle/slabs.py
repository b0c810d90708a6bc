"""Spatial decomposition of the oracle step into x-slabs (test infrastructure).

Only the tests may import this module. It strings the FP64 oracle's own
pieces together into the per-sub-domain loop of Sec. 4.2, run for every slab
in one process with the exchanges emulated by array copies:

  halo     each slab receives, as ghost particles, copies of the particles of
           its neighbours that lie in the neighbours' edge strips of width 2h
           next to the shared faces (Sec. 4.2: edges and halos of width 2h);
  step     each slab sorts its own particles and ghosts with the slab's cell
           grid (one extra cell layer of 2h outside each face), runs the
           interaction for its in-domain particles and forms its CFL limit;
  dt       the global time step is the minimum over the slabs (the paper's
           reduction of the per-process time steps);
  update   each slab advances its own particles with the global dt;
  migrate  each slab labels its updated particles (Sec. 4.3: 1 moved out
           through the low face, 2 through the high face) and hands the
           labelled ones to the neighbour on that side.

The slabs must be whole numbers of cells of side 2h wide. The union of the
slabs' particles after a step is the undecomposed step's state (up to the
order of floating-point sums), which is what the tests pin.
"""
from __future__ import annotations

import numpy as np

from . import FLUID, GHOST, cell_bits, keys, sort_state, interact, dt as _dt, verlet, to_f64

FIELDS = ("x", "y", "z", "vx", "vy", "vz", "rho", "vxp", "vyp", "vzp", "rhop", "type", "id")


def slab_params(p: dict, xlo: float, xhi: float) -> dict:
    """Parameters of the slab [xlo, xhi) of the whole-domain parameters p: the
    same y/z grid, an x grid from xlo - 2h with (xhi - xlo)/2h + 2 layers."""
    cs = 2.0 * p["h"]
    w = (xhi - xlo) / cs
    if abs(w - round(w)) > 1e-9 or round(w) < 1:
        raise ValueError("slab width must be a whole number of cells of side 2h")
    q = dict(p)
    q["origin"] = (xlo - cs, p["origin"][1], p["origin"][2])
    q["ncell"] = (int(round(w)) + 2, p["ncell"][1], p["ncell"][2])
    q["slab_mode"], q["slab_xlo"], q["slab_xhi"] = 1, float(xlo), float(xhi)
    return q


def _take(st: dict, sel) -> dict:
    return {k: np.ascontiguousarray(st[k][sel]) for k in FIELDS}


def _cat(parts) -> dict:
    return {k: np.ascontiguousarray(np.concatenate([s[k] for s in parts])) for k in FIELDS}


def split(st: dict, faces) -> list[dict]:
    """Own particles of each slab [faces[k], faces[k+1]) (FP64 state), decided
    in FP32 like the migration label of the slab's keys."""
    s = to_f64(st) if st["x"].dtype != np.float64 else st
    x32 = s["x"].astype(np.float32)
    out = []
    for k in range(len(faces) - 1):
        sel = ((x32 >= np.float32(faces[k])) & (x32 < np.float32(faces[k + 1]))
               & (s["type"] != GHOST))
        out.append(_take(s, sel))
    return out


def halo(own: list[dict], faces, h: float) -> list[tuple[dict, int]]:
    """Ghost copies for each slab, as (ghost state, number of copies of fluid
    particles): the particles of slab k-1 with x >= faces[k] - 2h and of slab
    k+1 with x < faces[k+1] + 2h (the neighbours' edge strips), typed ghost."""
    cs = 2.0 * h
    out = []
    for k in range(len(own)):
        parts = []
        if k > 0:
            s = own[k - 1]
            parts.append(_take(s, s["x"] >= faces[k] - cs))
        if k + 1 < len(own):
            s = own[k + 1]
            parts.append(_take(s, s["x"] < faces[k + 1] + cs))
        g = _cat(parts) if parts else _take(own[k], np.zeros(len(own[k]["x"]), bool))
        nf = int((g["type"] == FLUID).sum())
        g["type"] = np.full(len(g["x"]), GHOST, dtype=np.uint8)
        out.append((g, nf))
    return out


def decomposed_step(p: dict, own: list[dict], faces, step_index: int) -> dict:
    """One step of every slab with emulated exchanges. Returns dict(own=the
    slabs' particles after migration, dt=global dt, ghosts=ghost count per
    slab, migrants=[(to_lo, to_hi)] per slab)."""
    halos = halo(own, faces, p["h"])
    ghosts = [g for g, _ in halos]
    prm = [slab_params(p, faces[k], faces[k + 1]) for k in range(len(own))]
    srts, accs, dts = [], [], []
    for k in range(len(own)):
        st = _cat([own[k], ghosts[k]])
        srt = sort_state(prm[k], st)
        if srt["counts"][1] or srt["counts"][2] or srt["counts"][3]:
            raise AssertionError("a slab holds particles outside its faces before the step")
        acc = interact(prm[k], srt)
        srts.append(srt)
        accs.append(acc)
        dts.append(_dt(prm[k], srt, acc))
    dtg = min(dts)
    new_own = [[] for _ in own]
    migrants = []
    for k in range(len(own)):
        n0 = int(srts[k]["counts"][0])
        s = verlet(prm[k], srts[k]["state"], n0, step_index, dtg, accs[k])
        mine = _take(s, s["type"] != GHOST)
        lab = keys(prm[k], mine) >> np.uint32(cell_bits(prm[k]))
        if np.any(lab == 3):
            raise AssertionError("a particle left the slab grid in one step")
        stay, lo, hi = lab == 0, lab == 1, lab == 2
        new_own[k].append(_take(mine, stay))
        if k > 0:
            new_own[k - 1].append(_take(mine, lo))
        elif lo.any():
            raise AssertionError("a particle left the first slab through its outer face")
        if k + 1 < len(own):
            new_own[k + 1].append(_take(mine, hi))
        elif hi.any():
            raise AssertionError("a particle left the last slab through its outer face")
        migrants.append((int(lo.sum()), int(hi.sum())))
    return dict(own=[_cat(parts) for parts in new_own], dt=dtg,
                ghosts=[int(len(g["x"])) for g in ghosts],
                ghost_fluid=[nf for _, nf in halos], migrants=migrants)
