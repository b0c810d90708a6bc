"""Checkpoint and resume of a run of the plain FP32 step.

The per-process loop of the method (Sec. 4.2) saves particle data at output
steps; a checkpoint here holds everything a later step depends on. One step
(sph_step) is a function of the particle arrays alone (positions, velocities,
densities, the previous-step velocities and densities that the Verlet scheme
of Sec. 3.3 carries, type, id) and of the step index, which selects the
Euler or the leapfrog form; the context keeps nothing between steps that
changes a result (the cell-table search only starts from the previous
bounds, and is exact from any start). A checkpoint therefore stores the
structure of arrays of the n particles, the index of the next step and the
run parameters, and a resumed run continues bit for bit.

Format: one numpy .npz archive (no pickled objects; load with
allow_pickle=False): one array per field of the state and a UTF-8 JSON
header {"format", "version", "n", "step", "params"} as a uint8 array.
"""
from __future__ import annotations

import json

import numpy as np

from . import sph

FORMAT = "sph-checkpoint"
VERSION = 1
_DTYPES = {**{k: np.float32 for k in sph.F32_FIELDS}, "type": np.uint8, "id": np.int32}


def _plain(v):
    """Parameters as JSON values (numpy scalars and arrays to Python)."""
    if isinstance(v, dict):
        return {str(k): _plain(x) for k, x in v.items()}
    if isinstance(v, (list, tuple, np.ndarray)):
        return [_plain(x) for x in v]
    if isinstance(v, np.generic):
        return v.item()
    return v


def save(path, state: "sph.DeviceState", n: int, step: int, params: dict) -> None:
    """Write the first n particles of ``state``, the index of the next step and
    the run parameters to ``path`` (a .npz file). Synchronises with the device
    (the arrays are copied to the host)."""
    if n < 0 or step < 0:
        raise ValueError("n and step must be non-negative")
    arrays = state.to_numpy(n)
    head = {"format": FORMAT, "version": VERSION, "n": int(n), "step": int(step),
            "params": _plain(params)}
    raw = np.frombuffer(json.dumps(head, sort_keys=True).encode("utf-8"), dtype=np.uint8)
    with open(path, "wb") as f:
        np.savez(f, header=raw, **{k: np.ascontiguousarray(arrays[k]) for k in sph.SOA_FIELDS})


def load_arrays(path) -> tuple[dict, int, int, dict]:
    """Read a checkpoint: (host arrays, n, next step index, params). Raises
    ValueError on a file that is not a complete checkpoint of this format."""
    with np.load(path, allow_pickle=False) as z:
        if "header" not in z.files:
            raise ValueError(f"{path}: no checkpoint header")
        head = json.loads(bytes(z["header"]).decode("utf-8"))
        if head.get("format") != FORMAT or head.get("version") != VERSION:
            raise ValueError(f"{path}: not a {FORMAT} file of version {VERSION}")
        n = int(head["n"])
        arrays = {}
        for k in sph.SOA_FIELDS:
            if k not in z.files:
                raise ValueError(f"{path}: field {k} missing")
            a = z[k]
            if a.dtype != _DTYPES[k] or a.shape != (n,):
                raise ValueError(f"{path}: field {k} has dtype {a.dtype} and shape {a.shape}, "
                                 f"expected {np.dtype(_DTYPES[k])} and ({n},)")
            arrays[k] = a
    params = head["params"]
    return arrays, n, int(head["step"]), params


def load(path, capacity: int | None = None, device="cuda"):
    """Read a checkpoint into a device state of at least ``capacity``
    particles: (DeviceState, n, next step index, params)."""
    arrays, n, step, params = load_arrays(path)
    cap = n if capacity is None else capacity
    if cap < n:
        raise ValueError(f"capacity {cap} < {n} particles in the checkpoint")
    return sph.DeviceState.from_numpy(arrays, capacity=cap, device=device), n, step, params
