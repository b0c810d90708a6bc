"""Helpers for the GPU-vs-oracle parity tests (no arithmetic of the method)."""
import sys

import numpy as np

import oracle
from paper_1210_1017_amd import cases, sph

TOL = 1e-4  # normwise relative error bound of single-step FP32 results


def announce(msg: str):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def relnorm(got, ref) -> float:
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    num = np.linalg.norm(got - ref)
    return float(num / den) if den > 0 else float(num)


def ulp32(x):
    x = np.abs(np.asarray(x, dtype=np.float32))
    return (np.nextafter(x, np.float32(np.inf)) - x).astype(np.float64)


def gpu_sort(ctx: "sph.Context", state: dict, n: int):
    cur = sph.DeviceState.from_numpy(state, capacity=ctx.capacity)
    out = sph.DeviceState.empty(ctx.capacity)
    ctx.sort(cur, out, n)
    return cur, out


def assert_sorted_equal(out_np: dict, srt: dict, n: int):
    """Bit-exact comparison of a GPU-sorted state with the oracle's."""
    ref = srt["state"]
    for k in sph.SOA_FIELDS:
        r = ref[k]
        if r.dtype == np.float64:
            r = r.astype(np.float32)
        g = out_np[k][:n]
        assert np.array_equal(g.view(np.uint8), np.ascontiguousarray(r).view(np.uint8)), k


def interact_compare(p: dict, srt: dict, g: dict, sel=None, acc=None):
    """Normwise errors of GPU rates g (numpy, sorted order) against the oracle.
    Returns dict of relative errors and the oracle output used."""
    s = srt["state"]
    n0 = int(srt["counts"][0])
    if acc is None:
        acc = oracle.interact(p, srt, sel=sel)
    idx = np.arange(n0) if sel is None else np.asarray(sel)
    t = s["type"][idx]
    fl = t == cases.FLUID
    ng = t != cases.GHOST
    gvec = np.array(p["g"])
    a_ref = np.stack([acc["ax"], acc["ay"], acc["az"]], 1)[fl] - gvec
    a_gpu = np.stack([g["ax"][idx], g["ay"][idx], g["az"][idx]], 1)[fl].astype(np.float64) - gvec
    err = {
        "a_minus_g": relnorm(a_gpu, a_ref),
        "drho": relnorm(g["arho"][idx][ng], acc["drho"][ng]),
    }
    if "press" in g:
        err["p"] = relnorm(g["press"][idx][ng], acc["p"][ng])
    if "nu" in g:
        err["nu"] = relnorm(g["nu"][idx][ng], acc["nu"][ng])
    if "npair" in g:  # same FP32 support test on both sides: exact
        assert np.array_equal(g["npair"][idx][ng].astype(np.int64), acc["npair"][ng])
    # ghosts and non-fluid accelerations are exactly zero
    for k in ("ax", "ay", "az"):
        assert np.all(g[k][idx][~fl] == 0.0)
    assert np.all(g["arho"][idx][~ng] == 0.0)
    return err, acc
