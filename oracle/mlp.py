"""FP64 reference for the learned surrogate (test infrastructure only).

The surrogate is an addition to the paper's method: a multilayer perceptron
that maps the neighbourhood of a particle -- gathered through the cell list of
Sec. 3.1 with the distance test of Sec. 2.2, plus the pressure and continuity
sums of Sec. 2.2 over it -- to the change of its velocity and density over
four time steps. Beyond those two sections nothing
here comes from the paper; each piece follows a standard published definition:

* bfloat16: the upper half of an IEEE binary32 number, rounded to nearest with
  ties to even (8 significant bits, the binary32 exponent range);
* SiLU activation z * sigmoid(z) (Elfwing, Uchibe and Doya, 2018);
* mean squared error with one weight per output column, differentiated by the
  chain rule (back-propagation);
* Adam with bias correction (Kingma and Ba, 2015, Algorithm 1).

``emulate=False`` keeps every value in FP64 without rounding; the finite-
difference pins check that mode. ``emulate=True`` rounds to bfloat16 exactly
the tensors that the GPU path stores in bfloat16 between its kernels (the
activations after SiLU and the back-propagated pre-activation gradients),
with FP64 arithmetic in between, so that a comparison measures the GPU's FP32
accumulation alone.

Only the tests may import this module. It shares no code with the HIP path.
"""
from __future__ import annotations

import numpy as np


FLUID, BOUNDARY, GHOST = 0, 1, 2
SLOTS = 64          # neighbours per input row
SLOT_F = 8          # features per neighbour slot
OWN_F = 32          # own-particle block (10 used, rest zero)
N_IN = SLOTS * SLOT_F + OWN_F   # 544
N_OUT = 4           # (dv_x, dv_y, dv_z, drho), scaled
BF16_MAX = (2.0 - 2.0 ** -7) * 2.0 ** 127


def bf16_round(a) -> np.ndarray:
    """Round to the nearest bfloat16 value, ties to even; returned as FP64.

    A finite non-zero a = m 2^e (0.5 <= |m| < 1) has bfloat16 spacing
    2^(max(e, -125) - 8): 8 significant bits down to 2^-126, a fixed step of
    2^-133 below it. Results beyond the largest finite bfloat16 become inf."""
    a = np.array(a, dtype=np.float64, copy=True)
    fin = np.isfinite(a) & (a != 0.0)
    v = a[fin]
    _, e = np.frexp(v)
    sp = np.maximum(e, -125) - 8
    r = np.ldexp(np.round(np.ldexp(v, -sp)), sp)   # np.round: half to even
    big = np.abs(r) > BF16_MAX
    r[big] = np.copysign(np.inf, r[big])
    a[fin] = r
    return a


# ------------------------------------------------------------------ features

SUM_COLS = slice(SLOTS * SLOT_F + 6, SLOTS * SLOT_F + 10)   # own-block columns of the pair sums


def kind(t: np.ndarray) -> np.ndarray:
    """Particle kind as a feature: -1 for boundary particles, +1 otherwise."""
    return np.where(t == BOUNDARY, -1.0, 1.0)


def features(p: dict, srt: dict, sel, scales) -> np.ndarray:
    """Input rows of the surrogate for the sorted particles ``sel``.

    ``scales`` = (inv_len, inv_vel, rho_ref, inv_rho, r2f, inv_acc, inv_drho
    [, inv_dt]), FP32 numbers (inv_dt defaults to 0). The neighbours of i are the particles of the 27 cells of
    Sec. 3.1 whose FP32 squared distance (the expression of the support test
    of Sec. 2.2) is below r2f, in increasing sorted index (``nn_rows``); the
    first 64 fill the slots. Slot s holds
        (x_j - x_i) inv_len, (y_j - y_i) inv_len, (z_j - z_i) inv_len,
        (u_j - u_i) inv_vel (3 components), (rho_j - rho_ref) inv_rho, kind_j
    each an FP32 difference times an FP32 scale rounded to bfloat16; empty
    slots are zero. The own block is
        (rho_i - rho_ref) inv_rho, u_i inv_vel (3), count_i / 64, kind_i,
        ap_i inv_acc (3), dr_i inv_drho,
        ((u_i - u_prev_i) inv_dt) inv_acc (3), ((rho_i - rho_prev_i) inv_dt) inv_drho,
        0 ...
    with count_i the number of neighbours found, (ap_i, dr_i) the pressure
    acceleration and continuity rate of Sec. 2.2 summed over the slots
    (``nn_sums``, FP64 here) and u_prev, rho_prev the previous-step values of
    the Verlet scheme of Sec. 3.3 (FP32 arithmetic left to right). Ghost rows
    are zero. Returns an FP64 array of
    bfloat16 values, shape (len(sel), 544)."""
    from . import nn_rows, nn_sums
    s = srt["state"]
    n0 = int(srt["counts"][0])
    sel = np.asarray(sel, dtype=np.int64)
    assert np.all((sel >= 0) & (sel < n0))
    inv_len, inv_vel, rho_ref, inv_rho, r2f, inv_acc, inv_drho = (np.float32(v) for v in scales[:7])
    inv_dt = np.float32(scales[7] if len(scales) > 7 else 0.0)
    f = {k: s[k].astype(np.float32)
         for k in ("x", "y", "z", "vx", "vy", "vz", "rho", "vxp", "vyp", "vzp", "rhop")}
    typ = s["type"]
    nbr, cnt = nn_rows(p, srt, sel, r2f, SLOTS)
    valid = nbr >= 0
    j = np.where(valid, nbr, 0)
    i = sel[:, None]
    cols = []
    for k in ("x", "y", "z"):
        cols.append((f[k][j] - f[k][i]) * inv_len)
    for k in ("vx", "vy", "vz"):
        cols.append((f[k][j] - f[k][i]) * inv_vel)
    cols.append((f["rho"][j] - rho_ref) * inv_rho)
    cols.append(kind(typ[j]).astype(np.float32))
    slot = np.stack(cols, axis=2).astype(np.float64)          # (m, 64, 8)
    slot[~valid] = 0.0
    X = np.zeros((sel.shape[0], N_IN))
    X[:, : SLOTS * SLOT_F] = slot.reshape(sel.shape[0], -1)
    own = X[:, SLOTS * SLOT_F:]
    own[:, 0] = (f["rho"][sel] - rho_ref) * inv_rho
    own[:, 1] = f["vx"][sel] * inv_vel
    own[:, 2] = f["vy"][sel] * inv_vel
    own[:, 3] = f["vz"][sel] * inv_vel
    own[:, 4] = cnt.astype(np.float32) * np.float32(1.0 / 64.0)
    own[:, 5] = kind(typ[sel])
    sums = nn_sums(p, srt, sel, nbr)
    own[:, 6:9] = sums[:, :3] * float(inv_acc)
    own[:, 9] = sums[:, 3] * float(inv_drho)
    for c, (k, kp_, sc) in enumerate((("vx", "vxp", inv_acc), ("vy", "vyp", inv_acc),
                                      ("vz", "vzp", inv_acc), ("rho", "rhop", inv_drho))):
        own[:, 10 + c] = (f[k][sel] - f[kp_][sel]) * inv_dt * sc
    X[typ[sel] == GHOST] = 0.0
    return bf16_round(X)


def rates(p: dict, srt: dict, sel, scales) -> np.ndarray:
    """Pair-sum rates of the rows of ``sel`` (FP64, shape (len(sel), 4)): for
    a fluid particle the pressure acceleration of Sec. 2.2 over the row's
    neighbours plus gravity, (ap + g), for other particles 0; and the
    continuity rate dr over the same neighbours. Ghost rows are zero. These
    are the part of the four-step change that a residual network does not
    predict."""
    from . import nn_rows, nn_sums
    s = srt["state"]
    sel = np.asarray(sel, dtype=np.int64)
    r2f = np.float32(scales[4])
    nbr, _ = nn_rows(p, srt, sel, r2f, SLOTS)
    sums = nn_sums(p, srt, sel, nbr)
    typ = s["type"][sel]
    out = np.zeros((sel.shape[0], 4))
    fl = typ == FLUID
    out[fl, :3] = sums[fl, :3] + np.asarray(p["g"], dtype=np.float64)
    out[typ != GHOST, 3] = sums[typ != GHOST, 3]
    return out


def targets(a: dict, b_by_id: dict, rows, inv_dv: float, inv_dr: float,
            rts=None, span: float = 0.0) -> np.ndarray:
    """Training targets for particles ``rows`` of state ``a``: the FP32 changes
    ((u_b - u_a) - span rts[:, :3]) inv_dv (3 components) and
    ((rho_b - rho_a) - span rts[:, 3]) inv_dr, where b is the same particle
    (same id) in the later state, every operation rounded to FP32 in that
    order. ``b_by_id`` holds that state's FP32 arrays indexed by id; ``rts``
    (FP32 rates, one row per entry of ``rows``) defaults to zeros."""
    rows = np.asarray(rows, dtype=np.int64)
    ids = a["id"][rows]
    if rts is None:
        rts = np.zeros((rows.shape[0], 4), dtype=np.float32)
    rts = np.asarray(rts, dtype=np.float32)
    sp = np.float32(span)
    out = []
    for c, (k, sc) in enumerate((("vx", inv_dv), ("vy", inv_dv), ("vz", inv_dv),
                                 ("rho", inv_dr))):
        d = b_by_id[k][ids].astype(np.float32) - a[k][rows].astype(np.float32)
        out.append((d - sp * rts[:, c]) * np.float32(sc))
    return np.stack(out, axis=1)


# ----------------------------------------------------------------------- MLP

def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(W: list, b: list, X: np.ndarray, emulate: bool = False):
    """y = W_L phi(... phi(W_1 x + b_1) ...) + b_L with phi = SiLU on every
    layer but the last. W[l] has shape (out, in). Returns (Y, cache)."""
    A = [np.asarray(X, dtype=np.float64)]
    Z = []
    for l in range(len(W)):
        z = A[-1] @ W[l].T + b[l]
        Z.append(z)
        if l < len(W) - 1:
            a = silu(z)
            A.append(bf16_round(a) if emulate else a)
    return Z[-1], {"A": A, "Z": Z}


def mse(Y: np.ndarray, T: np.ndarray, wcol) -> tuple[float, np.ndarray]:
    """L = sum_{r,c} w_c (Y - T)^2 / (R C) and dL/dY."""
    R, Cn = Y.shape
    d = Y - T
    w = np.asarray(wcol, dtype=np.float64)
    return float(np.sum(w * d * d) / (R * Cn)), 2.0 * w * d / (R * Cn)


def backward(W: list, cache: dict, dY: np.ndarray, emulate: bool = False):
    """Gradients (dL/dW_l, dL/db_l) by the chain rule from dL/dY."""
    L = len(W)
    gW, gb = [None] * L, [None] * L
    dZ = bf16_round(dY) if emulate else dY
    for l in range(L - 1, -1, -1):
        gW[l] = dZ.T @ cache["A"][l]
        gb[l] = dZ.sum(axis=0)
        if l > 0:
            dZ = (dZ @ W[l]) * silu_grad(cache["Z"][l - 1])
            if emulate:
                dZ = bf16_round(dZ)
    return gW, gb


def adam(w, m, v, g, t: int, lr: float, b1: float = 0.9, b2: float = 0.999,
         eps: float = 1e-8):
    """One Adam step (step number t >= 1); returns (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
