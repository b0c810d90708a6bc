"""Migration injector for one GPU's slab of an x decomposition.

With one GPU there are no neighbouring sub-domains to exchange with, so this
driver stands in for them between steps (it is not part of the step):

* inject: before a step, ``nmig`` fluid particles per face, drawn with
  PCG64(seed_base + step) from the fluid of the layer of cells next to the
  face, are moved across it by U(0, dp); the step's sort then labels them as
  outgoing (labels 1 and 2 of the key, Sec. 4.3) and packs them behind the
  in-domain particles;
* wrap: after the step, the outgoing ranges of that sort are moved back in
  through the opposite face (x -/+ the slab width), as if the neighbours had
  sent the same number of particles back, so the particle count stays exact.
"""
from __future__ import annotations

import numpy as np


def inject(state, n: int, params: dict, step: int, nmig: int, seed_base: int = 5) -> int:
    """Move ``nmig`` fluid particles per face of the slab across the face
    (device state, in place). Returns the number moved."""
    import torch

    from .cases import FLUID
    xlo, xhi = params["slab_xlo"], params["slab_xhi"]
    cs, dp = 2.0 * params["h"], params["dp"]
    rng = np.random.Generator(np.random.PCG64(seed_base + step))
    x, typ = state.t["x"][:n], state.t["type"][:n]
    fl = typ == FLUID
    moved = 0
    for lo, hi, face, sign in ((xlo, xlo + cs, xlo, -1.0), (xhi - cs, xhi, xhi, 1.0)):
        idx = torch.nonzero(fl & (x >= lo) & (x < hi)).squeeze(1)
        if idx.numel() < nmig:
            raise ValueError(f"only {idx.numel()} fluid particles next to the face at {face}")
        pick = rng.choice(idx.numel(), size=nmig, replace=False)
        u = rng.uniform(0.0, dp, size=nmig)
        sel = idx[torch.from_numpy(pick).to(idx.device)]
        x[sel] = torch.from_numpy((face + sign * u).astype(np.float32)).to(x.device)
        moved += nmig
    return moved


def wrap(state, counts: dict, params: dict) -> int:
    """Move the outgoing ranges of the last sort (``counts`` of
    sph_get_counts) back in through the opposite face (device state of that
    sort's output, in place). Returns the number moved."""
    width = params["slab_xhi"] - params["slab_xlo"]
    x = state.t["x"]
    (l0, l1), (r0, r1) = counts["out_lo"], counts["out_hi"]
    if l1 > l0:
        x[l0:l1] += width
    if r1 > r0:
        x[r0:r1] -= width
    return (l1 - l0) + (r1 - r0)
