"""Seeded synthetic dam-break inputs: geometry, initial state and run parameters.

This module builds inputs only. It serves both the HIP path and the CPU
oracle, and holds none of the time step's arithmetic (no kernel, no equation
of state in the forward direction, no sums, no integrator). Every random draw
comes from ``numpy.random.Generator(PCG64(seed))``.

The paper's test problem is a 3-D dam break with three obstacles (Sec. 6,
weak/strong scaling runs); its geometry exists only in a figure, so the
recipes below stand in for it:

* particles sit on a cubic lattice of spacing ``dp``; one layer of fixed
  (dynamic-boundary, Sec. 2.3) particles on the floor and the four side walls,
  no lid;
* fluid lattice coordinates get a jitter of ``1e-4*dp*U(-1,1)`` per axis;
* the fluid starts at rest with a hydrostatic density profile: the Tait law
  of Sec. 2.2 inverted for ``p = rho0*|g|*(H - z)``, ``H`` the column top
  (an initial condition, not a step of the method);
* boundary particles start at ``rho0``;
* obstacles are hollow single-layer cuboids (side faces + top, no bottom).

Particle types: 0 fluid, 1 boundary, 2 ghost (halo copy of a neighbouring
sub-domain, Sec. 4.2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

FLUID, BOUNDARY, GHOST = 0, 1, 2
GRAVITY = 9.81

STATE_F32 = ("x", "y", "z", "vx", "vy", "vz", "rho", "vxp", "vyp", "vzp", "rhop")
STATE_KEYS = STATE_F32 + ("type", "id")


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def base_params(dp: float, *, h_over_dp: float = 1.3, alpha: float = 0.01,
                cfl: float = 0.2, euler_every: int = 40,
                c0: float | None = None) -> dict:
    """Physical constants of a run (SI units).

    rho0 = 1000 and gamma = 7 are the paper's (Sec. 2.2); h = 1.3 dp,
    c0 = 10*sqrt(g*0.3), alpha = 0.01 and CFL = 0.2 are the workload's
    settings; eta = 0.1 h (Sec. 2.2); m = rho0*dp^3 for every particle.
    """
    h = h_over_dp * dp
    return dict(
        dp=dp, h=h, rho0=1000.0, gamma=7.0,
        c0=(10.0 * math.sqrt(GRAVITY * 0.3)) if c0 is None else c0,
        alpha=alpha, eta_over_h=0.1, cfl=cfl, mass=1000.0 * dp ** 3,
        g=(0.0, 0.0, -GRAVITY), euler_every=euler_every,
        origin=(0.0, 0.0, 0.0), ncell=(1, 1, 1),
        slab_mode=0, slab_xlo=0.0, slab_xhi=0.0,
    )


def set_grid(params: dict, lo, hi) -> dict:
    """Cover the box [lo, hi) with cubic cells of side 2h starting at lo."""
    cs = 2.0 * params["h"]
    n = tuple(int(math.ceil((hi[a] - lo[a]) / cs - 1e-9)) for a in range(3))
    params["origin"] = tuple(float(v) for v in lo)
    params["ncell"] = tuple(max(1, v) for v in n)
    return params


def cell_bits(params: dict) -> int:
    """Bits needed for a linear cell index (smallest b with 2**b >= ncells)."""
    nc = params["ncell"][0] * params["ncell"][1] * params["ncell"][2]
    return max(1, int(nc - 1).bit_length())


def hydrostatic_rho(params: dict, depth: np.ndarray) -> np.ndarray:
    """Density whose Tait pressure equals rho0*|g|*depth (initial condition)."""
    rho0, gamma, c0 = params["rho0"], params["gamma"], params["c0"]
    B = c0 * c0 * rho0 / gamma
    return rho0 * np.power(1.0 + rho0 * GRAVITY * np.maximum(depth, 0.0) / B,
                           1.0 / gamma)


def _lattice(ii, jj, kk):
    I, J, K = np.meshgrid(ii, jj, kk, indexing="ij")
    return I.ravel(), J.ravel(), K.ravel()


def _make_state(pos: np.ndarray, typ: np.ndarray, rho: np.ndarray,
                vel: np.ndarray | None = None) -> dict:
    n = pos.shape[0]
    st = {}
    st["x"] = pos[:, 0].astype(np.float32)
    st["y"] = pos[:, 1].astype(np.float32)
    st["z"] = pos[:, 2].astype(np.float32)
    if vel is None:
        vel = np.zeros((n, 3))
    st["vx"] = vel[:, 0].astype(np.float32)
    st["vy"] = vel[:, 1].astype(np.float32)
    st["vz"] = vel[:, 2].astype(np.float32)
    st["rho"] = rho.astype(np.float32)
    st["vxp"] = st["vx"].copy()
    st["vyp"] = st["vy"].copy()
    st["vzp"] = st["vz"].copy()
    st["rhop"] = st["rho"].copy()
    st["type"] = typ.astype(np.uint8)
    st["id"] = np.arange(n, dtype=np.int32)
    return st


@dataclass
class Case:
    name: str
    params: dict
    state: dict
    pos64: np.ndarray | None = None  # the exact (FP64) positions the FP32 state rounds

    @property
    def n(self) -> int:
        return int(self.state["x"].shape[0])

    def counts(self) -> dict:
        t = self.state["type"]
        return {"fluid": int((t == FLUID).sum()), "boundary": int((t == BOUNDARY).sum()),
                "ghost": int((t == GHOST).sum()), "total": self.n}


def tank_walls(nx: int, ny: int, nz: int) -> np.ndarray:
    """Lattice indices (i,j,k) of one wall layer on x=0, x=nx, y=0, y=ny, z=0,
    each point once, in lexicographic order."""
    ii, jj, kk = np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1)
    faces = [np.stack(_lattice([0], jj, kk), 1), np.stack(_lattice([nx], jj, kk), 1),
             np.stack(_lattice(ii, [0], kk), 1), np.stack(_lattice(ii, [ny], kk), 1),
             np.stack(_lattice(ii, jj, [0]), 1)]
    return np.unique(np.concatenate(faces, axis=0), axis=0)


def obstacle_surface(i0: int, j0: int, side: int, height: int) -> np.ndarray:
    """Hollow cuboid on the floor: lattice points of its side faces and top."""
    I, J, K = _lattice(np.arange(i0, i0 + side + 1), np.arange(j0, j0 + side + 1),
                       np.arange(1, height + 1))
    on = (I == i0) | (I == i0 + side) | (J == j0) | (J == j0 + side) | (K == height)
    return np.stack([I[on], J[on], K[on]], axis=1)


def dam_break(dp: float, nx: int, ny: int, nz: int, nfx: int, nfz: int, *,
              jitter_seed: int, obstacles: int = 0, obstacle_seed: int = 2,
              obstacle_side: int = 0, obstacle_height: int = 0,
              name: str = "dam_break") -> Case:
    """Water column [1..nfx] x [1..ny-1] x [1..nfz] (lattice units) in a tank of
    nx x ny x nz lattice spacings, optionally with hollow obstacles."""
    params = base_params(dp)
    cs = 2.0 * params["h"]
    walls = tank_walls(nx, ny, nz)
    bnd = [walls]
    if obstacles:
        rng = _rng(obstacle_seed)
        ycent = [int(round(ny * f)) for f in (0.25, 0.5, 0.75)][:obstacles]
        placed = []
        for yc in ycent:
            while True:
                xc = int(round(rng.uniform(0.6, 1.4) / dp))
                i0, j0 = xc - obstacle_side // 2, yc - obstacle_side // 2
                box = (i0, i0 + obstacle_side, j0, j0 + obstacle_side)
                clash = any(not (box[1] < b[0] or b[1] < box[0] or box[3] < b[2] or b[3] < box[2])
                            for b in placed)
                if not clash:
                    placed.append(box)
                    break
            bnd.append(obstacle_surface(i0, j0, obstacle_side, min(obstacle_height, nz)))
    bidx = np.unique(np.concatenate(bnd, axis=0), axis=0)
    I, J, K = _lattice(np.arange(1, nfx + 1), np.arange(1, ny), np.arange(1, nfz + 1))
    fidx = np.stack([I, J, K], axis=1)
    rng = _rng(jitter_seed)
    fpos = fidx * dp + 1e-4 * dp * rng.uniform(-1.0, 1.0, size=fidx.shape)
    bpos = bidx.astype(np.float64) * dp
    H = nfz * dp
    frho = hydrostatic_rho(params, H - fpos[:, 2])
    pos = np.concatenate([bpos, fpos], axis=0)
    typ = np.concatenate([np.full(len(bpos), BOUNDARY), np.full(len(fpos), FLUID)])
    rho = np.concatenate([np.full(len(bpos), params["rho0"]), frho])
    Lx, Ly, Lz = nx * dp, ny * dp, nz * dp
    set_grid(params, (-cs, -cs, -cs), (Lx + cs, Ly + cs, 1.5 * Lz))
    return Case(name, params, _make_state(pos, typ, rho), pos)


def case_c1(seed: int = 1) -> Case:
    """Plain dam break at dp = 0.02 m: tank 1.6 x 0.68 x 0.4 m, column 0.4 x 0.66 x 0.3 m
    (9,900 fluid + 7,395 boundary particles)."""
    return dam_break(0.02, 80, 34, 20, 20, 15, jitter_seed=seed, name="dam_break_dp0.02")


def case_c2(jitter_seed: int = 3, obstacle_seed: int = 2) -> Case:
    """Dam break with three hollow 0.12 x 0.12 x 0.4 m obstacles at dp = 0.004 m
    (1,252,500 fluid particles, ~1.47M in total)."""
    return dam_break(0.004, 400, 168, 100, 100, 75, jitter_seed=jitter_seed,
                     obstacles=3, obstacle_seed=obstacle_seed, obstacle_side=30,
                     obstacle_height=100, name="dam_break_3obst_dp0.004")


def case_c4(seed: int = 7, obstacle_seed: int = 2) -> Case:
    """Dam break with three obstacles at dp = 0.0013 m: 308 x 514 x 231 = 36,570,072
    fluid particles (the nominal "32M" case) plus walls and obstacles (~38.5M)."""
    return dam_break(0.0013, 1231, 515, 308, 308, 231, jitter_seed=seed, obstacles=3,
                     obstacle_seed=obstacle_seed, obstacle_side=92, obstacle_height=308,
                     name="dam_break_3obst_dp0.0013")


def obstacle_tank(seed: int, *, dp: float = 0.004, nx: int = 200, ny: int = 84, nz: int = 100,
                  nfx: int = 50, nfz: int = 75, n_obstacles: int = 2, side: int = 30) -> Case:
    """Training layout for the learned surrogate: a 0.8 x 0.34 x 0.4 m tank at
    dp = 0.004 m with a 0.2 m long, 0.3 m high water column (the height of the
    1.47M-particle workload, so the same hydrostatic density range) and
    ``n_obstacles`` hollow square obstacles whose positions in front of the
    column are drawn from ``seed`` (non-overlapping, inside the tank)."""
    params = base_params(dp)
    cs = 2.0 * params["h"]
    rng = _rng(1000 + seed)
    placed, bnd = [], [tank_walls(nx, ny, nz)]
    tries = 0
    while len(placed) < n_obstacles:
        tries += 1
        if tries > 10000:
            raise ValueError("obstacle_tank: the obstacles do not fit into the tank")
        i0 = int(rng.integers(nfx + 10, nx - side - 5))
        j0 = int(rng.integers(3, ny - side - 3))
        box = (i0 - 2, i0 + side + 2, j0 - 2, j0 + side + 2)
        if any(not (box[1] < b[0] or b[1] < box[0] or box[3] < b[2] or b[3] < box[2])
               for b in placed):
            continue
        placed.append(box)
        bnd.append(obstacle_surface(i0, j0, side, nz))
    bidx = np.unique(np.concatenate(bnd, axis=0), axis=0)
    I, J, K = _lattice(np.arange(1, nfx + 1), np.arange(1, ny), np.arange(1, nfz + 1))
    fidx = np.stack([I, J, K], axis=1)
    fpos = fidx * dp + 1e-4 * dp * _rng(seed).uniform(-1.0, 1.0, size=fidx.shape)
    bpos = bidx.astype(np.float64) * dp
    frho = hydrostatic_rho(params, nfz * dp - fpos[:, 2])
    pos = np.concatenate([bpos, fpos], axis=0)
    typ = np.concatenate([np.full(len(bpos), BOUNDARY), np.full(len(fpos), FLUID)])
    rho = np.concatenate([np.full(len(bpos), params["rho0"]), frho])
    set_grid(params, (-cs, -cs, -cs), (nx * dp + cs, ny * dp + cs, 1.5 * nz * dp))
    return Case(f"obstacle_tank{seed}", params, _make_state(pos, typ, rho), pos)


def sub_block(case: Case, lo, side: float, margin: float) -> tuple[np.ndarray, np.ndarray]:
    """Indices of the particles inside the cube [lo, lo + side)^3 and of those
    inside the same cube grown by ``margin`` (the block and its halo)."""
    p = case.pos64 if case.pos64 is not None else np.stack(
        [case.state["x"], case.state["y"], case.state["z"]], 1).astype(np.float64)
    lo = np.asarray(lo, dtype=np.float64)
    inner = np.all((p >= lo) & (p < lo + side), axis=1)
    outer = np.all((p >= lo - margin) & (p < lo + side + margin), axis=1)
    return np.nonzero(inner)[0], np.nonzero(outer)[0]


def small_tank(dp: float = 0.02, nx: int = 24, ny: int = 10, nz: int = 12, nfx: int = 8,
               nfz: int = 8, seed: int = 11) -> Case:
    """A few-thousand-particle dam break for fast tests."""
    return dam_break(dp, nx, ny, nz, nfx, nfz, jitter_seed=seed, name="small_tank")


def slab_c3(*, dp: float = 0.0013, width_cells: int = 25, ny_fluid: int = 515,
            nz_fluid: int = 239, nz_wall: int = 308, ghost_layers: int = 3,
            migrants_per_face: int | None = None, ghost_seed: int = 4,
            migrant_seed: int = 5, name: str = "slab") -> Case:
    """One x-slab of a 4-slab decomposed dam break (slab 1 of 4: x in [W, 2W)).

    Fluid lattice x = x_lo + (i+1/2) dp, i < 25 cells * 2.6 = 65 layers; walls on
    y = 0, y = (ny_fluid+1) dp and z = 0. Ghost strips of ``ghost_layers``
    lattice layers (< 2h) continue fluid and walls on both x faces (type ghost;
    rho hydrostatic x (1 + U(+-1e-3)), v ~ U(+-0.1) m/s). A share of 0.25 % of
    the fluid per face, drawn from the edge layer, has just crossed the face by
    U(0, dp) (outgoing migrants).
    """
    params = base_params(dp)
    cs = 2.0 * params["h"]
    nxl = int(round(width_cells * cs / dp))
    W = width_cells * cs
    xlo, xhi = W, 2.0 * W
    nyw = ny_fluid + 1
    # fluid
    I, J, K = _lattice(np.arange(nxl), np.arange(1, ny_fluid + 1), np.arange(1, nz_fluid + 1))
    fpos = np.stack([xlo + (I + 0.5) * dp, J * dp, K * dp], axis=1)
    # walls (per x lattice layer: y=0, y=nyw (k=0..nz_wall), floor j=1..nyw-1)
    def wall_layer(xs):
        out = []
        Jw, Kw = np.meshgrid(np.array([0, nyw]), np.arange(nz_wall + 1), indexing="ij")
        Jf = np.arange(1, nyw)
        for xv in xs:
            out.append(np.stack([np.full(Jw.size, xv), Jw.ravel() * dp, Kw.ravel() * dp], 1))
            out.append(np.stack([np.full(Jf.size, xv), Jf * dp, np.zeros(Jf.size)], 1))
        return np.concatenate(out, 0)
    bpos = wall_layer(xlo + (np.arange(nxl) + 0.5) * dp)
    gx_l = xlo - (np.arange(ghost_layers) + 0.5) * dp
    gx_r = xhi + (np.arange(ghost_layers) + 0.5) * dp
    Jg, Kg = np.arange(1, ny_fluid + 1), np.arange(1, nz_fluid + 1)
    gpos = []
    for xs in (gx_l, gx_r):
        Ig, JJ, KK = _lattice(xs, Jg, Kg)
        gpos.append(np.stack([Ig, JJ * dp, KK * dp], 1))
        gpos.append(wall_layer(xs))
    gpos = np.concatenate(gpos, 0)
    H = nz_fluid * dp
    rng_g = _rng(ghost_seed)
    frho = hydrostatic_rho(params, H - fpos[:, 2])
    grho = np.where(gpos[:, 2] > 0.0, hydrostatic_rho(params, H - gpos[:, 2]), params["rho0"])
    grho = grho * (1.0 + rng_g.uniform(-1e-3, 1e-3, size=len(gpos)))
    gvel = rng_g.uniform(-0.1, 0.1, size=(len(gpos), 3))
    # migrants: fluid particles of the edge layers pushed across the faces
    nmig = int(round(0.0025 * len(fpos))) if migrants_per_face is None else migrants_per_face
    rng_m = _rng(migrant_seed)
    left = np.nonzero(fpos[:, 0] < xlo + cs)[0]
    right = np.nonzero(fpos[:, 0] >= xhi - cs)[0]
    if nmig:
        ml = rng_m.choice(left, size=nmig, replace=False)
        mr = rng_m.choice(right, size=nmig, replace=False)
        fpos[ml, 0] = xlo - rng_m.uniform(0.0, dp, size=nmig)
        fpos[mr, 0] = xhi + rng_m.uniform(0.0, dp, size=nmig)
    pos = np.concatenate([bpos, fpos, gpos], 0)
    typ = np.concatenate([np.full(len(bpos), BOUNDARY), np.full(len(fpos), FLUID),
                          np.full(len(gpos), GHOST)])
    rho = np.concatenate([np.full(len(bpos), params["rho0"]), frho, grho])
    vel = np.concatenate([np.zeros((len(bpos) + len(fpos), 3)), gvel], 0)
    set_grid(params, (xlo - cs, -cs, -cs), (xhi + cs, nyw * dp + cs, 1.5 * nz_wall * dp))
    params["slab_mode"] = 1
    params["slab_xlo"], params["slab_xhi"] = xlo, xhi
    return Case(name, params, _make_state(pos, typ, rho, vel), pos)


def small_slab(seed: int = 21) -> Case:
    """A ~10k-particle slab with ghosts and migrants (same recipe, smaller)."""
    return slab_c3(dp=0.01, width_cells=5, ny_fluid=20, nz_fluid=14, nz_wall=20,
                   migrants_per_face=12, ghost_seed=seed, migrant_seed=seed + 1,
                   name="small_slab")


def perturb(case: Case, seed: int, vamp: float = 0.5, rho_rel: float = 0.005,
            types=(FLUID,)) -> Case:
    """'Developed flow' state: v ~ U(-vamp, vamp) per component and
    rho *= 1 + U(-rho_rel, rho_rel) on the given particle types."""
    rng = _rng(seed)
    st = {k: v.copy() for k, v in case.state.items()}
    sel = np.isin(st["type"], np.array(types, dtype=np.uint8))
    n = int(sel.sum())
    for k in ("vx", "vy", "vz"):
        st[k][sel] = rng.uniform(-vamp, vamp, size=n).astype(np.float32)
    st["rho"][sel] = (st["rho"][sel] * (1.0 + rng.uniform(-rho_rel, rho_rel, size=n))).astype(np.float32)
    for a, b in (("vxp", "vx"), ("vyp", "vy"), ("vzp", "vz"), ("rhop", "rho")):
        st[a] = st[b].copy()
    return Case(case.name + f"+perturb{seed}", dict(case.params), st, case.pos64)


def shuffle(case: Case, seed: int) -> Case:
    """Same particles in a random storage order."""
    perm = _rng(seed).permutation(case.n)
    st = {k: v[perm].copy() for k, v in case.state.items()}
    return Case(case.name + f"+shuffle{seed}", dict(case.params), st,
                None if case.pos64 is None else case.pos64[perm].copy())


def random_cloud(n: int, dp: float, extent, seed: int, types=(FLUID,)) -> Case:
    """Uniform random particles in a box (no lattice, no ties at 2h)."""
    rng = _rng(seed)
    params = base_params(dp)
    ext = np.asarray(extent, dtype=np.float64)
    pos = rng.uniform(0.0, 1.0, size=(n, 3)) * ext
    typ = rng.choice(np.array(types), size=n)
    rho = 1000.0 * (1.0 + rng.uniform(-0.01, 0.01, size=n))
    vel = rng.uniform(-0.5, 0.5, size=(n, 3))
    cs = 2.0 * params["h"]
    set_grid(params, (-cs, -cs, -cs), tuple(ext + cs))
    return Case("random_cloud", params, _make_state(pos, typ, rho, vel), pos)


def isolated_clusters(seed: int, copies: int = 8, kmax: int = 12, dp: float = 0.02) -> Case:
    """`copies` clusters of each size k = 1..kmax, shuffled over a lattice of
    spacing 8h: a cluster's particles lie within 0.45h of its centre (so
    within 0.9h of each other) and 7h from any other cluster, so each has
    exactly k - 1 neighbours besides itself. Random fluid/boundary types,
    velocities and +-1 % densities."""
    rng = _rng(seed)
    params = base_params(dp)
    h = params["h"]
    sizes = np.repeat(np.arange(1, kmax + 1), copies)
    rng.shuffle(sizes)
    side = int(np.ceil(len(sizes) ** (1.0 / 3.0)))
    pos = []
    for c, k in enumerate(sizes):
        centre = (np.array([c % side, (c // side) % side, c // (side * side)]) + 0.5) * 8.0 * h
        d = rng.normal(size=(k, 3))
        d *= (0.45 * h * rng.uniform(0.0, 1.0, size=(k, 1)) ** (1.0 / 3.0)
              / np.linalg.norm(d, axis=1, keepdims=True))
        pos.append(centre + d)
    pos = np.concatenate(pos)
    n = pos.shape[0]
    typ = rng.choice(np.array([FLUID, BOUNDARY]), size=n)
    rho = 1000.0 * (1.0 + rng.uniform(-0.01, 0.01, size=n))
    vel = rng.uniform(-0.5, 0.5, size=(n, 3))
    ext = side * 8.0 * h
    set_grid(params, (-2.0 * h,) * 3, (ext + 2.0 * h,) * 3)
    return Case("isolated_clusters", params, _make_state(pos, typ, rho, vel), pos)


def periodic_block(n_side: int, dp: float, seed: int, jitter: float = 0.15) -> Case:
    """n_side^3 fluid particles on a jittered lattice filling a periodic cube of
    side n_side*dp, random velocities and +-1 % densities (for invariance pins)."""
    rng = _rng(seed)
    params = base_params(dp)
    I, J, K = _lattice(np.arange(n_side), np.arange(n_side), np.arange(n_side))
    pos = (np.stack([I, J, K], 1) + 0.5 + jitter * rng.uniform(-1, 1, size=(I.size, 3))) * dp
    rho = 1000.0 * (1.0 + rng.uniform(-0.01, 0.01, size=I.size))
    vel = rng.uniform(-0.5, 0.5, size=(I.size, 3))
    L = n_side * dp
    params["origin"] = (0.0, 0.0, 0.0)
    params["box"] = (L, L, L)
    return Case("periodic_block", params, _make_state(pos, np.full(I.size, FLUID), rho, vel))
