"""Pins of the sub-domain decomposition (Sec. 4.2-4.3) on the oracle.

The whole domain is cut into four x-slabs, each a whole number of cells of
side 2h wide, and every slab is stepped on its own with its halo of ghost
copies (the neighbours' edge strips of width 2h), the global time step as
the minimum over the slabs, and the migration of particles that cross a face
(labels 1 and 2 of the slab's sort key). The union of the slabs after each
step must be the undecomposed step's state: the decomposition is exact up to
the order of floating-point sums. The halo holds about 2 (2h)/W of a slab's
particles (Sec. 6, the halo ratio of the weak-scaling discussion).
"""
import numpy as np
import pytest

from paper_1210_1017_amd import cases

FIELDS = ("x", "y", "z", "vx", "vy", "vz", "rho", "vxp", "vyp", "vzp", "rhop")


def _long_tank():
    """Fluid along the whole 1.6 m tank (all four slabs hold fluid), developed flow."""
    base = cases.dam_break(0.02, 80, 8, 10, 79, 5, jitter_seed=31, name="long_tank")
    return cases.perturb(base, 32)


def _faces(p):
    cs = 2.0 * p["h"]
    W = 8 * cs                     # 8 cells of 2h per slab
    x0 = 20 * p["dp"] - W          # face 1 on the lattice plane i = 20: particles cross it
    return [x0 + k * W for k in range(5)], W


def _by_id(st):
    o = np.argsort(st["id"], kind="stable")
    return {k: v[o] for k, v in st.items()}


@pytest.mark.slow
def test_four_slab_steps_equal_undecomposed(orc):
    import oracle.slabs as slabs
    case = _long_tank()
    p = case.params
    faces, W = _faces(p)
    assert faces[0] < 0.0 and faces[-1] > 1.6  # both end walls inside the outer slabs
    whole = orc.to_f64(case.state)
    own = slabs.split(whole, faces)
    assert sum(len(s["x"]) for s in own) == case.n
    moved = 0
    for n in range(4):
        r = orc.step(p, whole, n)
        whole = r["state"]
        res = slabs.decomposed_step(p, own, faces, n)
        own = res["own"]
        moved += sum(a + b for a, b in res["migrants"])
        assert res["dt"] == pytest.approx(r["dt"], rel=1e-12, abs=0)
        union = _by_id({k: np.concatenate([s[k] for s in own]) for k in own[0]})
        ref = _by_id(whole)
        # every particle exactly once, same types
        assert np.array_equal(union["id"], ref["id"]) and np.array_equal(union["type"], ref["type"])
        for k in FIELDS:
            d = np.linalg.norm(union[k] - ref[k]) / np.linalg.norm(ref[k])
            assert d <= 1e-12, (n, k, d)
        # the increments of the step agree too (not only the states)
        prev = _by_id({k: np.concatenate([s[k] for s in own]) for k in own[0]})
        inc_u = union["vx"] - union["vxp"]
        inc_r = ref["vx"] - ref["vxp"]
        assert np.linalg.norm(inc_u - inc_r) <= 1e-10 * np.linalg.norm(inc_r)
        del prev
    assert moved > 0  # particles crossed faces and were handed over


def test_halo_share_matches_halo_ratio(orc):
    """Interior slabs: fluid ghosts / own fluid ~ 2 (2h)/W, within one lattice
    plane per face of the continuous relation (the strips of width 2h = 2.6 dp
    hold 2 or 3 lattice planes)."""
    import oracle.slabs as slabs
    case = _long_tank()
    p = case.params
    faces, W = _faces(p)
    own = slabs.split(orc.to_f64(case.state), faces)
    halos = slabs.halo(own, faces, p["h"])
    for k in (1, 2):
        nf_own = int((own[k]["type"] == cases.FLUID).sum())
        share = halos[k][1] / nf_own
        assert abs(share - 2 * 2 * p["h"] / W) <= 2 * p["dp"] / W, (k, share)
    # the ghosts are exactly the neighbours' particles within 2h of the faces
    cs = 2 * p["h"]
    g = halos[1][0]
    assert np.all((g["x"] >= faces[1] - cs) & (g["x"] < faces[2] + cs))
    assert np.all((g["x"] < faces[1]) | (g["x"] >= faces[2]))
    assert np.all(g["type"] == cases.GHOST)


def test_c3_slab_halo_ratio():
    """The one-GPU slab workload at real shape: 3 ghost lattice planes per face
    (planes at 0.5, 1.5, 2.5 dp are within 2h = 2.6 dp) against 65 planes of
    fluid: 6/65 = 9.2 %, one plane per face above 2 (2h)/W = 8.0 %."""
    dp, h = 0.0013, 1.3 * 0.0013
    planes_in_strip = sum(1 for k in range(10) if (k + 0.5) * dp < 2 * h)
    assert planes_in_strip == 3
    W_planes = int(round(25 * 2 * h / dp))
    assert W_planes == 65
    share = 2 * planes_in_strip / W_planes
    assert share == pytest.approx(0.0923, abs=1e-4)
    assert abs(share - 2 * 2 * h / (W_planes * dp)) <= 2 / W_planes
    # and the generator builds exactly that share of fluid ghosts (small slab, same recipe)
    sm = cases.small_slab()
    st = sm.state
    fl_own = int((st["type"] == cases.FLUID).sum())
    gh = st["type"] == cases.GHOST
    # ghost copies of fluid: off the floor (z > 0) and between the y walls
    ymax = st["y"][st["type"] == cases.FLUID].max()
    fluid_like = gh & (st["z"] > 0) & (st["y"] > 0) & (st["y"] <= ymax)
    assert fluid_like.sum() / fl_own == pytest.approx(2 * 3 / 13, abs=1e-12)
