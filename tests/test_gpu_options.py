"""GPU against the oracle for the step variants of sph_params.options: the
cubic spline kernel of Sec. 2.2, the boundary density floor and the
symplectic integrator (two interactions per step).

Same bars as the plain path: sort bit-exact, interaction within 1e-4
normwise with exact neighbour counts, update within one FP32 ulp plus 1e-5 of
the increment given the same rates, one full step within 1e-4 normwise.
"""
import numpy as np
import pytest

import oracle
from paper_1210_1017_amd import cases, sph
from parity_util import TOL, announce, gpu_sort, interact_compare, relnorm, ulp32

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    sph.lib()
    yield
    torch.cuda.synchronize()


def _with(case, options):
    p = dict(case.params)
    p["options"] = options
    return p


def _states():
    return {
        "c1_rest": lambda: cases.case_c1(),
        "c1_random": lambda: cases.perturb(cases.case_c1(), 6),
        "small_slab": lambda: cases.perturb(cases.small_slab(), 7),
        "dense_cloud": lambda: cases.random_cloud(4000, 0.02, (0.06, 0.06, 0.06), seed=17),
    }


@pytest.mark.parametrize("name", list(_states()))
def test_cubic_interaction_parity(name):
    case = _states()[name]()
    p, n = _with(case, sph.OPTION_CUBIC), case.n
    announce(f"cubic interact {name} n={n}")
    ctx = sph.Context(p, n)
    _, out = gpu_sort(ctx, case.state, n)
    rates = sph.make_rates(n)
    ctx.interact(out, n, rates)
    torch.cuda.synchronize()
    srt = oracle.sort_state(p, case.state)
    g = {k: v.cpu().numpy() for k, v in rates.items()}
    err, acc = interact_compare(p, srt, g)
    print(name, err, flush=True)
    for k, v in err.items():
        assert v <= TOL, (k, v)
    assert ctx.pairs() == int(acc["npair"].sum())
    dt_ref = oracle.dt(p, srt, acc)
    assert abs(ctx.dt() - dt_ref) <= 1e-4 * dt_ref
    # the variant really is another kernel
    w = oracle.interact(case.params, srt)
    n0 = int(srt["counts"][0])
    assert (relnorm(g["arho"][:n0], w["drho"]) > 10 * TOL or
            relnorm(g["ax"][:n0], w["ax"]) > 10 * TOL)


@pytest.mark.parametrize("step", [0, 1])
def test_floor_update_parity_same_rates(step):
    """Verlet kernel with the floor on a state where about half the boundary
    densities sit below rho0, with the oracle's rates rounded to FP32."""
    case = cases.perturb(cases.case_c1(), 6)
    p, n = _with(case, sph.OPTION_RHO_FLOOR), case.n
    announce(f"floor update step={step} n={n}")
    ctx = sph.Context(p, n)
    _, out = gpu_sort(ctx, case.state, n)
    rates = sph.make_rates(n)
    ctx.interact(out, n, rates)
    torch.cuda.synchronize()
    srt = oracle.sort_state(p, case.state)
    acc = oracle.interact(p, srt)
    for k in ("ax", "ay", "az"):
        rates[k].copy_(torch.from_numpy(acc[k].astype(np.float32)))
    rates["arho"].copy_(torch.from_numpy(acc["drho"].astype(np.float32)))
    acc32 = {k: acc[k].astype(np.float32).astype(np.float64) for k in ("ax", "ay", "az", "drho")}
    dt = ctx.dt()
    ctx.update(out, rates, n, step)
    torch.cuda.synchronize()
    got = out.to_numpy(n)
    ref = oracle.verlet(p, srt["state"], int(srt["counts"][0]), step, float(dt), acc32)
    s0 = srt["state"]
    for k in ("x", "y", "z", "vx", "vy", "vz", "rho", "vxp", "vyp", "vzp", "rhop"):
        inc = np.abs(ref[k] - s0[k])
        bound = 1.0 * ulp32(ref[k]) + 1e-5 * inc + 1e-30
        bad = np.abs(got[k].astype(np.float64) - ref[k]) > bound
        assert not bad.any(), (k, int(bad.sum()))
    bnd = s0["type"] == cases.BOUNDARY
    floored = bnd & (ref["rho"] == p["rho0"])
    assert floored.sum() > 100
    assert np.all(got["rho"][floored] == np.float32(p["rho0"]))
    assert np.all(got["rho"][bnd] >= np.float32(p["rho0"]))


def test_cubic_floor_step_matches_oracle():
    """sph_step with both options from an FP32 state against the oracle step."""
    case = cases.perturb(cases.case_c1(), 6)
    p, n = _with(case, sph.OPTION_CUBIC | sph.OPTION_RHO_FLOOR), case.n
    announce(f"cubic+floor step c1 n={n}")
    ctx = sph.Context(p, n)
    cur = sph.DeviceState.from_numpy(case.state, capacity=n)
    nxt = sph.DeviceState.empty(n)
    ctx.step(cur, nxt, n, 0)
    torch.cuda.synchronize()
    got = nxt.to_numpy(n)
    r = oracle.step(p, case.state, 0, dt_override=float(ctx.dt()))
    ref = r["state"]
    assert np.array_equal(got["id"], ref["id"])
    for k in ("x", "y", "z", "vx", "vy", "vz", "rho"):
        assert relnorm(got[k], ref[k]) <= TOL, k
    s0 = r["srt"]["state"]
    for k in ("vx", "vy", "vz", "rho"):
        inc_ref = ref[k] - s0[k]
        inc_gpu = got[k].astype(np.float64) - s0[k]
        excess = np.maximum(np.abs(inc_gpu - inc_ref) - ulp32(ref[k]), 0.0)
        assert np.linalg.norm(excess) <= 1e-3 * np.linalg.norm(inc_ref), k
    bnd = s0["type"] == cases.BOUNDARY
    assert np.all(got["rho"][bnd] >= np.float32(p["rho0"]))


def test_cubic_dam_break_runs_and_conserves():
    """100 steps of the small dam break with the cubic kernel and the floor:
    ids and counts conserved, walls fixed, no status flags, and the fluid
    moves (the front advances)."""
    case = cases.case_c1()
    p, n = _with(case, sph.OPTION_CUBIC | sph.OPTION_RHO_FLOOR), case.n
    announce(f"cubic+floor 100 steps c1 n={n}")
    ctx = sph.Context(p, n)
    a = sph.DeviceState.from_numpy(case.state, capacity=n)
    b = sph.DeviceState.empty(n)
    for s in range(100):
        ctx.step(a, b, n, s)
        a, b = b, a
    torch.cuda.synchronize()
    got = a.to_numpy(n)
    assert np.sort(got["id"]).tolist() == list(range(n))
    assert sum(ctx.counts()["n_label"]) == n
    assert ctx.status() & (sph.STATUS_NONFINITE | sph.STATUS_DT) == 0
    fl = got["type"] == cases.FLUID
    x0 = case.state["x"][case.state["type"] == cases.FLUID].max()
    assert got["x"][fl].max() > x0
    assert np.all(got["rho"][got["type"] == cases.BOUNDARY] >= np.float32(p["rho0"]))


@pytest.mark.parametrize("opts,state", [
    (sph.OPTION_SYMPLECTIC, "c1"),
    (sph.OPTION_SYMPLECTIC | sph.OPTION_CUBIC | sph.OPTION_RHO_FLOOR, "c1"),
    (sph.OPTION_SYMPLECTIC, "slab"),
])
def test_symplectic_step_matches_oracle(opts, state):
    """One symplectic sph_step (two interactions) from an FP32 state against
    the oracle's half step, half-state interaction and full step; the slab
    state has ghosts (untouched) and migrants (sorted behind the domain)."""
    case = (cases.perturb(cases.case_c1(), 6) if state == "c1"
            else cases.perturb(cases.small_slab(), 7))
    p, n = _with(case, opts), case.n
    announce(f"symplectic step opts={opts} {state} n={n}")
    ctx = sph.Context(p, n)
    cur = sph.DeviceState.from_numpy(case.state, capacity=n)
    nxt = sph.DeviceState.empty(n)
    ctx.step(cur, nxt, n, 0)
    torch.cuda.synchronize()
    assert ctx.status() & (sph.STATUS_NONFINITE | sph.STATUS_DT) == 0
    got = nxt.to_numpy(n)
    r = oracle.step(p, case.state, 0, dt_override=float(ctx.dt()))
    assert abs(ctx.dt() - r["dt_cfl"]) <= 1e-4 * r["dt_cfl"]
    assert ctx.pairs() == r["pairs"] or abs(ctx.pairs() - r["pairs"]) <= 2  # half-state edge pairs
    ref = r["state"]
    assert np.array_equal(got["id"], ref["id"])
    for k in ("x", "y", "z", "vx", "vy", "vz", "rho"):
        assert relnorm(got[k], ref[k]) <= TOL, k
    s0 = r["srt"]["state"]
    for k in ("vx", "vy", "vz", "rho"):
        inc_ref = ref[k] - s0[k]
        inc_gpu = got[k].astype(np.float64) - s0[k]
        excess = np.maximum(np.abs(inc_gpu - inc_ref) - ulp32(ref[k]), 0.0)
        assert np.linalg.norm(excess) <= 1e-3 * np.linalg.norm(inc_ref), k
    # previous-step arrays hold the state at n (velocity: fluid only)
    fl = s0["type"] == cases.FLUID
    ng = s0["type"] != cases.GHOST
    assert np.array_equal(got["vxp"][fl], s0["vx"][fl].astype(np.float32))
    assert np.array_equal(got["rhop"][ng], s0["rho"][ng].astype(np.float32))
    # the separate update call is refused for this integrator
    rates = sph.make_rates(n)
    with pytest.raises(sph.SphError):
        ctx.update(nxt, rates, n, 1)


def test_symplectic_dam_break_runs():
    """100 symplectic steps of the small dam break: ids and counts conserved,
    walls fixed, no status flags, the front advances, and the FP64 totals'
    energy changes little more than the Verlet run's."""
    case = cases.case_c1()
    p, n = _with(case, sph.OPTION_SYMPLECTIC), case.n
    announce(f"symplectic 100 steps c1 n={n}")
    ctx = sph.Context(p, n)
    a = sph.DeviceState.from_numpy(case.state, capacity=n)
    b = sph.DeviceState.empty(n)
    for s in range(100):
        ctx.step(a, b, n, s)
        a, b = b, a
    torch.cuda.synchronize()
    got = a.to_numpy(n)
    assert np.sort(got["id"]).tolist() == list(range(n))
    assert sum(ctx.counts()["n_label"]) == n
    assert ctx.status() & (sph.STATUS_NONFINITE | sph.STATUS_DT) == 0
    ref = case.state
    bnd_ids = ref["id"][ref["type"] == cases.BOUNDARY]
    order_g = np.argsort(got["id"])
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        assert np.array_equal(got[k][order_g][bnd_ids], ref[k][bnd_ids]), k
    fl = got["type"] == cases.FLUID
    assert got["x"][fl].max() > case.state["x"][case.state["type"] == cases.FLUID].max()
