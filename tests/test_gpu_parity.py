"""GPU (HIP, through the C ABI) against the FP64 oracle, element by element.

Sort, packing ranges and cell tables: bit-exact. Interaction: a - g, drho/dt,
p and nu within 1e-4 normwise relative error (FP32 arithmetic against FP64),
neighbour-pair counts exact (same FP32 support test on both sides). Update:
per element within one FP32 ulp of the result plus 1e-5 of the increment,
given the same rates.
"""
import numpy as np
import pytest

import oracle
from paper_1210_1017_amd import cases, sph
from parity_util import (TOL, announce, assert_sorted_equal, gpu_sort, interact_compare,
                         relnorm, ulp32)

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    sph.lib()
    yield
    torch.cuda.synchronize()


def _ctx(p, cap):
    return sph.Context(p, cap)


# ------------------------------------------------------------------ sort_kv

def _sort_kv(ctx, k, v, bits):
    n = k.shape[0]
    kd = torch.from_numpy(k.view(np.int32).copy()).cuda() if n else torch.empty(1, dtype=torch.int32, device="cuda")
    vd = torch.from_numpy(v.copy()).cuda() if n else torch.empty(1, dtype=torch.int32, device="cuda")
    ko = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    vo = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    ctx.sort_kv(kd, vd, ko, vo, n, bits)
    torch.cuda.synchronize()
    return ko[:n].cpu().numpy().view(np.uint32), vo[:n].cpu().numpy()


def test_sort_kv_paper_example():
    announce("sort_kv paper example n=8")
    ctx = _ctx(cases.small_tank().params, 64)
    k = np.array([0, 1, 1, 0, 1, 0, 0, 2], dtype=np.uint32)
    v = np.arange(1, 9, dtype=np.int32)
    ko, vo = _sort_kv(ctx, k, v, 2)
    assert ko.tolist() == [0, 0, 0, 0, 1, 1, 1, 2]
    assert vo.tolist() == [1, 4, 6, 7, 2, 3, 5, 8]


@pytest.mark.parametrize("n", [0, 1, 2, 63, 64, 65, 4095, 4096, 4097, 100003, (1 << 20) + 1])
@pytest.mark.parametrize("dist", ["random", "dups", "equal", "sorted", "reversed"])
def test_sort_kv_vs_oracle(n, dist):
    announce(f"sort_kv n={n} dist={dist}")
    rng = np.random.default_rng(1000 + n + len(dist))
    bits = 22
    if dist == "random":
        k = rng.integers(0, 1 << bits, size=n, dtype=np.uint32)
    elif dist == "dups":
        k = rng.integers(0, 5, size=n, dtype=np.uint32) << np.uint32(20)
    elif dist == "equal":
        k = np.full(n, 777, dtype=np.uint32)
    elif dist == "sorted":
        k = np.sort(rng.integers(0, 1 << bits, size=n, dtype=np.uint32))
    else:
        k = np.sort(rng.integers(0, 1 << bits, size=n, dtype=np.uint32))[::-1].copy()
    v = rng.permutation(n).astype(np.int32)
    ctx = _ctx(cases.small_tank().params, max(n, 1))
    ko, vo = _sort_kv(ctx, k, v, bits)
    rk, rv = oracle.stable_sort_kv(k, v)
    assert np.array_equal(ko, rk)
    assert np.array_equal(vo, rv)


@pytest.mark.parametrize("bits", [1, 7, 8, 9, 16, 24, 32])
def test_sort_kv_key_widths(bits):
    announce(f"sort_kv bits={bits}")
    rng = np.random.default_rng(bits)
    n = 50000
    hi = (1 << bits) - 1
    k = rng.integers(0, hi, size=n, dtype=np.uint64, endpoint=True).astype(np.uint32)
    v = np.arange(n, dtype=np.int32)
    ctx = _ctx(cases.small_tank().params, n)
    ko, vo = _sort_kv(ctx, k, v, bits)
    rk, rv = oracle.stable_sort_kv(k, v)
    assert np.array_equal(ko, rk) and np.array_equal(vo, rv)


# --------------------------------------------------------------- sort step

def _sort_cases():
    return {
        "small_tank_shuffled": lambda: cases.shuffle(cases.perturb(cases.small_tank(), 3), 4),
        "c1": cases.case_c1,
        "small_slab": cases.small_slab,
        "small_slab_shuffled": lambda: cases.shuffle(cases.small_slab(), 9),
    }


@pytest.mark.parametrize("name", list(_sort_cases()))
def test_sort_state_bit_exact(name):
    case = _sort_cases()[name]()
    p, n = case.params, case.n
    announce(f"sort {name} n={n}")
    ctx = _ctx(p, n + 5)
    _, out = gpu_sort(ctx, case.state, n)
    torch.cuda.synchronize()
    srt = oracle.sort_state(p, case.state)
    assert_sorted_equal(out.to_numpy(n), srt, n)
    assert np.array_equal(sph.u32(ctx.sorted_keys(n)), srt["keys"])
    b, e = ctx.cell_tables()
    assert np.array_equal(sph.u32(b), srt["begin"])
    assert np.array_equal(sph.u32(e), srt["end"])
    cnt = ctx.counts()
    assert cnt["n_label"] == srt["counts"].tolist()
    flat = cnt["halo_lo"] + cnt["edge_lo"] + cnt["edge_hi"] + cnt["halo_hi"] + cnt["out_lo"] + \
        cnt["out_hi"] + cnt["excluded"]
    assert flat == srt["ranges"].tolist()
    assert sum(cnt["n_label"]) == n


def test_tables_from_stale_bounds():
    """The cell-table search starts from the previous sort's bounds: one
    context sorts a full tank, then a third of it (every bound moves), then a
    shuffled full tank, then nothing; every table stays bit-exact."""
    case = cases.perturb(cases.small_tank(), 5)
    p, n = case.params, case.n
    announce(f"tables from stale bounds n={n}")
    ctx = _ctx(p, n)
    rng = np.random.default_rng(21)
    part = {k: v[np.sort(rng.choice(n, n // 3, replace=False))].copy() for k, v in case.state.items()}
    part["id"] = np.arange(n // 3, dtype=np.int32)
    shuf = cases.shuffle(case, 22).state
    for st in (case.state, part, shuf, {k: v[:0].copy() for k, v in case.state.items()}):
        m = st["x"].shape[0]
        _, out = gpu_sort(ctx, st, m)
        torch.cuda.synchronize()
        srt = oracle.sort_state(p, st)
        b, e = ctx.cell_tables()
        assert np.array_equal(sph.u32(b), srt["begin"]), m
        assert np.array_equal(sph.u32(e), srt["end"]), m
        assert ctx.counts()["n_label"] == srt["counts"].tolist()


def test_sort_outside_grid_and_nan():
    case = cases.small_tank()
    st = {k: v.copy() for k, v in case.state.items()}
    st["z"][:5] = 1e6
    st["x"][5] = np.nan
    st["y"][6] = -1.0
    st["x"][7] = np.inf
    n = case.n
    announce(f"sort outside-grid n={n}")
    ctx = _ctx(case.params, n)
    _, out = gpu_sort(ctx, st, n)
    srt = oracle.sort_state(case.params, st)
    assert_sorted_equal(out.to_numpy(n), srt, n)
    cnt = ctx.counts()
    assert cnt["n_label"][3] == 8 and sum(cnt["n_label"]) == n
    assert ctx.status() & sph.STATUS_EXCLUDED


@pytest.mark.parametrize("n", [0, 1])
def test_sort_and_step_tiny(n):
    case = cases.small_tank()
    st = {k: v[:n].copy() for k, v in case.state.items()}
    announce(f"tiny step n={n}")
    ctx = _ctx(case.params, 8)
    cur = sph.DeviceState.from_numpy(st, capacity=8)
    nxt = sph.DeviceState.empty(8)
    ctx.step(cur, nxt, n, 0)
    torch.cuda.synchronize()
    cnt = ctx.counts()
    assert sum(cnt["n_label"]) == n
    assert ctx.pairs() == 0
    if n == 1:  # isolated particle: a = g (boundary here: fixed) and dt from c0
        r = oracle.step(case.params, st, 0)
        assert abs(ctx.dt() - r["dt"]) <= 1e-6 * r["dt"]


# -------------------------------------------------------------- interaction

def _states():
    return {
        "c1_rest": lambda: cases.case_c1(),
        "c1_random": lambda: cases.perturb(cases.case_c1(), 6),
        "small_slab": lambda: cases.perturb(cases.small_slab(), 7),
        "cloud": lambda: cases.random_cloud(6000, 0.02, (0.4, 0.3, 0.3), seed=5,
                                            types=(cases.FLUID, cases.BOUNDARY)),
    }


@pytest.mark.parametrize("name", list(_states()))
def test_interact_parity(name):
    case = _states()[name]()
    p, n = case.params, case.n
    announce(f"interact {name} n={n}")
    ctx = _ctx(p, n)
    _, out = gpu_sort(ctx, case.state, n)
    rates = sph.make_rates(n)
    ctx.interact(out, n, rates)
    torch.cuda.synchronize()
    srt = oracle.sort_state(p, case.state)
    assert_sorted_equal(out.to_numpy(n), srt, n)
    g = {k: v.cpu().numpy() for k, v in rates.items()}
    err, acc = interact_compare(p, srt, g)
    print(name, err, flush=True)
    for k, v in err.items():
        assert v <= TOL, (k, v)
    assert ctx.pairs() == int(acc["npair"].sum())
    dt_ref = oracle.dt(p, srt, acc)
    assert abs(ctx.dt() - dt_ref) <= 1e-4 * dt_ref
    assert ctx.status() & (sph.STATUS_NONFINITE | sph.STATUS_DT | sph.STATUS_RUN_OVERFLOW) == 0


def test_interact_dense_cells_flush():
    """Hundreds of neighbours per particle: the per-lane neighbour buffer is
    flushed several times (more than 128 neighbours each)."""
    case = cases.random_cloud(4000, 0.02, (0.06, 0.06, 0.06), seed=17)
    p, n = case.params, case.n
    announce(f"interact dense n={n}")
    ctx = _ctx(p, n)
    _, out = gpu_sort(ctx, case.state, n)
    rates = sph.make_rates(n)
    ctx.interact(out, n, rates)
    torch.cuda.synchronize()
    srt = oracle.sort_state(p, case.state)
    g = {k: v.cpu().numpy() for k, v in rates.items()}
    err, acc = interact_compare(p, srt, g)
    assert acc["npair"].min() > 300
    for k, v in err.items():
        assert v <= TOL, (k, v)
    assert ctx.pairs() == int(acc["npair"].sum())


def test_interact_isolated_clusters_every_group_remainder():
    """Clusters of 1 to 12 particles, each far (7h) from the others: every
    particle has exactly k - 1 neighbours besides itself, so the lanes' hit
    counts take every remainder modulo the four neighbours evaluated together,
    and a lone particle has none but itself."""
    case = cases.isolated_clusters(23)
    p, n = case.params, case.n
    announce(f"interact isolated clusters n={n}")
    ctx = _ctx(p, n)
    _, out = gpu_sort(ctx, case.state, n)
    rates = sph.make_rates(n)
    ctx.interact(out, n, rates)
    torch.cuda.synchronize()
    srt = oracle.sort_state(p, case.state)
    assert_sorted_equal(out.to_numpy(n), srt, n)
    g = {k: v.cpu().numpy() for k, v in rates.items()}
    err, acc = interact_compare(p, srt, g)
    for k, v in err.items():
        assert v <= TOL, (k, v)
    # k x 8 particles have k - 1 neighbours, for k = 1..12
    counts = np.bincount(g["npair"][:n].astype(np.int64), minlength=12)
    assert np.array_equal(counts, 8 * np.arange(1, 13))
    assert ctx.pairs() == int(acc["npair"].sum()) == 8 * int((np.arange(1, 13) * np.arange(12)).sum())


def test_interact_deterministic():
    case = cases.perturb(cases.case_c1(), 6)
    p, n = case.params, case.n
    announce(f"determinism n={n}")
    outs = []
    for _ in range(2):
        ctx = _ctx(p, n)
        _, out = gpu_sort(ctx, case.state, n)
        rates = sph.make_rates(n)
        ctx.interact(out, n, rates)
        torch.cuda.synchronize()
        outs.append({k: v.cpu().numpy() for k, v in rates.items()})
    for k in outs[0]:
        assert np.array_equal(outs[0][k].view(np.uint32), outs[1][k].view(np.uint32)), k


# ------------------------------------------------------------------ update

@pytest.mark.parametrize("step", [0, 1, 40, 41])
def test_update_parity_same_rates(step):
    """Verlet kernel alone: the oracle's rates (rounded to FP32) and the GPU dt."""
    case = cases.perturb(cases.case_c1(), 6)
    st = {k: v.copy() for k, v in case.state.items()}
    rng = np.random.default_rng(step)
    for k in ("vxp", "vyp", "vzp"):
        st[k] = (st[k] + rng.uniform(-0.01, 0.01, size=case.n)).astype(np.float32)
    st["rhop"] = (st["rhop"] * (1 + rng.uniform(-1e-4, 1e-4, size=case.n))).astype(np.float32)
    p, n = case.params, case.n
    announce(f"update step={step} n={n}")
    ctx = _ctx(p, n)
    _, out = gpu_sort(ctx, st, n)
    rates = sph.make_rates(n)
    ctx.interact(out, n, rates)
    torch.cuda.synchronize()
    srt = oracle.sort_state(p, st)
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
    # boundary and ghost: position and velocity bit-unchanged
    fixed = s0["type"] != cases.FLUID
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        assert np.array_equal(got[k][fixed], s0[k][fixed].astype(np.float32))


def test_step_matches_oracle_single_step():
    """sph_step from an FP32 state against the oracle step (normwise 1e-4 on
    the new state and on its increments beyond FP32 rounding of the state)."""
    case = cases.perturb(cases.case_c1(), 6)
    p, n = case.params, case.n
    announce(f"step c1 n={n}")
    ctx = _ctx(p, n)
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
    fl = s0["type"] == cases.FLUID
    for k in ("vx", "vy", "vz", "rho"):
        inc_ref = ref[k] - s0[k]
        inc_gpu = got[k].astype(np.float64) - s0[k]
        excess = np.maximum(np.abs(inc_gpu - inc_ref) - ulp32(ref[k]), 0.0)
        assert np.linalg.norm(excess) <= 1e-3 * np.linalg.norm(inc_ref), k
    assert np.all(np.isfinite(got["x"][fl]))


def test_boundaries_fixed_over_steps():
    case = cases.case_c1()
    p, n = case.params, case.n
    announce(f"boundary fixed 60 steps n={n}")
    ctx = _ctx(p, n)
    a = sph.DeviceState.from_numpy(case.state, capacity=n)
    b = sph.DeviceState.empty(n)
    for s in range(60):
        ctx.step(a, b, n, s)
        a, b = b, a
    torch.cuda.synchronize()
    got = a.to_numpy(n)
    ref = case.state
    bnd_ids = ref["id"][ref["type"] == cases.BOUNDARY]
    order_g = np.argsort(got["id"])
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        gk = got[k][order_g][bnd_ids]
        assert np.array_equal(gk, ref[k][bnd_ids]), k
    assert np.sort(got["id"]).tolist() == list(range(n))
    assert sum(ctx.counts()["n_label"]) == n
    assert ctx.status() & (sph.STATUS_NONFINITE | sph.STATUS_DT) == 0
