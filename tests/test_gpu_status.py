"""Status bits raised by conditions of the input state, through the C ABI.

Every case here runs ordinary kernels to their end: the conditions come from
the data handed to the library (a NaN density, a state that imposes no time
step limit, a density whose sound speed overflows FP32, a cell holding more
particles than the surrogate rows' 12-bit run offsets can address), never
from a kernel made to fail.
"""
import numpy as np
import pytest

import oracle
from paper_1210_1017_amd import cases, sph
from parity_util import TOL, announce, gpu_sort, interact_compare

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    sph.lib()
    yield
    torch.cuda.synchronize()


def _step(case, step=0, features=0):
    p, n = case.params, case.n
    ctx = sph.Context(p, n, features)
    a = sph.DeviceState.from_numpy(case.state, capacity=n)
    b = sph.DeviceState.empty(n)
    ctx.step(a, b, n, step)
    torch.cuda.synchronize()
    return ctx, b


def test_nan_density_sets_nonfinite():
    """A NaN density of one interior fluid particle reaches its neighbours'
    accelerations through its pressure term (Sec. 2.2 momentum sum) and the
    update flags the result; the dt limit ignores the NaN, the count stays
    exact, and clearing the status works."""
    case = cases.case_c1()
    st = {k: v.copy() for k, v in case.state.items()}
    fl = np.nonzero(st["type"] == cases.FLUID)[0]
    k = fl[len(fl) // 2]
    st["rho"][k] = np.float32(np.nan)
    st["rhop"][k] = np.float32(np.nan)
    case = cases.Case("c1+nan", dict(case.params), st, case.pos64)
    announce("status: NaN density")
    ctx, b = _step(case)
    s = ctx.status()
    assert s & sph.STATUS_NONFINITE
    assert not s & sph.STATUS_DT
    dt = ctx.dt()
    assert np.isfinite(dt) and dt > 0.0
    assert sum(ctx.counts()["n_label"]) == case.n
    got = b.to_numpy(case.n)
    assert np.isnan(got["rho"]).sum() >= 1  # the particle itself
    assert np.isnan(got["vx"]).sum() > 10  # its neighbours
    ctx.clear_status()
    assert ctx.status() == 0


def test_no_limit_sets_dt():
    """Ghost particles only: nothing imposes a CFL limit (Sec. 3.3), the
    minimum stays +inf and the step reports a dt that is not finite."""
    case = cases.small_slab()
    gh = case.state["type"] == cases.GHOST
    st = {k: v[gh].copy() for k, v in case.state.items()}
    st["id"] = np.arange(int(gh.sum()), dtype=np.int32)
    case = cases.Case("ghosts", dict(case.params), st, case.pos64[gh])
    announce(f"status: ghosts only n={case.n}")
    ctx, _ = _step(case)
    assert ctx.status() & sph.STATUS_DT
    assert not np.isfinite(ctx.dt())
    assert ctx.pairs() == 0


def test_overflowing_sound_speed_sets_dt():
    """A density of 1e30 kg/m^3 makes c = c0 (rho/rho0)^3 overflow FP32, the
    acoustic limit h / (c + nu) becomes 0, and the step reports a dt that is
    not positive."""
    case = cases.case_c1()
    st = {k: v.copy() for k, v in case.state.items()}
    fl = np.nonzero(st["type"] == cases.FLUID)[0]
    st["rho"][fl[7]] = np.float32(1e30)
    case = cases.Case("c1+dense", dict(case.params), st, case.pos64)
    announce("status: overflowing sound speed")
    ctx, _ = _step(case)
    assert ctx.status() & sph.STATUS_DT
    assert ctx.dt() == 0.0


def _overfull_cloud():
    """5,000 fluid particles in a cube of side 0.8 h: one cell holds them all
    and every pair is within 2h."""
    dp = 0.02
    h = 1.3 * dp
    return cases.random_cloud(5000, dp, (0.8 * h, 0.8 * h, 0.8 * h), seed=31)


def test_overfull_cell_plain_interaction_exact():
    """The plain interaction addresses its candidates by full 32-bit indices:
    a run of 5,000 candidates is searched completely (every pair counted, the
    sums within the single-step tolerance) and no run overflow is reported."""
    case = _overfull_cloud()
    p, n = case.params, case.n
    announce(f"status: overfull cell, plain interaction n={n}")
    ctx = sph.Context(p, n)
    _, out = gpu_sort(ctx, case.state, n)
    rates = sph.make_rates(n)
    ctx.interact(out, n, rates)
    torch.cuda.synchronize()
    srt = oracle.sort_state(p, case.state)
    g = {k: v.cpu().numpy() for k, v in rates.items()}
    err, acc = interact_compare(p, srt, g)
    assert acc["npair"].min() == n - 1
    for k, v in err.items():
        assert v <= TOL, (k, v)
    assert ctx.pairs() == n * (n - 1)
    assert not ctx.status() & sph.STATUS_RUN_OVERFLOW


def test_overfull_cell_cell_path_exact():
    """The cell + offset interaction also addresses its candidates by full
    indices: the 5,000-candidate run is searched completely (every pair
    counted) and no run overflow is reported."""
    case = _overfull_cloud()
    p, n = case.params, case.n
    announce(f"status: overfull cell, cell path n={n}")
    ctx = sph.Context(p, n, sph.FEATURE_CELL)
    t64 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    ca, cb = sph.CellState.empty(n), sph.CellState.empty(n)
    ctx.cstate_from_positions(t64(case.pos64[:, 0]), t64(case.pos64[:, 1]), t64(case.pos64[:, 2]),
                              ca, n)
    for k in ("vx", "vy", "vz", "rho", "vxp", "vyp", "vzp", "rhop", "type", "id"):
        ca.t[k][:n].copy_(torch.from_numpy(np.ascontiguousarray(case.state[k])))
    ctx.csort(ca, cb, n)
    rates = sph.make_rates(n)
    ctx.cinteract(cb, n, rates)
    torch.cuda.synchronize()
    assert ctx.pairs() == n * (n - 1)
    assert not ctx.status() & sph.STATUS_RUN_OVERFLOW
    for k, v in rates.items():
        assert torch.isfinite(v[:n].float()).all(), k


def test_overfull_cell_flagged_in_surrogate_rows():
    """The surrogate's rows address a run with 12-bit offsets: a run of more
    than 4,096 particles is cut there and flagged (results of that call
    invalid), and the call still completes."""
    case = _overfull_cloud()
    p, n = case.params, case.n
    announce(f"status: overfull cell, surrogate rows n={n}")
    ctx2 = sph.Context(p, n)
    _, out = gpu_sort(ctx2, case.state, n)
    X = torch.empty(n, sph.NN_IN, dtype=torch.bfloat16, device="cuda")
    sc = (np.float32(1.0 / p["h"]), np.float32(2.0), np.float32(1000.0), np.float32(0.1),
          np.float32((1.85 * p["h"]) ** 2), np.float32(0.1), np.float32(1e-3), np.float32(0.0))
    ctx2.nn_features(out, None, n, sc, X)
    torch.cuda.synchronize()
    assert ctx2.status() & sph.STATUS_RUN_OVERFLOW
