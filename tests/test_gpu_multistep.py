"""GPU against the FP64 oracle over ten steps of the plain dam break (dp = 0.02 m).

Beyond one step the comparison is parity unpinned: the flow is chaotic and
FP32 rounding grows, so this test reports the divergence per step and the
drift of the conserved quantities, and bounds them loosely. Two runs from the
same perturbed FP32 state (v ~ U(-0.5, 0.5) m/s, rho within 0.5 %):

* locked: the oracle takes each step with the GPU's dt, so the divergence is
  the FP32 arithmetic alone;
* free: each side takes its own CFL dt (Sec. 2.4), so dt differences add.

Mass is conserved exactly on both sides (particle mass and count are fixed);
momentum and energy are not conserved by a walled, driven flow, so their
drift is reported beside the oracle's own drift over the same steps.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1210_1017_amd import cases, sph
from parity_util import announce

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

STEPS = 10
# Loose bound on the per-step divergence (parity unpinned; measured values
# stay near 1e-6 to 1e-5 over the ten steps).
DIV_BOUND = 1e-3


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    sph.lib()
    yield
    torch.cuda.synchronize()


def _by_id(st: dict) -> dict:
    o = np.argsort(st["id"], kind="stable")
    return {k: v[o] for k, v in st.items()}


def _rel(got, ref, base):
    """Normwise relative difference of the changes since the start state."""
    d_ref = np.asarray(ref, np.float64) - base
    d_got = np.asarray(got, np.float64) - base
    den = np.linalg.norm(d_ref)
    return float(np.linalg.norm(d_got - d_ref) / den) if den > 0 else float(np.linalg.norm(d_got))


def _run(locked: bool):
    case = cases.perturb(cases.case_c1(), 6)
    p, n = case.params, case.n
    announce(f"multistep c1 n={n} steps={STEPS} locked={locked}")
    ctx = sph.Context(p, n)
    a = sph.DeviceState.from_numpy(case.state, capacity=n)
    b = sph.DeviceState.empty(n)
    s0 = _by_id(oracle.to_f64(case.state))
    fl = s0["type"] == cases.FLUID
    ref = oracle.to_f64(case.state)
    tot0 = oracle.totals(p, s0)
    rows = []
    for s in range(STEPS):
        ctx.step(a, b, n, s)
        torch.cuda.synchronize()
        dtg = ctx.dt()
        r = oracle.step(p, ref, s, dt_override=dtg if locked else None)
        ref = r["state"]
        a, b = b, a
        got = _by_id(a.to_numpy(n))
        rr = _by_id(ref)
        assert np.array_equal(got["id"], rr["id"])
        row = {"step": s, "dt_gpu": dtg, "dt_oracle": r["dt"]}
        for k in ("x", "y", "z"):
            row[k] = _rel(got[k][fl], rr[k][fl], s0[k][fl])
        for k in ("vx", "vy", "vz", "rho"):
            row[k] = _rel(got[k][fl], rr[k][fl], 0.0 if k != "rho" else s0[k][fl])
        tg, to = oracle.totals(p, got), oracle.totals(p, rr)
        row["mass_gpu"] = float(tg[0] - tot0[0])
        row["mass_oracle"] = float(to[0] - tot0[0])
        for i, name in ((1, "px"), (2, "py"), (3, "pz")):
            row[name + "_gpu"] = float(tg[i] - tot0[i])
            row[name + "_oracle"] = float(to[i] - tot0[i])
        e0 = tot0[4] + tot0[5] + tot0[6]
        row["E_rel_gpu"] = float((tg[4] + tg[5] + tg[6] - e0) / abs(e0))
        row["E_rel_oracle"] = float((to[4] + to[5] + to[6] - e0) / abs(e0))
        rows.append(row)
        print(json.dumps(row), flush=True)
    return p, rows


def _check(rows, dt_tol):
    for row in rows:
        for k in ("x", "y", "z", "vx", "vy", "vz", "rho"):
            assert np.isfinite(row[k]) and row[k] <= DIV_BOUND, (row["step"], k, row[k])
        assert row["mass_gpu"] == 0.0 and row["mass_oracle"] == 0.0
        assert abs(row["dt_gpu"] - row["dt_oracle"]) <= dt_tol * row["dt_oracle"]
        # Energy drift of the FP32 run stays within 1e-4 of the initial
        # energy of the oracle's own drift.
        assert abs(row["E_rel_gpu"] - row["E_rel_oracle"]) <= 1e-4, row["step"]


def _save(name, rows):
    d = os.environ.get("SPH_REPORT_DIR")
    if d:
        os.makedirs(d, exist_ok=True)
        with open(os.path.join(d, name), "w") as f:
            json.dump(rows, f, indent=1)


def test_multistep_locked_dt():
    _, rows = _run(True)
    _save("multistep_c1_locked.json", rows)
    _check(rows, 0.0)


def test_multistep_free_dt():
    _, rows = _run(False)
    _save("multistep_c1_free.json", rows)
    _check(rows, 1e-4)
