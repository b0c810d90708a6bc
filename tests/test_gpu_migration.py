"""Repeated migration on a slab (Sec. 4.2-4.3), through the C ABI: before
each step the injector moves fluid particles across both faces, the sort of
that state (keys with migration labels, stable order, tables, counts and the
seven packing ranges) is bit-exact with the oracle's, the step runs, and the
outgoing ranges are wrapped back through the opposite faces; the particle
count stays exact over every step."""
import numpy as np
import pytest

import oracle
from paper_1210_1017_amd import cases, migration, sph
from parity_util import announce, assert_sorted_equal

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

STEPS = 12
NMIG = 10


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    sph.lib()
    yield
    torch.cuda.synchronize()


def test_repeated_migration_packing_and_count():
    case = cases.perturb(cases.small_slab(), 8)
    p, n = case.params, case.n
    announce(f"repeated migration small slab n={n}, {STEPS} steps, {NMIG} per face")
    ctx = sph.Context(p, n)
    a = sph.DeviceState.from_numpy(case.state, capacity=n)
    b = sph.DeviceState.empty(n)
    srt_buf = sph.DeviceState.empty(n)
    total_out = 0
    for s in range(STEPS):
        migration.inject(a, n, p, s, NMIG)
        torch.cuda.synchronize()
        host = a.to_numpy(n)
        # the sort of the injected state against the oracle's
        ctx.sort(a, srt_buf, n)
        c = ctx.counts()
        ref = oracle.sort_state(p, host)
        assert_sorted_equal(srt_buf.to_numpy(n), ref, n)
        assert c["n_label"] == [int(v) for v in ref["counts"]]
        got_ranges = [c[k] for k in ("halo_lo", "edge_lo", "edge_hi", "halo_hi", "out_lo",
                                     "out_hi", "excluded")]
        assert np.array_equal(np.asarray(got_ranges).ravel(), np.asarray(ref["ranges"]).ravel())
        assert c["n_label"][1] >= NMIG and c["n_label"][2] >= NMIG and c["n_label"][3] == 0
        assert sum(c["n_label"]) == n
        # the step (same sort inside), then the outgoing ranges wrapped back
        ctx.step(a, b, n, s)
        c2 = ctx.counts()
        assert c2 == c
        total_out += migration.wrap(b, c2, p)
        torch.cuda.synchronize()
        a, b = b, a
    assert total_out >= 2 * NMIG * STEPS
    assert ctx.status() & (sph.STATUS_NONFINITE | sph.STATUS_DT | sph.STATUS_EXCLUDED) == 0
    # every particle is still there, once
    ids = np.sort(a.t["id"][:n].cpu().numpy())
    assert np.array_equal(ids, np.arange(n))
