"""Resume from a checkpoint (GPU): 2N steps in one go equal N steps, a save,
a load into a new context and N more steps, bit for bit (every array of the
state, and the pair count and dt of the last step). N = 30 puts the periodic
Euler step of the Verlet scheme (every 40 steps, Sec. 3.3) in the resumed
half."""
import numpy as np
import pytest

from paper_1210_1017_amd import cases, checkpoint, sph
from parity_util import announce

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N = 30


def _run(ctx, a, b, n, s0, k):
    for s in range(s0, s0 + k):
        ctx.step(a, b, n, s)
        a, b = b, a
    torch.cuda.synchronize()
    return a, b


@pytest.mark.parametrize("name,make", [
    ("c1_developed", lambda: cases.perturb(cases.case_c1(), 6)),
    ("slab", lambda: cases.perturb(cases.small_slab(), 7)),
])
def test_resume_bit_identical(tmp_path, name, make):
    case = make()
    p, n = case.params, case.n
    announce(f"checkpoint resume {name} n={n}")
    ctx = sph.Context(p, n)
    a = sph.DeviceState.from_numpy(case.state, capacity=n)
    b = sph.DeviceState.empty(n)
    a, b = _run(ctx, a, b, n, 0, 2 * N)
    ref = a.to_numpy(n)
    ref_pairs, ref_dt = ctx.pairs(), ctx.dt()
    del ctx, a, b

    ctx1 = sph.Context(p, n)
    a = sph.DeviceState.from_numpy(case.state, capacity=n)
    b = sph.DeviceState.empty(n)
    a, b = _run(ctx1, a, b, n, 0, N)
    path = tmp_path / f"{name}.npz"
    checkpoint.save(path, a, n, N, p)
    del ctx1, a, b

    a, n2, s0, p2 = checkpoint.load(path)
    assert n2 == n and s0 == N
    ctx2 = sph.Context(p2, n)
    b = sph.DeviceState.empty(n)
    a, b = _run(ctx2, a, b, n, s0, N)
    got = a.to_numpy(n)
    for k in sph.SOA_FIELDS:
        assert np.array_equal(got[k].view(np.uint8), ref[k].view(np.uint8)), k
    assert ctx2.pairs() == ref_pairs and ctx2.dt() == ref_dt
    assert ctx2.status() & (sph.STATUS_NONFINITE | sph.STATUS_DT) == 0
