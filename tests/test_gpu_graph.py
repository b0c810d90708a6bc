"""Steps captured in a HIP graph. sph_step allocates nothing and issues no
memset (scratch comes from sph_create, counters and flags are cleared by
kernels), so a sequence of steps can be captured once and replayed; every
replay must give the bits of the same eager calls.

The step index decides the Euler/leapfrog choice of Sec. 3.3 on the host, so
a captured sequence keeps the indices it was captured with: here the Euler
step 0 runs eagerly and the graph holds two leapfrog steps (1, 2) that move
the state a -> b -> a.
"""
import numpy as np
import pytest

from paper_1210_1017_amd import cases, sph
from parity_util import announce

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

REPLAYS = 4


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    sph.lib()
    yield
    torch.cuda.synchronize()


def _start(case, n):
    ctx = sph.Context(case.params, n)
    a = sph.DeviceState.from_numpy(case.state, capacity=n)
    b = sph.DeviceState.empty(n)
    ctx.step(a, b, n, 0)  # Euler step, eager
    return ctx, b, a      # the state after step 0 is in b


def _same_bits(got, ref):
    for k in ref:
        g, r = got[k], ref[k]
        if g.dtype == np.float32:
            g, r = g.view(np.uint32), r.view(np.uint32)
        assert np.array_equal(g, r), k


@pytest.mark.parametrize("options", [0, sph.OPTION_SYMPLECTIC | sph.OPTION_CUBIC])
def test_step_graph_replays_match_eager(options):
    case = cases.perturb(cases.case_c1(), 6)
    case.params["options"] = options
    n = case.n
    announce(f"graph replay options={options} n={n}")

    ctx_e, a, b = _start(case, n)
    eager = []
    for _ in range(REPLAYS):
        ctx_e.step(a, b, n, 1)
        ctx_e.step(b, a, n, 2)
        torch.cuda.synchronize()
        eager.append((a.to_numpy(n), ctx_e.pairs(), ctx_e.dt(), ctx_e.counts()["n_label"]))

    ctx_g, a2, b2 = _start(case, n)
    torch.cuda.synchronize()
    before = a2.to_numpy(n)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(g, stream=s, capture_error_mode="relaxed"):
        ctx_g.step(a2, b2, n, 1, stream=s)
        ctx_g.step(b2, a2, n, 2, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    # capturing runs nothing
    _same_bits(a2.to_numpy(n), before)

    for r in range(REPLAYS):
        g.replay()
        torch.cuda.synchronize()
        # eager work between the replays: readbacks on the current stream
        got = a2.to_numpy(n)
        ref, pairs, dt, n_label = eager[r]
        _same_bits(got, ref)
        assert ctx_g.pairs() == pairs
        assert ctx_g.dt() == dt
        assert ctx_g.counts()["n_label"] == n_label
        assert ctx_g.status() & (sph.STATUS_NONFINITE | sph.STATUS_DT) == 0
    del g


def test_first_nn_advance_captured_in_graph():
    """A context created with SPH_F_SURROGATE holds every buffer of
    sph_nn_advance from sph_create on, so its very first call can be captured:
    the replays of that capture give the bits of an eager advance from the
    same state (each replay starts from the same cur, as the eager call did).
    Without the feature the advance is refused and allocates nothing."""
    from test_gpu_surrogate import _random_net, _scales

    case = cases.perturb(cases.case_c1(), 6)
    p, n = case.params, case.n
    announce(f"graph capture of the first nn_advance n={n}")
    net, _ = _random_net(128, 64, 23, out_gain=20.0)
    sc = _scales(p)
    dv, dr, dt4 = np.float32(0.02), np.float32(2.0), np.float32(4e-4)

    plain = sph.Context(p, n)
    plain.mlp_sync(net)
    cur0 = sph.DeviceState.from_numpy(case.state, capacity=n)
    out0 = sph.DeviceState.empty(n)
    with pytest.raises(RuntimeError, match="SPH_F_SURROGATE"):
        plain.nn_advance(net, cur0, out0, n, sc, dv, dr, dt4, 1.0)
    del plain

    ctx_e = sph.Context(p, n, sph.FEATURE_SURROGATE)
    ctx_e.mlp_sync(net)
    ctx_e.nn_advance(net, cur0, out0, n, sc, dv, dr, dt4, 1.0)
    torch.cuda.synchronize()
    ref = out0.to_numpy(n)
    ref_status = ctx_e.status()

    ctx_g = sph.Context(p, n, sph.FEATURE_SURROGATE)
    ctx_g.mlp_sync(net)
    cur = sph.DeviceState.from_numpy(case.state, capacity=n)
    out = sph.DeviceState.empty(n)
    torch.cuda.synchronize()
    before = out.to_numpy(n)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(g, stream=s, capture_error_mode="relaxed"):
        ctx_g.nn_advance(net, cur, out, n, sc, dv, dr, dt4, 1.0, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    _same_bits(out.to_numpy(n), before)  # capturing runs nothing
    for _ in range(REPLAYS):
        g.replay()
        torch.cuda.synchronize()
        _same_bits(out.to_numpy(n), ref)
        assert ctx_g.status() == ref_status
    del g
