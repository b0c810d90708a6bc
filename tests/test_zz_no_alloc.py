"""The stable key-value radix sort entry point that allocates nothing
(sph_sort_kv_noalloc: scratch in a fixed device array of the library)
against the context's sph_sort_kv, through the C ABI: bit-exact on two calls
in a row, the second with a smaller input (the array keeps the first call's
contents), for 3- and 4-pass key widths; sizes beyond the fixed scratch and
bad arguments are refused with a message."""
import numpy as np
import pytest

from paper_1210_1017_amd import cases, sph
from parity_util import announce

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    sph.lib()
    yield
    torch.cuda.synchronize()


def _keys(n, bits, seed):
    rng = np.random.default_rng(seed)
    k = rng.integers(0, 1 << bits, size=n, dtype=np.uint64).astype(np.uint32)
    k[: n // 8] = k[n // 8: 2 * (n // 8)]  # many duplicates: stability matters
    v = rng.permutation(n).astype(np.int32)
    return torch.from_numpy(k).cuda(), torch.from_numpy(v).cuda()


@pytest.mark.parametrize("bits", [22, 32])
def test_noalloc_sort_matches_context_sort(bits):
    cap = sph.SORT_NOALLOC_MAX
    ctx = sph.Context(cases.small_tank().params, cap)
    for n, seed in ((cap, 1), (100_003, 2)):  # second call smaller
        announce(f"noalloc sort n={n} bits={bits}")
        k, v = _keys(n, bits, seed + bits)
        kr, vr = torch.empty_like(k), torch.empty_like(v)
        kg, vg = torch.full_like(k, 7), torch.full_like(v, -1)
        ctx.sort_kv(k, v, kr, vr, n, bits)
        sph.sort_kv_noalloc(k, v, kg, vg, n, bits)
        torch.cuda.synchronize()
        assert torch.equal(kg, kr) and torch.equal(vg, vr)
        ko = k.cpu().numpy()
        order = np.argsort(ko, kind="stable")
        assert np.array_equal(vg.cpu().numpy(), v.cpu().numpy()[order])


def test_noalloc_sort_limits():
    k, v = _keys(16, 8, 3)
    kg, vg = torch.empty_like(k), torch.empty_like(v)
    sph.sort_kv_noalloc(k, v, kg, vg, 0, 8)  # empty input: nothing to do
    with pytest.raises(sph.SphError, match="fixed scratch"):
        sph.sort_kv_noalloc(k, v, kg, vg, sph.SORT_NOALLOC_MAX + 1, 8)
    with pytest.raises(sph.SphError, match="key_bits"):
        sph.sort_kv_noalloc(k, v, kg, vg, 16, 0)
    with pytest.raises(sph.SphError, match="alias"):
        sph.sort_kv_noalloc(k, v, k, vg, 16, 8)
    sph.sort_kv_noalloc(k, v, kg, vg, 16, 8)
    torch.cuda.synchronize()
    order = np.argsort(k.cpu().numpy(), kind="stable")
    assert np.array_equal(vg.cpu().numpy(), v.cpu().numpy()[order])
