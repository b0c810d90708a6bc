"""The machine probes that give the measured ceilings next to the roofline:
the FMA loop computes what it claims (so its FLOP count is real) and the
streaming copy is exact."""
import numpy as np
import pytest

from paper_1210_1017_amd import sph
from parity_util import announce

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    sph.lib()
    yield
    torch.cuda.synchronize()


def _fma32(a, b, c):
    # a*b of two floats is exact in FP64; the sum rounds once in FP64 and
    # again to FP32, which can differ from one fused rounding by one ulp
    return (np.asarray(a, np.float64) * np.float64(b) + np.float64(c)).astype(np.float32)


@pytest.mark.parametrize("blocks,iters", [(1, 1), (3, 7), (2, 100)])
def test_probe_fma_values(blocks, iters):
    announce(f"probe fma blocks={blocks} iters={iters}")
    out = torch.full((blocks * 256 + 5,), -1.0, dtype=torch.float32, device="cuda")
    sph.probe_fma(out, blocks, iters)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    b, c = np.float32(0.99999988), np.float32(1e-7)
    t = np.arange(256)
    a0 = (np.float32(1e-3) * t.astype(np.float32)).astype(np.float32)
    chains = [a0] + [(a0 + np.float32(k / 8)).astype(np.float32) for k in range(1, 8)]
    for _ in range(iters):
        chains = [_fma32(ch, b, c) for ch in chains]
    a = chains
    ref = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]))
    for blk in range(blocks):
        seg = got[blk * 256:(blk + 1) * 256]
        ulp = np.spacing(np.abs(ref)).astype(np.float64)
        assert np.all(np.abs(seg.astype(np.float64) - ref) <= 8 * iters * ulp + 1e-30)
    assert np.all(got[blocks * 256:] == -1.0)  # nothing written past blocks * 256


@pytest.mark.parametrize("nfloat,blocks", [(4, 1), (262_148, 7), (1 << 22, 4096)])
def test_probe_copy_exact(nfloat, blocks):
    announce(f"probe copy n={nfloat} blocks={blocks}")
    g = torch.Generator(device="cuda").manual_seed(nfloat)
    src = torch.randn(nfloat, generator=g, device="cuda")
    dst = torch.full((nfloat + 4,), 7.0, device="cuda")
    sph.probe_copy(src, dst, blocks)
    torch.cuda.synchronize()
    assert torch.equal(dst[:nfloat], src)
    assert torch.all(dst[nfloat:] == 7.0)


def test_probe_copy_refuses_overlap():
    x = torch.zeros(64, device="cuda")
    with pytest.raises(sph.SphError):
        sph.probe_copy(x[:32], x[16:], 1)
