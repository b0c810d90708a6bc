"""Checkpoint file format (no GPU): the arrays of a state, the next step
index and the parameters survive a save/load round trip bit for bit, and a
damaged or foreign file is refused."""
import numpy as np
import pytest

from paper_1210_1017_amd import cases, checkpoint, sph


def _cpu_state(case):
    return sph.DeviceState.from_numpy(case.state, capacity=case.n + 5, device="cpu")


def test_round_trip_bit_exact(tmp_path):
    case = cases.perturb(cases.small_slab(), 3)
    st = _cpu_state(case)
    path = tmp_path / "ck.npz"
    checkpoint.save(path, st, case.n, 41, case.params)
    arrays, n, step, params = checkpoint.load_arrays(path)
    assert n == case.n and step == 41
    for k in sph.SOA_FIELDS:
        a, b = arrays[k], case.state[k]
        assert a.dtype == b.dtype
        assert np.array_equal(a.view(np.uint8), np.ascontiguousarray(b).view(np.uint8)), k
    # parameters: same values (tuples come back as lists)
    for k, v in case.params.items():
        assert np.allclose(np.asarray(params[k], dtype=float), np.asarray(v, dtype=float),
                           rtol=0, atol=0), k
    # the parameters rebuild the same ABI structure
    a, b = sph.make_params(params, n), sph.make_params(case.params, n)
    assert bytes(a) == bytes(b)
    ds, n2, s2, _ = checkpoint.load(path, capacity=n + 10, device="cpu")
    assert n2 == n and s2 == 41 and ds.t["x"].shape[0] == n + 10
    assert np.array_equal(ds.t["rho"][:n].numpy(), case.state["rho"])


def test_refuses_damaged_files(tmp_path):
    case = cases.small_tank()
    st = _cpu_state(case)
    good = tmp_path / "good.npz"
    checkpoint.save(good, st, case.n, 0, case.params)
    arrays, n, _, _ = checkpoint.load_arrays(good)
    bad = tmp_path / "short.npz"
    np.savez(bad, header=np.load(good)["header"],
             **{k: (v[:-1] if k == "rho" else v) for k, v in arrays.items()})
    with pytest.raises(ValueError, match="rho"):
        checkpoint.load_arrays(bad)
    bad2 = tmp_path / "dtype.npz"
    np.savez(bad2, header=np.load(good)["header"],
             **{k: (v.astype(np.float64) if k == "x" else v) for k, v in arrays.items()})
    with pytest.raises(ValueError, match="x"):
        checkpoint.load_arrays(bad2)
    bad3 = tmp_path / "foreign.npz"
    np.savez(bad3, x=arrays["x"])
    with pytest.raises(ValueError, match="header"):
        checkpoint.load_arrays(bad3)
    with pytest.raises(ValueError, match="capacity"):
        checkpoint.load(good, capacity=n - 1, device="cpu")
