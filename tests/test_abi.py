"""C-ABI contract checks that need no GPU: the library loads, exports every
function that include/sph.h declares, and rejects bad parameters before it
touches the device."""
import ctypes as C

import pytest

from paper_1210_1017_amd import cases, sph


@pytest.fixture(scope="module")
def L():
    return sph.lib()


def test_exports_every_declared_function(L):
    names = sph.header_functions()
    assert "sph_step" in names and "sph_sort_kv" in names and len(names) >= 16
    for name in names:
        assert hasattr(L, name), name


def test_abi_version_and_error_strings(L):
    assert L.sph_abi_version() == 1
    for code in (0, -1, -2, -3, -4, -5, -99):
        assert isinstance(L.sph_error_string(code), bytes)


def _create(L, p: sph.Params):
    h = C.c_void_p()
    rc = L.sph_create(C.byref(p), C.byref(h))
    return rc, L.sph_last_error(None).decode()


def _good():
    return cases.small_tank().params


@pytest.mark.parametrize("field,value", [("gamma", 5.0), ("h", 0.0), ("cfl", -1.0),
                                         ("mass", 0.0), ("rho0", 0.0)])
def test_rejects_bad_physics(L, field, value):
    p = sph.make_params(_good(), 100)
    setattr(p, field, value)
    rc, msg = _create(L, p)
    assert rc == -1 and msg


def test_rejects_bad_capacity_and_grid(L):
    p = sph.make_params(_good(), 0)
    assert _create(L, p)[0] == -1
    p = sph.make_params(_good(), 100)
    p.ncell[1] = 0
    assert _create(L, p)[0] == -1
    p = sph.make_params(_good(), 100)
    p.ncell[0], p.ncell[1], p.ncell[2] = 2048, 1024, 1024  # 2^31 cells: 31 bits > 30
    rc, msg = _create(L, p)
    assert rc == -3 and "bits" in msg
    p = sph.make_params(_good(), 100)
    p.options = 8  # unknown option bit
    assert _create(L, p)[0] == -1
    p = sph.make_params(_good(), 100, features=sph.FEATURE_CELL)
    p.options = sph.OPTION_CUBIC  # the variant paths keep the Wendland kernel
    rc, msg = _create(L, p)
    assert rc == -1 and "Wendland" in msg


def test_rejects_misaligned_slab(L):
    prm = dict(cases.small_slab().params)
    p = sph.make_params(prm, 100)
    p.ncell[0] += 1
    rc, msg = _create(L, p)
    assert rc == -1 and "slab" in msg
    p = sph.make_params(prm, 100)
    p.origin[0] += 0.1 * prm["h"]
    assert _create(L, p)[0] == -1


def test_null_arguments(L):
    assert L.sph_create(None, None) == -1
    L.sph_destroy(None)
    assert L.sph_cell_bits(None) == -1
    assert L.sph_sort(None, None, None, 0, None) == -1
    assert L.sph_step(None, None, None, 0, 0, None) == -1
    assert L.sph_get_dt(None, None, None) == -1


def test_probes_reject_bad_arguments(L):
    """The machine probes validate before any launch (fake, never dereferenced
    addresses: every call below is refused on the host)."""
    a, b = C.c_void_p(1 << 20), C.c_void_p(1 << 30)
    assert L.sph_probe_fma(None, 1, 1, None) == -1
    assert L.sph_probe_fma(a, 0, 1, None) == -1
    assert L.sph_probe_fma(a, (1 << 20) + 1, 1, None) == -1
    assert L.sph_probe_fma(a, 1, 0, None) == -1
    assert "iters" in L.sph_last_error(None).decode()
    assert L.sph_probe_copy(None, b, 16, 1, None) == -1
    assert L.sph_probe_copy(a, b, 24, 1, None) == -1                  # not a multiple of 16
    assert L.sph_probe_copy(C.c_void_p((1 << 20) + 4), b, 16, 1, None) == -1  # misaligned
    assert L.sph_probe_copy(a, C.c_void_p((1 << 20) + 64), 128, 1, None) == -1  # overlap
    assert "overlap" in L.sph_last_error(None).decode()
    assert L.sph_probe_copy(a, b, 16, 0, None) == -1
