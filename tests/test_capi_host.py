"""Host-side checks of the C ABI that need no GPU: the library loads, exports every entry point
declared in include/elbm.h, sizes workspaces and rejects bad parameters with error codes."""
import ctypes

import pytest

from paper_1608_04658_amd import elbm


@pytest.fixture(scope="module")
def lib():
    return elbm.load()


def test_every_declared_symbol_is_exported(lib):
    names = elbm.header_symbols()
    assert "elbm_step" in names and "elbm_create" in names and "elbm_force" in names
    for name in names:
        assert hasattr(lib, name), name


def test_struct_sizes_match_header_layout():
    # the ctypes mirrors must have the C sizes (x86-64 SysV alignment)
    assert ctypes.sizeof(elbm.Params) == 4 * 8 + 8 + 8 + 8 + 24 + 8
    assert ctypes.sizeof(elbm.Body) == 8 + 24 + 8 + 24 + 8 + 8 + 24 + 24 + 24 + 8 + 24
    assert ctypes.sizeof(elbm.Info) == 8 + 8 + 8 + 8 + 8 + 8 + 4 + 4 + 8 + 8


def test_workspace_size_counts_two_population_arrays():
    p = elbm.make_params((32, 32, 32), 1e-3)
    n = elbm.elbm_workspace_bytes(p)
    assert n >= 2 * 27 * 32 ** 3 * 4
    p16 = elbm.make_params((32, 32, 32), 1e-3, storage="f16")
    assert elbm.elbm_workspace_bytes(p16) < n
    pg = elbm.make_params((32, 32, 32), 1e-3, max_bodies=2, channel=True)
    assert elbm.elbm_workspace_bytes(pg) > n


@pytest.mark.parametrize("kw,msg", [
    (dict(shape=(0, 4, 4)), "lattice size"),
    (dict(shape=(4, 4, 4), nu=-1.0), "nu"),
    (dict(shape=(2, 4, 4), channel=True), "channel"),
    (dict(shape=(4, 4, 4), max_bodies=9), "max_bodies"),
    (dict(shape=(4, 4, 4), storage=7), "storage"),
])
def test_bad_parameters_are_rejected(kw, msg):
    shape = kw.pop("shape")
    nu = kw.pop("nu", 0.1)
    p = elbm.make_params(shape, nu, **kw)
    with pytest.raises(elbm.ElbmError, match=msg):
        elbm.elbm_workspace_bytes(p)


def test_create_rejects_small_or_misaligned_workspace(lib):
    p = elbm.make_params((8, 8, 8), 0.1)
    ctx = ctypes.c_void_p()
    n = elbm.elbm_workspace_bytes(p)
    assert lib.elbm_create(ctypes.byref(p), None, ctypes.c_void_p(256), n - 1, ctypes.byref(ctx)) == -2
    assert "needs" in elbm.elbm_last_error(None)
    assert lib.elbm_create(ctypes.byref(p), None, ctypes.c_void_p(257), n, ctypes.byref(ctx)) == -1
    assert lib.elbm_create(ctypes.byref(p), None, None, n, ctypes.byref(ctx)) == -1
