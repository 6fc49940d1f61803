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


def _c_layout(struct: str, fields):
    """sizeof and offsetof of a header struct, from a C compiler reading include/elbm.h."""
    import os
    import subprocess
    import tempfile
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    body = "".join(f'  printf("%zu\\n", offsetof({struct}, {f}));\n' for f in fields)
    src = ("#include <stddef.h>\n#include <stdio.h>\n#include \"elbm.h\"\nint main(void) {\n"
           f'  printf("%zu\\n", sizeof({struct}));\n{body}  return 0;\n}}\n')
    with tempfile.TemporaryDirectory() as d:
        c, exe = os.path.join(d, "l.c"), os.path.join(d, "l")
        with open(c, "w") as fh:
            fh.write(src)
        subprocess.run(["gcc", "-I", inc, "-o", exe, c], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    return [int(v) for v in out]


@pytest.mark.parametrize("struct,mirror", [("elbm_params", elbm.Params), ("elbm_body", elbm.Body),
                                           ("elbm_info", elbm.Info)])
def test_struct_layout_matches_header(struct, mirror):
    # the ctypes mirrors must have the C layout: size and every field offset
    names = [f[0] for f in mirror._fields_]
    got = _c_layout(struct, names)
    assert got[0] == ctypes.sizeof(mirror)
    for name, off in zip(names, got[1:]):
        assert getattr(mirror, name).offset == off, name


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
    (dict(shape=(4, 4, 4), flags=64 | 16), "CENTRAL"),
    (dict(shape=(4, 4, 4), flags=64 | 8), "CENTRAL"),
    (dict(shape=(4, 4, 4), flags=16 | 32), "EXACT_GAMMA"),
    (dict(shape=(4, 4, 4), max_bodies=1, max_mesh_vertices=10), "mesh capacity"),
    (dict(shape=(2048, 1024, 1025)), "2\\^31"),
    (dict(shape=(8192, 8192, 1)), "z plane"),
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


@pytest.mark.parametrize("kw,msg", [
    (dict(shape=(256, 256, 129)), "exceed"),
    (dict(shape=(16, 16, 16), channel=True), "periodic box without bodies"),
    (dict(shape=(16, 16, 16), max_bodies=1), "periodic box without bodies"),
    (dict(shape=(16, 16, 16), flags=1), "no body force"),
    (dict(shape=(16, 16, 16), flags=8), "no body force"),
])
def test_noalloc_step_rejects_what_it_does_not_serve(lib, kw, msg):
    # rejected on the host before any device call: no GPU needed
    shape = kw.pop("shape")
    p = elbm.make_params(shape, 0.1, **kw)
    with pytest.raises(elbm.ElbmError, match=msg):
        elbm.elbm_step_periodic_noalloc(p, 256, 1 << 40, stream=0)


def test_noalloc_step_rejects_overlap(lib):
    p = elbm.make_params((8, 8, 8), 0.1)
    with pytest.raises(elbm.ElbmError, match="overlap"):
        elbm.elbm_step_periodic_noalloc(p, 4096, 4096 + 64, stream=0)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 (or a WORLD_SIZE above 1) exits with status 2 and a
    message, before it touches a device."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, WORLD_SIZE="1")
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, env=env, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    env["WORLD_SIZE"] = "4"
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py")], capture_output=True, text=True, env=env,
                       timeout=120)
    assert r.returncode == 2 and "WORLD_SIZE=4" in r.stderr
