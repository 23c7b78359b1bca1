"""The C ABI library loads and exports every entry point include/hydro.h
declares; host-only entry points behave as documented (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1511_02137_amd import hydro as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "hydro.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hydro_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(H.LIB_PATH):
        from paper_1511_02137_amd import build
        build.build()
    return H.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert "hydro_rk3_step" in names and "hydro_init" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(H.EXPORTED) <= set(names)


def test_struct_layout_matches_the_c_compiler(tmp_path):
    # Compile the header with gcc and compare every field offset with ctypes.
    checks = []
    for cname, pyt in (("hydro_config", H.Config), ("hydro_jet", H.JetC), ("hydro_freezeout_params", H.FreezeoutParams)):
        checks.append((cname, "sizeof", ctypes.sizeof(pyt)))
        for fname, _ in pyt._fields_:
            checks.append((cname, fname, getattr(pyt, fname).offset))
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "hydro.h"', "int main(void) {"]
    for cname, fname, _ in checks:
        expr = "sizeof(%s)" % cname if fname == "sizeof" else "offsetof(%s, %s)" % (cname, fname)
        lines.append('  printf("%%zu\\n", (size_t)(%s));' % expr)
    lines.append("  return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    assert got == [c[2] for c in checks]


def test_default_config(lib):
    c = H.Config()
    lib.hydro_default_config(ctypes.byref(c))
    assert list(c.n) == [256, 256, 256]
    assert list(c.dx) == [0.1, 0.1, 0.1]
    assert c.dt == 0.02 and c.t0 == 1.0
    assert c.weno == 0 and c.weno_p == 2 and c.weno_eps == 1e-6
    assert c.eos_dof == 47.5 and c.hbarc == 0.1973269804


def test_workspace_bytes(lib):
    c = H.make_config((32, 32, 32))
    b64 = H.workspace_bytes(c)
    assert b64 >= 15 * 32 ** 3 * 8
    c32 = H.make_config((32, 32, 32), precision="f32")
    assert H.workspace_bytes(c32) < b64
    bad = H.make_config((32, 32, 32))
    bad.dt = -1.0
    assert H.workspace_bytes(bad) == 0
    bad = H.make_config((2000, 4, 4))
    assert H.workspace_bytes(bad) == 0


@pytest.mark.parametrize("field,value", [("dt", 0.0), ("weno", 7), ("deposit", 3), ("weno_p", 3),
                                         ("precision", 5), ("weno_eps", 0.0), ("weno_eps", 1e-40),
                                         ("weno_eps", float("inf")), ("f32_weno_eps", 1e-13)])
def test_init_rejects_bad_config_without_side_effects(lib, field, value):
    # weno_eps below 1e-30 (FP64) or 1e-12 (FP32): the weights' common
    # denominator (a product of four squared indicators) would leave the
    # normal range, or tau / b squared would overflow FP32
    c = H.make_config((16, 16, 16), precision="f32" if field.startswith("f32_") else "f64")
    setattr(c, field.replace("f32_", ""), value)
    h = ctypes.c_void_p(123)
    rc = lib.hydro_init(ctypes.byref(c), None, ctypes.c_void_p(1), ctypes.c_void_p(256), 1 << 30, None,
                        ctypes.byref(h))
    assert rc == H.HYDRO_EINVAL
    assert h.value is None
    assert lib.hydro_last_error(None)


def test_init_rejects_small_or_misaligned_workspace(lib):
    c = H.make_config((16, 16, 16))
    h = ctypes.c_void_p()
    need = H.workspace_bytes(c)
    assert lib.hydro_init(ctypes.byref(c), None, ctypes.c_void_p(256), ctypes.c_void_p(512), need - 1, None,
                          ctypes.byref(h)) == H.HYDRO_EINVAL
    assert b"small" in lib.hydro_last_error(None)
    assert lib.hydro_init(ctypes.byref(c), None, ctypes.c_void_p(256), ctypes.c_void_p(520), need, None,
                          ctypes.byref(h)) == H.HYDRO_EINVAL
    assert b"aligned" in lib.hydro_last_error(None)


def test_null_context_is_rejected(lib):
    assert lib.hydro_rk3_step(None, ctypes.c_void_p(256), 1, None) == H.HYDRO_EINVAL
    assert lib.hydro_add_jet(None, None, None) == H.HYDRO_EINVAL
    lib.hydro_destroy(None)


def test_product_fails_loudly_without_library_or_gpu(tmp_path):
    """No fallback: a missing libhydro.so raises, and so does a context
    without a GPU (checked in fresh interpreters; the second check only
    where torch sees no GPU)."""
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("from paper_1511_02137_amd import hydro as H\n"
            "try:\n    H.load_library(%r)\nexcept RuntimeError as e:\n    print('raised', e)\n" % str(tmp_path / "none.so"))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=300)
    assert "raised libhydro.so is not built" in r.stdout, r.stdout + r.stderr
    code = ("import torch\nfrom paper_1511_02137_amd import hydro as H\n"
            "if torch.cuda.is_available():\n    print('gpu present')\nelse:\n"
            "    try:\n        H.Hydro(H.make_config((8, 8, 8)), None)\n"
            "    except RuntimeError as e:\n        print('raised', e)\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=300)
    assert "gpu present" in r.stdout or "raised libhydro needs a GPU" in r.stdout, r.stdout + r.stderr


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), ([], {"WORLD_SIZE": "2"})])
def test_bench_refuses_more_than_one_gpu(argv, env):
    """bench.py measures one GPU: asked for more (flag or a launcher's
    WORLD_SIZE) it exits with status 2 and says so, before touching a GPU."""
    e = dict(os.environ, **env)
    r = subprocess.run(["python3", os.path.join(ROOT, "bench.py")] + argv, capture_output=True, text=True,
                       env=e, timeout=120)
    assert r.returncode == 2
    assert "measures one GPU" in r.stderr and r.stdout == ""
