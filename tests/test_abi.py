"""The C-ABI library loads and exports every entry point its headers declare (CPU only)."""
import ctypes
import glob
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1506_06039_amd", "libmoco.so")


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(moco_\w+)\s*\(", txt, re.M):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1506_06039_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for need in ("moco_create", "moco_destroy", "moco_template_create", "moco_template_destroy",
                 "moco_align", "moco_last_error"):
        assert need in names


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.check_output(["nm", "-D", "--defined-only", LIB]).decode()
    exported = {l.split()[-1] for l in out.splitlines() if l.strip()}
    for name in sorted(_declared()):
        assert name in exported, name
        assert hasattr(lib, name)


def test_version_and_error_string_without_gpu(lib):
    lib.moco_version.restype = ctypes.c_char_p
    lib.moco_last_error.restype = ctypes.c_char_p
    assert lib.moco_version().decode().startswith("moco")
    assert isinstance(lib.moco_last_error(), bytes)


def test_null_arguments_rejected_without_gpu(lib):
    lib.moco_create.argtypes = [ctypes.c_int, ctypes.c_size_t, ctypes.c_void_p]
    assert lib.moco_create(0, 0, None) == -1
    lib.moco_align.restype = ctypes.c_int
    assert lib.moco_align(None, None, None, 1, 8, 8, 2, 0, 1, 0, None, None) == -1
    lib.moco_last_error.restype = ctypes.c_char_p
    assert b"null" in lib.moco_last_error()


def test_binding_fails_loudly_without_library(tmp_path):
    # the product binding has no CPU path: without libmoco.so it refuses to import
    code = ("import sys, importlib.util; sys.path.insert(0, %r);"
            "import paper_1506_06039_amd.moco as m" % ROOT)
    env = dict(os.environ)
    # point the package at an empty copy of itself that has no library
    pkg = tmp_path / "paper_1506_06039_amd"
    pkg.mkdir()
    for f in ("__init__.py", "moco.py"):
        (pkg / f).write_text(open(os.path.join(ROOT, "paper_1506_06039_amd", f)).read())
    code = "import sys; sys.path.insert(0, %r); import paper_1506_06039_amd.moco" % str(tmp_path)
    r = subprocess.run(["python", "-c", code], capture_output=True, env=env)
    assert r.returncode != 0
    assert b"libmoco.so is not built" in r.stderr


def test_apply_rejects_bad_arguments_without_gpu(lib):
    lib.moco_apply.restype = ctypes.c_int
    lib.moco_apply.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int] * 4 + [ctypes.c_void_p] * 3
    assert lib.moco_apply(None, None, None, 1, 8, 8, 1, None, None, None) == -1   # null ctx
    lib.moco_last_error.restype = ctypes.c_char_p
    assert b"null" in lib.moco_last_error()


def test_default_params_follow_the_paper_without_gpu(lib):
    # sec. 3: downsample once iff the frame is larger than 256x256; window
    # min(m', n')/3 on the searched grid
    lib.moco_default_params.restype = ctypes.c_int
    lib.moco_default_params.argtypes = [ctypes.c_int, ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    w, ds = ctypes.c_int(), ctypes.c_int()
    for (m, n), want in [((512, 512), (85, 1)), ((256, 256), (85, 0)), ((416, 460), (69, 1)),
                         ((800, 300), (50, 1)), ((10, 4), (1, 0)), ((1, 1), (1, 0))]:
        assert lib.moco_default_params(m, n, ctypes.byref(w), ctypes.byref(ds)) == 0
        assert (w.value, ds.value) == want, (m, n)
    assert lib.moco_default_params(0, 5, ctypes.byref(w), ctypes.byref(ds)) == -1


def test_fft_bound_null_arguments_rejected_without_gpu(lib):
    lib.moco_template_fft_bound.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.moco_template_fft_bound.restype = ctypes.c_int
    assert lib.moco_template_fft_bound(None, None, None) == -1
    lib.moco_template_int8_products.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    lib.moco_template_int8_products.restype = ctypes.c_int
    assert lib.moco_template_int8_products(None, None) == -1


def test_binding_structs_match_the_header(lib, tmp_path):
    """The ctypes records of the binding have the header's sizes and field offsets."""
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "moco.h"\n'
        "int main(void) {\n"
        '  printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(moco_outputs),\n'
        "         offsetof(moco_outputs, recomputed), sizeof(moco_stack),\n"
        "         offsetof(moco_stack, out), sizeof(moco_result), offsetof(moco_result, latency_us));\n"
        "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    from paper_1506_06039_amd import moco
    want = [ctypes.sizeof(moco._Outputs), moco._Outputs.recomputed.offset,
            ctypes.sizeof(moco._Stack), moco._Stack.out.offset,
            ctypes.sizeof(moco.ServerResult), moco.ServerResult.latency_us.offset]
    assert got == want


def test_tune_table_without_gpu(lib):
    """The per-process table of tuned forms: set, get, reject AUTO, clear."""
    c_int = ctypes.c_int
    lib.moco_tune_set.argtypes = [c_int] * 6
    lib.moco_tune_get.argtypes = [c_int] * 5 + [ctypes.POINTER(c_int)]
    lib.moco_tune_clear()
    f = c_int(-7)
    try:
        assert lib.moco_tune_get(512, 512, 32, 1, 1, ctypes.byref(f)) == -1
        assert lib.moco_tune_set(512, 512, 32, 1, 1, 4) == 0
        assert lib.moco_tune_get(512, 512, 32, 1, 1, ctypes.byref(f)) == 0 and f.value == 4
        assert lib.moco_tune_get(512, 512, 32, 1, 2, ctypes.byref(f)) == -1   # other dtype
        assert lib.moco_tune_set(512, 512, 32, 1, 1, 0) == -1   # AUTO is not a concrete form
        assert lib.moco_tune_set(512, 512, 32, 1, 9, 3) == -1   # unknown dtype
        assert lib.moco_tune_set(512, 512, 32, 1, 1, 2) == 0    # replaced
        assert lib.moco_tune_get(512, 512, 32, 1, 1, ctypes.byref(f)) == 0 and f.value == 2
    finally:
        lib.moco_tune_clear()
    assert lib.moco_tune_get(512, 512, 32, 1, 1, ctypes.byref(f)) == -1


def test_tune_json_roundtrip_without_gpu(lib, tmp_path):
    from paper_1506_06039_amd import moco
    moco.tune_clear()
    try:
        moco.tune_set(256, 256, 64, 0, "f32", "fft_cert")
        moco.tune_set(512, 512, 32, 1, "u16", "int8")
        path = str(tmp_path / "tune.json")
        moco.tune_save(path, [(256, 256, 64, 0, "f32"), (512, 512, 32, 1, "u16"),
                              (128, 128, 10, 0, "f32")])
        moco.tune_clear()
        assert moco.tune_get(512, 512, 32, 1, "u16") is None
        assert moco.tune_load(path) == 2
        assert moco.tune_get(256, 256, 64, 0, "f32") == "fft_cert"
        assert moco.tune_get(512, 512, 32, 1, "u16") == "int8"
        assert moco.tune_get(128, 128, 10, 0, "f32") is None
    finally:
        moco.tune_clear()
