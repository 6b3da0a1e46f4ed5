"""C-ABI contract checks that need no GPU: the library loads, exports every
symbol include/jso.h declares, and its pure host functions behave."""
import os
import re
import subprocess

import pytest

import oracle as O
from paper_2309_15676_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "jso.h")) as f:
        src = f.read()
    return sorted(set(re.findall(r"^\s*(?:int|uint64_t|const char\*)\s+(jso_\w+)\s*\(", src,
                                 re.M)))


def test_header_and_binding_agree():
    assert _declared() == sorted(L.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = L.load()
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (jso_\w+)", out))
    assert set(_declared()) <= exported


def test_stream_key_matches_oracle():
    for seed in (0, 1, 0xDEADBEEFCAFEF00D):
        for it in (0, 1, 999, 2 ** 31):
            for tag in range(1, 9):
                assert L.jso_stream_key(seed, it, tag) == O.stream_key(seed, it, tag)


def test_null_context_errors():
    lib = L.load()
    assert lib.jso_destroy(None) == 0
    assert lib.jso_set_debug(None, 0) == L.JSO_E_INVALID
    assert lib.jso_synchronize(None) == L.JSO_E_INVALID
    assert lib.jso_grad_step(None, None, 0, None, None) == L.JSO_E_INVALID
    assert lib.jso_create(None, 0, None) == L.JSO_E_INVALID
    assert lib.jso_last_error(None) == b"null context"


def test_create_without_gpu_reports_unsupported():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import ctypes
    ctx = ctypes.c_void_p()
    rc = L.load().jso_create(ctypes.byref(ctx), 0, None)
    assert rc in (L.JSO_E_UNSUPPORTED, L.JSO_E_INVALID)
    assert not ctx.value


def test_header_constants_match_the_binding():
    with open(os.path.join(ROOT, "include", "jso.h")) as f:
        src = f.read()
    defs = dict(re.findall(r"^#define (JSO_\w+)\s+(-?\d+)\b", src, re.M))
    shared = [k for k in defs if hasattr(L, k)]
    assert len(shared) >= 40
    for k in shared:
        assert getattr(L, k) == int(defs[k]), k


def _c_layout(struct, fields):
    """sizeof and field offsets of a header struct, from the C compiler."""
    import tempfile
    body = "\n".join('  printf("%%zu\\n", offsetof(%s, %s));' % (struct, f) for f in fields)
    prog = ('#include <stddef.h>\n#include <stdio.h>\n#include "jso.h"\nint main(void) {\n'
            '  printf("%%zu\\n", sizeof(%s));\n%s\n  return 0;\n}\n' % (struct, body))
    with tempfile.TemporaryDirectory() as d:
        c, exe = os.path.join(d, "l.c"), os.path.join(d, "l")
        with open(c, "w") as f:
            f.write(prog)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    return int(out[0]), [int(x) for x in out[1:]]


@pytest.mark.parametrize("struct", ["jso_scene_desc", "jso_render_opts", "jso_step_opts",
                                    "jso_step_stats"])
def test_ctypes_structs_match_the_c_layout(struct):
    cls = getattr(L, struct)
    names = [f[0] for f in cls._fields_]
    size, offs = _c_layout(struct, names)
    assert ctypes_size(cls) == size, struct
    for name, off in zip(names, offs):
        assert getattr(cls, name).offset == off, (struct, name)


def ctypes_size(cls):
    import ctypes
    return ctypes.sizeof(cls)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run(["python", os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
