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
