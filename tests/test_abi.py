"""The C-ABI library builds, loads and exports every symbol include/tsvd.h
declares; host-only entry points behave (CPU only, no compute calls)."""

import ctypes
import os
import re

import pytest

import paper_2208_08410_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include"))) if f.endswith(".h")]


def declared_functions():
    names = []
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(tsvd_\w+)\s*\(", text, flags=re.M):
            names.append(m.group(1))
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(P.library_path()):
        from paper_2208_08410_amd import build
        build.build()
    return ctypes.CDLL(P.library_path())


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["tsvd_ctx_create", "tsvd_ctx_destroy", "tsvd_dense", "tsvd_gram_dense", "tsvd_power_gram",
                 "tsvd_finish_dense", "tsvd_status_string", "tsvd_last_error", "tsvd_opts_default"]:
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_opts_default_matches_binding_layout(lib):
    P.load_library()
    o = P.TsvdOpts()
    lib.tsvd_opts_default(ctypes.byref(o))
    assert o.k == -1 and o.eps == 1e-8 and o.max_iter == 10000 and o.gram == 0 and o.queue_depth == 2
    assert o.rows_per_block == 0 and o.hbm_budget == 0 and o.branch == 0 and not o.v0


def test_status_strings(lib):
    lib.tsvd_status_string.restype = ctypes.c_char_p
    assert lib.tsvd_status_string(0) == b"ok"
    assert lib.tsvd_status_string(3) == b"not converged"
    assert lib.tsvd_status_string(99) == b"unknown status"


def test_no_gpu_fails_loudly(lib):
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert lib.tsvd_ctx_create(0, ctypes.byref(h)) != 0
    with pytest.raises(RuntimeError):
        P.Context(0)
