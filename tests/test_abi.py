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


LAYOUT_C = r"""
#include <stddef.h>
#include <stdio.h>
#include "tsvd.h"
#define F(T, f) printf("%s.%s %zu %zu\n", #T, #f, offsetof(T, f), sizeof(((T*)0)->f));
#define Z(T) printf("%s.sizeof %zu 0\n", #T, sizeof(T));
int main(void) {
  F(tsvd_opts, k) F(tsvd_opts, eps) F(tsvd_opts, max_iter) F(tsvd_opts, fixed_iters) F(tsvd_opts, v0)
  F(tsvd_opts, gram) F(tsvd_opts, rows_per_block) F(tsvd_opts, hbm_budget) F(tsvd_opts, branch)
  F(tsvd_opts, queue_depth) F(tsvd_opts, method) F(tsvd_opts, factor_loc) F(tsvd_opts, factor_batches)
  Z(tsvd_opts)
  F(tsvd_tuning, gram_tile) F(tsvd_tuning, gram_chunks) F(tsvd_tuning, power_blocks) F(tsvd_tuning, team_kib)
  F(tsvd_tuning, group_kchunk) F(tsvd_tuning, sparse_row_bits) F(tsvd_tuning, sparse_col_bits) F(tsvd_tuning, power_path)
  F(tsvd_tuning, group_tile) F(tsvd_tuning, group_kchunk_cls)
  Z(tsvd_tuning)
  F(tsvd_info, k_done) F(tsvd_info, iters) F(tsvd_info, lambda) F(tsvd_info, t_gram_ms) F(tsvd_info, h2d_bytes) F(tsvd_info, latency_ms)
  F(tsvd_info, t_stream_copy_ms) F(tsvd_info, t_stream_compute_ms) F(tsvd_info, t_stream_overlap_ms)
  Z(tsvd_info)
  F(tsvd_problem, A) F(tsvd_problem, dtype) F(tsvd_problem, m) F(tsvd_problem, lda) F(tsvd_problem, opts)
  F(tsvd_problem, U) F(tsvd_problem, ldu) F(tsvd_problem, S) F(tsvd_problem, V) F(tsvd_problem, ldv)
  Z(tsvd_problem)
  F(tsvd_server_config, hbm_budget) F(tsvd_server_config, max_slots) F(tsvd_server_config, max_batch)
  F(tsvd_server_config, lanes)
  Z(tsvd_server_config)
  F(tsvd_server_stats, submitted) F(tsvd_server_stats, batches) F(tsvd_server_stats, mean_batch)
  F(tsvd_server_stats, p50_ms) F(tsvd_server_stats, max_ms) F(tsvd_server_stats, peak_bytes)
  F(tsvd_server_stats, waiting) F(tsvd_server_stats, lanes_busy_max) F(tsvd_server_stats, overlapped)
  Z(tsvd_server_stats)
  return 0;
}
"""


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of the public structs have the C compiler's offsets
    and sizes (host gcc on the same header)."""
    import shutil
    import subprocess
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    src = tmp_path / "layout.c"
    src.write_text(LAYOUT_C)
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    mirrors = {"tsvd_opts": P.TsvdOpts, "tsvd_tuning": P.TsvdTuning, "tsvd_info": P.TsvdInfo,
               "tsvd_problem": P.TsvdProblem, "tsvd_server_config": P.TsvdServerConfig,
               "tsvd_server_stats": P.TsvdServerStats}
    rename = {"lambda": "lambda_"}
    checked = 0
    for line in out:
        if not line.strip():
            continue
        name, off, size = line.split()
        sname, field = name.split(".")
        cls = mirrors[sname]
        if field == "sizeof":
            assert ctypes.sizeof(cls) == int(off), sname
        else:
            desc = getattr(cls, rename.get(field, field))
            assert (desc.offset, desc.size) == (int(off), int(size)), name
        checked += 1
    assert checked >= 40


def test_gram_class_boundaries():
    """Gram-dimension classes of the batched Gram's unit shapes: 0 up to 128,
    then one per power of two, the last class open-ended."""
    assert P.GRAM_CLASSES == 8
    cases = {1: 0, 128: 0, 129: 1, 256: 1, 257: 2, 512: 2, 1024: 3, 1025: 4, 4096: 5, 8192: 6, 8193: 7, 10**6: 7}
    for d, c in cases.items():
        assert P.gram_class(d) == c, d
