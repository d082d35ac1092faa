"""Whole t-SVD (tsvd_dense: Gram -> power iteration -> FP64 finish) against
the oracle and against spectra known in closed form."""

import math

import numpy as np
import pytest

import oracle as O
import paper_2208_08410_amd as P
import synth
from gpu_util import line_angle, stop_model, to_dev

pytestmark = pytest.mark.gpu


def run(ctx, A, k, eps, st, **kw):
    U, S, V, info = P.tsvd_dense(ctx, to_dev(A), k, eps, to_dev(st), **kw)
    return U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy(), info


def test_c1_plain_fp64(ctx):
    """2000 x 500 FP64, s_i = 10^(-i/100), k = 10, eps = 1e-8 (the plain method)."""
    m, n, k, eps = 2000, 500, 10, 1e-8
    dk = synth.dense_known(m, n, synth.spectrum_pow10(n), seed=1)
    st = synth.start_vectors(k, n, seed=11)
    ref = O.tsvd_gram(dk.A, eps, k, st)
    U, S, V, info = run(ctx, dk.A, k, eps, st)
    assert info["converged"] and info["k_done"] == k
    assert info["iters"] == list(ref.iters)
    assert np.allclose(S, ref.S, rtol=1e-11, atol=0)
    Ur, Vr = O.canonical(ref.U, ref.V)
    assert np.allclose(V, Vr, atol=1e-9) and np.allclose(U, Ur, atol=1e-9)
    r = 10 ** (-2 / 100)
    theta, srel = stop_model(eps, r)
    assert np.max(np.abs(S - dk.s[:k]) / dk.s[:k]) < 1e-6
    for l in range(k):
        assert line_angle(V[:, l], dk.V[:, l]) < 3 * theta


@pytest.mark.parametrize("gram", ["bf16x3", "fp32"])
def test_fp32_paths_closed_form_and_trajectory(ctx, gram):
    """Reduced C2 shape: FP32 A with s_i = 0.97^i; sigma within 1e-6 of the
    closed form, and vectors within 1e-4 rad of the FP64 oracle run for the
    same number of steps (trajectory mode)."""
    m, n, k, eps = 20000, 512, 16, 5e-8
    dk = synth.dense_known(m, n, synth.spectrum_geometric(0.97, n), seed=2, dtype=np.float32)
    st = synth.start_vectors(k, n, seed=12)
    ref = O.tsvd_gram(dk.A, eps, k, st)
    U, S, V, info = run(ctx, dk.A, k, eps, st, gram=gram)
    assert info["converged"]
    assert np.max(np.abs(S - dk.s[:k]) / dk.s[:k]) < 1e-6
    U2, S2, V2, info2 = run(ctx, dk.A, k, eps, st, gram=gram, fixed_iters=ref.iters)
    Ur, Vr = O.canonical(ref.U, ref.V)
    for l in range(k):
        assert line_angle(V2[:, l], Vr[:, l]) < 1e-4
        assert line_angle(U2[:, l], Ur[:, l]) < 1e-4
    assert np.max(np.abs(S2 - ref.S) / ref.S) < 1e-6
    assert np.linalg.norm(V.T @ V - np.eye(k)) < 1e-10


@pytest.mark.parametrize("m,n,k,branch", [(300, 1000, 6, 0), (777, 333, 7, 0), (200, 200, 5, 0), (200, 200, 5, 1),
                                          (60, 40, -1, 0), (40, 60, -1, 0), (500, 1, 1, 0), (1, 300, 1, 0)])
def test_shapes_and_branches_fp64(ctx, m, n, k, branch):
    """Ragged shapes, both branches, k = min(m, n), single row/column.  The
    stopping decision at eps = 1e-12 may flip by one step between two FP64
    Grams that differ in rounding, so iteration counts are compared to +-1 and
    results in trajectory mode (the oracle's counts imposed)."""
    d = min(m, n)
    dk = synth.dense_known(m, n, synth.spectrum_geometric(0.85, d), seed=m + n)
    kk = d if k == -1 else k
    right = (m > n) if branch == 1 else (m >= n)
    st = synth.start_vectors(kk, n if right else m, seed=5)
    ref = O.tsvd_gram(dk.A, 1e-12, k, st, branch="paper" if branch == 1 else "ge", max_iter=20000)
    U, S, V, info = run(ctx, dk.A, k, 1e-12, st, branch=branch, max_iter=20000)
    assert info["branch_right"] == right
    assert np.max(np.abs(np.array(info["iters"]) - ref.iters)) <= 1
    assert np.allclose(S, ref.S, rtol=1e-9, atol=0)
    U, S, V, info = run(ctx, dk.A, k, 1e-12, st, branch=branch, fixed_iters=ref.iters)
    assert np.allclose(S, ref.S, rtol=1e-11, atol=0)
    Ur, Vr = O.canonical(ref.U, ref.V)
    assert np.allclose(V, Vr, atol=1e-8)
    assert np.allclose(U, Ur, atol=1e-8)


def test_zero_matrix_rank_deficient(ctx):
    A = np.zeros((30, 20), dtype=np.float32)
    U, S, V, info = run(ctx, A, 3, 1e-8, synth.start_vectors(3, 20, 1), gram="bf16x3")
    assert info["k_done"] == 0 and info["rank_deficient"]
    assert np.all(S == 0) and np.all(U == 0) and np.all(V == 0)


@pytest.mark.parametrize("gram", ["bf16x3", "fp32"])
def test_rank_below_k_keeps_v_orthonormal(ctx, gram):
    """A of exact rank 3 (FP32, 1500 x 300, s = 3, 2, 1) asked for k = 6 with
    200 fixed iterations per triplet.  The first three triplets meet the
    closed form; after them the deflated Gram is at rounding level, so the
    later triplets have sigma at that level, while V stays orthonormal to
    FP64 rounding (each v is re-orthogonalised against the earlier ones and
    normalised through the gather that carries its norm) and U stays finite.
    A rank-deficiency stop after the third triplet is also a valid outcome."""
    m, n, k = 1500, 300, 6
    s = np.zeros(n)
    s[:3] = [3.0, 2.0, 1.0]
    dk = synth.dense_known(m, n, s, seed=5, dtype=np.float32)
    st = synth.start_vectors(k, n, seed=21)
    U, S, V, info = run(ctx, dk.A, k, 1e-8, st, fixed_iters=[200] * k, gram=gram)
    assert info["status"] == "TSVD_OK"
    kd = info["k_done"]
    assert kd == k or (info["rank_deficient"] and kd >= 3)
    assert np.max(np.abs(S[:3] - s[:3]) / s[:3]) < 1e-6
    assert np.all(S[3:kd] < 1e-5 * s[0])
    assert np.linalg.norm(V[:, :kd].T @ V[:, :kd] - np.eye(kd)) < 1e-10
    assert np.all(np.isfinite(U))
    for l in range(3):
        assert line_angle(V[:, l], dk.V[:, l]) < 1e-4


def test_nan_is_nonfinite(ctx):
    A = synth.gaussian_dense(100, 40, seed=1)
    A[17, 3] = np.nan
    with pytest.raises(P.TsvdError) as e:
        run(ctx, A, 2, 1e-8, synth.start_vectors(2, 40, 1))
    assert e.value.status == P.NONFINITE


def test_invalid_arguments(ctx):
    import torch
    A = to_dev(synth.gaussian_dense(50, 20, seed=1))
    st = to_dev(synth.start_vectors(3, 20, 1))
    lib = P.load_library()
    with pytest.raises(P.TsvdError) as e:
        P.tsvd_dense(ctx, A, 21, 1e-8, to_dev(synth.start_vectors(21, 20, 1)))
    assert e.value.status == P.INVALID_ARG
    o = P.TsvdOpts()
    lib.tsvd_opts_default(__import__("ctypes").byref(o))
    o.k = 0
    o.v0 = st.data_ptr()
    U = torch.zeros(50 * 3, dtype=torch.float64, device="cuda")
    S = torch.zeros(3, dtype=torch.float64, device="cuda")
    V = torch.zeros(20 * 3, dtype=torch.float64, device="cuda")
    import ctypes
    st_code = lib.tsvd_dense(ctx.handle, ctypes.c_void_p(A.data_ptr()), 0, 0, 50, 20, 20, ctypes.byref(o),
                             ctypes.c_void_p(U.data_ptr()), 50, ctypes.c_void_p(S.data_ptr()),
                             ctypes.c_void_p(V.data_ptr()), 20, None, None)
    assert st_code == P.INVALID_ARG
    o.k = 3
    st_code = lib.tsvd_dense(ctx.handle, ctypes.c_void_p(A.data_ptr()), 0, 0, 50, 20, 19, ctypes.byref(o),
                             ctypes.c_void_p(U.data_ptr()), 50, ctypes.c_void_p(S.data_ptr()),
                             ctypes.c_void_p(V.data_ptr()), 20, None, None)
    assert st_code == P.INVALID_ARG  # lda < n
    o.gram = 2  # BF16X3 needs FP32 A: an FP64 A is refused before anything runs
    st_code = lib.tsvd_dense(ctx.handle, ctypes.c_void_p(A.data_ptr()), 1, 0, 50, 20, 20, ctypes.byref(o),
                             ctypes.c_void_p(U.data_ptr()), 50, ctypes.c_void_p(S.data_ptr()),
                             ctypes.c_void_p(V.data_ptr()), 20, None, None)
    assert st_code == P.UNSUPPORTED


def test_hbm_budget(ctx):
    A = synth.gaussian_dense(1000, 200, seed=1)
    with pytest.raises(P.TsvdError) as e:
        run(ctx, A, 2, 1e-8, synth.start_vectors(2, 200, 1), hbm_budget=1024)
    assert e.value.status == P.OUT_OF_MEMORY
