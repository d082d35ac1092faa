"""The allocation-free finishing pass (tsvd_finish_dense_noalloc) against the
finishing pass that uses the context's workspace (tsvd_finish_dense), called
through the C ABI.  Both run the same kernels on the same inputs, so W and S
must agree bit for bit; two calls in a row (the second with a smaller input)
check that the shared device scratch left by one call does not leak into the
next.  Sizes beyond the scratch array are refused."""

import ctypes

import numpy as np
import pytest

import paper_2208_08410_amd as P
import synth

pytestmark = pytest.mark.gpu


def _noalloc_fn(lib):
    fn = lib.tsvd_finish_dense_noalloc
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    fn.argtypes = [vp, vp, i32, i64, i64, i64, i32, vp, i64, i32, vp, i64, vp, vp]
    fn.restype = ctypes.c_int
    return fn


def _inputs(m, n, k, side, dtype, seed):
    import torch
    A = synth.gaussian_dense(m, n, seed=seed, dtype=dtype)
    K = n if side == "right" else m
    X = synth.start_vectors(k, K, seed=seed + 1)  # k x K row-major = K x k column-major
    return torch.from_numpy(A).cuda(), torch.from_numpy(X).cuda().T


def _noalloc(ctx, A, side, X, k):
    import torch
    m, n = A.shape
    M = m if side == "right" else n
    W = torch.full((k, M), 7.0, dtype=torch.float64, device=A.device).T
    S = torch.full((k,), 7.0, dtype=torch.float64, device=A.device)
    st = _noalloc_fn(ctx.lib)(ctx.handle, ctypes.c_void_p(A.data_ptr()), P._dtype_code(A), m, n, A.stride(0),
                              P.SIDE[side], ctypes.c_void_p(X.data_ptr()), X.stride(1), k,
                              ctypes.c_void_p(W.data_ptr()), W.stride(1), ctypes.c_void_p(S.data_ptr()),
                              P._stream(None))
    return st, W, S


@pytest.mark.parametrize("side,dtype", [("right", np.float32), ("left", np.float32), ("right", np.float64)])
def test_noalloc_finish_equals_workspace_finish(ctx, side, dtype):
    import torch
    for (m, n, k, seed) in [(5000, 700, 24, 3), (777, 300, 9, 4)]:  # second call smaller
        A, X = _inputs(m, n, k, side, dtype, seed)
        st, W, S = _noalloc(ctx, A, side, X, k)
        assert st == P.OK, ctx.last_error()
        Wr, Sr = P.tsvd_finish_dense(ctx, A, side, X, k)
        torch.cuda.synchronize()
        assert np.array_equal(S.cpu().numpy(), Sr.cpu().numpy()), (m, n, k)
        assert np.array_equal(W.cpu().numpy(), Wr.cpu().numpy()), (m, n, k)


def test_noalloc_finish_refuses_oversize(ctx):
    import torch
    # (ceil(m / 128) + 2) * k doubles: 8194 tiles x 128 columns exceeds 2^20
    m, n, k = 1_048_576, 128, 128
    A = torch.empty((m, n), dtype=torch.float32, device="cuda")
    X = torch.zeros((k, n), dtype=torch.float64, device="cuda").T
    st, W, S = _noalloc(ctx, A, "right", X, k)
    assert st == P.UNSUPPORTED
    assert "scratch" in ctx.last_error()
