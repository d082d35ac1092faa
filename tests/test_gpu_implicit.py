"""The power paths whose Gram is not held on chip, against the FP64 oracle:

* the dense product applied implicitly, A^T (A x) every iteration (Equation 2
  evaluated right to left, no Gram), with A in HBM or streamed from pinned
  host memory once per iteration;
* an explicit Gram in HBM iterated by HBM-streamed B x products (the path for
  iterates the on-chip kernel cannot hold), forced at small sizes through the
  tuning and taken by itself at n = 40,000;
* the iterated factor kept in pinned host memory and batched to the device
  for every projection (the paper's out-of-memory handling of the heavy
  co-factor, Sec. V-C): bitwise equal to the device-resident factor.
"""

import numpy as np
import pytest

import oracle as O
import paper_2208_08410_amd as P
import synth
from gpu_util import line_angle, to_dev

pytestmark = pytest.mark.gpu


def compare(ref, U, S, V, k, s_rtol, ang):
    S = S.cpu().numpy()
    U = U.cpu().numpy()
    V = V.cpu().numpy()
    assert np.allclose(S[:k], ref.S[:k], rtol=s_rtol, atol=0), (S[:k], ref.S[:k])
    Ur, Vr = O.canonical(ref.U, ref.V)
    worst = 0.0
    for l in range(k):
        worst = max(worst, line_angle(V[:, l], Vr[:, l]), line_angle(U[:, l], Ur[:, l]))
    assert worst < ang, worst
    return worst


@pytest.mark.parametrize("m,n,dt", [(3000, 700, np.float64), (700, 2500, np.float64), (5000, 900, np.float32),
                                    (900, 3000, np.float32), (4097, 4097, np.float32)])
def test_dense_implicit_vs_oracle(ctx, m, n, dt):
    """Trajectory mode (the oracle's iteration counts imposed): FP64 A agrees
    to rounding; FP32 A rounds the iterate to FP32 for the first product."""
    k = 5
    r = min(m, n)
    dk = synth.dense_known(m, n, synth.spectrum_geometric(0.9, r), seed=m + n, dtype=dt)
    d = n if m >= n else m
    st = synth.start_vectors(k, d, seed=3)
    A64 = dk.A.astype(np.float64)
    ref = O.tsvd_implicit(lambda x: A64 @ x, lambda y: A64.T @ y, (m, n), 1e-10, k, st)
    U, S, V, info = P.tsvd_dense(ctx, to_dev(dk.A), k, 1e-10, to_dev(st), fixed_iters=ref.iters, method="implicit")
    assert info["t_gram_ms"] == 0.0 and info["k_done"] == k
    assert info["iters"] == list(ref.iters)
    if dt == np.float64:
        compare(ref, U, S, V, k, 1e-11, 1e-8)
    else:
        compare(ref, U, S, V, k, 1e-8, 1e-5)


def test_dense_implicit_eps_mode_closed_form(ctx):
    """eps mode on a C2-shaped matrix: every sigma within 1e-6 of the closed form."""
    m, n, k = 20000, 512, 8
    s = synth.spectrum_geometric(0.97, n)
    dk = synth.dense_known(m, n, s, seed=21, dtype=np.float32)
    st = synth.start_vectors(k, n, seed=22)
    U, S, V, info = P.tsvd_dense(ctx, to_dev(dk.A), k, 5e-8, to_dev(st), method="implicit")
    assert info["converged"]
    S = S.cpu().numpy()
    assert np.max(np.abs(S - s[:k]) / s[:k]) < 1e-6


@pytest.mark.parametrize("qd,rows", [(1, 700), (2, 700), (3, 1000)])
def test_pinned_implicit_vs_oracle(ctx, qd, rows):
    """A in pinned host memory, streamed once per iteration in several row
    batches (ragged last batch) through queue_depth device buffers."""
    import torch
    m, n, k = 4500, 600, 4
    dk = synth.dense_known(m, n, synth.spectrum_geometric(0.9, n), seed=31, dtype=np.float32)
    st = synth.start_vectors(k, n, seed=32)
    A64 = dk.A.astype(np.float64)
    ref = O.tsvd_implicit(lambda x: A64 @ x, lambda y: A64.T @ y, (m, n), 1e-10, k, st)
    Ah = torch.from_numpy(dk.A).pin_memory()
    U, S, V, info = P.tsvd_dense(ctx, Ah, k, 1e-10, to_dev(st), fixed_iters=ref.iters, method="implicit",
                                 rows_per_block=rows, queue_depth=qd)
    it = int(np.sum(ref.iters))
    # one pass over A per iteration plus the finishing pass
    assert info["h2d_bytes"] == m * n * 4 * (it + 1)
    compare(ref, U, S, V, k, 1e-8, 1e-5)
    # the device-resident implicit path: the same t = A x rows, slab partials cut differently
    Ud, Sd, Vd, _ = P.tsvd_dense(ctx, to_dev(dk.A), k, 1e-10, to_dev(st), fixed_iters=ref.iters, method="implicit")
    assert np.allclose(S.cpu().numpy(), Sd.cpu().numpy(), rtol=1e-12)


@pytest.mark.parametrize("qd,cols", [(1, 700), (2, 700), (3, 1000)])
def test_pinned_implicit_left_branch_vs_oracle(ctx, qd, cols):
    """m < n with A in pinned host memory: streamed once per iteration in
    pitched column batches (ragged last batch), z = sum_c A_c (A_c^T u),
    against the oracle's left branch (Eq. 3); the same run on the
    device-resident A agrees to rounding."""
    import torch
    m, n, k = 600, 4500, 4
    dk = synth.dense_known(m, n, synth.spectrum_geometric(0.9, m), seed=33, dtype=np.float32)
    st = synth.start_vectors(k, m, seed=34)
    A64 = dk.A.astype(np.float64)
    ref = O.tsvd_implicit(lambda x: A64 @ x, lambda y: A64.T @ y, (m, n), 1e-10, k, st)
    Ah = torch.from_numpy(dk.A).pin_memory()
    U, S, V, info = P.tsvd_dense(ctx, Ah, k, 1e-10, to_dev(st), fixed_iters=ref.iters, method="implicit",
                                 rows_per_block=cols, queue_depth=qd)
    assert not info["branch_right"]
    it = int(np.sum(ref.iters))
    assert info["h2d_bytes"] == m * n * 4 * (it + 1)
    compare(ref, U, S, V, k, 1e-8, 1e-5)
    Ud, Sd, Vd, _ = P.tsvd_dense(ctx, to_dev(dk.A), k, 1e-10, to_dev(st), fixed_iters=ref.iters, method="implicit")
    assert np.allclose(S.cpu().numpy(), Sd.cpu().numpy(), rtol=1e-12)


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_gram_loop_power_vs_oracle(ctx, dt):
    """tsvd_power_gram on the host-driven loop (B streamed from HBM per
    iteration, deflation by projection) against Algorithm 2 on the same B."""
    import torch
    d, k = 1500, 6
    dk = synth.dense_known(3000, d, synth.spectrum_geometric(0.9, d), seed=41)
    B64 = dk.A.T @ dk.A
    B = B64.astype(dt)
    st = synth.start_vectors(k, d, seed=42)
    Bt = B.astype(np.float64)
    ref = O.tsvd_gram(np.eye(d), 1e-11, k, st, B0=Bt)  # A = I: the finishing step returns the vectors
    P.set_tuning(ctx, power_path=1)
    try:
        X, info = P.tsvd_power_gram(ctx, to_dev(B), k, 1e-11, to_dev(st), fixed_iters=ref.iters)
    finally:
        P.set_tuning(ctx)
    assert info["iters"] == list(ref.iters)
    X = X.cpu().numpy()
    tol = 1e-9 if dt == np.float64 else 1e-4
    for l in range(k):
        assert line_angle(X[:, l], ref.V[:, l]) < tol
    lam = np.array(info["lambda"])
    assert np.allclose(lam, ref.lam, rtol=1e-12 if dt == np.float64 else 1e-6)


def test_gram_loop_dense_matches_onchip(ctx):
    """The whole dense t-SVD with the power phase forced onto the loop agrees
    with the on-chip kernel and with the oracle (same Gram, same iterations)."""
    m, n, k = 20000, 512, 8
    s = synth.spectrum_geometric(0.97, n)
    dk = synth.dense_known(m, n, s, seed=51, dtype=np.float32)
    st = synth.start_vectors(k, n, seed=52)
    ref = O.tsvd_gram(dk.A.astype(np.float64), 5e-8, k, st)
    U0, S0, V0, i0 = P.tsvd_dense(ctx, to_dev(dk.A), k, 5e-8, to_dev(st), fixed_iters=ref.iters, gram="fp32")
    P.set_tuning(ctx, power_path=1)
    try:
        U1, S1, V1, i1 = P.tsvd_dense(ctx, to_dev(dk.A), k, 5e-8, to_dev(st), fixed_iters=ref.iters, gram="fp32")
    finally:
        P.set_tuning(ctx)
    assert i1["iters"] == list(ref.iters)
    compare(ref, U1, S1, V1, k, 1e-6, 1e-4)
    V0 = V0.cpu().numpy(); V1 = V1.cpu().numpy()
    for l in range(k):
        assert line_angle(V0[:, l], V1[:, l]) < 1e-4


def test_large_gram_beyond_onchip(ctx):
    """n = 40,000: the iterate exceeds what the on-chip power kernel holds, so
    the Gram (6.4 GB in HBM) is iterated by the streamed loop; the implicit
    product on the same A agrees.  A = H_L [diag(0.9^i); 0] H_R (Householder
    factors), so sigma is known in closed form."""
    import torch
    m, n, k = 48000, 40000, 4
    s = synth.spectrum_geometric(0.9, n)
    print(f"[large] building A {m}x{n}", flush=True)
    A = synth.householder_known_torch(m, n, s, seed=61, device=torch.device("cuda:0"))
    st = synth.start_vectors(k, n, seed=62)
    print("[large] gram route", flush=True)
    U, S, V, info = P.tsvd_dense(ctx, A, k, 1e-10, to_dev(st), gram="bf16x3")
    assert info["t_gram_ms"] > 0 and info["converged"]
    Sg = S.cpu().numpy()
    assert np.max(np.abs(Sg - s[:k]) / s[:k]) < 1e-6
    Vg = V.cpu().numpy()
    assert np.linalg.norm(Vg.T @ Vg - np.eye(k)) < 1e-10
    print("[large] implicit route", flush=True)
    Ui, Si, Vi, info_i = P.tsvd_dense(ctx, A, k, 1e-10, to_dev(st), method="implicit")
    assert info_i["t_gram_ms"] == 0.0
    assert np.max(np.abs(Si.cpu().numpy() - s[:k]) / s[:k]) < 1e-6
    Vi = Vi.cpu().numpy()
    for l in range(k):
        assert line_angle(Vg[:, l], Vi[:, l]) < 1e-4
    # residual of each triplet of the Gram route against A itself, in FP64:
    # ||A v - sigma u|| / sigma (the finishing step's u = A v / sigma)
    A64 = A.double()
    del A
    R = A64 @ V - U * S
    assert float(torch.max(torch.linalg.norm(R, dim=0) / S)) < 1e-9
    del A64, R


def test_auto_falls_back_to_implicit(ctx):
    """method AUTO under an hbm_budget too small for the Gram route takes the
    implicit product and still meets the oracle."""
    m, n, k = 6000, 1200, 4
    dk = synth.dense_known(m, n, synth.spectrum_geometric(0.9, n), seed=71, dtype=np.float32)
    st = synth.start_vectors(k, n, seed=72)
    A64 = dk.A.astype(np.float64)
    ref = O.tsvd_implicit(lambda x: A64 @ x, lambda y: A64.T @ y, (m, n), 1e-10, k, st)
    budget = 4 * n * n  # less than the Gram alone
    U, S, V, info = P.tsvd_dense(ctx, to_dev(dk.A), k, 1e-10, to_dev(st), fixed_iters=ref.iters, hbm_budget=budget)
    assert info["t_gram_ms"] == 0.0 and info["workspace_bytes"] <= budget
    compare(ref, U, S, V, k, 1e-8, 1e-5)
    with pytest.raises(P.TsvdError, match="OUT_OF_MEMORY"):
        P.tsvd_dense(ctx, to_dev(dk.A), k, 1e-10, to_dev(st), hbm_budget=budget, method="gram")


@pytest.mark.parametrize("nb,qd", [(1, 1), (3, 1), (3, 2), (5, 8)])
def test_host_factor_sparse_bitwise(ctx, nb, qd):
    """Sparse t-SVD with V in pinned host memory, batched per projection:
    bitwise the device-resident result (the batches align with the
    projection's 4096-row blocks), and V really crossed the link."""
    import scipy.sparse as sp
    import torch
    m, n, k = 9000, 14000, 5
    rp, ci, va = synth.csr_uniform(m, n, 0.002, seed=81)
    M = sp.csr_matrix((va.astype(np.float64), ci, rp), shape=(m, n))
    c = P.tsvd_csr_create(ctx, to_dev(rp), to_dev(ci), to_dev(va), (m, n))
    d = m  # m < n: the left branch iterates on u
    st = synth.start_vectors(k, d, seed=82)
    U0, S0, V0, i0 = P.tsvd_sparse(ctx, c, k, 0.0, to_dev(st), max_iter=30)
    U1, S1, V1, i1 = P.tsvd_sparse(ctx, c, k, 0.0, to_dev(st), max_iter=30, factor="host", factor_batches=nb,
                                   queue_depth=qd)
    assert not U1.is_cuda and U1.is_pinned()
    assert torch.equal(S0.cpu(), S1.cpu())
    assert torch.equal(U0.cpu(), U1.cpu())
    assert torch.equal(V0.cpu(), V1.cpu())
    assert i1["h2d_bytes"] > 0
    ref = O.tsvd_implicit(lambda x: M @ x, lambda y: M.T @ y, (m, n), 0.0, k, st, max_iter=30)
    compare(ref, U1, S1, V1, k, 1e-6, 1e-4)
    c.close()


def test_host_factor_dense_implicit(ctx):
    """Dense implicit product with V in pinned host memory (right branch, three
    batches, two buffers): bitwise the device-resident factor."""
    import torch
    m, n, k = 8999, 5000, 4
    dk = synth.dense_known(m, n, synth.spectrum_geometric(0.9, n), seed=91, dtype=np.float32)
    st = synth.start_vectors(k, n, seed=92)
    U0, S0, V0, _ = P.tsvd_dense(ctx, to_dev(dk.A), k, 1e-9, to_dev(st), method="implicit")
    U1, S1, V1, i1 = P.tsvd_dense(ctx, to_dev(dk.A), k, 1e-9, to_dev(st), method="implicit", factor="host",
                                  factor_batches=3, queue_depth=2)
    assert V1.is_pinned()
    # the iterates and V are bitwise those of the device factor; the finishing
    # product runs per column here (a mat-vec) instead of one FP64 GEMM
    assert torch.equal(V0.cpu(), V1.cpu())
    assert np.allclose(S0.cpu().numpy(), S1.cpu().numpy(), rtol=1e-13)
    assert np.allclose(U0.cpu().numpy(), U1.cpu().numpy(), rtol=0, atol=1e-12)
    assert i1["h2d_bytes"] > 0


def test_host_factor_rejects_device_pointer(ctx):
    """factor_loc = PINNED_HOST with a device V is an argument error."""
    import ctypes
    import torch
    m, n, k = 300, 200, 2
    A = torch.randn(m, n, device="cuda", dtype=torch.float32)
    st = to_dev(synth.start_vectors(k, n, seed=1))
    U = torch.zeros((k, m), dtype=torch.float64, device="cuda").T
    V = torch.zeros((k, n), dtype=torch.float64, device="cuda").T
    S = torch.zeros(k, dtype=torch.float64, device="cuda")
    o, keep = P._make_opts(ctx.lib, k, 1e-8, st, 100, None, "auto", 0, 0, 0)
    o.method = 2
    o.factor_loc = P.LOC_PINNED_HOST
    torch.cuda.synchronize()
    st_code = ctx.lib.tsvd_dense(ctx.handle, ctypes.c_void_p(A.data_ptr()), P.F32, P.LOC_DEVICE, m, n, n,
                                 ctypes.byref(o), ctypes.c_void_p(U.data_ptr()), m, ctypes.c_void_p(S.data_ptr()),
                                 ctypes.c_void_p(V.data_ptr()), n, None, None)
    assert st_code == P.INVALID_ARG
    assert "pinned host" in ctx.last_error()
