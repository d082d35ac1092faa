"""Parity at the streaming workload's size (the default bench run's streaming
leg: FP32 A of 1,000,000 x 8,192 in pinned host memory, N(0, 1) plus a
rank-32 spike, k = 32, eps = 5e-8, 4 GiB row batches through two device
buffers).  The streamed t-SVD (Alg. 3's batches through a stream queue, Sec.
V-C) gives the same bits as the same computation on the device-resident A
with the same chunking, and its outputs meet properties that hold at any
size: unit and orthonormal factors, and u = A v / sigma on sampled rows."""

import numpy as np
import pytest

import paper_2208_08410_amd as P
import synth

pytestmark = pytest.mark.gpu

M, N, K, EPS, SEED = 1_000_000, 8192, 32, 5e-8, 2
R = (4 << 30) // (N * 4) // 128 * 128  # rows per 4 GiB batch


@pytest.fixture(scope="module")
def c3():
    import torch
    dev = torch.device("cuda:0")
    print(f"[stream full size] A {M}x{N} ({M * N * 4 / 1e9:.1f} GB), {R}-row batches", flush=True)
    y, _ = synth.spiked_factors(M, N, 32, SEED)
    yd = torch.as_tensor(y, device=dev)
    Ad = torch.empty((M, N), dtype=torch.float32, device=dev)
    for r0 in range(0, M, R):
        rows = min(R, M - r0)
        Ad[r0:r0 + rows] = synth.spiked_rows_torch(M, N, 32, SEED, r0, rows, dev, yfac=yd)
    Ah = torch.empty((M, N), dtype=torch.float32, pin_memory=True)
    Ah.copy_(Ad)
    v0 = torch.from_numpy(synth.start_vectors(K, N, seed=SEED + 5)).to(dev)
    yield Ad, Ah, v0
    del Ad, Ah
    torch.cuda.empty_cache()


def test_streamed_equals_resident_and_properties(ctx, c3):
    import torch
    Ad, Ah, v0 = c3
    Us, Ss, Vs, info = P.tsvd_dense(ctx, Ah, K, EPS, v0, rows_per_block=R, queue_depth=2)
    assert info["status"] == "TSVD_OK" and info["k_done"] == K
    assert info["h2d_bytes"] >= 2 * M * N * 4  # both passes streamed A
    Ud, Sd, Vd, infod = P.tsvd_dense(ctx, Ad, K, EPS, v0, rows_per_block=R)
    assert infod["iters"] == info["iters"]
    assert torch.equal(Ss, Sd) and torch.equal(Vs, Vd) and torch.equal(Us, Ud)
    S, U, V = Ss.cpu().numpy(), Us.cpu().numpy(), Vs.cpu().numpy()
    assert np.all(S[:-1] >= S[1:]) and S[-1] > 0
    assert np.linalg.norm(V.T @ V - np.eye(K)) < 1e-10
    assert np.max(np.abs(np.linalg.norm(U, axis=0) - 1.0)) < 1e-12
    An = Ah.numpy()
    rng = np.random.default_rng(3)
    for i in [0, R - 1, R, M - 1] + [int(t) for t in rng.integers(0, M, 40)]:
        a = An[i].astype(np.float64)
        ref = (a @ V) / S                 # u_i = (A v)_i / sigma, FP64
        mag = (np.abs(a) @ np.abs(V)) / S
        assert np.all(np.abs(U[i] - ref) <= 1e-12 * mag + 1e-15), i
