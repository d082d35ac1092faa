"""Parity at the benchmark's full size (dense in-HBM FP32 A of 200,000 x 4,096,
k = 64, BF16X3 Gram, the launch configuration bench.py times): outputs the
oracle can compute one by one are checked one by one, the rest through
properties that hold at any size."""

import numpy as np
import pytest

import oracle as O
import paper_2208_08410_amd as P
import synth

pytestmark = pytest.mark.gpu

M, N, K, EPS, Q = 200000, 4096, 64, 5e-8, 0.97


@pytest.fixture(scope="module")
def c2():
    import torch
    s = synth.spectrum_geometric(Q, N)
    A, U, V = synth.dense_known_torch(M, N, s, 2, torch.device("cuda:0"), keep_factors=K)
    v0 = torch.from_numpy(synth.start_vectors(K, N, seed=102)).cuda()
    Ah = A.cpu().numpy()
    yield A, Ah, s, V.cpu().numpy(), v0
    del A


def test_gram_sampled_entries(ctx, c2):
    """Sampled entries of the full-size BF16X3 Gram against the oracle's FP64
    dot products of the same columns: |error| <= 1e-5 sqrt(B_ii B_jj) (the
    dropped lo*lo term is 2^-18 relative, FP32 accumulation ~sqrt(chunk) 2^-24)."""
    A, Ah, s, Vt, v0 = c2
    B = P.tsvd_gram_dense(ctx, A, gram="bf16x3", side="right").cpu().numpy()
    rng = np.random.default_rng(0)
    pairs = [(0, 0), (N - 1, N - 1), (0, N - 1), (N - 1, 0), (127, 128), (255, 256)]
    pairs += [tuple(int(x) for x in rng.integers(0, N, 2)) for _ in range(40)]
    cols = sorted({c for p in pairs for c in p})
    Ac = Ah[:, cols].astype(np.float64)
    idx = {c: i for i, c in enumerate(cols)}
    for i, j in pairs:
        ref = O.gram_rowblocks(Ac[:, [idx[i], idx[j]]])
        scale = np.sqrt(ref[0, 0] * ref[1, 1])
        assert abs(B[i, j] - ref[0, 1]) <= 1e-5 * scale, (i, j)
    assert np.array_equal(B, B.T)


def test_tsvd_full_size(ctx, c2):
    """sigma within 1e-6 of the closed form for all 64 triplets; V orthonormal
    to FP64 rounding; for sampled triplets the oracle's u = A v / ||A v|| from
    the GPU's v matches the GPU's u and sigma; vectors within the stopping
    model's angle of the true singular vectors."""
    A, Ah, s, Vt, v0 = c2
    U, S, V, info = P.tsvd_dense(ctx, A, K, EPS, v0, gram="bf16x3")
    assert info["status"] == "TSVD_OK" and info["converged"] and info["k_done"] == K
    S, U, V = S.cpu().numpy(), U.cpu().numpy(), V.cpu().numpy()
    assert np.max(np.abs(S - s[:K]) / s[:K]) < 1e-6
    assert np.linalg.norm(V.T @ V - np.eye(K)) < 1e-10
    sample = [0, 1, 17, 40, K - 1]
    Uo, So = O.rayleigh(Ah, V[:, sample])  # the oracle's finishing step (Alg. 1) from the GPU's v
    for i, l in enumerate(sample):
        assert abs(So[i] - S[l]) <= 1e-12 * So[i]
        assert np.max(np.abs(Uo[:, i] - U[:, l])) < 1e-12
    r = Q * Q
    theta = np.sqrt(2 * EPS) * r / (1 - r)
    for l in range(K):
        c = abs(float(V[:, l] @ Vt[:, l]))
        assert np.arccos(min(1.0, c)) < 3 * theta, l
