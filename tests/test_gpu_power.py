"""Power iteration with deflation (persistent kernel) against the oracle."""

import numpy as np
import pytest

import oracle as O
import paper_2208_08410_amd as P
import synth
from gpu_util import line_angle, to_dev

pytestmark = pytest.mark.gpu


def gram_case(m, n, q, seed):
    dk = synth.dense_known(m, n, synth.spectrum_geometric(q, min(m, n)), seed=seed)
    return dk, O.gram_rowblocks(dk.A)


@pytest.mark.parametrize("n,k", [(300, 8), (513, 5), (64, 64), (1000, 3)])
def test_power_fp64_trajectory(ctx, n, k):
    import torch
    dk, B0 = gram_case(2 * n, n, 0.9, seed=n)
    st = synth.start_vectors(k, n, seed=3)
    ref = O.tsvd_gram(dk.A, 1e-10, k, st, B0=B0)
    X, info = P.tsvd_power_gram(ctx, to_dev(B0.copy()), k, 1e-10, to_dev(st), fixed_iters=ref.iters)
    X = X.cpu().numpy()
    assert info["k_done"] == k
    assert info["iters"] == list(ref.iters)
    assert np.allclose(info["lambda"], ref.lam, rtol=1e-11)
    for l in range(k):
        assert line_angle(X[:, l], ref.V[:, l]) < 1e-9
    assert np.linalg.norm(X.T @ X - np.eye(k)) < 1e-12


def test_power_fp64_eps_mode_same_decisions(ctx):
    dk, B0 = gram_case(800, 300, 0.9, seed=5)
    st = synth.start_vectors(6, 300, seed=8)
    ref = O.tsvd_gram(dk.A, 1e-9, 6, st, B0=B0)
    X, info = P.tsvd_power_gram(ctx, to_dev(B0.copy()), 6, 1e-9, to_dev(st))
    assert info["converged"]
    assert info["iters"] == list(ref.iters)
    X = X.cpu().numpy()
    for l in range(6):
        assert line_angle(X[:, l], ref.V[:, l]) < 1e-9


@pytest.mark.parametrize("n,k", [(512, 16), (257, 7)])
def test_power_fp32_trajectory(ctx, n, k):
    """B rounded to FP32: vectors within 1e-4 rad of the FP64 oracle run for the
    same number of steps from the same start vectors."""
    dk, B0 = gram_case(4 * n, n, 0.97, seed=n + 1)
    st = synth.start_vectors(k, n, seed=4)
    ref = O.tsvd_gram(dk.A, 5e-8, k, st, B0=B0)
    X, info = P.tsvd_power_gram(ctx, to_dev(B0.astype(np.float32)), k, 5e-8, to_dev(st), fixed_iters=ref.iters)
    X = X.cpu().numpy()
    for l in range(k):
        assert line_angle(X[:, l], ref.V[:, l]) < 1e-4
    assert np.allclose(info["lambda"], ref.lam, rtol=1e-5)
    assert np.linalg.norm(X.T @ X - np.eye(k)) < 1e-12


def test_fixed_mode_and_not_converged(ctx):
    dk, B0 = gram_case(300, 100, 0.99, seed=2)
    st = synth.start_vectors(3, 100, seed=1)
    X, info = P.tsvd_power_gram(ctx, to_dev(B0.copy()), 3, 0.0, to_dev(st), max_iter=7)
    assert info["iters"] == [7, 7, 7] and info["converged"]
    X, info = P.tsvd_power_gram(ctx, to_dev(B0.copy()), 3, 1e-14, to_dev(st), max_iter=5)
    assert info["status"] == "TSVD_ERR_NOT_CONVERGED" and not info["converged"]
    assert info["iters"] == [5, 5, 5]


def test_zero_gram_is_rank_deficient(ctx):
    st = synth.start_vectors(2, 50, seed=1)
    X, info = P.tsvd_power_gram(ctx, to_dev(np.zeros((50, 50))), 2, 1e-8, to_dev(st))
    assert info["k_done"] == 0 and info["rank_deficient"]
    assert np.all(X.cpu().numpy() == 0)


def test_nonfinite_gram(ctx):
    B = np.eye(40); B[3, 5] = np.nan
    st = synth.start_vectors(2, 40, seed=1)
    with pytest.raises(P.TsvdError) as e:
        P.tsvd_power_gram(ctx, to_dev(B), 2, 1e-8, to_dev(st))
    assert e.value.status == P.NONFINITE


@pytest.mark.parametrize("d,k", [(3999, 3), (4096, 3), (6000, 2), (9001, 2)])
def test_power_fp32_register_rows(ctx, d, k):
    """Large d: a block's rows are split over LDS, registers and HBM (d = 9001:
    no register rows, most rows streamed from HBM, and an odd leading dimension
    that takes the scalar load and deflation paths); the result must match the
    FP64 oracle run for the same number of steps."""
    g = synth.rng(d, 3)
    lam = 0.8 ** np.arange(d, dtype=np.float64)
    Q = synth.haar_orthonormal(d, 8, seed=d, tag=1)
    # B = Q diag(lam[:8]) Q^T + small symmetric noise: a well-separated top
    Bn = g.standard_normal((d, d)) * 1e-5
    B0 = (Q * lam[:8]) @ Q.T + (Bn + Bn.T)
    st = synth.start_vectors(k, d, seed=5)
    ref = O.tsvd_gram(np.eye(d), 1e-9, k, st, B0=B0, max_iter=2000)
    X, info = P.tsvd_power_gram(ctx, to_dev(B0.astype(np.float32)), k, 1e-9, to_dev(st), fixed_iters=ref.iters)
    X = X.cpu().numpy()
    for l in range(k):
        assert line_angle(X[:, l], ref.V[:, l]) < 1e-5
    assert np.allclose(info["lambda"], ref.lam, rtol=1e-5)
