"""Pins for the oracle's precision-mode definitions (CPU only)."""

import numpy as np
import pytest

import oracle as O
import synth


def test_bf16_round_matches_torch():
    torch = pytest.importorskip("torch")
    x = synth.gaussian_dense(300, 200, seed=1, dtype=np.float32) * np.float32(37.0)
    x[0, :5] = [1.0, 1.00390625, 1.005859375, -3.0078125, 0.0]  # exact ties and representable values
    ours = O.bf16_round(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(ours, ref)


def _exact_split_matrix(m, n, seed):
    """A = H + L with H in {+-1, +-2, +-3} and L = j 2^-10, |j| <= 1: |L| is
    below half a bf16 ulp of H on either side of it, so bf16(a) = H and
    bf16(a - H) = L exactly, and every product and partial sum of the BF16X3
    Gram is a multiple of 2^-10 small enough to be exact in FP32."""
    g = synth.rng(seed, 99)
    H = g.choice(np.array([-3, -2, -1, 1, 2, 3], dtype=np.float64), size=(m, n))
    L = g.integers(-1, 2, size=(m, n)).astype(np.float64) * 2.0 ** -10
    return (H + L).astype(np.float32), H, L


def test_gram_bf16x3_definition_on_exact_split():
    A, H, L = _exact_split_matrix(200, 40, seed=3)
    assert np.array_equal(O.bf16_round(A).astype(np.float64), H)
    B = O.gram_bf16x3(A)
    assert np.array_equal(B, H.T @ H + H.T @ L + L.T @ H)
    # and it differs from the exact Gram by exactly the dropped lo^T lo term
    A64 = A.astype(np.float64)
    assert np.allclose(A64.T @ A64 - B, L.T @ L, rtol=0, atol=1e-12)
    Bl = O.gram_bf16x3(A, side="left")
    assert np.array_equal(Bl, H @ H.T + H @ L.T + L @ H.T)


def test_gram_bf16x3_error_bound_gaussian():
    A = synth.gaussian_dense(500, 64, seed=5)
    A64 = A.astype(np.float64)
    exact = A64.T @ A64
    B = O.gram_bf16x3(A)
    absA = np.abs(A64)
    # dropped terms per product are bounded by about 3 * 2^-16 |a_i a_j|
    assert np.all(np.abs(B - exact) <= 3.1 * 2.0 ** -16 * (absA.T @ absA))
