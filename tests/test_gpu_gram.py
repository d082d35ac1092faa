"""Gram step (MFMA SYRK) against the oracle, through the C ABI."""

import numpy as np
import pytest

import oracle as O
import paper_2208_08410_amd as P
import synth
from gpu_util import to_dev

pytestmark = pytest.mark.gpu


def int_matrix(m, n, seed, lo=-7, hi=7):
    return synth.rng(seed, 5).integers(lo, hi + 1, size=(m, n)).astype(np.float64)


def exact_split(m, n, seed):
    g = synth.rng(seed, 99)
    H = g.choice(np.array([-3, -2, -1, 1, 2, 3], dtype=np.float64), size=(m, n))
    L = g.integers(-1, 2, size=(m, n)).astype(np.float64) * 2.0 ** -10
    return (H + L).astype(np.float32)


# shapes: ragged tiles (not multiples of 128/64), a single column/row, chunking
SHAPES = [(1000, 300, "right", 0), (1000, 300, "right", 96), (257, 1000, "left", 0), (1700, 129, "right", 64),
          (5, 1, "right", 0), (1, 5, "left", 0), (64, 64, "right", 0), (333, 700, "right", 0),
          # d >= 1024: the 256-wide BF16X3 tiles (ragged last tile, both sides)
          (1700, 1100, "right", 0), (1300, 1030, "left", 0), (1024, 1024, "right", 320)]


@pytest.mark.parametrize("m,n,side,rpb", SHAPES)
def test_bf16x3_exact_split_bit_exact(ctx, m, n, side, rpb):
    A = exact_split(m, n, seed=m + n)
    ref = O.gram_bf16x3(A, side=side)
    B = P.tsvd_gram_dense(ctx, to_dev(A), gram="bf16x3", side=side, rows_per_block=rpb).cpu().numpy()
    assert np.array_equal(B.astype(np.float64), ref)


@pytest.mark.parametrize("m,n,side,rpb", SHAPES)
def test_fp32_integer_bit_exact(ctx, m, n, side, rpb):
    A = int_matrix(m, n, seed=m * 7 + n)
    ref = A.T @ A if side == "right" else A @ A.T
    B = P.tsvd_gram_dense(ctx, to_dev(A.astype(np.float32)), gram="fp32", side=side, rows_per_block=rpb)
    assert np.array_equal(B.cpu().numpy().astype(np.float64), ref)


@pytest.mark.parametrize("m,n,side,rpb", SHAPES)
def test_fp64_integer_bit_exact(ctx, m, n, side, rpb):
    A = int_matrix(m, n, seed=m * 3 + n)
    ref = A.T @ A if side == "right" else A @ A.T
    B = P.tsvd_gram_dense(ctx, to_dev(A), gram="fp64", side=side, rows_per_block=rpb)
    assert np.array_equal(B.cpu().numpy(), ref)


def test_accumulate_adds(ctx):
    import torch
    A1 = int_matrix(300, 150, seed=1).astype(np.float32)
    A2 = int_matrix(200, 150, seed=2).astype(np.float32)
    B = P.tsvd_gram_dense(ctx, to_dev(A1), gram="fp32")
    B = P.tsvd_gram_dense(ctx, to_dev(A2), gram="fp32", B=B, accumulate=True)
    ref = O.gram_rowblocks(np.vstack([A1, A2]).astype(np.float64), 300)
    assert np.array_equal(B.cpu().numpy().astype(np.float64), ref)


@pytest.mark.parametrize("gram,tol", [("fp32", 5e-6), ("bf16x3", 5e-6)])
def test_gaussian_normwise(ctx, gram, tol):
    """Random data: the only remaining difference from the mode's definition is
    FP32 rounding of the accumulation, about sqrt(chunk) * 2^-24 relative."""
    A = synth.gaussian_dense(20000, 512, seed=4)
    ref = O.gram_bf16x3(A) if gram == "bf16x3" else O.gram_rowblocks(A)
    B = P.tsvd_gram_dense(ctx, to_dev(A), gram=gram).cpu().numpy().astype(np.float64)
    assert np.linalg.norm(B - ref) / np.linalg.norm(ref) < tol
    assert np.array_equal(B, B.T)


def test_lda_padding_and_misaligned(ctx):
    import torch
    A = int_matrix(400, 130, seed=9)
    big = torch.zeros((400, 133), dtype=torch.float32, device="cuda")
    big[:, :130] = torch.from_numpy(A.astype(np.float32)).cuda()
    B = P.tsvd_gram_dense(ctx, big[:, :130], gram="bf16x3")          # lda = 133
    assert np.array_equal(B.cpu().numpy().astype(np.float64), A.T @ A)
    big.zero_()
    big[:, 1:131] = torch.from_numpy(A.astype(np.float32)).cuda()
    B = P.tsvd_gram_dense(ctx, big[:, 1:131], gram="bf16x3")          # 4-byte aligned base
    assert np.array_equal(B.cpu().numpy().astype(np.float64), A.T @ A)
    B = P.tsvd_gram_dense(ctx, big[:, 1:131], gram="fp32", side="left")
    assert np.array_equal(B.cpu().numpy().astype(np.float64), A @ A.T)


@pytest.mark.parametrize("tile", [128, 256])
def test_tuning_tiles_agree(ctx, tile):
    """Both BF16X3 tile shapes give the mode's definition bit for bit."""
    A = exact_split(1500, 700, seed=21)
    ref = O.gram_bf16x3(A)
    P.set_tuning(ctx, gram_tile=tile, gram_chunks=5)
    try:
        B = P.tsvd_gram_dense(ctx, to_dev(A), gram="bf16x3").cpu().numpy()
    finally:
        P.set_tuning(ctx)
    assert np.array_equal(B.astype(np.float64), ref)


def test_tuning_rejects_bad_values(ctx):
    with pytest.raises(P.TsvdError):
        P.set_tuning(ctx, gram_tile=64)
    with pytest.raises(P.TsvdError):
        P.set_tuning(ctx, power_blocks=100000)
    with pytest.raises(P.TsvdError):
        P.set_tuning(ctx, team_kib=4)
    with pytest.raises(P.TsvdError):
        P.set_tuning(ctx, group_kchunk=16)
    with pytest.raises(P.TsvdError):
        P.set_tuning(ctx, sparse_row_bits=12)
    with pytest.raises(P.TsvdError):
        P.set_tuning(ctx, sparse_row_bits=11, sparse_col_bits=22)
    with pytest.raises(P.TsvdError):
        P.set_tuning(ctx, group_tile={2: 256})
    with pytest.raises(P.TsvdError):
        P.set_tuning(ctx, group_kchunk_cls={7: 16})
    with pytest.raises(ValueError):
        P.set_tuning(ctx, group_tile={8: 64})
    zero = {f: 0 for f in P.TUNING_FIELDS}
    zero.update(group_tile=[0] * P.GRAM_CLASSES, group_kchunk_cls=[0] * P.GRAM_CLASSES)
    assert P.get_tuning(ctx) == zero
