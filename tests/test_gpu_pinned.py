"""Dense t-SVD with A in pinned host memory (double-buffered H2D row batches)."""

import numpy as np
import pytest

import oracle as O
import paper_2208_08410_amd as P
import synth
from gpu_util import line_angle, to_dev

pytestmark = pytest.mark.gpu


def pinned(x):
    import torch
    t = torch.empty(x.shape, dtype=torch.float32, pin_memory=True)
    t.copy_(torch.from_numpy(np.ascontiguousarray(x)))
    return t


@pytest.mark.parametrize("rpb,q,gram", [(3072, 2, "bf16x3"), (2048, 3, "fp32"), (768, 2, "bf16x3"), (20480, 2, "fp32")])
def test_pinned_bitwise_equals_device(ctx, rpb, q, gram):
    """Streaming the rows in batches of rpb (a multiple of 128, the finishing
    pass's row tile) with one Gram chunk per batch gives the same bits as the
    in-HBM path with the same row blocking; the last batch is ragged."""
    m, n, k = 20000, 384, 6
    dk = synth.dense_known(m, n, synth.spectrum_geometric(0.9, n), seed=3, dtype=np.float32)
    st = to_dev(synth.start_vectors(k, n, seed=2))
    Ud, Sd, Vd, infd = P.tsvd_dense(ctx, to_dev(dk.A), k, 1e-9, st, gram=gram, rows_per_block=rpb)
    Up, Sp, Vp, infp = P.tsvd_dense(ctx, pinned(dk.A), k, 1e-9, st, gram=gram, rows_per_block=rpb, queue_depth=q)
    assert infp["h2d_bytes"] == 2 * m * n * 4
    assert infp["iters"] == infd["iters"]
    assert np.array_equal(Sp.cpu().numpy(), Sd.cpu().numpy())
    assert np.array_equal(Vp.cpu().numpy(), Vd.cpu().numpy())
    assert np.array_equal(Up.cpu().numpy(), Ud.cpu().numpy())


@pytest.mark.parametrize("rpb,q", [(0, 2), (4000, 2), (2500, 3)])
def test_pinned_batches_vs_oracle(ctx, rpb, q):
    """Default batches (one batch here) and rows_per_block well below m, so
    that 8 or 12 batches stream through 2 or 3 device buffers with a ragged
    last batch: sigma, v and u against the FP64 oracle in trajectory mode."""
    m, n, k, eps = 30000, 256, 5, 1e-9
    dk = synth.dense_known(m, n, synth.spectrum_geometric(0.9, n), seed=4, dtype=np.float32)
    st = synth.start_vectors(k, n, seed=1)
    ref = O.tsvd_gram(dk.A, eps, k, st)
    U, S, V, info = P.tsvd_dense(ctx, pinned(dk.A), k, eps, to_dev(st), fixed_iters=ref.iters, rows_per_block=rpb,
                                 queue_depth=q)
    assert info["h2d_bytes"] == 2 * m * n * 4
    S = S.cpu().numpy(); V = V.cpu().numpy(); U = U.cpu().numpy()
    assert np.max(np.abs(S - ref.S) / ref.S) < 1e-6
    Ur, Vr = O.canonical(ref.U, ref.V)
    for l in range(k):
        assert line_angle(V[:, l], Vr[:, l]) < 1e-4
        assert line_angle(U[:, l], Ur[:, l]) < 1e-4


def test_pinned_rejects_pageable_and_host_factor(ctx):
    import torch
    A = torch.from_numpy(synth.gaussian_dense(100, 50, seed=1))
    st = to_dev(synth.start_vectors(2, 50, seed=1))
    with pytest.raises(ValueError):
        P.tsvd_dense(ctx, A, 2, 1e-8, st)  # pageable memory is refused by the binding
    # with A streamed from the host, the iterated factor stays on the device
    Ap = pinned(synth.gaussian_dense(100, 50, seed=1))
    with pytest.raises(P.TsvdError) as e:
        P.tsvd_dense(ctx, Ap, 2, 1e-8, st, method="implicit", factor="host")
    assert e.value.status == P.UNSUPPORTED


@pytest.mark.parametrize("cpb,q,gram", [(3072, 2, "bf16x3"), (2048, 3, "fp32"), (768, 2, "bf16x3")])
def test_pinned_left_branch_bitwise_equals_device(ctx, cpb, q, gram):
    """m < n (the A A^T branch, Eq. 3): A streams in column batches of cpb
    (pitched copies, a multiple of 128) with one Gram chunk per batch, and
    gives the same bits as the in-HBM path with the same column blocking; the
    last batch is ragged."""
    m, n, k = 384, 20000, 6
    dk = synth.dense_known(m, n, synth.spectrum_geometric(0.9, m), seed=13, dtype=np.float32)
    st = to_dev(synth.start_vectors(k, m, seed=12))
    Ud, Sd, Vd, infd = P.tsvd_dense(ctx, to_dev(dk.A), k, 1e-9, st, gram=gram, rows_per_block=cpb)
    Up, Sp, Vp, infp = P.tsvd_dense(ctx, pinned(dk.A), k, 1e-9, st, gram=gram, rows_per_block=cpb, queue_depth=q)
    assert not infp["branch_right"] and not infd["branch_right"]
    assert infp["h2d_bytes"] == 2 * m * n * 4
    assert infp["iters"] == infd["iters"]
    assert np.array_equal(Sp.cpu().numpy(), Sd.cpu().numpy())
    assert np.array_equal(Vp.cpu().numpy(), Vd.cpu().numpy())
    assert np.array_equal(Up.cpu().numpy(), Ud.cpu().numpy())


@pytest.mark.parametrize("cpb,q", [(0, 2), (2500, 3)])
def test_pinned_left_branch_vs_oracle(ctx, cpb, q):
    """m < n streamed in column batches (one batch, or 12 through 3 buffers):
    sigma, u and v against the FP64 oracle's left branch in trajectory mode."""
    m, n, k, eps = 256, 30000, 5, 1e-9
    dk = synth.dense_known(m, n, synth.spectrum_geometric(0.9, m), seed=14, dtype=np.float32)
    st = synth.start_vectors(k, m, seed=15)
    ref = O.tsvd_gram(dk.A, eps, k, st)
    U, S, V, info = P.tsvd_dense(ctx, pinned(dk.A), k, eps, to_dev(st), fixed_iters=ref.iters, rows_per_block=cpb,
                                 queue_depth=q)
    assert info["h2d_bytes"] == 2 * m * n * 4
    S = S.cpu().numpy(); V = V.cpu().numpy(); U = U.cpu().numpy()
    assert np.max(np.abs(S - ref.S) / ref.S) < 1e-6
    Ur, Vr = O.canonical(ref.U, ref.V)
    for l in range(k):
        assert line_angle(V[:, l], Vr[:, l]) < 1e-4
        assert line_angle(U[:, l], Ur[:, l]) < 1e-4


def test_pinned_stream_timing_is_consistent(ctx):
    """The Gram pass reports its copy and compute busy times and their overlap
    from per-batch HIP events: each is positive, the overlap fits inside both,
    with 12 batches through two buffers some copy runs beside a Gram, and the
    pass cannot be shorter than the busy time of either stream."""
    m, n, k = 48000, 1024, 2
    dk = synth.dense_known(m, n, synth.spectrum_geometric(0.9, n), seed=5, dtype=np.float32)
    st = to_dev(synth.start_vectors(k, n, seed=6))
    U, S, V, info = P.tsvd_dense(ctx, pinned(dk.A), k, 1e-6, st, rows_per_block=4000, queue_depth=2)
    c, g, o = info["t_stream_copy_ms"], info["t_stream_compute_ms"], info["t_stream_overlap_ms"]
    assert c > 0 and g > 0 and o > 0
    assert o <= min(c, g) + 1e-3
    assert info["t_gram_ms"] >= max(c, g) - 1e-3
    # the in-HBM path has no streamed pass
    _, _, _, infd = P.tsvd_dense(ctx, to_dev(dk.A), k, 1e-6, st)
    assert infd["t_stream_copy_ms"] == 0 and infd["t_stream_overlap_ms"] == 0
