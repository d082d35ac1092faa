"""The autotuner measures real launches, stores a valid choice, and the chosen
launch shapes leave the results unchanged (to FP32 reduction-order rounding)."""

import numpy as np
import pytest

import paper_2208_08410_amd as P
import synth
from gpu_util import line_angle, to_dev
from paper_2208_08410_amd import autotune as T

pytestmark = pytest.mark.gpu


@pytest.fixture
def tuner(ctx, tmp_path):
    t = T.Tuner(ctx, str(tmp_path / "tuning.json"), reps=2)
    yield t
    P.set_tuning(ctx)


def test_tune_dense_then_same_results(ctx, tuner):
    m, n, k = 16384, 1024, 6
    dk = synth.dense_known(m, n, synth.spectrum_geometric(0.9, n), seed=8, dtype=np.float32)
    A, st = to_dev(dk.A), to_dev(synth.start_vectors(k, n, seed=3))
    it = [30] * k
    U0, S0, V0, _ = P.tsvd_dense(ctx, A, k, 0.0, st, gram="bf16x3", fixed_iters=it)
    choice = tuner.tune_dense(A, gram="bf16x3", k=4, power_iters=10)
    assert (choice["gram_tile"], choice["gram_chunks"]) in T.gram_candidates("bf16x3", n, m, ctx.num_cu)
    assert choice["power_blocks"] in T.power_candidates(n, ctx.num_cu)
    assert P.get_tuning(ctx)["team_kib"] == 0  # the tuner restores the context's tuning
    assert tuner.apply_dense(m, n, "bf16x3")
    assert {k2: P.get_tuning(ctx)[k2] for k2 in choice} == choice
    U1, S1, V1, _ = P.tsvd_dense(ctx, A, k, 0.0, st, gram="bf16x3", fixed_iters=it)
    assert np.max(np.abs(S1.cpu().numpy() - S0.cpu().numpy()) / S0.cpu().numpy()) < 1e-6
    for l in range(k):
        assert line_angle(V1[:, l].cpu().numpy(), V0[:, l].cpu().numpy()) < 1e-4
    # a second tuner reads the stored choice back
    t2 = T.Tuner(ctx, tuner.path)
    assert t2.lookup(T.dense_class(m, n, "bf16x3")) == choice


def test_tune_batch(ctx, tuner):
    probs = []
    for i, (m, n, k) in enumerate([(3000, 200, 4), (800, 1500, 3), (5000, 700, 4), (1200, 64, 2)]):
        dk = synth.dense_known(m, n, synth.spectrum_geometric(0.85, min(m, n)), seed=i, dtype=np.float32)
        st = synth.start_vectors(k, n if m >= n else m, seed=10 + i)
        probs.append(dict(A=to_dev(dk.A), k=k, eps=0.0, v0=to_dev(st), fixed_iters=[15] * k))
    ref = P.tsvd_dense_batched(ctx, probs, raise_errors=True)
    choice = tuner.tune_batch(probs)
    assert (choice["team_kib"], choice["group_kchunk"]) in T.batch_candidates()
    assert tuner.apply_batch([tuple(p["A"].shape) for p in probs])
    out = P.tsvd_dense_batched(ctx, probs, raise_errors=True)
    for (U, S, V, _), (Ur, Sr, Vr, _) in zip(out, ref):
        assert np.max(np.abs(S.cpu().numpy() - Sr.cpu().numpy()) / Sr.cpu().numpy()) < 1e-6


def test_tune_gram_classes(ctx, tuner):
    """Per-class batched-Gram unit shapes: the tuner picks each class's (tile
    edge, chunk rows) among the candidates, apply_batch sets them beside the
    batch class's team rule, and the results keep to FP32 rounding of the
    default shapes."""
    shapes = [(3000, 100), (4000, 257), (300, 2600), (2500, 1000), (5000, 700)]
    chosen = tuner.tune_gram_classes(shapes, per_class=2)
    assert set(chosen) == {P.gram_class(min(m, n)) for m, n in shapes}
    for c, (tile, kc) in chosen.items():
        K_max = max(max(m, n) for m, n in shapes if P.gram_class(min(m, n)) == c)
        assert (tile, kc) in T.gram_unit_candidates(K_max)
    assert P.get_tuning(ctx)["group_tile"] == [0] * P.GRAM_CLASSES  # restored
    probs = []
    for i, (m, n) in enumerate(shapes):
        k = 3
        dk = synth.dense_known(m, n, synth.spectrum_geometric(0.85, min(m, n)), seed=20 + i, dtype=np.float32)
        st = synth.start_vectors(k, min(m, n), seed=30 + i)
        probs.append(dict(A=to_dev(dk.A), k=k, eps=0.0, v0=to_dev(st), fixed_iters=[15] * k))
    ref = P.tsvd_dense_batched(ctx, probs, raise_errors=True)
    assert not tuner.apply_batch(shapes)  # no team-rule entry for this batch class, only class shapes
    got = P.get_tuning(ctx)
    for c, (tile, kc) in chosen.items():
        assert (got["group_tile"][c], got["group_kchunk_cls"][c]) == (tile, kc)
    out = P.tsvd_dense_batched(ctx, probs, raise_errors=True)
    for (U, S, V, _), (Ur, Sr, Vr, _) in zip(out, ref):
        assert np.max(np.abs(S.cpu().numpy() - Sr.cpu().numpy()) / Sr.cpu().numpy()) < 1e-6
        for l in range(S.shape[0]):
            assert line_angle(V[:, l].cpu().numpy(), Vr[:, l].cpu().numpy()) < 1e-4
    t2 = T.Tuner(ctx, tuner.path)
    ct = t2.class_tuning()
    assert {c: (ct["group_tile"][c], ct["group_kchunk_cls"][c]) for c in chosen} == chosen
