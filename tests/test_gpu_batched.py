"""Batched dense t-SVD (tsvd_dense_batched: grouped Gram, team power kernel,
grouped FP64 finish) against the oracle, per problem, for mixes of shapes."""

import numpy as np
import pytest

import oracle as O
import paper_2208_08410_amd as P
import synth
from gpu_util import line_angle, to_dev

pytestmark = pytest.mark.gpu

# (m, n, k, gram): both sides, ragged tiles, a Gram of 1 x 1, rank-1 shapes
MIX = [(3000, 300, 6, "bf16x3"), (500, 1200, 4, "fp32"), (2000, 1000, 8, "bf16x3"), (700, 700, 5, "fp32"),
       (4096, 128, 3, "bf16x3"), (257, 2100, 2, "bf16x3"), (1, 300, 1, "fp32"), (500, 1, 1, "bf16x3")]


def make_problem(m, n, k, gram, seed, q=0.9):
    d = min(m, n)
    dk = synth.dense_known(m, n, synth.spectrum_geometric(q, d), seed=seed, dtype=np.float32)
    right = m >= n
    st = synth.start_vectors(k, n if right else m, seed=seed + 100)
    return dk, st


@pytest.fixture
def tuned(ctx):
    yield ctx
    P.set_tuning(ctx)  # back to library defaults


@pytest.mark.parametrize("team_kib", [0, 8, 65536])
def test_batched_mix_trajectory_vs_oracle(tuned, team_kib):
    """Each problem of a mixed batch follows the FP64 oracle's trajectory
    (fixed iteration counts): vectors within 1e-4 rad, sigma within 1e-6.
    team_kib 8 gives every problem the largest team it can use (up to the
    whole chip), 65536 one-workgroup teams, 0 the default rule."""
    ctx = tuned
    P.set_tuning(ctx, team_kib=team_kib)
    probs, refs = [], []
    for i, (m, n, k, gram) in enumerate(MIX):
        dk, st = make_problem(m, n, k, gram, seed=40 + i)
        ref = O.tsvd_gram(dk.A, 1e-10, k, st)
        refs.append((dk, ref))
        probs.append(dict(A=to_dev(dk.A), k=k, eps=1e-10, v0=to_dev(st), gram=gram, fixed_iters=ref.iters))
    out = P.tsvd_dense_batched(ctx, probs, raise_errors=True)
    for (m, n, k, gram), (dk, ref), (U, S, V, info) in zip(MIX, refs, out):
        U, S, V = U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy()
        assert info["status"] == "TSVD_OK" and info["k_done"] == k
        assert info["iters"] == list(ref.iters)
        assert info["branch_right"] == (m >= n)
        assert np.max(np.abs(S - ref.S) / ref.S) < 1e-6, (m, n)
        Ur, Vr = O.canonical(ref.U, ref.V)
        for l in range(k):
            assert line_angle(V[:, l], Vr[:, l]) < 1e-4, (m, n, l)
            assert line_angle(U[:, l], Ur[:, l]) < 1e-4, (m, n, l)
            # sign convention: largest |v| entry positive
            assert V[np.argmax(np.abs(V[:, l])), l] > 0


def test_batched_equals_single_calls(ctx):
    """The batch gives each problem what a single tsvd_dense call gives it, to
    the rounding of a different reduction order (same fixed iteration counts)."""
    probs, singles = [], []
    for i, (m, n, k, gram) in enumerate(MIX[:6]):
        dk, st = make_problem(m, n, k, gram, seed=70 + i)
        it = [25] * k
        A, v0 = to_dev(dk.A), to_dev(st)
        probs.append(dict(A=A, k=k, eps=0.0, v0=v0, gram=gram, fixed_iters=it))
        singles.append(P.tsvd_dense(ctx, A, k, 0.0, v0, gram=gram, fixed_iters=it))
    out = P.tsvd_dense_batched(ctx, probs, raise_errors=True)
    for (Ub, Sb, Vb, _), (Us, Ss, Vs, _) in zip(out, singles):
        Sb, Ss = Sb.cpu().numpy(), Ss.cpu().numpy()
        assert np.max(np.abs(Sb - Ss) / Ss) < 1e-6
        for l in range(len(Ss)):
            assert line_angle(Vb[:, l].cpu().numpy(), Vs[:, l].cpu().numpy()) < 1e-4
            assert line_angle(Ub[:, l].cpu().numpy(), Us[:, l].cpu().numpy()) < 1e-4


def test_batched_many_small_converged(ctx):
    """48 small problems (more than fit one per CU at the default team size is
    not needed here: they share teams by the LPT rule); eps mode, sigma within
    1e-6 of the closed form and the iterated factor orthonormal."""
    rng = np.random.default_rng(5)
    probs, dks = [], []
    for i in range(48):
        m = int(rng.integers(200, 2000))
        n = int(rng.integers(16, 300))
        if i % 5 == 0:
            m, n = n, m  # some wide problems (left branch)
        k = int(min(4, m, n))
        dk, st = make_problem(m, n, k, "bf16x3", seed=200 + i, q=0.8)
        dks.append(dk)
        probs.append(dict(A=to_dev(dk.A), k=k, eps=1e-12, v0=to_dev(st), gram="bf16x3"))
    out = P.tsvd_dense_batched(ctx, probs, raise_errors=True)
    for dk, p, (U, S, V, info) in zip(dks, probs, out):
        k = p["k"]
        assert info["converged"]
        S = S.cpu().numpy()
        assert np.max(np.abs(S - dk.s[:k]) / dk.s[:k]) < 1e-6
        Q = (V if info["branch_right"] else U).cpu().numpy()
        assert np.linalg.norm(Q.T @ Q - np.eye(k)) < 1e-10


def test_batched_one_bad_problem(ctx):
    """A NaN in one problem fails that problem only; the others are exact."""
    probs, dks = [], []
    for i, (m, n, k) in enumerate([(800, 200, 3), (600, 150, 2), (900, 300, 3)]):
        dk, st = make_problem(m, n, k, "fp32", seed=300 + i, q=0.8)
        A = dk.A.copy()
        if i == 1:
            A[5, 7] = np.nan
        dks.append(dk)
        probs.append(dict(A=to_dev(A), k=k, eps=1e-12, v0=to_dev(st), gram="fp32"))
    out = P.tsvd_dense_batched(ctx, probs)
    assert out[1][3]["status"] == "TSVD_ERR_NONFINITE"
    for i in (0, 2):
        U, S, V, info = out[i]
        assert info["status"] == "TSVD_OK"
        k = probs[i]["k"]
        assert np.max(np.abs(S.cpu().numpy() - dks[i].s[:k]) / dks[i].s[:k]) < 1e-6


def test_batched_zero_problem_rank_deficient(ctx):
    A0 = np.zeros((64, 32), dtype=np.float32)
    dk, st = make_problem(500, 100, 2, "bf16x3", seed=9)
    probs = [dict(A=to_dev(A0), k=3, eps=1e-8, v0=to_dev(synth.start_vectors(3, 32, 1))),
             dict(A=to_dev(dk.A), k=2, eps=1e-12, v0=to_dev(st))]
    out = P.tsvd_dense_batched(ctx, probs, raise_errors=True)
    U, S, V, info = out[0]
    assert info["k_done"] == 0 and info["rank_deficient"]
    assert float(S.abs().max()) == 0 and float(U.abs().max()) == 0 and float(V.abs().max()) == 0
    assert np.max(np.abs(out[1][1].cpu().numpy() - dk.s[:2]) / dk.s[:2]) < 1e-6


def test_batched_rank_below_k(ctx):
    """In a batch: an exact rank-3 FP32 A (1,500 x 300, s = 3, 2, 1) asked for
    k = 6 with fixed iterations, next to a wide rank-2 A (200 x 900, left
    side) asked for k = 4.  The nonzero triplets meet the closed form, the
    rest have sigma at rounding level, U and V stay finite and the iterate
    side of each problem (V for the tall one, U for the wide one) stays
    orthonormal to 1e-10 (or the problem stops rank-deficient after its
    nonzero triplets)."""
    specs = [(1500, 300, 6, [3.0, 2.0, 1.0], 5), (200, 900, 4, [2.0, 0.5], 6)]
    probs, truth = [], []
    for m, n, k, sv, seed in specs:
        s = np.zeros(min(m, n))
        s[:len(sv)] = sv
        dk = synth.dense_known(m, n, s, seed=seed, dtype=np.float32)
        st = synth.start_vectors(k, n if m >= n else m, seed=seed + 50)
        probs.append(dict(A=to_dev(dk.A), k=k, eps=1e-8, v0=to_dev(st), fixed_iters=[200] * k, gram="bf16x3"))
        truth.append((len(sv), s))
    out = P.tsvd_dense_batched(ctx, probs, raise_errors=True)
    for (U, S, V, info), (r, s), p in zip(out, truth, probs):
        U, S, V = U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy()
        k, kd = p["k"], info["k_done"]
        assert kd == k or (info["rank_deficient"] and kd >= r)
        assert np.max(np.abs(S[:r] - s[:r]) / s[:r]) < 1e-6
        assert np.all(S[r:kd] < 1e-5 * s[0])
        W = V if info["branch_right"] else U
        assert np.linalg.norm(W[:, :kd].T @ W[:, :kd] - np.eye(kd)) < 1e-10
        assert np.all(np.isfinite(U)) and np.all(np.isfinite(V))


def test_batched_invalid_arguments_and_budget(ctx):
    dk, st = make_problem(300, 100, 2, "fp32", seed=3)
    good = dict(A=to_dev(dk.A), k=2, eps=1e-8, v0=to_dev(st))
    with pytest.raises(P.TsvdError) as e:
        P.tsvd_dense_batched(ctx, [good, dict(good, k=101, v0=to_dev(synth.start_vectors(101, 100, 1)))])
    assert e.value.status == P.INVALID_ARG
    with pytest.raises(P.TsvdError) as e:
        P.tsvd_dense_batched(ctx, [good, dict(good, A=to_dev(dk.A.astype(np.float64)))])
    assert e.value.status == P.UNSUPPORTED
    with pytest.raises(P.TsvdError) as e:
        P.tsvd_dense_batched(ctx, [good], hbm_budget=1 << 12)
    assert e.value.status == P.OUT_OF_MEMORY
    assert P.tsvd_dense_batched(ctx, []) == []


@pytest.mark.parametrize("team_kib", [512, 1024])
def test_batched_random_mix_team_rules(tuned, team_kib):
    """Forty random shapes per batch under larger team_kib rules (teams read
    most Gram rows from HBM, and some plans fill a workgroup's LDS to the last
    row): every problem meets the closed form; two batches in a row on one
    context both succeed."""
    ctx = tuned
    P.set_tuning(ctx, team_kib=team_kib)
    rng = np.random.default_rng(team_kib)
    for rep in range(2):
        probs, dks = [], []
        for i in range(40):
            m = int(np.exp(rng.uniform(np.log(256), np.log(4096))))
            n = int(np.exp(rng.uniform(np.log(64), np.log(1500))))
            k = int(min(rng.choice([2, 4, 8]), m, n))
            dk, st = make_problem(m, n, k, "bf16x3", seed=1000 * rep + i, q=0.8)
            dks.append(dk)
            probs.append(dict(A=to_dev(dk.A), k=k, eps=1e-12, v0=to_dev(st), gram="bf16x3"))
        out = P.tsvd_dense_batched(ctx, probs, raise_errors=True)
        for dk, p, (U, S, V, info) in zip(dks, probs, out):
            k = p["k"]
            assert info["status"] == "TSVD_OK"
            assert np.max(np.abs(S.cpu().numpy() - dk.s[:k]) / dk.s[:k]) < 1e-6


# one or two shapes per Gram-dimension class 0..5, both sides, ragged tiles;
# the last one has enough contraction rows for the cap on its chunk count to
# bind (24 x 24 tiles of edge 128)
CLASS_MIX = [(3000, 100, 3), (90, 2500, 2), (4000, 257, 4), (200, 5000, 3), (2500, 1000, 4), (700, 1500, 3),
             (6000, 2100, 2), (129, 129, 2), (40000, 3000, 2)]


@pytest.mark.parametrize("gram", ["bf16x3", "fp32"])
def test_batched_tile_edge_same_bits(tuned, gram):
    """The batched Gram's tile edge changes no bit of any result: every Gram
    entry sums the same contraction steps in the same order whichever tile
    holds it (64-wide and 128-wide tiles in every class, both sides, ragged
    edges)."""
    import torch
    ctx = tuned
    probs = []
    g = torch.Generator(device="cuda:0").manual_seed(300)
    for i, (m, n, k) in enumerate(CLASS_MIX):
        A = torch.randn((m, n), generator=g, dtype=torch.float32, device="cuda:0")
        st = synth.start_vectors(k, min(m, n), seed=300 + i)
        probs.append(dict(A=A, k=k, eps=0.0, v0=to_dev(st), gram=gram, fixed_iters=[12] * k))
    outs = []
    for tile in (64, 128):
        P.set_tuning(ctx, group_tile=[tile] * P.GRAM_CLASSES)
        outs.append(P.tsvd_dense_batched(ctx, probs, raise_errors=True))
    for (m, n, k), a, b in zip(CLASS_MIX, outs[0], outs[1]):
        for x, y in zip(a[:3], b[:3]):
            assert torch_equal(x, y), (m, n, P.gram_class(min(m, n)))


def test_batched_class_chunk_alone_equals_mixed(tuned):
    """A class's own chunk length (group_kchunk_cls) applies per problem: a
    problem gives the same bits alone and in a mix, and the chunk length
    changes only FP32 rounding (sigma within 1e-6 of the default's)."""
    ctx = tuned
    probs = []
    for i, (m, n, k) in enumerate(CLASS_MIX[:6]):
        dk, st = make_problem(m, n, k, "bf16x3", seed=400 + i)
        probs.append(dict(A=to_dev(dk.A), k=k, eps=0.0, v0=to_dev(st), gram="bf16x3", fixed_iters=[20] * k))
    ref = P.tsvd_dense_batched(ctx, probs, raise_errors=True)
    cls = P.gram_class(1000)  # the (2500, 1000) problem's class
    kc = [0] * P.GRAM_CLASSES
    kc[cls] = 256
    P.set_tuning(ctx, group_kchunk_cls=kc, group_tile={cls: 64})
    mixed = P.tsvd_dense_batched(ctx, probs, raise_errors=True)
    alone = P.tsvd_dense_batched(ctx, [probs[4]], raise_errors=True)[0]
    for x, y in zip(mixed[4][:3], alone[:3]):
        assert torch_equal(x, y)
    Sm, Sr = mixed[4][1].cpu().numpy(), ref[4][1].cpu().numpy()
    assert np.max(np.abs(Sm - Sr) / Sr) < 1e-6
    for (m, n, k), a, b in zip(CLASS_MIX[:6], mixed, ref):
        if P.gram_class(min(m, n)) != cls:
            for x, y in zip(a[:3], b[:3]):
                assert torch_equal(x, y), (m, n)


def torch_equal(x, y):
    import torch
    return bool(torch.equal(x, y))
