"""Sparse path (CSR validation, CSC build, SpMV, implicit t-SVD) against the oracle."""

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import paper_2208_08410_amd as P
import synth
from gpu_util import line_angle, to_dev

pytestmark = pytest.mark.gpu


def make(m, n, density, seed):
    rp, ci, va = synth.csr_uniform(m, n, density, seed)
    M = sp.csr_matrix((va.astype(np.float64), ci, rp), shape=(m, n))
    return rp, ci, va, M


def register(ctx, rp, ci, va, shape):
    import torch
    return P.tsvd_csr_create(ctx, to_dev(rp), to_dev(ci), to_dev(va), shape)


@pytest.mark.parametrize("m,n,dens", [(3000, 2000, 0.01), (500, 4000, 0.02), (1, 50, 0.5), (50, 1, 0.5), (10000, 10000, 0.0005)])
def test_csc_build_bit_exact(ctx, m, n, dens):
    rp, ci, va, M = make(m, n, dens, seed=m + n)
    c = register(ctx, rp, ci, va, (m, n))
    cp, ri, cv = P.tsvd_csr_get_csc(ctx, c)
    T = sp.csr_matrix((va, ci, rp), shape=(m, n)).tocsc()
    T.sort_indices()
    assert np.array_equal(cp.cpu().numpy(), T.indptr.astype(np.int64))
    assert np.array_equal(ri.cpu().numpy(), T.indices.astype(np.int32))
    assert np.array_equal(cv.cpu().numpy(), T.data.astype(np.float32))


@pytest.mark.parametrize("trans", [0, 1])
@pytest.mark.parametrize("xdt", [np.float32, np.float64])
def test_spmv_matches_fp64(ctx, trans, xdt):
    m, n = 7000, 5000
    rp, ci, va, M = make(m, n, 0.004, seed=3)
    c = register(ctx, rp, ci, va, (m, n))
    nin = n if trans == 0 else m
    x = synth.start_vectors(1, nin, seed=4)[0].astype(xdt)
    y = P.tsvd_spmv(ctx, c, to_dev(x), trans=trans).cpu().numpy()
    ref = (M @ x.astype(np.float64)) if trans == 0 else (M.T @ x.astype(np.float64))
    # every FP32 x FP32 (or FP32 x FP64) product is exact in FP64; only the
    # summation order differs
    assert np.allclose(y, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def awkward_csr(m=500, n=700, seed=11):
    """Random entries plus the cases the sliced tiles must get right: a full
    row (many entries of one row in every tile), a long column, empty rows,
    an empty band of columns, repeated column indices inside a row, and rows
    whose columns are not sorted."""
    rng = np.random.default_rng(seed)
    rows = []
    for r in range(m):
        if r % 37 == 0:
            rows.append(np.array([], dtype=np.int64))  # empty row
        elif r == 7:
            rows.append(rng.permutation(n))  # full row, unsorted
        else:
            k = rng.poisson(0.03 * n)
            cols = rng.integers(0, n, k)
            cols = cols[(cols < 128) | (cols >= 192)]  # no entries in columns 128..191
            if r % 11 == 0 and len(cols):
                cols = np.concatenate([cols, cols[:2]])  # repeats
            if r % 3 == 0:
                cols = np.concatenate([cols, [300]])  # a long column
            rows.append(cols)
    rp = np.zeros(m + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(c) for c in rows])
    ci = np.concatenate(rows).astype(np.int32)
    va = rng.standard_normal(len(ci)).astype(np.float32)
    # scipy sums repeated entries, as the CSR definition does
    M = sp.csr_matrix((va.astype(np.float64), ci, rp), shape=(m, n))
    return rp, ci, va, M


@pytest.mark.parametrize("bits", [(4, 6), (1, 1), (0, 0), (11, 19)])
def test_tiled_products_awkward_matrix(ctx, bits):
    """Both products of the sliced-tile kernels (tiny tiles put one row's
    entries across many tiles and many 64-entry chunks) against FP64 SciPy;
    products are exact in FP64, so only summation order can differ; two runs
    give the same bits."""
    P.set_tuning(ctx, sparse_row_bits=bits[0], sparse_col_bits=bits[1])
    try:
        rp, ci, va, M = awkward_csr()
        c = register(ctx, rp, ci, va, M.shape)
    finally:
        P.set_tuning(ctx)
    for trans in (0, 1):
        nin = M.shape[1] if trans == 0 else M.shape[0]
        for xdt in (np.float32, np.float64):
            x = synth.start_vectors(1, nin, seed=5 + trans)[0].astype(xdt)
            y = P.tsvd_spmv(ctx, c, to_dev(x), trans=trans).cpu().numpy()
            y2 = P.tsvd_spmv(ctx, c, to_dev(x), trans=trans).cpu().numpy()
            ref = (M @ x.astype(np.float64)) if trans == 0 else (M.T @ x.astype(np.float64))
            absref = (abs(M) @ np.abs(x.astype(np.float64))) if trans == 0 else (abs(M).T @ np.abs(x.astype(np.float64)))
            assert np.all(np.abs(y - ref) <= 1e-13 * absref + 1e-300), (bits, trans, xdt)
            assert np.array_equal(y, y2)


def test_invalid_csr_rejected(ctx):
    import torch
    rp, ci, va, M = make(100, 80, 0.05, seed=1)
    bad = ci.copy(); bad[3] = 80
    with pytest.raises(P.TsvdError) as e:
        register(ctx, rp, bad, va, (100, 80))
    assert e.value.status == P.INVALID_ARG
    badp = rp.copy(); badp[10], badp[11] = badp[11], badp[10] - 1
    with pytest.raises(P.TsvdError) as e:
        register(ctx, badp, ci, va, (100, 80))
    assert e.value.status == P.INVALID_ARG


def test_permuted_diagonal_closed_form(ctx):
    """A = P diag(s) Q (permutations): singular values s and unit singular vectors."""
    m, n, k = 3000, 2000, 6
    g = synth.rng(5, 1)
    s = synth.spectrum_geometric(0.8, n)
    rows = g.permutation(m)[:n]
    cols = g.permutation(n)
    M = sp.csr_matrix((s.astype(np.float32).astype(np.float64), (rows, cols)), shape=(m, n))
    M.sort_indices()
    c = register(ctx, M.indptr.astype(np.int64), M.indices.astype(np.int32), M.data.astype(np.float32), (m, n))
    st = synth.start_vectors(k, n, seed=2)
    U, S, V, info = P.tsvd_sparse(ctx, c, k, 1e-14, to_dev(st), max_iter=5000)
    S = S.cpu().numpy(); V = V.cpu().numpy(); U = U.cpu().numpy()
    sf = s.astype(np.float32).astype(np.float64)
    assert np.allclose(S, sf[:k], rtol=1e-9)
    for l in range(k):
        e = np.zeros(n); e[cols[l]] = 1.0
        assert line_angle(V[:, l], e) < 1e-5
        assert V[cols[l], l] > 0  # sign convention
        f = np.zeros(m); f[rows[l]] = 1.0
        assert line_angle(U[:, l], f) < 1e-5


@pytest.mark.parametrize("m,n", [(6000, 4000), (3000, 5000)])
def test_sparse_trajectory_vs_oracle(ctx, m, n):
    """Random sparse matrix, fixed iteration counts (the paper's benchmark
    mode): the GPU gathers x in FP32, so trajectories agree to ~1e-6."""
    k, iters = 4, 60
    rp, ci, va, M = make(m, n, 0.003, seed=m)
    c = register(ctx, rp, ci, va, (m, n))
    d = min(m, n) if m < n else n
    st = synth.start_vectors(k, d, seed=6)
    ref = O.tsvd_implicit(lambda x: M @ x, lambda y: M.T @ y, (m, n), 0.0, k, st, max_iter=iters)
    U, S, V, info = P.tsvd_sparse(ctx, c, k, 0.0, to_dev(st), max_iter=iters)
    assert info["iters"] == [iters] * k
    S = S.cpu().numpy()
    assert np.allclose(S, ref.S, rtol=1e-6)
    V = V.cpu().numpy(); U = U.cpu().numpy()
    Ur, Vr = O.canonical(ref.U, ref.V)
    for l in range(k):
        assert line_angle(V[:, l], Vr[:, l]) < 1e-4
        assert line_angle(U[:, l], Ur[:, l]) < 1e-4
    # the iterated factor is orthonormal to rounding; the other one only as far
    # as the iterates have converged
    Q = V if m >= n else U
    assert np.linalg.norm(Q.T @ Q - np.eye(k)) < 1e-10


def test_sparse_trajectory_many_tiles_vs_oracle(ctx):
    """The library's default tiling at a size where it spans many row chunks
    (2^8-row chunks, 4,297 of them) and five column slices (2^18 columns each,
    the last ragged): m = n = 1.1e6 with Poisson(50) uniform columns per row
    (draw order, repeats kept), k = 4 triplets of 20 fixed iterations each,
    against the implicit oracle on the same matrix (Eq. 2 in factored form,
    Alg. 4's benchmark mode)."""
    import torch
    m = n = 1_100_000
    k, iters = 4, 20
    print(f"[sparse] CSR {m}x{n}, 50 nonzeros per row", flush=True)
    rp, ci, va = synth.csr_uniform_torch(m, n, 50.0 / n, 13, torch.device("cuda:0"))
    M = sp.csr_matrix((va.cpu().numpy().astype(np.float64), ci.cpu().numpy(), rp.cpu().numpy()), shape=(m, n))
    c = P.tsvd_csr_create(ctx, rp, ci, va, (m, n))
    st = synth.start_vectors(k, n, seed=8)
    print("[sparse] oracle", flush=True)
    ref = O.tsvd_implicit(lambda x: M @ x, lambda y: M.T @ y, (m, n), 0.0, k, st, max_iter=iters)
    print("[sparse] GPU", flush=True)
    U, S, V, info = P.tsvd_sparse(ctx, c, k, 0.0, to_dev(st), max_iter=iters)
    assert info["iters"] == [iters] * k
    S = S.cpu().numpy(); V = V.cpu().numpy(); U = U.cpu().numpy()
    assert np.allclose(S, ref.S, rtol=1e-6)
    Ur, Vr = O.canonical(ref.U, ref.V)
    for l in range(k):
        assert line_angle(V[:, l], Vr[:, l]) < 1e-4
        assert line_angle(U[:, l], Ur[:, l]) < 1e-4
    c.close()


def test_sparse_matches_dense_route(ctx):
    """The dense (Gram) and sparse (implicit) routes give the same triplets for
    a sparse matrix small enough to densify (FP64 Gram, tight eps)."""
    m, n, k = 800, 500, 5
    rp, ci, va, M = make(m, n, 0.02, seed=9)
    c = register(ctx, rp, ci, va, (m, n))
    st = synth.start_vectors(k, n, seed=7)
    Us, Ss, Vs, _ = P.tsvd_sparse(ctx, c, k, 0.0, to_dev(st), max_iter=400)
    D = M.toarray()
    Ud, Sd, Vd, _ = P.tsvd_dense(ctx, to_dev(D), k, 0.0, to_dev(st), max_iter=400)
    assert np.allclose(Ss.cpu().numpy(), Sd.cpu().numpy(), rtol=1e-6)


def test_zero_values_rank_deficient(ctx):
    rp, ci, va, M = make(300, 200, 0.02, seed=2)
    c = register(ctx, rp, ci, np.zeros_like(va), (300, 200))
    U, S, V, info = P.tsvd_sparse(ctx, c, 2, 1e-8, to_dev(synth.start_vectors(2, 200, 1)))
    assert info["k_done"] == 0 and info["rank_deficient"]
