"""Parity at the sparse benchmark's full size (CSR 50,000,000 x 50,000,000,
density 1e-6, about 2.5e9 nonzeros, uniform random columns; the library's
default tiles, which bench.py's sparse workload times): sampled outputs of
both products are checked one by one against FP64 dot products of the
matrix's own entries, and the finishing step u = A v / sigma of a short
t-SVD on sampled rows (Alg. 4, Eq. 2 in factored form)."""

import numpy as np
import pytest

import paper_2208_08410_amd as P
import synth

pytestmark = pytest.mark.gpu

N, DENS, SEED = 50_000_000, 1e-6, 2


@pytest.fixture(scope="module")
def c4(ctx):
    import torch
    dev = torch.device("cuda:0")
    print(f"[sparse full size] CSR {N}x{N}, density {DENS}", flush=True)
    rowptr, col, val = synth.csr_uniform_torch(N, N, DENS, SEED, dev)
    csr = P.tsvd_csr_create(ctx, rowptr, col, val, (N, N))
    yield rowptr, col, val, csr
    csr.close()
    del rowptr, col, val
    torch.cuda.empty_cache()


def _row_ref(rowptr, col, val, i, x):
    """FP64 sum over row i's entries of a_ij x_j, and the sum of |a_ij x_j|."""
    a, b = int(rowptr[i]), int(rowptr[i + 1])
    c = col[a:b].long()
    t = val[a:b].double().cpu().numpy() * x[c].double().cpu().numpy()
    return float(np.sum(t)), float(np.sum(np.abs(t)))


def _col_ref(rowptr, col, val, j, x):
    """FP64 sum over column j's entries of a_ij x_i (entries found by a scan
    of the column indices; rows by a search of the row pointers)."""
    import torch
    # (scanned in pieces of 2^30 entries: one nonzero() over all 2.5e9 of
    # them overflows the library's size arithmetic)
    step = 1 << 30
    idx = torch.cat([torch.nonzero(col[s:s + step] == j).flatten() + s for s in range(0, col.numel(), step)])
    rows = torch.searchsorted(rowptr, idx, right=True) - 1
    t = val[idx].double().cpu().numpy() * x[rows].double().cpu().numpy()
    return float(np.sum(t)), float(np.sum(np.abs(t)))


def test_products_sampled(ctx, c4):
    """y = A x and A^T x at full size: every FP32 x FP32 product is exact in
    FP64, so each sampled entry agrees with the FP64 sum to 1e-12 of
    sum |a x| (only the order of the additions differs)."""
    import torch
    rowptr, col, val, csr = c4
    g = torch.Generator(device="cuda:0").manual_seed(11)
    x = torch.randn(N, generator=g, dtype=torch.float32, device="cuda:0")
    y = P.tsvd_spmv(ctx, csr, x, trans=0)
    yt = P.tsvd_spmv(ctx, csr, x, trans=1)
    rng = np.random.default_rng(5)
    picks = [0, 1, 1023, 1024, (1 << 18) - 1, 1 << 18, N // 2, N - 2, N - 1]
    picks += [int(v) for v in rng.integers(0, N, 40)]
    for i in picks:
        ref, mag = _row_ref(rowptr, col, val, i, x)
        assert abs(float(y[i]) - ref) <= 1e-12 * max(mag, 1e-300), ("A x", i)
    for j in picks[:24]:
        ref, mag = _col_ref(rowptr, col, val, j, x)
        assert abs(float(yt[j]) - ref) <= 1e-12 * max(mag, 1e-300), ("A^T x", j)


def test_finish_sampled(ctx, c4):
    """A short t-SVD at full size (one triplet, 5 fixed iterations): v is a
    unit vector, sigma > 0, and sampled rows of u equal (A v)_i / sigma formed
    in FP64 from the matrix's entries and the returned v."""
    import torch
    rowptr, col, val, csr = c4
    g = torch.Generator(device="cuda:0").manual_seed(12)
    v0 = torch.randn((1, N), generator=g, dtype=torch.float64, device="cuda:0")
    U, S, V, info = P.tsvd_sparse(ctx, csr, 1, 0.0, v0, fixed_iters=[5])
    assert info["status"] == "TSVD_OK" and info["iters"] == [5]
    sigma = float(S[0])
    assert sigma > 0
    v = V[:, 0].double()
    assert abs(float(torch.dot(v, v)) - 1.0) < 1e-12
    u = U[:, 0].double()
    rng = np.random.default_rng(6)
    for i in [0, N - 1] + [int(t) for t in rng.integers(0, N, 30)]:
        ref, mag = _row_ref(rowptr, col, val, i, v)
        assert abs(float(u[i]) - ref / sigma) <= 1e-6 * (mag / sigma) + 1e-12, i
