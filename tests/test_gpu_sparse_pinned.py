"""Sparse matrices kept out of HBM (the paper's out-of-memory case of degree 1,
Sec. III and Sec. V-C): the CSR in pinned host memory, its sliced tiles built
on the device batch by batch into pinned host memory and streamed back for
every product.  The tiles are the device handle's tiles, so every product and
every t-SVD must be bitwise those of the device handle; the oracle pins both."""

import ctypes

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import paper_2208_08410_amd as P
import synth
from gpu_util import line_angle, to_dev

pytestmark = pytest.mark.gpu


def pinned(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).pin_memory()


def handles(ctx, rp, ci, va, shape, batch_bytes, qd):
    dev = P.tsvd_csr_create(ctx, to_dev(rp), to_dev(ci), to_dev(va), shape)
    pin = P.tsvd_csr_create_pinned(ctx, pinned(rp), pinned(ci), pinned(va), shape, batch_bytes=batch_bytes,
                                   queue_depth=qd)
    return dev, pin


def awkward(m=3000, n=2500, seed=5):
    """Random entries plus a full row, a long column, empty rows and an empty
    band of columns (distinct columns per row, sorted)."""
    rng = np.random.default_rng(seed)
    rows = []
    for r in range(m):
        if r % 97 == 3:
            cols = np.arange(n)  # a full row
        elif r % 13 == 0 or 1000 <= r < 1200:
            cols = np.array([], dtype=np.int64)  # empty rows
        else:
            cols = rng.choice(n, size=int(rng.integers(1, 12)), replace=False)
        cols = np.union1d(cols, [7]) if r % 5 == 0 else cols  # column 7 is long
        cols = cols[(cols < 1500) | (cols >= 1700)]  # an empty band of columns
        rows.append(np.sort(cols))
    rp = np.zeros(m + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(c) for c in rows])
    ci = np.concatenate(rows).astype(np.int32)
    va = rng.standard_normal(ci.size).astype(np.float32)
    return rp, ci, va


@pytest.mark.parametrize("bits", [(0, 0), (5, 9)])
@pytest.mark.parametrize("batch_kib,qd", [(64, 1), (64, 2), (512, 3), (0, 0)])
def test_pinned_products_bitwise(ctx, bits, batch_kib, qd):
    m, n = 3000, 2500
    rp, ci, va = awkward(m, n)
    M = sp.csr_matrix((va.astype(np.float64), ci, rp), shape=(m, n))
    P.set_tuning(ctx, sparse_row_bits=bits[0], sparse_col_bits=bits[1])
    try:
        dev, pin = handles(ctx, rp, ci, va, (m, n), batch_kib * 1024, qd)
    finally:
        P.set_tuning(ctx)
    info = pin.info()
    assert info["loc"] == "pinned_host"
    if batch_kib == 64:
        assert info["batches"] > 1
    for trans in (0, 1):
        for xdt in (np.float32, np.float64):
            nin = n if trans == 0 else m
            x = to_dev(synth.start_vectors(1, nin, seed=trans + 7)[0].astype(xdt))
            yd = P.tsvd_spmv(ctx, dev, x, trans=trans).cpu().numpy()
            yp = P.tsvd_spmv(ctx, pin, x, trans=trans).cpu().numpy()
            assert np.array_equal(yd, yp)
            xr = x.cpu().numpy().astype(np.float64)
            ref = M @ xr if trans == 0 else M.T @ xr
            assert np.allclose(yp, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    dev.close()
    pin.close()


@pytest.mark.parametrize("m,n", [(6000, 4000), (3000, 5000)])
def test_pinned_tsvd_bitwise_and_oracle(ctx, m, n):
    import torch
    k, iters = 4, 40
    rp, ci, va = synth.csr_uniform(m, n, 0.003, seed=m + 1)
    M = sp.csr_matrix((va.astype(np.float64), ci, rp), shape=(m, n))
    dev, pin = handles(ctx, rp, ci, va, (m, n), 48 * 1024, 2)
    d = n if m >= n else m
    st = synth.start_vectors(k, d, seed=9)
    Ud, Sd, Vd, idv = P.tsvd_sparse(ctx, dev, k, 0.0, to_dev(st), max_iter=iters)
    Up, Sp, Vp, ipn = P.tsvd_sparse(ctx, pin, k, 0.0, to_dev(st), max_iter=iters)
    assert torch.equal(Sd.cpu(), Sp.cpu()) and torch.equal(Ud.cpu(), Up.cpu()) and torch.equal(Vd.cpu(), Vp.cpu())
    # every iteration streams both tile sets (8 bytes per nonzero each), plus one product per finished triplet
    nnz = ci.size
    assert ipn["h2d_bytes"] == (2 * k * iters + k) * 8 * nnz
    ref = O.tsvd_implicit(lambda x: M @ x, lambda y: M.T @ y, (m, n), 0.0, k, st, max_iter=iters)
    S = Sp.cpu().numpy()
    assert np.allclose(S, ref.S, rtol=1e-6)
    Ur, Vr = O.canonical(ref.U, ref.V)
    U = Up.cpu().numpy(); V = Vp.cpu().numpy()
    for l in range(k):
        assert line_angle(V[:, l], Vr[:, l]) < 1e-4
        assert line_angle(U[:, l], Ur[:, l]) < 1e-4
    dev.close()
    pin.close()


def test_pinned_many_tiles_with_host_factor(ctx):
    """Library default tiling over many row chunks and five column slices
    (m = n = 1.1e6, Poisson(50) columns per row), tiles streamed in 64 MiB
    batches and V in pinned host memory as well (every array that grows with
    the matrix stays on the host): bitwise the all-device result."""
    import torch
    m = n = 1_100_000
    k, iters = 3, 12
    print(f"[pinned] CSR {m}x{n}", flush=True)
    rp, ci, va = synth.csr_uniform_torch(m, n, 50.0 / n, 17, torch.device("cuda:0"))
    dev = P.tsvd_csr_create(ctx, rp, ci, va, (m, n))
    print("[pinned] pinned build", flush=True)
    pin = P.tsvd_csr_create_pinned(ctx, rp.cpu().pin_memory(), ci.cpu().pin_memory(), va.cpu().pin_memory(), (m, n),
                                   batch_bytes=64 << 20, queue_depth=2)
    info = pin.info()
    assert info["batches"] >= 4 and info["device_bytes"] < dev.info()["device_bytes"] / 4
    st = synth.start_vectors(k, n, seed=19)
    print("[pinned] solves", flush=True)
    Ud, Sd, Vd, _ = P.tsvd_sparse(ctx, dev, k, 0.0, to_dev(st), max_iter=iters)
    Up, Sp, Vp, ip = P.tsvd_sparse(ctx, pin, k, 0.0, to_dev(st), max_iter=iters, factor="host", factor_batches=4)
    assert Vp.is_pinned()
    assert torch.equal(Sd.cpu(), Sp.cpu()) and torch.equal(Ud.cpu(), Up.cpu()) and torch.equal(Vd.cpu(), Vp.cpu())
    dev.close()
    pin.close()


def test_pinned_rejects_bad_structure(ctx):
    m, n = 500, 400
    rp, ci, va = synth.csr_uniform(m, n, 0.01, seed=3)
    bad_col = ci.copy()
    bad_col[17] = n + 5
    with pytest.raises(P.TsvdError, match="INVALID_ARG"):
        P.tsvd_csr_create_pinned(ctx, pinned(rp), pinned(bad_col), pinned(va), (m, n), batch_bytes=4096)
    bad_rp = rp.copy()
    bad_rp[200] = bad_rp[201] + 3  # decreasing inside a chunk
    with pytest.raises(P.TsvdError, match="INVALID_ARG"):
        P.tsvd_csr_create_pinned(ctx, pinned(bad_rp), pinned(ci), pinned(va), (m, n), batch_bytes=4096)
    bad_end = rp.copy()
    bad_end[-1] += 1
    with pytest.raises(P.TsvdError, match="INVALID_ARG"):
        P.tsvd_csr_create_pinned(ctx, pinned(bad_end), pinned(ci), pinned(va), (m, n))
    # device arrays are not pinned host memory
    h = ctypes.c_void_p()
    drp, dci, dva = to_dev(rp), to_dev(ci), to_dev(va)
    st = ctx.lib.tsvd_csr_create_pinned(ctx.handle, m, n, ci.size, ctypes.c_void_p(drp.data_ptr()),
                                        ctypes.c_void_p(dci.data_ptr()), ctypes.c_void_p(dva.data_ptr()), 0, 0,
                                        ctypes.byref(h), None)
    assert st == P.INVALID_ARG and "pinned host" in ctx.last_error()
    # the CSC copy is a device-handle feature
    pin = P.tsvd_csr_create_pinned(ctx, pinned(rp), pinned(ci), pinned(va), (m, n))
    with pytest.raises(P.TsvdError, match="UNSUPPORTED"):
        P.tsvd_csr_get_csc(ctx, pin)
    pin.close()
