"""Seeded synthetic inputs for the truncated-SVD path.

This module only *makes inputs*: matrices with a known spectrum, spiked noise
matrices, random CSR matrices, start vectors and request streams.  It holds
none of the method's arithmetic (no Gram products, no power steps, no
projections), so both the FP64 oracle and the GPU path can take their inputs
from here without sharing any of the computation they are compared on.

Every generator is a pure function of its integer seed(s): sub-streams are
derived with ``numpy.random.SeedSequence`` keyed by (seed, tag, ...), and the
underlying bit generator is Philox (counter based), so any piece can be
regenerated on its own.

Workload recipes (shapes and distributions follow the paper's synthetic
random inputs, Sec. VI-A, and the five configurations this library is
measured on):

* ``dense_known``: A = U diag(s) V^T with U (m x r) and V (n x r) orthonormal
  factors from the Householder QR of a seeded N(0,1) matrix, column signs fixed
  by sign(diag R) (Haar distribution), r = min(m, n).
* ``spectrum_pow10``  s_i = 10^(-i/100);  ``spectrum_geometric`` s_i = q^i
  (i = 0, 1, ...).
* ``spiked_rows``: G + sum_j theta_j x_j y_j^T with G i.i.d. N(0,1),
  orthonormal spike factors and theta_j = strength * sqrt(m) * decay^j;
  rows are generated block by block from counter-based streams.
* ``csr_uniform``: each row has Poisson(density * n) distinct, sorted column
  indices drawn uniformly; values N(0,1) in FP32; int64 row pointers and
  int32 column indices.
* ``start_vectors``: i.i.d. N(0,1) entries (the method normalises them).
* ``request_stream``: Poisson arrivals with log-uniform m, n and k drawn from
  a given set.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "rng",
    "spectrum_pow10",
    "spectrum_geometric",
    "haar_orthonormal",
    "dense_known",
    "dense_known_torch",
    "spiked_factors",
    "spiked_rows",
    "csr_uniform",
    "start_vectors",
    "Request",
    "request_stream",
    "gaussian_dense",
]


def rng(seed: int, *tags: int) -> np.random.Generator:
    """A Philox generator keyed by (seed, *tags)."""
    ss = np.random.SeedSequence([int(seed) & 0xFFFFFFFF, *[int(t) & 0xFFFFFFFF for t in tags]])
    return np.random.Generator(np.random.Philox(ss))


# --- spectra -----------------------------------------------------------------

def spectrum_pow10(count: int) -> np.ndarray:
    """s_i = 10^(-i/100), i = 0..count-1 (FP64)."""
    return 10.0 ** (-np.arange(count, dtype=np.float64) / 100.0)


def spectrum_geometric(q: float, count: int) -> np.ndarray:
    """s_i = q^i, i = 0..count-1 (FP64)."""
    return np.power(float(q), np.arange(count, dtype=np.float64))


# --- dense matrices with a known spectrum -------------------------------------

TAG_U, TAG_V, TAG_START, TAG_NOISE, TAG_SPIKE_X, TAG_SPIKE_Y, TAG_CSR, TAG_REQ = range(1, 9)


def haar_orthonormal(rows: int, cols: int, seed: int, tag: int) -> np.ndarray:
    """rows x cols FP64 matrix with orthonormal columns, Haar distributed.

    Householder QR (LAPACK geqrf/orgqr through numpy) of a seeded N(0,1)
    matrix; column signs are fixed by sign(diag R).
    """
    if cols > rows:
        raise ValueError("need rows >= cols")
    g = rng(seed, tag).standard_normal((rows, cols))
    q, r = np.linalg.qr(g, mode="reduced")
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d


@dataclass
class DenseKnown:
    A: np.ndarray      # m x n, row-major, dtype as requested
    U: np.ndarray      # m x r FP64 (left singular vectors, exact up to FP64)
    s: np.ndarray      # r FP64, non-increasing
    V: np.ndarray      # n x r FP64


def dense_known(m: int, n: int, s: np.ndarray, seed: int, dtype=np.float64) -> DenseKnown:
    """A = U diag(s) V^T with Haar orthonormal factors (see module docstring)."""
    r = min(m, n)
    s = np.asarray(s, dtype=np.float64)
    if s.shape != (r,):
        raise ValueError(f"spectrum must have min(m, n) = {r} entries")
    U = haar_orthonormal(m, r, seed, TAG_U)
    V = haar_orthonormal(n, r, seed, TAG_V)
    A = (U * s) @ V.T
    return DenseKnown(np.ascontiguousarray(A.astype(dtype)), U, s, V)


def dense_known_torch(m: int, n: int, s: np.ndarray, seed: int, device, keep_factors: int = 0):
    """Same recipe as ``dense_known`` on a torch device (FP64 QR), returns FP32 A.

    Used where an m x n FP64 QR is too slow on the host.  The random stream
    is torch's, so A differs from ``dense_known``'s for the same seed; the
    spectrum s is the same.  Returns (A_fp32 [m, n], U[:, :keep], V[:, :keep])
    with the factors in FP64 on the device.
    """
    import torch

    r = min(m, n)
    s_t = torch.as_tensor(np.asarray(s, dtype=np.float64), device=device)
    gen = torch.Generator(device=device)

    def haar(rows, cols, tag):
        gen.manual_seed((int(seed) * 1000003 + tag) & 0x7FFFFFFFFFFFFFFF)
        g = torch.randn(rows, cols, generator=gen, dtype=torch.float64, device=device)
        q, rr = torch.linalg.qr(g, mode="reduced")
        d = torch.sign(torch.diagonal(rr))
        d[d == 0] = 1.0
        del g, rr
        return q * d

    U = haar(m, r, TAG_U)
    V = haar(n, r, TAG_V)
    U.mul_(s_t)
    A = (U @ V.T).to(torch.float32)
    U.div_(s_t)
    Uk = U[:, :keep_factors].clone() if keep_factors else None
    Vk = V[:, :keep_factors].clone() if keep_factors else None
    del U, V
    return A, Uk, Vk


def householder_known_torch(m: int, n: int, s: np.ndarray, seed: int, device, reflectors: int = 2):
    """A = H_L [diag(s); 0] H_R with H_L (m x m) and H_R (n x n) products of
    `reflectors` Householder reflections I - 2 w w^T, w uniform on the sphere:
    exactly orthogonal factors in O(mn) work (no QR), so the singular values
    are s.  Built in FP64 on the device, returned as FP32 [m, n]."""
    import torch

    d = min(m, n)
    g = rng(seed, TAG_U)
    X = torch.zeros((m, n), dtype=torch.float64, device=device)
    idx = torch.arange(d, device=device)
    X[idx, idx] = torch.as_tensor(np.asarray(s[:d], dtype=np.float64), device=device)
    for _ in range(reflectors):
        w = g.standard_normal(n)
        w = torch.as_tensor(w / np.linalg.norm(w), device=device)
        X.sub_(torch.outer(2.0 * (X @ w), w))
    for _ in range(reflectors):
        u = g.standard_normal(m)
        u = torch.as_tensor(u / np.linalg.norm(u), device=device)
        X.sub_(torch.outer(u, 2.0 * (u @ X)))
    A = X.to(torch.float32)
    del X
    return A


def gaussian_dense(m: int, n: int, seed: int, dtype=np.float32) -> np.ndarray:
    """i.i.d. N(0,1) m x n matrix."""
    return rng(seed, TAG_NOISE).standard_normal((m, n)).astype(dtype)


# --- spiked noise matrices (streamed, row block by row block) -----------------

def spiked_factors(m: int, n: int, rank: int, seed: int, strength: float = 50.0, decay: float = 0.9):
    """Orthonormal spike factors x (m x rank), y (n x rank) and strengths theta.

    theta_j = strength * sqrt(m) * decay^j.  x is generated block-wise so that
    very tall m need not be held at once: callers that stream rows ask
    ``spiked_rows`` for a block and get the matching rows of x.
    """
    y = haar_orthonormal(n, rank, seed, TAG_SPIKE_Y)
    theta = strength * math.sqrt(m) * decay ** np.arange(rank, dtype=np.float64)
    return y, theta


def _spike_x_rows(m: int, rank: int, seed: int, row0: int, rows: int) -> np.ndarray:
    """Rows [row0, row0+rows) of an m x rank matrix with orthonormal columns.

    The columns are N(0,1)/sqrt(m) Gaussian vectors, which are orthonormal to
    within O(1/sqrt(m)); callers that need the exact singular values use the
    oracle on the assembled matrix, not a closed form.
    """
    block = 1 << 16
    out = np.empty((rows, rank))
    r = row0
    while r < row0 + rows:
        b = r // block
        off = r - b * block
        take = min(block - off, row0 + rows - r)
        g = rng(seed, TAG_SPIKE_X, b).standard_normal((block, rank))
        out[r - row0:r - row0 + take] = g[off:off + take] / math.sqrt(m)
        r += take
    return out


def spiked_rows(m: int, n: int, rank: int, seed: int, row0: int, rows: int,
                strength: float = 50.0, decay: float = 0.9, dtype=np.float32) -> np.ndarray:
    """Rows [row0, row0+rows) of A = G + sum_j theta_j x_j y_j^T (see module docstring)."""
    y, theta = spiked_factors(m, n, rank, seed, strength, decay)
    block = 1 << 14
    out = np.empty((rows, n), dtype=dtype)
    r = row0
    while r < row0 + rows:
        b = r // block
        off = r - b * block
        take = min(block - off, row0 + rows - r)
        g = rng(seed, TAG_NOISE, b).standard_normal((block, n))[off:off + take]
        x = _spike_x_rows(m, rank, seed, r, take)
        out[r - row0:r - row0 + take] = (g + (x * theta) @ y.T).astype(dtype)
        r += take
    return out


def spiked_rows_torch(m: int, n: int, rank: int, seed: int, row0: int, rows: int, device,
                      strength: float = 50.0, decay: float = 0.9, yfac=None):
    """Rows [row0, row0+rows) of the same spiked recipe, generated on a torch
    device (torch's random stream, seeded per 2^14-row block, so any row range
    is reproducible): A = G + sum_j theta_j x_j y_j^T with G, x i.i.d. N(0, 1)
    (x scaled by 1/sqrt(m)), y the Haar factor of ``spiked_factors`` (pass it
    as ``yfac`` on the device to skip its QR).  FP32."""
    import torch

    if yfac is None:
        y, _ = spiked_factors(m, n, rank, seed, strength, decay)
        yfac = torch.as_tensor(y, device=device)
    theta = torch.as_tensor(strength * math.sqrt(m) * decay ** np.arange(rank, dtype=np.float64), device=device)
    gen = torch.Generator(device=device)
    block = 1 << 14
    out = torch.empty((rows, n), dtype=torch.float32, device=device)
    r = row0
    while r < row0 + rows:
        b = r // block
        off = r - b * block
        take = min(block - off, row0 + rows - r)
        gen.manual_seed((int(seed) * 1000003 + TAG_NOISE * 7919 + b) & 0x7FFFFFFFFFFFFFFF)
        g = torch.randn((block, n), generator=gen, dtype=torch.float32, device=device)[off:off + take]
        gen.manual_seed((int(seed) * 1000003 + TAG_SPIKE_X * 7919 + b) & 0x7FFFFFFFFFFFFFFF)
        x = torch.randn((block, rank), generator=gen, dtype=torch.float64, device=device)[off:off + take]
        x = x / math.sqrt(m)
        out[r - row0:r - row0 + take] = g + ((x * theta) @ yfac.T).to(torch.float32)
        r += take
    return out


def csr_uniform_torch(m: int, n: int, density: float, seed: int, device):
    """CSR on a torch device with the recipe of ``csr_uniform`` except that the
    columns of a row are uniform draws kept in draw order (not sorted; a
    repeated column, probability ~(density n)^2 / 2n per row, stays a repeated
    entry): row lengths Poisson(density * n), values N(0, 1) FP32, int64 row
    pointers, int32 columns.  For sizes too large for the host generator."""
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed((int(seed) * 1000003 + TAG_CSR) & 0x7FFFFFFFFFFFFFFF)
    lam = torch.full((m,), float(density) * n, dtype=torch.float32, device=device)
    counts = torch.poisson(lam, generator=gen).to(torch.int64)
    rowptr = torch.zeros(m + 1, dtype=torch.int64, device=device)
    torch.cumsum(counts, 0, out=rowptr[1:])
    del counts, lam
    nnz = int(rowptr[-1])
    col = torch.randint(0, n, (nnz,), generator=gen, dtype=torch.int32, device=device)
    val = torch.randn(nnz, generator=gen, dtype=torch.float32, device=device)
    return rowptr, col, val


# --- sparse CSR -----------------------------------------------------------------

def csr_uniform(m: int, n: int, density: float, seed: int):
    """Random CSR matrix: Poisson(density*n) distinct sorted columns per row.

    Returns (rowptr int64 [m+1], col int32 [nnz], val float32 [nnz]).
    """
    g = rng(seed, TAG_CSR)
    lam = density * n
    lens = g.poisson(lam, size=m).astype(np.int64)
    lens = np.minimum(lens, n)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(lens, out=rowptr[1:])
    nnz = int(rowptr[-1])
    col = np.empty(nnz, dtype=np.int32)
    # draw with replacement, then redraw the (rare) duplicates row by row
    cols = g.integers(0, n, size=nnz, dtype=np.int64)
    rows_of = np.repeat(np.arange(m, dtype=np.int64), lens)
    key = rows_of * n + cols
    order = np.argsort(key, kind="stable")
    key = key[order]
    dup = np.nonzero(key[1:] == key[:-1])[0] + 1
    cols_sorted = (key - rows_of * n).astype(np.int64)  # rows_of is already row-sorted
    if dup.size:
        for i in np.unique(rows_of[dup]):
            a, b = rowptr[i], rowptr[i + 1]
            L = b - a
            cols_sorted[a:b] = np.sort(g.choice(n, size=L, replace=False))
    col[:] = cols_sorted.astype(np.int32)
    val = g.standard_normal(nnz).astype(np.float32)
    return rowptr, col, val


# --- start vectors ------------------------------------------------------------------

def start_vectors(k: int, dim: int, seed: int) -> np.ndarray:
    """k x dim FP64, i.i.d. N(0,1): row l is the (unnormalised) start vector of triplet l."""
    return rng(seed, TAG_START).standard_normal((k, dim))


# --- request streams -----------------------------------------------------------------

@dataclass
class Request:
    t: float        # arrival time, seconds from stream start
    m: int
    n: int
    k: int
    seed: int


def request_stream(count: int, rate: float, seed: int, m_range=(1024, 65536), n_range=(128, 4096),
                   k_choices=(8, 16, 32, 64)) -> list:
    """Poisson arrivals (exponential gaps, mean 1/rate) with log-uniform shapes."""
    g = rng(seed, TAG_REQ)
    gaps = g.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    lm = g.uniform(math.log(m_range[0]), math.log(m_range[1]), size=count)
    ln = g.uniform(math.log(n_range[0]), math.log(n_range[1]), size=count)
    ks = g.choice(np.asarray(k_choices), size=count)
    out = []
    for i in range(count):
        m = int(round(math.exp(lm[i])))
        n = int(round(math.exp(ln[i])))
        k = int(min(ks[i], m, n))
        out.append(Request(float(t[i]), m, n, k, int(seed) * 100003 + i))
    return out
