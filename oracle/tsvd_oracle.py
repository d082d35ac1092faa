"""FP64 CPU oracle for the power-method truncated SVD.

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports this module; only
the test suite, the smoke check and the CPU-baseline leg of the benchmark do.
It shares no code with the GPU path: every step below is plain NumPy/SciPy in
float64, written to be read against the paper (Boureima et al., "Distributed
Out-of-Memory SVD on CPU/GPU Architectures"):

* Algorithm 1 (SVD, the truncated-SVD driver with deflation),
* Algorithm 2 (SVD_1D, the power method on a Gram matrix),
* Equations 1-3 (the expanded Gram of the deflated residual and its
  right-to-left matrix-vector evaluation),
* Algorithm 3 (dist_gram: the Gram as a sum of block products),
* Algorithm 4 (dist_Compute_v0: the deflated product for a sparse matrix,
  evaluated batch by batch).

Four forms of the method are given, equal in exact arithmetic:

``tsvd_literal``   Deflation by the explicit residual (Algorithm 1): for every
                   triplet the residual X = A - sum_j sigma_j u_j v_j^T is
                   formed in full and the power method runs on its Gram.
                   Memory O(m n) per triplet: small inputs only.
``tsvd_gram``      The Gram B0 = A^T A (or A A^T) is formed once (the paper's
                   dense path reuses the Gram for every iteration, Sec. VI-A)
                   and each triplet runs the power method on P B0 P, with
                   P = I - V V^T applied as two projections.  Because
                   u_j sigma_j = A v_j (Algorithm 1), X_l = A P and
                   X_l^T X_l = P B0 P exactly.
``tsvd_implicit``  The same with B0 x = A^T (A x) from mat-vecs (Equation 2
                   in factored form), for sparse A.
``eq2_apply``      Equation 2's four-term product, kept to show which reading
                   the GPU implements.

Readings taken where the paper is silent, ambiguous or garbled (each is also
listed in the design notes):

R1  The "R_+" in the Require clauses is read as "any real": inputs and the
    normal start vector are signed.
R2  The Ensure clause "U U^T = I_m, V V^T = I_n" is read as U^T U = V^T V = I_k.
R3  U[:l], V[:l], sigma[:l] mean all l-1 triplets already found.
R4  Algorithm 1 computes U^l = A V^l from A, not from the residual X.
R5  The Gram is formed once and deflation is applied by projection (equal to
    re-forming the residual's Gram for every l).
R6  A square A (m == n) takes the A^T A branch (branch on m >= n), as
    Algorithm 4 does; the printed Algorithm 1 uses m > n.  ``branch='paper'``
    keeps the printed test.
R7  Algorithm 2 has no iteration cap; ``max_iter`` is added, and ``eps <= 0``
    means "run exactly max_iter iterations" (the paper's benchmark mode with
    the convergence test disabled).  ``fixed_iters`` imposes a per-triplet
    count (trajectory mode).
R8  The stopping test |v0 . v1| >= 1 - eps is evaluated in float64.
R9  sigma = 0 (a zero product) stops the factorisation: the triplets found so
    far are returned and the rest are zero (rank deficiency).
R10 Start vectors: one N(0, I) draw per triplet, supplied by the caller as
    rows of ``starts`` so that the oracle and the GPU use the same ones.
R11 Several results are equally correct ((u, v) and (-u, -v)); ``canonical``
    fixes the sign so that the largest-magnitude entry of each v is positive
    (ties: lowest index).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "PowerResult",
    "TSVDResult",
    "power_1d",
    "gram_rowblocks",
    "gram_colblocks",
    "tsvd_literal",
    "tsvd_gram",
    "tsvd_implicit",
    "rayleigh",
    "eq1_expanded_gram",
    "eq2_apply",
    "eq3_apply",
    "alg4_compute_v0",
    "alg3_gram_tasks",
    "bf16_round",
    "gram_bf16x3",
    "canonical",
    "subspace_angles",
]


# ----------------------------------------------------------------------------
# Algorithm 2: the power method
# ----------------------------------------------------------------------------

@dataclass
class PowerResult:
    v: np.ndarray       # the returned unit vector v1
    iters: int          # number of products B @ v0 taken
    converged: bool     # the test |v0 . v1| >= 1 - eps was met (always True in fixed mode)
    lam: float          # ||B v0|| at the last step (the eigenvalue estimate)
    zero: bool = False  # B v0 was exactly zero (R9)


def power_1d(apply_B, x0: np.ndarray, eps: float, max_iter: int = 10000,
             fixed_iters: int | None = None) -> PowerResult:
    """Algorithm 2 (SVD_1D) after the Gram is available.

    ``apply_B(x)`` returns B @ x for the symmetric B of Algorithm 2 (X^T X or
    X X^T).  The start vector x0 (a N(0, I) draw) is normalised, then the loop
    takes v1 = B v0, normalises it, and returns v1 once |v0 . v1| >= 1 - eps;
    otherwise v0 = v1 and the loop repeats.  ``eps <= 0`` or ``fixed_iters``
    runs an exact number of iterations instead (R7).
    """
    v0 = np.asarray(x0, dtype=np.float64)
    v0 = v0 / np.linalg.norm(v0)
    fixed = fixed_iters if fixed_iters is not None else (max_iter if eps <= 0 else None)
    it = 0
    while True:
        v1 = apply_B(v0)
        it += 1
        nrm = np.linalg.norm(v1)
        if nrm == 0.0 or not np.isfinite(nrm):
            return PowerResult(v1 * 0.0, it, False, float(nrm), zero=(nrm == 0.0))
        v1 = v1 / nrm
        if fixed is not None:
            if it >= fixed:
                return PowerResult(v1, it, True, float(nrm))
        else:
            if abs(float(v0 @ v1)) >= 1.0 - eps:
                return PowerResult(v1, it, True, float(nrm))
            if it >= max_iter:
                return PowerResult(v1, it, False, float(nrm))
        v0 = v1


# ----------------------------------------------------------------------------
# Algorithm 3: the Gram as a sum of block products
# ----------------------------------------------------------------------------

def gram_rowblocks(A: np.ndarray, rows_per_block: int | None = None) -> np.ndarray:
    """B = sum_b A_b^T A_b over row blocks A_b of A (collinear batching, Alg. 3).

    Equal to A^T A; the row blocks are the batches a host-resident A is
    streamed in.  float64 throughout.
    """
    A = np.asarray(A)
    m, n = A.shape
    rb = m if not rows_per_block else int(rows_per_block)
    B = np.zeros((n, n))
    for r0 in range(0, m, rb):
        Ab = A[r0:r0 + rb].astype(np.float64)
        B += Ab.T @ Ab
    return B


def gram_colblocks(A: np.ndarray, cols_per_block: int | None = None) -> np.ndarray:
    """B = sum_b A_b A_b^T over column blocks A_b (the m < n Gram X X^T)."""
    A = np.asarray(A)
    m, n = A.shape
    cb = n if not cols_per_block else int(cols_per_block)
    B = np.zeros((m, m))
    for c0 in range(0, n, cb):
        Ab = A[:, c0:c0 + cb].astype(np.float64)
        B += Ab @ Ab.T
    return B


def alg3_gram_tasks(A: np.ndarray, n_b: int) -> np.ndarray:
    """Algorithm 3's task list on one device, orthogonal batching.

    A is split into n_b column batches X_j of width b_s = n / n_b; task (i, j)
    with i <= j computes B_ij = X_i^T X_j and its mirror B_ji = B_ij^T
    (the reduced task list of the Gram's symmetric half).  With one device
    the Reduce_sum is the identity.
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    edges = np.linspace(0, n, n_b + 1).astype(int)
    B = np.zeros((n, n))
    for j in range(n_b):
        j0, j1 = edges[j], edges[j + 1]
        Xj = A[:, j0:j1]
        for i in range(j + 1):
            i0, i1 = edges[i], edges[i + 1]
            Bij = A[:, i0:i1].T @ Xj
            B[i0:i1, j0:j1] = Bij
            B[j0:j1, i0:i1] = Bij.T
    return B


def bf16_round(x) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest, ties to even),
    returned as float32.  bfloat16 keeps the top 16 bits of the float32
    pattern; rounding adds 0x7FFF plus the lowest kept bit before truncating.
    (Finite inputs only.)"""
    x = np.ascontiguousarray(x, dtype=np.float32)
    b = x.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def gram_bf16x3(A: np.ndarray, side: str = "right") -> np.ndarray:
    """The Gram of the BF16X3 precision mode, by definition.

    Every FP32 element is split as hi = bf16(a), lo = bf16(a - hi) (a - hi is
    exact in FP32), and B = hi^T hi + hi^T lo + lo^T hi (lo^T lo dropped),
    here accumulated in float64.  side 'left' gives the A A^T analogue.
    """
    a = np.asarray(A, dtype=np.float32)
    hi = bf16_round(a)
    lo = bf16_round(a - hi)
    h = hi.astype(np.float64)
    l_ = lo.astype(np.float64)
    if side == "right":
        return h.T @ h + h.T @ l_ + l_.T @ h
    return h @ h.T + h @ l_.T + l_ @ h.T


# ----------------------------------------------------------------------------
# Algorithm 1: the driver
# ----------------------------------------------------------------------------

@dataclass
class TSVDResult:
    U: np.ndarray            # m x k
    S: np.ndarray            # k
    V: np.ndarray            # n x k
    iters: np.ndarray        # k, power iterations per triplet
    converged: np.ndarray    # k, bool
    lam: np.ndarray          # k, ||B v0|| at the last step of each power loop
    k_done: int = 0          # triplets found before a zero product (R9)
    branch: str = "right"    # "right": v first (A^T A); "left": u first (A A^T)
    extra: dict = field(default_factory=dict)


def _branch_right(m: int, n: int, branch: str) -> bool:
    if branch == "paper":
        return m > n
    if branch == "ge":
        return m >= n
    if branch in ("right", "left"):
        return branch == "right"
    raise ValueError(branch)


def _resolve_k(m: int, n: int, k: int) -> int:
    if k == -1:
        return min(m, n)
    if k <= 0 or k > min(m, n):
        raise ValueError("k must be -1 or in [1, min(m, n)]")
    return k


def _fixed_for(l: int, fixed_iters):
    if fixed_iters is None:
        return None
    return int(fixed_iters[l])


def tsvd_literal(A: np.ndarray, eps: float, k: int = -1, starts: np.ndarray | None = None,
                 max_iter: int = 10000, fixed_iters=None, branch: str = "ge") -> TSVDResult:
    """Truncated SVD with deflation by the explicit residual (Algorithm 1).

    Triplet l is the dominant singular triplet of the residual that remains
    once the l - 1 rank-one terms already found are subtracted from A,
    X_l = A - sum_{j<l} sigma_j u_j v_j^T.  Its right (or left) singular
    vector is the dominant eigenvector of the Gram X_l^T X_l (or X_l X_l^T),
    found by the power method (Algorithm 2); the other vector and sigma then
    come from A itself (reading R4): u = A v / ||A v||, sigma = ||A v||, or
    the mirror for the left branch.  Memory O(m n) per triplet: small inputs
    only.
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    k = _resolve_k(m, n, k)
    right = _branch_right(m, n, branch)
    d = n if right else m
    if starts is None:
        raise ValueError("start vectors are required (R10)")
    U = np.zeros((m, k)); V = np.zeros((n, k)); S = np.zeros(k)
    iters = np.zeros(k, dtype=np.int64); conv = np.zeros(k, dtype=bool); lam = np.zeros(k)
    k_done = k
    for l in range(k):
        X = A.copy()
        if l > 0:
            X = X - (U[:, :l] * S[:l]) @ V[:, :l].T
        B = X.T @ X if right else X @ X.T
        pr = power_1d(lambda x: B @ x, starts[l, :d], eps, max_iter, _fixed_for(l, fixed_iters))
        iters[l], conv[l], lam[l] = pr.iters, pr.converged, pr.lam
        if pr.zero:
            k_done = l
            break
        if right:
            u = A @ pr.v
            s = np.linalg.norm(u)
            if s == 0.0:
                k_done = l
                break
            U[:, l], V[:, l], S[l] = u / s, pr.v, s
        else:
            v = A.T @ pr.v
            s = np.linalg.norm(v)
            if s == 0.0:
                k_done = l
                break
            U[:, l], V[:, l], S[l] = pr.v, v / s, s
    return TSVDResult(U, S, V, iters, conv, lam, k_done, "right" if right else "left")


def _project(Q: np.ndarray, x: np.ndarray) -> np.ndarray:
    """P x = x - Q (Q^T x): projection out of the span of the found vectors (R5)."""
    if Q.shape[1] == 0:
        return x
    return x - Q @ (Q.T @ x)


def tsvd_gram(A: np.ndarray, eps: float, k: int = -1, starts: np.ndarray | None = None,
              max_iter: int = 10000, fixed_iters=None, branch: str = "ge",
              rows_per_block: int | None = None, B0: np.ndarray | None = None) -> TSVDResult:
    """Algorithm 1 with the Gram formed once and deflation by projection (R5).

    B0 = sum_b A_b^T A_b (Algorithm 3, right branch) or A A^T (left branch).
    Triplet l runs Algorithm 2 on P B0 P, P = I - Q Q^T with Q the l-1
    vectors found on the iterated side, then finishes as Algorithm 1 does
    (u = A v, sigma = ||u||, u = u / sigma, or the mirror).
    """
    A = np.asarray(A)
    m, n = A.shape
    k = _resolve_k(m, n, k)
    right = _branch_right(m, n, branch)
    d = n if right else m
    if starts is None:
        raise ValueError("start vectors are required (R10)")
    if B0 is None:
        B0 = gram_rowblocks(A, rows_per_block) if right else gram_colblocks(A)
    A64 = A.astype(np.float64, copy=False)
    Q = np.zeros((d, 0))
    U = np.zeros((m, k)); V = np.zeros((n, k)); S = np.zeros(k)
    iters = np.zeros(k, dtype=np.int64); conv = np.zeros(k, dtype=bool); lam = np.zeros(k)
    k_done = k
    for l in range(k):
        Ql = Q
        pr = power_1d(lambda x: _project(Ql, B0 @ _project(Ql, x)), starts[l, :d], eps, max_iter,
                      _fixed_for(l, fixed_iters))
        iters[l], conv[l], lam[l] = pr.iters, pr.converged, pr.lam
        if pr.zero:
            k_done = l
            break
        w = A64 @ pr.v if right else A64.T @ pr.v
        s = np.linalg.norm(w)
        if s == 0.0:
            k_done = l
            break
        if right:
            U[:, l], V[:, l], S[l] = w / s, pr.v, s
        else:
            U[:, l], V[:, l], S[l] = pr.v, w / s, s
        Q = np.column_stack([Q, pr.v])
    return TSVDResult(U, S, V, iters, conv, lam, k_done, "right" if right else "left")


def tsvd_implicit(matvec, rmatvec, shape, eps: float, k: int = -1, starts: np.ndarray | None = None,
                  max_iter: int = 10000, fixed_iters=None, branch: str = "ge") -> TSVDResult:
    """Algorithm 1 with the implicit deflated product (Equation 2/3, Algorithm 4).

    B0 is never formed.  Right branch: B x = P A^T (A (P x)) -- the factored
    form X'^T (X' x) of Equation 2 with X' = A P; left branch: Q A (A^T (Q x)).
    ``matvec(x)`` = A x and ``rmatvec(y)`` = A^T y in float64.
    """
    m, n = shape
    k = _resolve_k(m, n, k)
    right = _branch_right(m, n, branch)
    d = n if right else m
    if starts is None:
        raise ValueError("start vectors are required (R10)")
    Q = np.zeros((d, 0))
    U = np.zeros((m, k)); V = np.zeros((n, k)); S = np.zeros(k)
    iters = np.zeros(k, dtype=np.int64); conv = np.zeros(k, dtype=bool); lam = np.zeros(k)
    k_done = k
    for l in range(k):
        Ql = Q
        if right:
            op = lambda x: _project(Ql, rmatvec(matvec(_project(Ql, x))))
        else:
            op = lambda x: _project(Ql, matvec(rmatvec(_project(Ql, x))))
        pr = power_1d(op, starts[l, :d], eps, max_iter, _fixed_for(l, fixed_iters))
        iters[l], conv[l], lam[l] = pr.iters, pr.converged, pr.lam
        if pr.zero:
            k_done = l
            break
        w = matvec(pr.v) if right else rmatvec(pr.v)
        s = np.linalg.norm(w)
        if s == 0.0:
            k_done = l
            break
        if right:
            U[:, l], V[:, l], S[l] = w / s, pr.v, s
        else:
            U[:, l], V[:, l], S[l] = pr.v, w / s, s
        Q = np.column_stack([Q, pr.v])
    return TSVDResult(U, S, V, iters, conv, lam, k_done, "right" if right else "left")


def rayleigh(A: np.ndarray, V: np.ndarray):
    """Algorithm 1's finishing step for all triplets at once: U = A V, sigma_j =
    ||U[:, j]||, U[:, j] /= sigma_j (float64)."""
    W = np.asarray(A, dtype=np.float64) @ np.asarray(V, dtype=np.float64)
    s = np.linalg.norm(W, axis=0)
    return W / np.where(s == 0, 1.0, s), s


# ----------------------------------------------------------------------------
# Equations 1-3 and Algorithm 4
# ----------------------------------------------------------------------------

def eq1_expanded_gram(X, U, S, V):
    """Equation 1: X'^T X' expanded as X^T X - V S U^T X - X^T U S V^T + V S^2 V^T.

    The last term uses U^T U = I, as the paper does.
    """
    X = np.asarray(X, dtype=np.float64)
    Sd = np.diag(S)
    return X.T @ X - V @ Sd @ U.T @ X - X.T @ U @ Sd @ V.T + V @ Sd @ Sd @ V.T


def eq2_apply(X, U, S, V, v0):
    """Equation 2: v1 = X^T X v0 - V S U^T X v0 - X^T U S V^T v0 + V S^2 V^T v0,
    each product evaluated right to left (matrix-vector products only)."""
    X = np.asarray(X, dtype=np.float64)
    Xv = X @ v0
    t1 = X.T @ Xv
    t2 = V @ (S * (U.T @ Xv))
    t3 = X.T @ (U @ (S * (V.T @ v0)))
    t4 = V @ (S * S * (V.T @ v0))
    return t1 - t2 - t3 + t4


def eq3_apply(X, U, S, V, v0):
    """Equation 3 (m < n): v1 = X X^T v0 - U S V^T X^T v0 - X V S U^T v0 + U S^2 U^T v0."""
    X = np.asarray(X, dtype=np.float64)
    Xtv = X.T @ v0
    t1 = X @ Xtv
    t2 = U @ (S * (V.T @ Xtv))
    t3 = X @ (V @ (S * (U.T @ v0)))
    t4 = U @ (S * S * (U.T @ v0))
    return t1 - t2 - t3 + t4


def alg4_compute_v0(X, U, S, V, v0, n_b: int):
    """Algorithm 4 (m >= n) on one device (N = 1) with n_b column batches.

    The steps follow the algorithm's order: per batch j the partial products
    X_j (v0)_j are summed to X v0; then (X^T X v0)_j = X_j^T (X v0);
    U^T X v0 and Sigma^T U^T X v0; (V Sigma^T U^T X v0)_j = V_j (...);
    V^T v0 = sum_j V_j^T (v0)_j; Sigma V^T v0; U Sigma V^T v0;
    (X^T U Sigma V^T v0)_j = X_j^T (...); Sigma^2 V^T v0 and
    (V Sigma^2 V^T v0)_j = V_j (...); finally the four terms are combined.
    Printed typos are read as: the batch sums run over n_b batches, V_j is
    V_j^T where it multiplies (v0)_j, the k x 1 sizes, "Sigma^T V^T v0" is
    Sigma^2 V^T v0 and the last term is (V Sigma^2 V^T v0)_j.  The
    all-reduces over devices are identities for N = 1.
    """
    X = np.asarray(X, dtype=np.float64)
    m, n = X.shape
    edges = np.linspace(0, n, n_b + 1).astype(int)
    batches = [(edges[j], edges[j + 1]) for j in range(n_b)]
    Xv0 = np.zeros(m)
    for a, b in batches:                       # X_ij @ (v0)_j, summed over batches
        Xv0 += X[:, a:b] @ v0[a:b]
    XtXv0 = [X[:, a:b].T @ Xv0 for a, b in batches]
    UtXv0 = U.T @ Xv0
    SUtXv0 = S * UtXv0
    VSUtXv0 = [V[a:b] @ SUtXv0 for a, b in batches]
    Vtv0 = np.zeros(len(S))
    for a, b in batches:
        Vtv0 += V[a:b].T @ v0[a:b]
    SVtv0 = S * Vtv0
    USVtv0 = U @ SVtv0
    XtUSVtv0 = [X[:, a:b].T @ USVtv0 for a, b in batches]
    S2Vtv0 = S * SVtv0
    VS2Vtv0 = [V[a:b] @ S2Vtv0 for a, b in batches]
    out = np.empty(n)
    for j, (a, b) in enumerate(batches):
        out[a:b] = XtXv0[j] - VSUtXv0[j] - XtUSVtv0[j] + VS2Vtv0[j]
    return out


# ----------------------------------------------------------------------------
# comparison helpers (conventions, not method arithmetic)
# ----------------------------------------------------------------------------

def canonical(U: np.ndarray, V: np.ndarray):
    """Sign convention (R11): flip (u_j, v_j) so that the largest-|.| entry of
    v_j is positive (ties: lowest index)."""
    U = np.array(U, dtype=np.float64, copy=True)
    V = np.array(V, dtype=np.float64, copy=True)
    for j in range(V.shape[1]):
        i = int(np.argmax(np.abs(V[:, j])))
        if V[i, j] < 0:
            V[:, j] *= -1.0
            U[:, j] *= -1.0
    return U, V


def subspace_angles(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Principal angles (radians, ascending) between span(X) and span(Y).

    Both are orthonormalised first; the sines are the singular values of the
    part of Y's basis outside span(X), which is accurate for small angles.
    """
    qx, _ = np.linalg.qr(np.asarray(X, dtype=np.float64))
    qy, _ = np.linalg.qr(np.asarray(Y, dtype=np.float64))
    r = qy - qx @ (qx.T @ qy)
    sn = np.linalg.svd(r, compute_uv=False)
    return np.sort(np.arcsin(np.clip(sn, 0.0, 1.0)))
