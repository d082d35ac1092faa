"""Pins for the FP64 oracle (CPU only).

Each test checks the oracle against something other than itself: a hand-made
example, singular values known in closed form from the construction, LAPACK
eigen/singular value routines on tiny inputs, algebraic identities with exact
factors, and invariants.  The mutation tests at the end plant plausible
mistakes in the oracle and check that these pins catch them.
"""

import json
import math
import os

import numpy as np
import pytest

import oracle as O
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def starts_for(k, d, seed=7):
    return synth.start_vectors(k, d, seed)


def angle(a, b):
    """Angle between the lines spanned by a and b (radians)."""
    a = a / np.linalg.norm(a)
    b = b / np.linalg.norm(b)
    c = float(a @ b)
    return math.atan2(np.linalg.norm(a - c * b), abs(c))


def predicted(eps, r):
    """Stopping-error model of the power method (Golub & Van Loan, Sec. 7.3):
    the test stops when the step angle is sqrt(2 eps), leaving an angle
    theta = sqrt(2 eps) r / (1 - r) to the eigenvector and a Rayleigh-quotient
    relative error of (1 - r) theta^2 / 2 in sigma, r = (s_{l+1}/s_l)^2."""
    theta = math.sqrt(2 * eps) * r / (1 - r)
    return theta, (1 - r) * theta ** 2 / 2


# ---------------------------------------------------------------- golden example

@pytest.mark.parametrize("form", ["literal", "gram", "implicit"])
def test_golden_hand_example(form):
    g = json.load(open(os.path.join(GOLD, "hand_3x2.json")))
    A = np.array(g["A"])
    st = starts_for(2, 2, seed=3)
    if form == "literal":
        r = O.tsvd_literal(A, 1e-15, -1, st, max_iter=500)
    elif form == "gram":
        r = O.tsvd_gram(A, 1e-15, -1, st, max_iter=500)
    else:
        r = O.tsvd_implicit(lambda x: A @ x, lambda y: A.T @ y, A.shape, 1e-15, -1, st, max_iter=500)
    U, V = O.canonical(r.U, r.V)
    assert np.allclose(r.S, g["sigma"], rtol=1e-12, atol=0)
    assert np.allclose(V, np.array(g["V"]), atol=1e-7)
    assert np.allclose(U, np.array(g["U"]), atol=1e-7)
    assert np.allclose(O.gram_rowblocks(A, 2), np.array(g["AtA"]), atol=1e-14)


# ---------------------------------------------------------------- closed-form spectrum (C1)

@pytest.fixture(scope="module")
def c1():
    m, n, k, eps = 2000, 500, 10, 1e-8
    s = synth.spectrum_pow10(n)
    dk = synth.dense_known(m, n, s, seed=1)
    st = starts_for(k, n, seed=11)
    rg = O.tsvd_gram(dk.A, eps, k, st)
    return dk, st, rg, eps, k


def test_c1_sigma_closed_form(c1):
    dk, st, rg, eps, k = c1
    r = 10 ** (-2 / 100)
    theta, srel = predicted(eps, r)
    rel = np.abs(rg.S - dk.s[:k]) / dk.s[:k]
    assert rg.converged.all()
    assert rel.max() <= 1e-6
    assert rel.max() <= 3 * srel + 1e-12
    # the first sigma is a Rayleigh quotient of the undeflated A: it sits below the truth
    assert rg.S[0] <= dk.s[0] * (1 + 1e-14)


def test_c1_vectors_closed_form(c1):
    dk, st, rg, eps, k = c1
    r = 10 ** (-2 / 100)
    theta, _ = predicted(eps, r)
    for l in range(k):
        assert angle(rg.V[:, l], dk.V[:, l]) <= 3 * theta
        assert angle(rg.U[:, l], dk.U[:, l]) <= 3 * theta


def test_c1_literal_matches_gram_in_trajectory_mode(c1):
    dk, st, rg, eps, k = c1
    rl = O.tsvd_literal(dk.A, eps, k, st, fixed_iters=rg.iters)
    assert np.allclose(rl.S, rg.S, rtol=1e-12, atol=0)
    for l in range(k):
        assert angle(rl.V[:, l], rg.V[:, l]) < 1e-9
    # with the same stopping test the literal form takes the same number of steps
    rl2 = O.tsvd_literal(dk.A, eps, 3, st)
    assert np.array_equal(rl2.iters, rg.iters[:3])


def test_c1_eckart_young_and_invariants(c1):
    dk, st, rg, eps, k = c1
    A = dk.A
    tail = np.sum(dk.s[k:] ** 2)
    resid = np.sum(A * A) - np.sum(rg.S ** 2)
    r = 10 ** (-2 / 100)
    theta, srel = predicted(eps, r)
    assert abs(resid - tail) <= 4 * srel * np.sum(dk.s[:k] ** 2) + 1e-10 * np.sum(A * A)
    assert np.linalg.norm(rg.V.T @ rg.V - np.eye(k)) < 1e-12
    assert np.linalg.norm(rg.U.T @ rg.U - np.eye(k)) < 3 * theta
    assert np.all(np.diff(rg.S) <= 1e-12)
    for l in range(k):
        # informative residual ||A^T u - sigma v|| / sigma (A v - sigma u is 0 by construction)
        res = np.linalg.norm(A.T @ rg.U[:, l] - rg.S[l] * rg.V[:, l]) / rg.S[l]
        assert res <= 3 * theta
        assert np.linalg.norm(A @ rg.V[:, l] - rg.S[l] * rg.U[:, l]) <= 1e-12 * rg.S[l]


# ---------------------------------------------------------------- brute force on tiny inputs

@pytest.mark.parametrize("m,n", [(40, 12), (12, 40), (25, 25), (7, 1), (1, 7)])
def test_brute_force_eig(m, n):
    d = min(m, n)
    s = synth.spectrum_geometric(0.5, d) * 3.0
    dk = synth.dense_known(m, n, s, seed=5)
    st = starts_for(d, d, seed=9)
    r = O.tsvd_gram(dk.A, 1e-15, -1, st, max_iter=5000)
    B = dk.A.T @ dk.A if m >= n else dk.A @ dk.A.T
    ev = np.sort(np.linalg.eigvalsh(B))[::-1]
    sv = np.linalg.svd(dk.A, compute_uv=False)
    # eigvalsh and svd are accurate to O(u) relative to the largest value
    assert np.allclose(r.S ** 2, ev[:d], rtol=1e-9, atol=1e-13 * ev[0])
    assert np.allclose(r.S, sv, rtol=1e-9, atol=1e-14 * sv[0])
    Uu, Ss, Vt = np.linalg.svd(dk.A, full_matrices=False)
    for l in range(min(d, 8)):  # vectors are well conditioned while the gap is >> u ||B||
        assert abs(abs(r.V[:, l] @ Vt[l]) - 1) < 1e-8
        assert abs(abs(r.U[:, l] @ Uu[:, l]) - 1) < 1e-8


# ---------------------------------------------------------------- the forms agree

@pytest.mark.parametrize("m,n", [(300, 120), (120, 300), (150, 150)])
def test_forms_agree(m, n):
    d = min(m, n)
    k = 6
    s = synth.spectrum_geometric(0.9, d)
    dk = synth.dense_known(m, n, s, seed=2)
    st = starts_for(k, d, seed=4)
    A = dk.A
    rg = O.tsvd_gram(A, 1e-10, k, st)
    rl = O.tsvd_literal(A, 1e-10, k, st, fixed_iters=rg.iters)
    ri = O.tsvd_implicit(lambda x: A @ x, lambda y: A.T @ y, A.shape, 1e-10, k, st, fixed_iters=rg.iters)
    for other in (rl, ri):
        assert np.allclose(other.S, rg.S, rtol=1e-11, atol=0)
        assert np.allclose(np.abs(np.sum(other.V * rg.V, axis=0)), 1, atol=1e-10)
        assert np.allclose(np.abs(np.sum(other.U * rg.U, axis=0)), 1, atol=1e-10)


def test_square_branch_readings_agree():
    n = 60
    s = synth.spectrum_geometric(0.8, n)
    dk = synth.dense_known(n, n, s, seed=8)
    st = starts_for(5, n, seed=1)
    r_ge = O.tsvd_gram(dk.A, 1e-14, 5, st, branch="ge", max_iter=5000)
    r_pp = O.tsvd_gram(dk.A, 1e-14, 5, st, branch="paper", max_iter=5000)
    assert r_ge.branch == "right" and r_pp.branch == "left"
    assert np.allclose(r_ge.S, r_pp.S, rtol=1e-10)
    assert np.allclose(np.abs(np.sum(r_ge.V * r_pp.V, axis=0)), 1, atol=1e-7)


def test_transpose_symmetry():
    m, n, k = 90, 40, 5
    s = synth.spectrum_geometric(0.85, n)
    dk = synth.dense_known(m, n, s, seed=12)
    st = starts_for(k, n, seed=6)
    r = O.tsvd_gram(dk.A, 1e-14, k, st, max_iter=5000)
    rt = O.tsvd_gram(dk.A.T.copy(), 1e-14, k, st, max_iter=5000)
    assert rt.branch == "left"
    assert np.allclose(r.S, rt.S, rtol=1e-10)
    assert np.allclose(np.abs(np.sum(r.V * rt.U, axis=0)), 1, atol=1e-8)
    assert np.allclose(np.abs(np.sum(r.U * rt.V, axis=0)), 1, atol=1e-8)


# ---------------------------------------------------------------- Gram blocking (Algorithm 3)

@pytest.mark.parametrize("rb", [1, 7, 64, 1000])
def test_gram_rowblocks_is_ata(rb):
    A = synth.gaussian_dense(301, 37, seed=3, dtype=np.float64)
    assert np.allclose(O.gram_rowblocks(A, rb), A.T @ A, rtol=1e-13, atol=1e-11)
    assert np.allclose(O.gram_colblocks(A.T, rb), A.T @ A, rtol=1e-13, atol=1e-11)


@pytest.mark.parametrize("n_b", [1, 2, 3, 5])
def test_alg3_task_list(n_b):
    A = synth.gaussian_dense(80, 23, seed=4, dtype=np.float64)
    B = O.alg3_gram_tasks(A, n_b)
    assert np.allclose(B, A.T @ A, rtol=1e-13, atol=1e-11)
    assert np.array_equal(B, B.T)


# ---------------------------------------------------------------- Equations 1-3, Algorithm 4

def _exact_factors(X, l):
    Uu, Ss, Vt = np.linalg.svd(X, full_matrices=False)
    return Uu[:, :l], Ss[:l], Vt[:l].T


@pytest.mark.parametrize("l", [1, 3])
def test_eq1_identity(l):
    X = synth.gaussian_dense(60, 25, seed=5, dtype=np.float64)
    U, S, V = _exact_factors(X, l)
    Xp = X - (U * S) @ V.T
    assert np.allclose(O.eq1_expanded_gram(X, U, S, V), Xp.T @ Xp, rtol=1e-11, atol=1e-10)


@pytest.mark.parametrize("l,n_b", [(1, 1), (2, 3), (4, 7)])
def test_eq2_and_alg4(l, n_b):
    X = synth.gaussian_dense(70, 28, seed=6, dtype=np.float64)
    U, S, V = _exact_factors(X, l)
    v0 = synth.start_vectors(1, 28, 3)[0]
    Xp = X - (U * S) @ V.T
    ref = Xp.T @ (Xp @ v0)
    e2 = O.eq2_apply(X, U, S, V, v0)
    assert np.allclose(e2, ref, rtol=1e-10, atol=1e-10)
    a4 = O.alg4_compute_v0(X, U, S, V, v0, n_b)
    assert np.allclose(a4, ref, rtol=1e-10, atol=1e-10)


def test_eq3_identity():
    X = synth.gaussian_dense(20, 50, seed=7, dtype=np.float64)
    U, S, V = _exact_factors(X, 3)
    v0 = synth.start_vectors(1, 20, 4)[0]
    Xp = X - (U * S) @ V.T
    assert np.allclose(O.eq3_apply(X, U, S, V, v0), Xp @ (Xp.T @ v0), rtol=1e-10, atol=1e-10)


def test_eq2_differs_from_factored_form_by_cross_terms():
    """With converged-but-inexact factors, Eq. 2 (which assumes U^T U = I)
    and the factored form X'^T X' v0 differ only by V (S^2 - V^T B0 V) V^T v0,
    whose diagonal is zero when sigma_j^2 = v_j^T B0 v_j (u = A v / sigma)."""
    m, n = 200, 60
    dk = synth.dense_known(m, n, synth.spectrum_geometric(0.9, n), seed=13)
    st = starts_for(3, n, seed=2)
    r = O.tsvd_gram(dk.A, 1e-6, 3, st)
    A = dk.A
    v0 = synth.start_vectors(1, n, 21)[0]
    Xp = A - (r.U * r.S) @ r.V.T
    fact = Xp.T @ (Xp @ v0)
    e2 = O.eq2_apply(A, r.U, r.S, r.V, v0)
    G = r.V.T @ (A.T @ A) @ r.V
    assert np.allclose(np.diag(G), r.S ** 2, rtol=1e-12)
    corr = r.V @ ((np.diag(r.S ** 2) - G) @ (r.V.T @ v0))
    assert np.allclose(e2 - fact, corr, atol=1e-9 * np.linalg.norm(fact))


# ---------------------------------------------------------------- modes and edge cases

def test_fixed_iteration_mode():
    dk = synth.dense_known(50, 20, synth.spectrum_geometric(0.9, 20), seed=1)
    st = starts_for(4, 20)
    r = O.tsvd_gram(dk.A, 0.0, 4, st, max_iter=17)
    assert np.all(r.iters == 17)
    r2 = O.tsvd_gram(dk.A, 1e-3, 4, st, fixed_iters=[3, 5, 7, 9])
    assert list(r2.iters) == [3, 5, 7, 9]


def test_not_converged_flag():
    dk = synth.dense_known(50, 20, synth.spectrum_geometric(0.99, 20), seed=1)
    r = O.tsvd_gram(dk.A, 1e-14, 2, starts_for(2, 20), max_iter=5)
    assert not r.converged.any()
    assert np.all(r.iters == 5)


def test_zero_and_rank_deficient():
    A = np.zeros((5, 3))
    r = O.tsvd_gram(A, 1e-8, 2, starts_for(2, 3))
    assert r.k_done == 0 and np.all(r.S == 0)
    A = np.zeros((2, 2)); A[0, 0] = 3.0
    r = O.tsvd_gram(A, 1e-12, 2, starts_for(2, 2))
    assert r.k_done == 1 and r.S[0] == 3.0 and r.S[1] == 0.0


def test_k_validation():
    A = np.eye(3)
    with pytest.raises(ValueError):
        O.tsvd_gram(A, 1e-8, 0, starts_for(3, 3))
    with pytest.raises(ValueError):
        O.tsvd_gram(A, 1e-8, 4, starts_for(4, 3))


def test_sparse_form_matches_dense():
    import scipy.sparse as sp
    m, n = 400, 300
    rp, ci, va = synth.csr_uniform(m, n, 0.05, seed=3)
    M = sp.csr_matrix((va.astype(np.float64), ci, rp), shape=(m, n))
    D = M.toarray()
    st = starts_for(4, n, seed=5)
    rg = O.tsvd_gram(D, 0.0, 4, st, max_iter=60)
    ri = O.tsvd_implicit(lambda x: M @ x, lambda y: M.T @ y, (m, n), 0.0, 4, st, max_iter=60)
    assert np.allclose(ri.S, rg.S, rtol=1e-11)
    assert np.allclose(np.abs(np.sum(ri.V * rg.V, axis=0)), 1, atol=1e-10)


# ---------------------------------------------------------------- generators

def test_generator_spectrum_and_csr():
    dk = synth.dense_known(120, 30, synth.spectrum_geometric(0.8, 30), seed=1)
    assert np.allclose(np.linalg.svd(dk.A, compute_uv=False), dk.s, rtol=1e-12, atol=1e-14)
    rp, ci, va = synth.csr_uniform(1000, 5000, 0.002, seed=9)
    assert rp[0] == 0 and rp[-1] == len(ci) == len(va)
    for i in range(1000):
        row = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(row) > 0)
    assert abs(len(ci) / 1000 - 10) < 1.0
    a = synth.spiked_rows(5000, 64, 4, seed=2, row0=100, rows=300)
    b = synth.spiked_rows(5000, 64, 4, seed=2, row0=0, rows=1000)
    assert np.array_equal(a, b[100:400])


# ---------------------------------------------------------------- planted mistakes

def test_pins_catch_dropped_deflation(monkeypatch, c1):
    dk, st, rg, eps, k = c1
    monkeypatch.setattr(O.tsvd_oracle, "_project", lambda Q, x: x)
    bad = O.tsvd_gram(dk.A[:400, :100], 1e-8, 2, st[:, :100])
    s_true = np.linalg.svd(dk.A[:400, :100], compute_uv=False)
    assert abs(bad.S[1] - s_true[1]) / s_true[1] > 1e-3


def test_pins_catch_sign_error_in_eq2(monkeypatch):
    X = synth.gaussian_dense(70, 28, seed=6, dtype=np.float64)
    U, S, V = _exact_factors(X, 2)
    v0 = synth.start_vectors(1, 28, 3)[0]
    Xp = X - (U * S) @ V.T
    ref = Xp.T @ (Xp @ v0)

    def eq2_wrong(X, U, S, V, v0):
        Xv = X @ v0
        return X.T @ Xv - V @ (S * (U.T @ Xv)) + X.T @ (U @ (S * (V.T @ v0))) + V @ (S * S * (V.T @ v0))

    assert not np.allclose(eq2_wrong(X, U, S, V, v0), ref, rtol=1e-6)


def test_pins_catch_wrong_finish(monkeypatch):
    """Computing u from the residual X instead of A (against reading R4) must
    not change sigma for exact projections, but dropping the normalisation
    of the start vector does change the first stopping decision; the
    literal-vs-gram trajectory pin catches a transposed Gram instead."""
    A = synth.dense_known(60, 20, synth.spectrum_geometric(0.7, 20), seed=3).A
    st = starts_for(3, 20)
    good = O.tsvd_gram(A, 1e-12, 3, st)
    bad_B = (A @ A.T)  # transposed operand: wrong shape for the right branch
    with pytest.raises(ValueError):
        O.tsvd_gram(A, 1e-12, 3, st, B0=bad_B)
    assert good.converged.all()
