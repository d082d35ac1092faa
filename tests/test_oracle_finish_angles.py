"""Pins for the oracle's finishing step (``rayleigh``) and its subspace-angle
helper (``subspace_angles``), CPU only.

``rayleigh`` is Algorithm 1's finish for all triplets at once: u = A v,
sigma = ||u||, u = u / sigma.  It is pinned to the hand-computed 3 x 2 SVD of
tests/golden/hand_3x2.json (exact sigma and U from the exact V), to the
closed-form factors of a constructed matrix, and to the zero-column rule.
``subspace_angles`` is pinned to subspaces built at known angles (including
one below the resolution of an arccos formula and a right angle, where an
unclipped arcsine would return NaN), to invariance under a change of basis,
and to SciPy's independent implementation.  The planted-mistake tests at the
end check that plausible slips fail these pins.
"""

import json
import math
import os

import numpy as np
import pytest

import oracle as O
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold():
    return json.load(open(os.path.join(GOLD, "hand_3x2.json")))


# ---------------------------------------------------------------- rayleigh

def test_rayleigh_hand_example():
    g = _gold()
    A, V = np.array(g["A"]), np.array(g["V"])
    U, s = O.rayleigh(A, V)
    assert s.shape == (2,)
    assert np.allclose(s, g["sigma"], rtol=0, atol=1e-14)
    assert np.allclose(U, np.array(g["U"]), rtol=0, atol=1e-14)


def test_rayleigh_closed_form_factors():
    """A = U diag(s) V^T with exact orthonormal factors: rayleigh(A, V) returns
    (U, s) to FP64 rounding, for the leading columns and for a permuted,
    sign-flipped subset (columns are independent)."""
    s = synth.spectrum_geometric(0.8, 40)
    dk = synth.dense_known(300, 40, s, seed=4)
    U, sv = O.rayleigh(dk.A, dk.V[:, :7])
    assert np.allclose(sv, s[:7], rtol=1e-13, atol=0)
    assert np.allclose(U, dk.U[:, :7], atol=1e-12)
    cols = [5, 0, 3]
    U2, s2 = O.rayleigh(dk.A, -dk.V[:, cols])
    assert np.allclose(s2, s[cols], rtol=1e-13, atol=0)
    assert np.allclose(U2, -dk.U[:, cols], atol=1e-12)


def test_rayleigh_zero_column_left_zero():
    """A v = 0 gives sigma = 0 and a zero u (Algorithm 1 would divide by zero;
    the library and the oracle leave the column zero)."""
    A = np.array([[1.0, 0.0], [0.0, 0.0], [2.0, 0.0]])
    V = np.array([[0.0, 1.0], [1.0, 0.0]])
    U, s = O.rayleigh(A, V)
    assert s[0] == 0.0 and np.all(U[:, 0] == 0.0)
    assert abs(s[1] - math.sqrt(5.0)) < 1e-15
    assert np.allclose(U[:, 1], np.array([1.0, 0.0, 2.0]) / math.sqrt(5.0), atol=1e-15)


def test_rayleigh_left_branch_by_transpose():
    """The m < n branch finishes with A^T u: rayleigh(A^T, U) returns (V, s)."""
    g = _gold()
    A, U = np.array(g["A"]), np.array(g["U"])
    V, s = O.rayleigh(A.T, U)
    assert np.allclose(s, g["sigma"], rtol=0, atol=1e-14)
    assert np.allclose(V, np.array(g["V"]), atol=1e-14)


# ---------------------------------------------------------------- subspace_angles

def _pair_at(theta, d=6):
    """span(e0, e1) and span(cos t e0 + sin t e2, e1): principal angles (0, t)."""
    X = np.zeros((d, 2)); X[0, 0] = 1.0; X[1, 1] = 1.0
    Y = np.zeros((d, 2)); Y[0, 0] = math.cos(theta); Y[2, 0] = math.sin(theta); Y[1, 1] = 1.0
    return X, Y


@pytest.mark.parametrize("theta", [0.3, 1e-3, 1e-9, math.pi / 2])
def test_subspace_angles_known(theta):
    X, Y = _pair_at(theta)
    a = O.subspace_angles(X, Y)
    assert a.shape == (2,)
    assert np.all(np.isfinite(a))
    assert abs(a[0]) < 1e-15
    assert abs(a[1] - theta) <= 1e-14 * max(1.0, theta) + 1e-24


def test_subspace_angles_basis_invariant():
    """A change of basis (scaling, mixing) of either side leaves the angles."""
    X, Y = _pair_at(0.25, d=9)
    R = np.array([[2.0, 1.0], [-0.5, 3.0]])
    a0 = O.subspace_angles(X, Y)
    a1 = O.subspace_angles(X @ R, Y @ R.T)
    assert np.allclose(a0, a1, atol=1e-14)


def test_subspace_angles_against_scipy():
    scipy_linalg = pytest.importorskip("scipy.linalg")
    g = synth.rng(5, 3)
    X = g.standard_normal((30, 4))
    Y = X + 1e-2 * g.standard_normal((30, 4))
    ours = O.subspace_angles(X, Y)
    ref = np.sort(scipy_linalg.subspace_angles(X, Y))
    assert np.allclose(ours, ref, rtol=1e-9, atol=1e-14)


# ---------------------------------------------------------------- planted mistakes

def test_pins_catch_rayleigh_row_norms():
    """Row norms in place of column norms (a transposed reduction axis) fail
    the hand-example pin."""
    g = _gold()
    A, V = np.array(g["A"]), np.array(g["V"])

    def wrong(A, V):
        W = A @ V
        s = np.linalg.norm(W, axis=1)
        return W, s

    _, s = wrong(A, V)
    assert s.shape != (2,) or not np.allclose(s, g["sigma"], atol=1e-12)


def test_pins_catch_rayleigh_from_transposed_operand():
    """u = A^T v is shape-incompatible for a tall A, and for a square A gives
    the wrong singular values of a non-normal matrix."""
    A = np.array([[2.0, 1.0], [0.0, 1.0]])
    V = np.linalg.svd(A)[2].T
    s_true = np.linalg.svd(A, compute_uv=False)
    good = O.rayleigh(A, V)[1]
    wrong = np.linalg.norm(A.T @ V, axis=0)
    assert np.allclose(good, s_true, rtol=1e-14)
    assert not np.allclose(wrong, s_true, rtol=1e-6)


def test_pins_catch_unclipped_or_arccos_angles():
    """An arccos of the cosines loses small angles; an unclipped arcsine of the
    sines returns NaN at a right angle when rounding pushes a sine past 1."""
    X, Y = _pair_at(1e-9)
    qx, _ = np.linalg.qr(X)
    qy, _ = np.linalg.qr(Y)
    cos = np.linalg.svd(qx.T @ qy, compute_uv=False)
    via_acos = np.sort(np.arccos(np.clip(cos, -1, 1)))
    assert abs(via_acos[1] - 1e-9) > 1e-10  # would fail test_subspace_angles_known
    sn = np.array([1.0 + 2.0 ** -52])
    with np.errstate(invalid="ignore"):
        assert np.isnan(np.arcsin(sn)[0])  # what the clip guards against
