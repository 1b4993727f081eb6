"""Pins for the oracle's Householder steps (Sec. 2.3) and small SVD.

The LAPACK routines are checked against what the paper and the mathematics
fix: Q orthogonal with Q R = A, R upper trapezoidal, the compact reflector
form ``H_i = I - tau_i v_i v_i^T`` with ``v_i(i) = 1`` and ``tau`` in
``{0} ∪ [1, 2]``, the dlarfg sign rule (R_jj opposite in sign to the pivot it
replaces), and the zero-column case giving ``H = I``.
"""
import numpy as np
import pytest

from oracle.hqr import apply_q, form_q, hqr
from oracle.small_svd import small_svd


@pytest.mark.parametrize("m,k", [(7, 3), (12, 12), (40, 9), (5, 1)])
def test_hqr_factorizes(m, k):
    rng = np.random.default_rng(m * 100 + k)
    A = rng.standard_normal((m, k))
    W, tau = hqr(A)
    Q = form_q(W, tau, m)
    R = np.triu(W)
    np.testing.assert_allclose(Q @ R, A, atol=1e-13 * np.abs(A).max())
    np.testing.assert_allclose(Q.T @ Q, np.eye(m), atol=1e-14 * m)
    assert np.all((tau == 0) | ((tau >= 1) & (tau <= 2)))


def test_reflectors_are_explicit_products():
    """Q equals H_1 H_2 ... H_k built from the stored v_i and tau_i."""
    rng = np.random.default_rng(3)
    A = rng.standard_normal((9, 4))
    W, tau = hqr(A)
    Q = np.eye(9)
    for i in range(4):
        v = np.zeros(9)
        v[i] = 1.0
        v[i + 1:] = W[i + 1:, i]
        Q = Q @ (np.eye(9) - tau[i] * np.outer(v, v))
    np.testing.assert_allclose(Q, form_q(W, tau, 9), atol=1e-14)


def test_dlarfg_sign_rule():
    A = np.array([[3.0, 1.0], [4.0, 2.0], [0.0, 5.0]])
    W, _ = hqr(A)
    # beta = -sign(alpha) * ||x||: alpha = 3 > 0 -> R11 = -5
    assert W[0, 0] == pytest.approx(-5.0, rel=1e-15)
    W2, _ = hqr(-A)
    assert W2[0, 0] == pytest.approx(5.0, rel=1e-15)


def test_zero_subcolumn_gives_identity_reflector():
    A = np.array([[2.0, 1.0], [0.0, 3.0], [0.0, 4.0]])
    W, tau = hqr(A)
    assert tau[0] == 0.0
    assert W[0, 0] == 2.0  # H_1 = I keeps the entry (no sign flip)


def test_apply_q_matches_explicit_q():
    rng = np.random.default_rng(5)
    Y = rng.standard_normal((10, 4))
    W, tau = hqr(Y)
    Q = form_q(W, tau, 10)
    C = rng.standard_normal((6, 10))
    np.testing.assert_allclose(apply_q(W, tau, C, "R", "N"), C @ Q, atol=1e-13)
    D = rng.standard_normal((10, 3))
    np.testing.assert_allclose(apply_q(W, tau, D, "L", "T"), Q.T @ D, atol=1e-13)


def test_compact_wy_form():
    """Sec. 2.3: Q = I - Y T Y^T with T upper triangular (Schreiber-Van Loan).

    T is built by the forward recurrence T(1:i-1, i) = -tau_i T Y^T v_i,
    T(i, i) = tau_i and checked against the explicit Q.
    """
    rng = np.random.default_rng(8)
    A = rng.standard_normal((12, 5))
    W, tau = hqr(A)
    Y = np.tril(W, -1)[:, :5] + np.eye(12, 5)
    T = np.zeros((5, 5))
    for i in range(5):
        T[:i, i] = -tau[i] * T[:i, :i] @ (Y[:, :i].T @ Y[:, i])
        T[i, i] = tau[i]
    np.testing.assert_allclose(np.eye(12) - Y @ T @ Y.T, form_q(W, tau, 12), atol=1e-14)


@pytest.mark.parametrize("shape", [(6, 6), (9, 4), (1, 1), (3, 2)])
def test_small_svd_order_signs_reconstruction(shape):
    rng = np.random.default_rng(sum(shape))
    B = rng.standard_normal(shape)
    Us, d, Vs = small_svd(B)
    D = np.zeros(shape)
    D[: d.size, : d.size] = np.diag(d)
    np.testing.assert_allclose(Us @ D @ Vs.T, B, atol=1e-14 * 10)
    assert np.all(np.diff(d) <= 0)
    for j in range(Vs.shape[1]):
        assert Vs[np.argmax(np.abs(Vs[:, j])), j] > 0


def test_small_svd_matches_textbook_2x2():
    # closed form: singular values of [[a, b], [0, c]]
    a, b, c = 3.0, 4.0, 0.5
    B = np.array([[a, b], [0.0, c]])
    s2 = (a * a + b * b + c * c)
    disc = np.sqrt(s2 * s2 - 4 * (a * c) ** 2)
    expect = np.sqrt([(s2 + disc) / 2, (s2 - disc) / 2])
    _, d, _ = small_svd(B)
    np.testing.assert_allclose(d, expect, rtol=1e-14)
