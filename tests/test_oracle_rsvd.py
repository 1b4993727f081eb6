"""Pins of the RSVD oracle (oracle/rsvd.py) against what fixes it
independently: exact recovery of matrices of rank <= l, Eckart-Young's lower
bound on its error and near-optimality with power steps, invariances, and
Theorem 1 of the paper (the rank-l projector of the RSVD equals that of the
first l columns of powerURV's U, computed by the powerURV oracle on the same
Gaussian)."""
import numpy as np
import pytest

import oracle
from oracle import metrics as M
from synthetic import gaussian_matrix, spectral_matrix, spectrum


@pytest.mark.parametrize("m,n,l,q", [(80, 50, 50, 0), (50, 80, 50, 1), (120, 70, 20, 2)])
def test_rsvd_exact_on_rank_le_l(m, n, l, q):
    r = min(l, 12)
    A = gaussian_matrix(m, r, seed=1) @ gaussian_matrix(r, n, seed=2)
    U, s, V = oracle.rsvd(A, l, q, 5)
    assert M.orth_error(U) < 1e-13 and M.orth_error(V) < 1e-13
    np.testing.assert_allclose(U @ np.diag(s) @ V.T, A, atol=1e-12 * np.linalg.norm(A, 2))
    np.testing.assert_allclose(s[:r], np.linalg.svd(A, compute_uv=False)[:r], rtol=1e-12)
    assert np.all(np.diff(s) <= 0)


@pytest.mark.parametrize("q", [0, 1, 2])
def test_rsvd_error_bounds(q):
    m, n, l = 200, 150, 20
    sv = spectrum("geometric", n, decades=6.0)
    A = spectral_matrix(m, n, sv, seed=3)
    U, s, V = oracle.rsvd(A, l, q, 7)
    err = np.linalg.norm(A - U @ np.diag(s) @ V.T, 2)
    assert err >= sv[l] * (1 - 1e-12)       # Eckart-Young
    # no oversampling: measured 2.1-2.7, 1.23-1.34 and 1.07-1.14 sigma_{l+1}
    # over sketch seeds at q = 0, 1, 2 (power steps drive the factor to 1)
    assert err <= {0: 4.0, 1: 1.6, 2: 1.3}[q] * sv[l]
    # the approximate singular values never exceed the true ones
    assert np.all(s <= sv[:l] * (1 + 1e-12))


def test_rsvd_theorem1_matches_powerurv():
    """U_rsvd U_rsvd^T A = U(:, 1:l) U(:, 1:l)^T A with U from powerURV on the
    same G (stream 0, first l columns)."""
    m, n = 120, 90
    A = spectral_matrix(m, n, spectrum("geometric", n, decades=4.0), seed=4)
    for l, q in ((10, 0), (25, 1), (40, 2)):
        Ur, _, _ = oracle.rsvd(A, l, q, 9)
        Up, _, _ = oracle.powerurv(A, q, 9)
        Pl = Up[:, :l] @ (Up[:, :l].T @ A)
        Pr = Ur @ (Ur.T @ A)
        np.testing.assert_allclose(Pr, Pl, atol=1e-9 * np.linalg.norm(A, 2))


def test_rsvd_scaling_invariance():
    A = gaussian_matrix(60, 40, seed=6)
    U, s, V = oracle.rsvd(A, 10, 1, 3)
    U2, s2, V2 = oracle.rsvd(A * 2.0 ** 40, 10, 1, 3)
    np.testing.assert_allclose(s2, s * 2.0 ** 40, rtol=1e-12)
    np.testing.assert_allclose(np.abs(U2.T @ U), np.eye(10), atol=1e-10)
