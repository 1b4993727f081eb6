"""Pins of the early-stopped randUTV oracle (oracle.randutv_partial, Sec.
4.1) against the full factorization it truncates: the stopping index is the
first multiple of b at which the full run's trailing Frobenius norm meets
the tolerance (or the rank cap), the reduced leading block is bitwise the
full run's, the paper's update formula for e_i agrees with the direct norm,
and the limiting cases (tol >= 1, kmax = 0, tol = 0) reduce to the identity
and to the full factorization."""
import numpy as np
import pytest

import oracle
from oracle import metrics as M
from synthetic import gaussian_matrix, spectral_matrix, spectrum

U64 = np.finfo(np.float64).eps / 2


def _full(A, b, q, seed):
    return oracle.randutv(A, b, q, seed)


@pytest.mark.parametrize("tol,kmax", [(1e-2, 10 ** 6), (1e-5, 10 ** 6), (1e-9, 10 ** 6),
                                      (0.0, 48), (1e-5, 40), (0.0, 10 ** 6)])
def test_partial_stops_where_the_full_run_meets_the_tolerance(tol, kmax):
    m, n, b = 250, 200, 16
    A = spectral_matrix(m, n, spectrum("geometric", n, decades=8.0), seed=1)
    e0 = np.linalg.norm(A)
    _, Tf, _ = _full(A, b, 1, 3)
    U, T, V, k = oracle.randutv_partial(A, b, 1, 3, tol, kmax)
    # expected k: the first c0 = 0, b, 2b, ... with c0 >= kmax or e(c0) <= tol e0
    # (n itself when no earlier step qualifies)
    want = n
    for c0 in range(0, n, b):
        if c0 >= kmax or np.linalg.norm(Tf[c0:, c0:]) <= tol * e0:
            want = c0
            break
    assert k == want
    # the reduced block is bitwise the full run's; the remainder is unreduced
    np.testing.assert_array_equal(T[:k, :k], Tf[:k, :k])
    assert np.all(T[k:, :k] == 0.0)
    assert abs(np.linalg.norm(T[k:, k:]) - np.linalg.norm(Tf[k:, k:])) <= 100 * n * U64 * e0
    assert M.orth_error(U) < 1e-13 and M.orth_error(V) < 1e-13
    assert M.recon_error(A, U, T, V) < 1e-13


def test_partial_limits():
    A = gaussian_matrix(60, 40, seed=2)
    U, T, V, k = oracle.randutv_partial(A, 8, 1, 5, 1.0, 10 ** 6)
    assert k == 0 and np.array_equal(T, A)
    assert np.array_equal(U, np.eye(60)) and np.array_equal(V, np.eye(40))
    U, T, V, k = oracle.randutv_partial(A, 8, 1, 5, 0.0, 0)
    assert k == 0 and np.array_equal(T, A)
    Uf, Tf, Vf = oracle.randutv(A, 8, 1, 5)
    U, T, V, k = oracle.randutv_partial(A, 8, 1, 5, 0.0, 10 ** 6)
    assert k == 40
    np.testing.assert_array_equal(T, Tf)
    np.testing.assert_array_equal(U, Uf)
    Z = np.zeros((30, 20))
    _, T, _, k = oracle.randutv_partial(Z, 4, 1, 5, 1e-8, 10 ** 6)
    assert k == 0 and np.all(T == 0.0)


def test_frobenius_update_formula_of_the_paper():
    """e_i^2 = e_{i-1}^2 - ||T^(i)(I2, J2 u J3)||_F^2 with e_0 = ||A||_F
    (Sec. 4.1) equals the direct ||T(ib:, ib:)||_F^2 after each step, to
    rounding relative to ||A||_F^2."""
    m, n, b = 120, 96, 16
    A = gaussian_matrix(m, n, seed=3)
    e0sq = np.linalg.norm(A) ** 2
    rec = [e0sq]
    direct = [e0sq]

    def on_step(i, T):
        c0 = b * (i - 1)
        rec.append(rec[-1] - np.linalg.norm(T[c0:c0 + b, c0:]) ** 2)
        direct.append(np.linalg.norm(T[c0 + b:, c0 + b:]) ** 2)

    oracle.randutv(A, b, 1, 7, on_step=on_step)
    np.testing.assert_allclose(rec[:-1], direct[:-1], rtol=0, atol=100 * n * U64 * e0sq)


@pytest.mark.parametrize("tol,kmax", [(1e-5, 10 ** 6), (0.0, 32)])
def test_partial_wide_through_the_transpose(tol, kmax):
    """m < n (Sec. 3.2, as for the full run): the transpose's early stop,
    transposed back. k is where the full wide run's trailing norm first meets
    the criteria, T(:k, :k) is the full run's (lower triangular), T(:k, k:) = 0
    and A = U T V^T."""
    m, n, b = 120, 200, 16
    A = spectral_matrix(n, m, spectrum("geometric", m, decades=8.0), seed=2).T.copy()
    e0 = np.linalg.norm(A)
    _, Tf, _ = _full(A, b, 1, 3)
    U, T, V, k = oracle.randutv_partial(A, b, 1, 3, tol, kmax)
    Ut, Tt, Vt, kt = oracle.randutv_partial(A.T, b, 1, 3, tol, kmax)
    assert k == kt
    np.testing.assert_array_equal(T, Tt.T)
    np.testing.assert_array_equal(U, Vt)
    np.testing.assert_array_equal(V, Ut)
    want = m
    for c0 in range(0, m, b):
        if c0 >= kmax or np.linalg.norm(Tf[c0:, c0:]) <= tol * e0:
            want = c0
            break
    assert k == want and 0 < k < m
    np.testing.assert_array_equal(T[:k, :k], Tf[:k, :k])
    assert np.all(np.triu(T[:k, :k], 1) == 0.0) and np.all(T[:k, k:] == 0.0)
    assert M.orth_error(U) < 1e-13 and M.orth_error(V) < 1e-13
    assert M.recon_error(A, U, T, V) < 1e-13
