"""Pins for the powerURV oracle (Alg. 1).

* factorization facts: U (m x m), V (n x n) orthogonal, A = U T V^T with T
  upper trapezoidal (Alg. 1 contract);
* q = 0 is RURV (Sec. 3.1): V is the orthogonal factor of the Gaussian, so
  V^T G is upper triangular;
* for q >= 1 the leading l columns of V span (A^T A)^q G(:, 1:l) (the first
  QR of Sec. 3.3 restricted to l columns), checked on a well-conditioned A;
* Theorem 1 (Sec. 3.3): U(:,1:l) U(:,1:l)^T A equals Q Q^T A for the
  randomized SVD basis Q of (A A^T)^q A G(:, 1:l), computed independently;
* T(k,k) magnitudes equal the R diagonal of A V (definition check by
  Gram-Schmidt on the explicit product).
"""
import types

import numpy as np
import pytest

import oracle
from oracle import metrics as M
from oracle.philox import gaussian

EPS = np.finfo(np.float64).eps


def _well_conditioned(m, n, seed):
    from synthetic import spectral_matrix
    s = np.linspace(2.0, 1.0, n)
    return spectral_matrix(m, n, s, seed=seed)


def pin_failures(fn, A, q, seed=1):
    fails = []
    U, T, V = fn(A, q, seed)
    m, n = A.shape
    tol = 50 * m * EPS
    if M.orth_error(U) > tol:
        fails.append("U not orthogonal")
    if M.orth_error(V) > tol:
        fails.append("V not orthogonal")
    if M.recon_error(A, U, T, V) > tol:
        fails.append("A != U T V^T")
    if np.any(np.tril(T, -1) != 0):
        fails.append("T not upper trapezoidal")
    G = gaussian(seed, 0, n, n)
    if q == 0:
        if np.max(np.abs(np.tril(V.T @ G, -1))) > 1e-12 * np.abs(G).max() * n:
            fails.append("q=0: V is not Q of G")
    else:
        Z = G.copy()
        for _ in range(q):
            Z = A.T @ (A @ Z)
        Z /= np.linalg.norm(Z, axis=0)
        for l in (1, n // 3, n // 2):
            if M.spec(V[:, l:].T @ Z[:, :l]) > 1e-9:
                fails.append(f"V(:,1:{l}) does not span (A^T A)^q G(:,1:{l})")
                break
    for l in (1, n // 4, n // 2):
        Gl = G[:, :l]
        Y = A @ Gl
        for _ in range(q):
            Y = A @ (A.T @ Y)
        Qr, _ = np.linalg.qr(Y)
        lhs = U[:, :l] @ (U[:, :l].T @ A)
        rhs = Qr @ (Qr.T @ A)
        if M.spec(lhs - rhs) > 1e-9 * M.spec(A):
            fails.append(f"Theorem 1 fails at l={l}")
            break
    return fails


@pytest.mark.parametrize("m,n", [(20, 20), (31, 17), (64, 48)])
@pytest.mark.parametrize("q", [0, 1, 2])
def test_pins_well_conditioned(m, n, q):
    A = _well_conditioned(m, n, seed=m + n)
    assert pin_failures(oracle.powerurv, A, q) == []


def test_gaussian_input_factorization():
    A = np.random.default_rng(2).standard_normal((50, 40))
    U, T, V = oracle.powerurv(A, 2, 1)
    assert M.orth_error(U) < 1e-13 and M.orth_error(V) < 1e-13
    assert M.recon_error(A, U, T, V) < 1e-13
    # singular values preserved
    np.testing.assert_allclose(np.linalg.svd(T, compute_uv=False),
                               np.linalg.svd(A, compute_uv=False), atol=1e-12)


def test_r_diagonal_is_gram_schmidt_of_AV():
    A = _well_conditioned(12, 6, seed=3)
    U, T, V = oracle.powerurv(A, 1, 1)
    AV = A @ V
    # classical Gram-Schmidt norms of successive residuals of A V
    Qg = np.zeros_like(AV)
    norms = []
    for j in range(6):
        r = AV[:, j] - Qg[:, :j] @ (Qg[:, :j].T @ AV[:, j])
        r = r - Qg[:, :j] @ (Qg[:, :j].T @ r)
        norms.append(np.linalg.norm(r))
        Qg[:, j] = r / norms[-1]
    np.testing.assert_allclose(np.abs(np.diag(T)), norms, rtol=1e-12)


MUTANTS = {
    "no_rurv_qr_for_q0": ("        V = form_q(W, tau, n)\n    else:", "        V = G\n    else:"),
    "A_instead_of_AT": ("Y = A.T @ V_hat", "Y = A @ V_hat"),
    "skip_final_product": ("A_hat = A @ V\n", "A_hat = A @ G\n"),
    "one_round_less": ("for j in range(q):", "for j in range(max(q - 1, 0)):"),
}


def _mutant(name):
    old, new = MUTANTS[name]
    src = open(oracle.powerurv.__code__.co_filename).read()
    assert src.count(old) == 1, name
    mod = types.ModuleType("oracle._pmutant_" + name)
    mod.__package__ = "oracle"
    exec(compile(src.replace(old, new), "mutant:" + name, "exec"), mod.__dict__)
    return mod.powerurv


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name):
    A = _well_conditioned(24, 24, seed=5)
    q = 0 if name == "no_rurv_qr_for_q0" else 2
    assert pin_failures(_mutant(name), A, q) != [], name
