"""The Lanczos norm estimators used where a full SVD is too costly (the
n = 8192 parity tests and their expected values) agree with exact spectral
norms: clustered top singular values (square Gaussian), fast decay, rank one,
tiny and zero matrices, and the triangular trailing blocks of a factorization."""
import numpy as np
import pytest
import torch

from oracle import metrics as M
import device_norms as D

CASES = ["gauss_square", "gauss_tall", "power_decay", "rank_one", "tiny", "zero", "upper_tri"]


def _matrix(kind):
    rng = np.random.default_rng(3)
    if kind == "gauss_square":
        return rng.standard_normal((1500, 1500))
    if kind == "gauss_tall":
        return rng.standard_normal((1200, 700))
    if kind == "power_decay":
        Q1, _ = np.linalg.qr(rng.standard_normal((800, 800)))
        Q2, _ = np.linalg.qr(rng.standard_normal((800, 800)))
        s = np.arange(1, 801, dtype=float) ** -2.0
        return (Q1 * s) @ Q2.T
    if kind == "rank_one":
        return np.outer(rng.standard_normal(300), rng.standard_normal(200))
    if kind == "tiny":
        return rng.standard_normal((5, 3))
    if kind == "zero":
        return np.zeros((90, 70))
    if kind == "upper_tri":
        return np.triu(rng.standard_normal((900, 900)))
    raise ValueError(kind)


@pytest.mark.parametrize("kind", CASES)
def test_oracle_lanczos_matches_exact(kind):
    X = _matrix(kind)
    exact = np.linalg.norm(X, 2) if X.size else 0.0
    est = M.lanczos_norm(lambda x: X @ x, lambda y: X.T @ y, X.shape[1])
    assert abs(est - exact) <= 1e-13 * max(exact, 1e-300) + 1e-300


@pytest.mark.parametrize("kind", CASES)
def test_torch_gkl_matches_exact(kind):
    X = _matrix(kind)
    exact = np.linalg.norm(X, 2) if X.size else 0.0
    est = D.spec(torch.from_numpy(X))
    assert abs(est - exact) <= 1e-13 * max(exact, 1e-300) + 1e-300


def test_torch_helpers_on_a_factorization():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((400, 300))
    Q, R = np.linalg.qr(A, mode="complete")
    U, T, V = Q, R, np.eye(300)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x))
    assert abs(D.orth_error(t(U)) - M.orth_error(U)) <= 1e-17 + 1e-3 * M.orth_error(U)
    rec = D.recon_error(t(A), t(U), t(T), t(V), np.linalg.norm(A, 2))
    # both are rounding noise of the product (the operator form rounds differently)
    assert rec <= 1e-14 and abs(rec - M.recon_error(A, U, T, V)) <= 1e-15
    # a planted error of known size is measured exactly
    E = np.zeros_like(A)
    E[7, 9] = 1e-9
    rec = D.recon_error(t(A + E), t(U), t(T), t(V), 1.0)
    assert abs(rec - 1e-9) <= 1e-12
