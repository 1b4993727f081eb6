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
    "A_instead_of_AT": ("Y = Ap.T @ rnd(V_hat)", "Y = Ap @ rnd(V_hat)"),
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


# ------------------------------------------------ mixed mode (bfloat16 power)
def _spectral(m, n, s, seed=0):
    from synthetic import spectral_matrix
    return spectral_matrix(m, n, s, seed=seed)


def test_mixed_q0_is_fp64():
    """q = 0 has no power products: the mixed mode is the FP64 RURV."""
    A = np.random.default_rng(3).standard_normal((40, 30))
    U1, T1, V1 = oracle.powerurv(A, 0, 5)
    U2, T2, V2 = oracle.powerurv(A, 0, 5, precision="bf16")
    assert np.array_equal(T1, T2) and np.array_equal(V1, V2) and np.array_equal(U1, U2)


def test_mixed_power_of_two_invariance():
    """Scaling A by 2^k leaves the rounded power products' column spaces,
    hence V, unchanged bit for bit, and scales T exactly."""
    A = _spectral(60, 48, np.exp(-np.arange(48) / 6.0))
    U1, T1, V1 = oracle.powerurv(A, 2, 7, precision="bf16")
    U2, T2, V2 = oracle.powerurv(A * 2.0 ** 37, 2, 7, precision="bf16")
    assert np.array_equal(V1, V2) and np.array_equal(U1, U2)
    assert np.array_equal(T2, T1 * 2.0 ** 37)


def test_mixed_rounds_and_keeps_the_subspace():
    """The bfloat16 products move the dominant subspace of V (a gap of 10^3
    after k = 8) by the rounding level, not by zero (the rounding is applied)
    and not by more (it is still captured); the factorization stays exact.
    The trailing columns span singular values below bfloat16's resolution
    relative to the leading ones and may rotate freely."""
    n = 64
    s = np.r_[np.linspace(1.0, 0.5, 8), 1e-3 * np.linspace(1.0, 0.5, n - 8)]
    A = _spectral(80, n, s, seed=2)
    _, _, V64 = oracle.powerurv(A, 1, 3)
    U, T, V = oracle.powerurv(A, 1, 3, precision="bf16")
    assert M.orth_error(U) < 1e-13 and M.orth_error(V) < 1e-13
    assert M.recon_error(A, U, T, V) < 1e-13
    P, P64 = V[:, :8] @ V[:, :8].T, V64[:, :8] @ V64[:, :8].T
    d = np.linalg.norm(P - P64, 2)
    assert 1e-7 < d < 2e-2, d
    _, _, Vt = np.linalg.svd(A)
    Pd = Vt[:8].T
    sin_b = np.linalg.norm(Pd - V[:, :8] @ (V[:, :8].T @ Pd), 2)
    assert sin_b < 2e-2, sin_b


@pytest.mark.parametrize("q", [1, 2])
def test_mixed_rank_revealing_gate(q):
    """e_k of the mixed mode within max(1.5 sigma_{k+1}, 1.1 x the FP64
    envelope over 5 sketch seeds) where sigma_{k+1} is well above rounding."""
    n = 160
    s = np.exp(-np.arange(n) / 40.0)
    A = _spectral(n, n, s, seed=4)
    ks = list(range(0, n, 8))
    env = np.zeros(len(ks))
    for seed in range(5):
        _, T, _ = oracle.powerurv(A, q, 100 + seed)
        env = np.maximum(env, [M.spec(T[k:, k:]) for k in ks])
    _, Tb, _ = oracle.powerurv(A, q, 1, precision="bf16")
    ek = np.array([M.spec(Tb[k:, k:]) for k in ks])
    ok = [i for i, k in enumerate(ks) if s[k] >= 1e-10]
    bad = [ks[i] for i in ok if ek[i] > max(1.5 * s[ks[i]], 1.1 * env[i])]
    assert not bad, bad


def test_mixed_resolution_limit():
    """Below about 1e-3 sigma_1 the bfloat16 power products (rounded relative
    to ||A||) no longer separate directions: e_k there exceeds the FP64
    value, by a bounded factor (here spectrum exp(-j/40), q = 2, e_k at
    sigma ~ 1e-5 is 2-3x the FP64 envelope), while above it the gate holds."""
    n = 512
    s = np.exp(-np.arange(n) / 40.0)
    A = _spectral(n, n, s, seed=3)
    ks = list(range(0, n, 32))
    env = np.zeros(len(ks))
    for seed in range(3):
        _, T, _ = oracle.powerurv(A, 2, 100 + seed)
        env = np.maximum(env, [M.spec(T[k:, k:]) for k in ks])
    _, Tb, _ = oracle.powerurv(A, 2, 1, precision="bf16")
    ek = np.array([M.spec(Tb[k:, k:]) for k in ks])
    hi = [i for i, k in enumerate(ks) if s[k] >= 1e-3]
    lo = [i for i, k in enumerate(ks) if s[k] < 1e-4]
    assert all(ek[i] <= max(1.5 * s[ks[i]], 1.1 * env[i]) for i in hi)
    r = ek[lo] / env[lo]
    assert 1.2 < r.max() < 6.0, r


@pytest.mark.parametrize("precision", ["fp64", "bf16"])
def test_wide_matrix_through_the_transpose(precision):
    """m < n (the reading of Sec. 3.2 used for randUTV): A = U T V^T with
    T = T'^T lower trapezoidal, A^T = U' T' V'^T being the tall transpose's
    factorization; U, V orthogonal, the singular values kept."""
    A = np.random.default_rng(13).standard_normal((30, 52))
    U, T, V = oracle.powerurv(A, 1, 4, precision=precision)
    Ut, Tt, Vt = oracle.powerurv(A.T, 1, 4, precision=precision)
    np.testing.assert_array_equal(T, Tt.T)
    np.testing.assert_array_equal(U, Vt)
    np.testing.assert_array_equal(V, Ut)
    assert U.shape == (30, 30) and T.shape == (30, 52) and V.shape == (52, 52)
    assert np.all(np.triu(T, 1) == 0.0)
    nA = np.linalg.norm(A, 2)
    assert M.orth_error(U) < 1e-13 and M.orth_error(V) < 1e-13
    assert np.linalg.norm(A - U @ T @ V.T, 2) < 1e-13 * nA
    np.testing.assert_allclose(np.linalg.svd(T, compute_uv=False),
                               np.linalg.svd(A, compute_uv=False), atol=1e-13 * nA)
    with pytest.raises(ValueError):
        oracle.powerurv(A, 1, 4, rounds=1)
