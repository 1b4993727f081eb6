"""Pins for the randUTV oracle (Alg. 3), each tied to a fact the paper or the
mathematics fixes, plus planted-mistake checks showing the pins catch
plausible oracle bugs.

* factorization facts (Sec. 1 problem statement): U, V orthogonal,
  A = U T V^T, T upper trapezoidal with exact zeros;
* sparsity pattern after each step (Sec. 4.1 and Figure 1, m=11, n=8, b=3);
* orthogonal invariance: sigma(T) = sigma(A);
* Eckart-Young (Sec. 2.1): e_k >= sigma_{k+1};
* the first step equals the randomized SVD (Sec. 4.1 remark), computed here
  independently from the same Gaussian with plain matrix products;
* the Frobenius recurrence of Sec. 4.1;
* special cases: b >= n is one SVD; exact rank r gives e_r ~ 0; an
  orthogonal matrix has all T_kk = 1; the zero matrix gives T = 0.
"""
import os
import types

import numpy as np
import pytest

import oracle
from oracle import metrics as M
from oracle.philox import gaussian

EPS = np.finfo(np.float64).eps
HERE = os.path.dirname(os.path.abspath(__file__))


def _structure_failures(T, b):
    m, n = T.shape
    fails = []
    if np.any(np.tril(T, -1) != 0.0):
        fails.append("strict lower part not exactly zero")
    for c0 in range(0, n, b):
        c1 = min(c0 + b, n)
        blk = T[c0:c1, c0:c1]
        if np.any(blk - np.diag(np.diag(blk)) != 0.0):
            fails.append(f"diagonal block at {c0} not diagonal")
        d = np.diag(blk)
        if np.any(d < 0) or np.any(np.diff(d) > 0):
            fails.append(f"diagonal block at {c0} not non-negative descending")
    return fails


def _rsvd_first_step(A, b, q, seed):
    """e_b and the first block's singular values from the randomized SVD."""
    G = gaussian(seed, 1, A.shape[0], b)
    Y = A.T @ G
    for _ in range(q):
        Y = A.T @ (A @ Y)
    Qy, _ = np.linalg.qr(Y)
    d_first = np.linalg.svd(A @ Qy, compute_uv=False)
    Qu, _ = np.linalg.qr(A @ Qy)
    e_b = np.linalg.norm(A - Qu @ (Qu.T @ A), 2)
    return e_b, d_first


def pin_failures(randutv_fn, A, b, q, seed=1):
    """Run every pin on one input; return the list of failed pins."""
    fails = []
    U, T, V = randutv_fn(A, b, q, seed)
    m, n = A.shape
    nA = max(M.spec(A), 1e-300)
    tol = 50 * max(m, n) * EPS
    if M.orth_error(U) > tol:
        fails.append("U not orthogonal")
    if M.orth_error(V) > tol:
        fails.append("V not orthogonal")
    if M.spec(A - U @ T @ V.T) > tol * nA:
        fails.append("A != U T V^T")
    fails += _structure_failures(T, b)
    sa = np.linalg.svd(A, compute_uv=False)
    st = np.linalg.svd(T, compute_uv=False)
    if np.max(np.abs(sa - st)) > tol * nA:
        fails.append("sigma(T) != sigma(A)")
    ks = range(0, n)
    ek = M.trailing_norms(T, ks)
    if np.any(ek < sa[: len(ek)] - tol * nA):
        fails.append("Eckart-Young violated")
    if n > b and m > b:
        e_b, d_first = _rsvd_first_step(A, b, q, seed)
        if abs(ek[b] - e_b) > 1e-9 * nA:
            fails.append("first step != RSVD error")
        if np.max(np.abs(np.diag(T)[:b] - d_first)) > 1e-9 * nA:
            fails.append("first block != sigma(A orth(Y))")
    return fails


SHAPES = [(11, 8, 3), (8, 8, 8), (9, 4, 4), (40, 30, 7), (64, 64, 16), (33, 17, 5), (20, 20, 6)]


@pytest.mark.parametrize("m,n,b", SHAPES)
@pytest.mark.parametrize("q", [0, 1, 2])
def test_pins_gaussian(m, n, b, q):
    A = np.random.default_rng(m * 7 + n + b).standard_normal((m, n))
    assert pin_failures(oracle.randutv, A, b, q) == []


def test_pins_config1_shape_spectrum():
    """512 x 512, s_j = 10^(-12 (j-1)/511), b = 32, q = 1 (first config)."""
    from synthetic import spectral_matrix, spectrum
    n = 512
    s = spectrum("geometric", n, decades=12.0)
    A = spectral_matrix(n, n, s, seed=0)
    U, T, V = oracle.randutv(A, 32, 1, 1)
    assert M.orth_error(U) < 1e-13 and M.orth_error(V) < 1e-13
    assert M.recon_error(A, U, T, V) < 1e-13
    assert _structure_failures(T, 32) == []
    ks = np.arange(0, 512, 16)
    ek = M.trailing_norms(T, ks)
    # Eckart-Young against the known spectrum (floor: reconstruction error)
    assert np.all(ek >= s[ks] * (1 - 1e-6) - 1e-14)
    # rank-revealing quality on a geometric spectrum: e_k within 10x sigma_k+1
    assert np.all(ek <= 10 * s[ks] + 1e-13)


def test_pattern_golden_m11_n8_b3():
    path = os.path.join(HERE, "golden", "randutv_pattern_m11_n8_b3.txt")
    pats, cur = {}, None
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("step"):
            cur = int(line.split()[1])
            pats[cur] = []
        else:
            pats[cur].append(line)
    A = np.random.default_rng(42).standard_normal((11, 8))
    seen = {0: A.copy()}
    oracle.randutv(A, 3, 1, 1, on_step=lambda i, T: seen.__setitem__(i, T.copy()))
    assert sorted(seen) == sorted(pats)
    for i, rows in pats.items():
        T = seen[i]
        for r, row in enumerate(rows):
            for c, ch in enumerate(row):
                if ch == "0":
                    assert T[r, c] == 0.0, (i, r, c)
                else:
                    assert T[r, c] != 0.0, (i, r, c)


@pytest.mark.parametrize("q", [0, 2])
def test_frobenius_recurrence(q):
    A = np.random.default_rng(9).standard_normal((30, 24))
    b = 5
    prev = {"e2": np.linalg.norm(A, "fro") ** 2, "ok": True}

    def hook(i, T):
        c0, c2 = b * (i - 1), min(b * i, 24)
        if c2 >= 24:
            return
        e2 = prev["e2"] - np.linalg.norm(T[c0:c2, c0:], "fro") ** 2
        direct = np.linalg.norm(T[c2:, c2:], "fro") ** 2
        if abs(e2 - direct) > 1e-11 * np.linalg.norm(A, "fro") ** 2:
            prev["ok"] = False
        prev["e2"] = direct

    oracle.randutv(A, b, q, 1, on_step=hook)
    assert prev["ok"]


def test_block_at_least_n_is_svd():
    A = np.random.default_rng(1).standard_normal((12, 7))
    U, T, V = oracle.randutv(A, 8, 1, 1)
    sa = np.linalg.svd(A, compute_uv=False)
    np.testing.assert_allclose(np.diag(T), sa, rtol=1e-13)
    D = np.zeros_like(T)
    np.fill_diagonal(D, sa)
    np.testing.assert_allclose(T, D, atol=1e-13 * sa[0])


def test_exact_rank_deficient():
    rng = np.random.default_rng(4)
    r = 10
    A = rng.standard_normal((48, r)) @ rng.standard_normal((r, 40))
    U, T, V = oracle.randutv(A, 5, 1, 1)
    nA = M.spec(A)
    assert M.spec(T[r:, r:]) < 1e-12 * nA
    assert np.all(np.diag(T)[:r] > 1e-6 * nA)


def test_orthogonal_input():
    from synthetic import haar
    A = haar(32, 32, seed=3)
    U, T, V = oracle.randutv(A, 8, 2, 1)
    np.testing.assert_allclose(np.diag(T), np.ones(32), atol=1e-13)
    np.testing.assert_allclose(T, np.eye(32), atol=1e-13)


def test_zero_matrix():
    A = np.zeros((20, 16))
    U, T, V = oracle.randutv(A, 4, 1, 1)
    assert np.all(T == 0.0)
    assert M.orth_error(U) < 1e-14 and M.orth_error(V) < 1e-14


# ---------------------------------------------------------------- mutants
# Each mutant plants one plausible mistake in a copy of the oracle's source;
# the pins above must reject every one of them.
MUTANTS = {
    "sketch_not_transposed": ("Y = T22.T @ G", "Y = T22 @ G"),
    "one_extra_power_step": ("for _ in range(q):\n                Y = T22.T", "for _ in range(q + 1):\n                Y = T22.T"),
    "dropped_I1_J2_update": ("T[:c0, c0:c2] = T[:c0, c0:c2] @ Vs", "pass"),
    "left_update_not_transposed": ('T[c0:, c2:], "L", "T")', 'T[c0:, c2:], "L", "N")'),
    "dropped_V_accumulation": ('V[:, c0:] = apply_q(Wv, tv, V[:, c0:], "R", "N")', "pass"),
    "Us_not_transposed": ("T[c0:r2, c2:] = Us.T @ T[c0:r2, c2:]", "T[c0:r2, c2:] = Us @ T[c0:r2, c2:]"),
    "zeroing_off_by_one": ("T[r2:, c0:c2] = 0.0", "T[r2 + 1:, c0:c2] = 0.0"),
    "wrong_stream": ("G = gaussian(seed, i, m - c0, b)", "G = gaussian(seed, i + 1, m - c0, b)"),
}


def _mutant(name):
    old, new = MUTANTS[name]
    src = open(oracle.randutv.__code__.co_filename).read()
    assert src.count(old) == 1, name
    mod = types.ModuleType("oracle._mutant_" + name)
    mod.__package__ = "oracle"
    exec(compile(src.replace(old, new), "mutant:" + name, "exec"), mod.__dict__)
    return mod.randutv


def test_real_oracle_passes_all_pins():
    A = np.random.default_rng(77).standard_normal((24, 24))
    assert pin_failures(oracle.randutv, A, 6, 1) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name):
    A = np.random.default_rng(77).standard_normal((24, 24))
    fn = _mutant(name)
    assert pin_failures(fn, A, 6, 1) != [], name


def test_wide_matrix_through_the_transpose():
    """m < n (Sec. 3.2): A = U T V^T with T = T'^T lower trapezoidal, where
    A^T = U' T' V'^T is the factorization of the tall transpose; the
    singular values survive and the diagonal blocks are diagonal."""
    A = np.random.default_rng(12).standard_normal((40, 70))
    U, T, V = oracle.randutv(A, 8, 1, 3)
    Ut, Tt, Vt = oracle.randutv(A.T, 8, 1, 3)
    np.testing.assert_array_equal(T, Tt.T)
    np.testing.assert_array_equal(U, Vt)
    np.testing.assert_array_equal(V, Ut)
    assert U.shape == (40, 40) and V.shape == (70, 70)
    assert np.all(np.triu(T, 1) == 0.0)
    assert M.orth_error(U) < 1e-13 and M.orth_error(V) < 1e-13
    assert np.linalg.norm(A - U @ T @ V.T, 2) < 1e-13 * np.linalg.norm(A, 2)
    np.testing.assert_allclose(np.linalg.svd(T, compute_uv=False),
                               np.linalg.svd(A, compute_uv=False), atol=1e-13 * np.linalg.norm(A, 2))
