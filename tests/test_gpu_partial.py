"""GPU parity of rrf_randutv_partial (randUTV halted early, Sec. 4.1)
against the oracle's early-stopped run (oracle.randutv_partial): the same
number of reduced columns k, |T| (the reduced part and the unreduced
remainder T(k:, k:)) within 1e-9 ||A|| of the oracle's, U and V orthogonal
and A = U T V^T to 1e-13."""
import numpy as np
import pytest

import oracle
from oracle import metrics as M
from synthetic import gaussian_matrix, spectral_matrix, spectrum

from test_gpu_factorizations import _check_blocks, _host, _to_dev

pytestmark = pytest.mark.gpu


def _run(A, b, q, seed, tol, kmax, gpu, **kw):
    from paper_2106_13402_amd import randutv_partial
    U, T, V, k = randutv_partial(_to_dev(A, gpu), b, q, seed, tol, kmax, **kw)
    return (_host(U) if U is not None else None, _host(T),
            _host(V) if V is not None else None, k)


@pytest.mark.parametrize("tol,kmax", [(1e-2, None), (1e-5, None), (1e-9, None), (0.0, 48),
                                      (1e-5, 40), (0.0, None), (1.0, None)])
def test_partial_parity(gpu, tol, kmax):
    print(f"case: partial tol={tol} kmax={kmax}", flush=True)
    m, n, b = 250, 200, 16
    A = spectral_matrix(m, n, spectrum("geometric", n, decades=8.0), seed=1)
    U, T, V, k = _run(A, b, 1, 3, tol, kmax, gpu)
    Uo, To, Vo, ko = oracle.randutv_partial(A, b, 1, 3, tol, n if kmax is None else kmax)
    assert k == ko
    assert M.orth_error(U) <= 1e-13 and M.orth_error(V) <= 1e-13
    assert M.recon_error(A, U, T, V) <= 1e-13
    assert np.all(np.tril(T[:, :k], -1) == 0.0)
    _check_blocks(T[:k, :k], b)
    np.testing.assert_allclose(np.abs(T), np.abs(To), rtol=0, atol=1e-9 * M.spec(A))


def test_partial_large_rank_cap(gpu):
    """2048 x 1536, b = 128, q = 2, Gaussian: stop at the rank cap k = 512;
    the remainder's norm is that of the full run's trailing block."""
    from paper_2106_13402_amd import randutv
    print("case: partial 2048 x 1536 kmax=512", flush=True)
    A = gaussian_matrix(2048, 1536, seed=4)
    U, T, V, k = _run(A, 128, 2, 9, 0.0, 512, gpu)
    assert k == 512
    assert M.recon_error(A, U, T, V) <= 1e-13
    Tf = _host(randutv(_to_dev(A, gpu), 128, 2, 9, want_u=False, want_v=False)[1])
    np.testing.assert_array_equal(T[:512, :512], Tf[:512, :512])
    np.testing.assert_allclose(np.linalg.norm(T[512:, 512:]), np.linalg.norm(Tf[512:, 512:]),
                               rtol=1e-12)


def test_partial_zero_and_mixed(gpu):
    print("case: partial zero matrix and mixed modes", flush=True)
    U, T, V, k = _run(np.zeros((64, 48)), 16, 1, 1, 1e-8, None, gpu)
    assert k == 0 and np.all(T == 0.0)
    n = 1024
    A = spectral_matrix(n, n, spectrum("exp", n, scale=100.0), seed=5)
    nA = np.linalg.norm(A)
    for precision in ("bf16_sketch", "bf16_x3"):
        U, T, V, k = _run(A, 64, 1, 2, 1e-3, None, gpu, precision=precision)
        assert 0 < k < n and np.linalg.norm(T[k:, k:]) <= 1e-3 * nA * (1 + 1e-4)
        assert np.linalg.norm(T[k - 64:, k - 64:]) > 1e-3 * nA
        rec = M.recon_error(A, U, T, V)
        assert rec <= (1e-13 if precision == "bf16_sketch" else 1e-4), rec


@pytest.mark.parametrize("tol1,tol2,kmax2", [(1e-2, 1e-6, None), (1e-3, 0.0, 96), (1e-5, 1e-5, None),
                                             (1e-2, 0.0, None)])
def test_resume_matches_one_partial_run(gpu, tol1, tol2, kmax2):
    """partial(tol1) then resume(tol2, kmax2) equals one partial run with
    (tol2, kmax2): same k, |T| within 1e-9 ||A|| of the oracle's single run,
    U and V orthogonal and A = U T V^T to 1e-13."""
    from paper_2106_13402_amd import randutv_partial, randutv_resume
    print(f"case: resume tol1={tol1} tol2={tol2} kmax2={kmax2}", flush=True)
    m, n, b = 250, 200, 16
    A = spectral_matrix(m, n, spectrum("geometric", n, decades=8.0), seed=1)
    U, T, V, k1 = randutv_partial(_to_dev(A, gpu), b, 1, 3, tol1)
    k2 = randutv_resume(U, T, V, k1, b, 1, 3, tol2, kmax2)
    Uo, To, Vo, ko = oracle.randutv_partial(A, b, 1, 3, tol2, n if kmax2 is None else kmax2)
    assert k2 == max(k1, ko)
    U, T, V = _host(U), _host(T), _host(V)
    assert M.orth_error(U) <= 1e-13 and M.orth_error(V) <= 1e-13
    assert M.recon_error(A, U, T, V) <= 1e-13
    if k2 == ko:
        np.testing.assert_allclose(np.abs(T), np.abs(To), rtol=0, atol=1e-9 * M.spec(A))


@pytest.mark.parametrize("tol,kmax", [(1e-5, None), (0.0, 32)])
def test_partial_wide_parity(gpu, tol, kmax):
    """m < n through the transpose: same k as the oracle (which takes the
    same route), T(:k, k:) = 0, |T| within 1e-9 ||A||, A = U T V^T."""
    print(f"case: partial wide tol={tol} kmax={kmax}", flush=True)
    m, n, b = 120, 200, 16
    A = spectral_matrix(n, m, spectrum("geometric", m, decades=8.0), seed=2).T.copy(order="F")
    U, T, V, k = _run(A, b, 1, 3, tol, kmax, gpu)
    _, To, _, ko = oracle.randutv_partial(A, b, 1, 3, tol, n if kmax is None else kmax,
                                          want_u=False, want_v=False)
    assert k == ko and 0 < k < m
    assert U.shape == (m, m) and V.shape == (n, n)
    assert M.orth_error(U) <= 1e-13 and M.orth_error(V) <= 1e-13
    assert M.recon_error(A, U, T, V) <= 1e-13
    assert np.all(T[:k, k:] == 0.0)
    _check_blocks(T[:k, :k].T, b)
    np.testing.assert_allclose(np.abs(T), np.abs(To), rtol=0, atol=1e-9 * M.spec(A))


def test_resume_wide(gpu):
    """m < n: partial(1e-2) then resume(1e-6) equals the oracle's single
    partial run at 1e-6."""
    from paper_2106_13402_amd import randutv_partial, randutv_resume
    print("case: resume wide", flush=True)
    m, n, b = 120, 200, 16
    A = spectral_matrix(n, m, spectrum("geometric", m, decades=8.0), seed=2).T.copy(order="F")
    U, T, V, k1 = randutv_partial(_to_dev(A, gpu), b, 1, 3, 1e-2)
    k2 = randutv_resume(U, T, V, k1, b, 1, 3, 1e-6)
    _, To, _, ko = oracle.randutv_partial(A, b, 1, 3, 1e-6, n, want_u=False, want_v=False)
    assert 0 < k1 < k2 == ko
    U, T, V = _host(U), _host(T), _host(V)
    assert M.orth_error(U) <= 1e-13 and M.orth_error(V) <= 1e-13
    assert M.recon_error(A, U, T, V) <= 1e-13
    np.testing.assert_allclose(np.abs(T), np.abs(To), rtol=0, atol=1e-9 * M.spec(A))
