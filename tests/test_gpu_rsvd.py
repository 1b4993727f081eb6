"""GPU parity of rrf_rsvd (the randomized SVD, Sec. 3.3) against the oracle
(oracle/rsvd.py: the plain definition with numpy's QR and SVD) on the same
Gaussian: singular values within 1e-10 relative (+ 1e-13 ||A||), the
approximation U diag(S) V^T within 1e-12 ||A|| + 10 u kappa(Y) sigma_l sqrt(l)
of the oracle's (kappa(Y) the sample's conditioning), U and V
orthonormal to 1e-13; and the paper's Theorem 1 on the GPU: the projector of
the RSVD's U equals that of the first l columns of rrf_powerurv's U."""
import numpy as np
import pytest

import oracle
from oracle import metrics as M
from synthetic import gaussian_matrix, spectral_matrix, spectrum

from test_gpu_factorizations import _host, _to_dev, U64

pytestmark = pytest.mark.gpu


def _rsvd(A, l, q, seed, gpu, **kw):
    from paper_2106_13402_amd import rsvd
    U, S, V = rsvd(_to_dev(A, gpu), l, q, seed, **kw)
    return (_host(U) if U is not None else None, _host(S), _host(V) if V is not None else None)


# The sample (A A^T)^q A G only resolves directions above about
# u^(1/(2q+1)) sigma_1 (Sec. 3.3); the cases keep the top l singular values
# above it, so that they are well posed (the l = 256 case with 6 decades and
# q = 1 would leave its last ~30 values to rounding in any implementation).
@pytest.mark.parametrize("m,n,l,q,dec", [(300, 200, 20, 0, 6.0), (300, 200, 20, 1, 6.0),
                                         (300, 200, 20, 2, 6.0), (150, 400, 30, 1, 6.0),
                                         (1000, 800, 128, 2, 6.0), (64, 64, 64, 0, 6.0),
                                         (513, 257, 256, 1, 2.0)])
def test_rsvd_parity(gpu, m, n, l, q, dec):
    print(f"case: rsvd m={m} n={n} l={l} q={q}", flush=True)
    k = min(m, n)
    A = spectral_matrix(max(m, n), k, spectrum("geometric", k, decades=dec), seed=m + l)
    if m < n:
        A = np.asfortranarray(A.T)
    U, S, V = _rsvd(A, l, q, 7, gpu)
    Uo, So, Vo = oracle.rsvd(A, l, q, 7)
    nA = M.spec(A)
    assert M.orth_error(U) <= 1e-13 and M.orth_error(V) <= 1e-13
    assert np.all(np.diff(S) <= 0) and np.all(S >= 0)
    np.testing.assert_allclose(S, So, rtol=1e-10, atol=1e-13 * nA)
    # rounding moves the projector Q Q^T A by about u kappa(Y) sigma_l per
    # direction, kappa(Y) = (sigma_1 / sigma_l)^(2q+1)
    kappa = (So[0] / So[-1]) ** (2 * q + 1)
    tol = 1e-12 * nA + 10 * U64 * kappa * So[-1] * np.sqrt(l)
    np.testing.assert_allclose(U @ np.diag(S) @ V.T, Uo @ np.diag(So) @ Vo.T, rtol=0, atol=tol)
    if l == min(m, n) and q == 0:  # full rank sample: exact
        np.testing.assert_allclose(U @ np.diag(S) @ V.T, A, rtol=0, atol=1e-12 * nA)


def test_rsvd_theorem1_against_powerurv(gpu):
    """U_rsvd U_rsvd^T A = U(:, 1:l) U(:, 1:l)^T A, both from the GPU, same
    seed (stream 0 Gaussian)."""
    from paper_2106_13402_amd import powerurv
    print("case: rsvd theorem 1", flush=True)
    n = 512
    A = spectral_matrix(n, n, spectrum("geometric", n, decades=4.0), seed=3)
    Up = _host(powerurv(_to_dev(A, gpu), 1, 11, b=64)[0])
    for l in (16, 100):
        U, _, _ = _rsvd(A, l, 1, 11, gpu)
        np.testing.assert_allclose(U @ (U.T @ A), Up[:, :l] @ (Up[:, :l].T @ A),
                                   atol=1e-9 * M.spec(A))


def test_rsvd_options(gpu):
    import torch
    from paper_2106_13402_amd import RRFError, rsvd
    print("case: rsvd options", flush=True)
    A = gaussian_matrix(90, 70, seed=5)
    U, S, V = _rsvd(A, 12, 1, 3, gpu)
    U2, S2, V2 = _rsvd(A, 12, 1, 3, gpu, want_u=False, want_v=False)
    assert U2 is None and V2 is None
    np.testing.assert_array_equal(S2, S)
    bad = _to_dev(A, gpu).clone()
    bad[5, 6] = float("inf")
    with pytest.raises(RRFError) as e:
        rsvd(bad, 12, 1, 3, check_finite=True)
    assert e.value.status == 4
