"""Thin U (rrf_opts.thin_u): for a tall A only U(:, 1:n) is formed. It must
equal the first n columns of the full U (the same reflectors applied to the
first n columns of the identity; the GEMM splits may differ, so to rounding),
have orthonormal columns, and reproduce A = U(:, 1:n) T(1:n, :) V^T."""
import numpy as np
import pytest

from oracle import metrics as M
from synthetic import gaussian_matrix, spectral_matrix, spectrum

from test_gpu_factorizations import _host, _to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("m,n,b,q,precision", [(1000, 300, 64, 1, "fp64"),
                                               (2049, 512, 128, 2, "fp64"),
                                               (700, 700, 96, 1, "fp64"),
                                               (1500, 400, 64, 1, "bf16_x3")])
def test_thin_u(gpu, m, n, b, q, precision):
    from paper_2106_13402_amd import randutv
    print(f"case: thin U m={m} n={n} b={b} q={q} {precision}", flush=True)
    A = spectral_matrix(m, n, spectrum("geometric", n, decades=8.0), seed=m)
    Uf, Tf, Vf = (_host(x) for x in randutv(_to_dev(A, gpu), b, q, 3, precision=precision))
    Ut, Tt, Vt = (_host(x) for x in randutv(_to_dev(A, gpu), b, q, 3, precision=precision,
                                              thin_u=True))
    assert Ut.shape == (m, n)
    tol = 1e-13 if precision == "fp64" else 1e-4
    np.testing.assert_array_equal(Tt, Tf)
    np.testing.assert_array_equal(Vt, Vf)
    assert np.abs(Ut - Uf[:, :n]).max() <= (1e-13 if precision == "fp64" else 1e-5)
    assert M.orth_error(Ut) <= tol
    nA = M.spec(A)
    assert np.linalg.norm(A - Ut @ Tt[:n] @ Vt.T, 2) <= tol * nA
