"""rrf_randutv_noalloc (the library's static scratch, no device allocation
in the call) against rrf_randutv_ex (caller workspace) on the same inputs:
bitwise equal U, T, V on consecutive calls, the second one smaller, then a
mixed-precision and a wide call."""
import numpy as np
import pytest

from synthetic import gaussian_matrix, spectral_matrix, spectrum

pytestmark = pytest.mark.gpu


def _dev(x, gpu):
    import torch
    from paper_2106_13402_amd import colmajor
    return colmajor(torch.as_tensor(np.asfortranarray(x), device=gpu))


CALLS = [  # (m, n, b, q, precision, input)
    (1000, 900, 64, 1, "fp64", "geometric"),
    (300, 260, 32, 2, "fp64", "gaussian"),
    (700, 700, 128, 1, "bf16_sketch", "geometric"),
    (200, 513, 32, 1, "fp64", "gaussian"),
]


def _input(m, n, kind, seed):
    if kind == "gaussian":
        return gaussian_matrix(m, n, seed=seed)
    k = min(m, n)
    A = spectral_matrix(max(m, n), k, spectrum("geometric", k, decades=10.0), seed=seed)
    return A if m >= n else np.asfortranarray(A.T)


def test_noalloc_matches_workspace_entry_point(gpu):
    import torch
    import paper_2106_13402_amd as rrf
    for i, (m, n, b, q, prec, kind) in enumerate(CALLS):
        print(f"case: noalloc call {i}: m={m} n={n} b={b} q={q} {prec}", flush=True)
        A = _dev(_input(m, n, kind, 10 + i), gpu)
        U0, T0, V0 = rrf.randutv(A, b, q, 3 + i, precision=prec)
        U1, T1, V1 = rrf.randutv_noalloc(A, b, q, 3 + i, precision=prec)
        torch.cuda.synchronize()
        assert torch.equal(T0, T1) and torch.equal(U0, U1) and torch.equal(V0, V1), i


def test_noalloc_without_factors_and_repeat(gpu):
    import torch
    import paper_2106_13402_amd as rrf
    A = _dev(gaussian_matrix(500, 400, seed=4), gpu)
    _, T0, _ = rrf.randutv(A, 32, 1, 9, want_u=False, want_v=False)
    for _ in range(2):
        U, T1, V = rrf.randutv_noalloc(A, 32, 1, 9, want_u=False, want_v=False)
        assert U is None and V is None
        assert torch.equal(T0, T1)


def test_noalloc_rejects_oversize(gpu):
    import paper_2106_13402_amd as rrf
    A = _dev(np.zeros((2048, 2048)), gpu)
    with pytest.raises(rrf.RRFError) as e:
        rrf.randutv_noalloc(A, 128, 1, 1)
    assert e.value.status == 2
