#!/usr/bin/env python3
"""Write the expected values of the n = 8192 parity tests (the second
configuration of the benchmark set: plain randUTV (Alg. 3) and powerURV
(Alg. 1) in FP64 on an 8192 x 8192 matrix, b = 128, q in {0, 1, 2}; input
(a) i.i.d. N(0, 1), input (b) Q1 diag(j^-2) Q2^T with Haar Q1, Q2; matrix
seed 0, sketch seed 1).

Only ``oracle/`` and ``synthetic/`` are called; nothing here touches the
GPU library. For each case the file records

* fingerprints of the input (2-norm, Frobenius norm, eight entries) so a
  test can check that it regenerated the same matrix;
* |T_kk| of the oracle on a subset of k (the first and last 16 and every
  13th; 13 is prime to b, so every position inside a block is sampled);
* the spread of |T_kk| under three backward-error-sized perturbations of A
  (||E||_2 = n eps ||A||_2, Gaussian E from numpy's PCG64 seed 12345): the
  amount by which any correct FP64 run may differ where the sketch of a
  block is numerically rank deficient;
* e_k = ||T(k:, k:)||_2 on a k-grid (Golub-Kahan-Lanczos, 200 steps with full
  reorthogonalisation) and, for input (b), the known sigma_{k+1} = (k+1)^-2.

    python tests/golden/make_c2_goldens.py [--only NAME ...]

Takes about an hour on 8 host cores (24 randUTV and 24 powerURV oracle runs
at n = 8192).
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import metrics as M  # noqa: E402
from synthetic import gaussian_matrix, spectral_matrix, spectrum  # noqa: E402

N, B, MATRIX_SEED, SKETCH_SEED = 8192, 128, 0, 1
EPS = np.finfo(np.float64).eps
K_GRID = (0, 64, 128, 1024, 2048, 4096, 6144, 8064)
PROBES = ((0, 0), (1, 0), (0, 1), (4095, 17), (17, 4095), (8191, 8191), (5000, 123), (77, 7777))
PERTURB_SEED, PERTURB_DRAWS = 12345, 3


def k_subset(n: int) -> list[int]:
    return sorted(set(range(16)) | set(range(0, n, 13)) | set(range(n - 16, n)))


def make_input(kind: str) -> np.ndarray:
    if kind == "gaussian":
        return gaussian_matrix(N, N, seed=MATRIX_SEED, stream=0)
    if kind == "power":
        return spectral_matrix(N, N, spectrum("power", N, p=2.0), seed=MATRIX_SEED)
    raise ValueError(kind)


def factor_T(alg: str, A: np.ndarray, q: int) -> np.ndarray:
    if alg == "randutv":
        _, T, _ = oracle.randutv(A, B, q, SKETCH_SEED, want_u=False, want_v=False)
    else:
        _, T, _ = oracle.powerurv(A, q, SKETCH_SEED)
    return T


def write_case(path, alg, kind, q, A, nA, fro, T0, spread, ks, eks, secs):
    lines = [
        f"# {alg} FP64 oracle, {N}x{N} input '{kind}', b={B}, q={q}, matrix seed "
        f"{MATRIX_SEED}, sketch seed {SKETCH_SEED}",
        "# randUTV: Alg. 3 (Appendix B); powerURV: Alg. 1 (Sec. 3.2). Written by "
        "tests/golden/make_c2_goldens.py from oracle/ and synthetic/ only.",
        "# columns: k |T_kk| spread (max change of |T_kk| over three perturbations "
        "||E||_2 = n eps ||A||_2)",
        f"#: alg {alg}", f"#: input {kind}", f"#: m {N}", f"#: n {N}", f"#: b {B}", f"#: q {q}",
        f"#: matrix_seed {MATRIX_SEED}", f"#: sketch_seed {SKETCH_SEED}",
        f"#: A_norm2 {nA:.17e}", f"#: A_fro {fro:.17e}",
        f"#: oracle_seconds {secs:.1f}",
    ]
    for i, j in PROBES:
        lines.append(f"#: A_probe {i} {j} {A[i, j]:.17e}")
    for k, e in zip(K_GRID, eks):
        lines.append(f"#: ek {k} {e:.17e}")
    d0 = np.abs(np.diag(T0))
    for k in ks:
        lines.append(f"{k} {d0[k]:.17e} {spread[k]:.3e}")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def run_case(alg: str, kind: str, q: int, A: np.ndarray, nA: float, fro: float,
             perturbations) -> str:
    name = f"c2_{alg}_{kind}_q{q}"
    path = os.path.join(HERE, name + ".txt")
    t0 = time.perf_counter()
    T0 = factor_T(alg, A, q)
    secs = time.perf_counter() - t0
    d0 = np.abs(np.diag(T0))
    spread = np.zeros_like(d0)
    for E in perturbations:
        Tp = factor_T(alg, A + E, q)
        spread = np.maximum(spread, np.abs(np.abs(np.diag(Tp)) - d0))
        del Tp
    eks = [M.spec_lanczos(T0[k:, k:]) for k in K_GRID]
    write_case(path, alg, kind, q, A, nA, fro, T0, spread, k_subset(N), eks, secs)
    print(f"{name}: oracle {secs:.0f} s, spread max {spread.max() / nA:.2e} ||A||, "
          f"total {time.perf_counter() - t0:.0f} s", flush=True)
    return path


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--only", nargs="*", default=None,
                    help="case names such as c2_randutv_gaussian_q1")
    args = ap.parse_args()
    cases = [(alg, kind, q) for kind in ("gaussian", "power") for alg in ("randutv", "powerurv")
             for q in (0, 1, 2)]
    if args.only:
        cases = [c for c in cases if f"c2_{c[0]}_{c[1]}_q{c[2]}" in args.only]
    for kind in sorted({c[1] for c in cases}):
        A = make_input(kind)
        nA = M.spec_lanczos(A)
        fro = float(np.linalg.norm(A))
        rng = np.random.default_rng(PERTURB_SEED)
        perts = []
        for _ in range(PERTURB_DRAWS):
            E = rng.standard_normal(A.shape)
            E *= N * EPS * nA / M.spec_lanczos(E)
            perts.append(np.asfortranarray(E))
        for alg, k2, q in cases:
            if k2 == kind:
                run_case(alg, kind, q, A, nA, fro, perts)
        del A, perts
    return 0


if __name__ == "__main__":
    sys.exit(main())
