"""Seeded synthetic test matrices, shared by the tests, the smoke check and
the benchmark. Holds none of the factorization's arithmetic: only the input
recipes (Gaussian matrices and ``Q1 diag(s) Q2^T`` with Haar-distributed
orthogonal factors, Sec. 5.2 "fast decay" construction).
"""
from .matrices import (
    SPECTRA,
    batch_gaussians,
    batch_shapes,
    batch_spectral,
    gaussian_matrix,
    haar,
    spectral_matrix,
    spectrum,
)

__all__ = ["SPECTRA", "batch_gaussians", "batch_shapes", "batch_spectral", "gaussian_matrix", "haar", "spectral_matrix", "spectrum"]
