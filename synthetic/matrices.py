"""Synthetic input matrices (column-major float64).

Recipes, after the test matrices of Sec. 5 (numerical results):

* ``gaussian_matrix``: i.i.d. N(0, 1) entries (the speed experiments use a
  standard Gaussian n x n matrix);
* ``spectral_matrix``: ``Q1 diag(s) Q2^T (+ noise * N(0,1))`` with Q1, Q2
  Haar-distributed, made as the QR factor of an i.i.d. Gaussian matrix with
  the sign fix ``Q <- Q diag(sign(R_ii))`` (sign(0) = +1) so that the
  distribution is exactly Haar (Mezzadri 2007). The "fast decay" matrix of
  Sec. 5.2 is this construction with ``s_i = beta^((i-1)/(n-1))``.

Streams of one seed: Q1 uses stream 1, Q2 stream 2, the noise stream 3, a
plain Gaussian stream 0. On the CPU the numbers come from numpy's PCG64
seeded with ``[seed, stream]``; on a GPU device from a torch generator seeded
with ``seed * 8 + stream``. The two devices therefore give different (equally
distributed) matrices; every comparison hands one matrix to both sides.
"""
from __future__ import annotations

import numpy as np


def spectrum(kind: str, n: int, **kw) -> np.ndarray:
    """Singular values s_1 >= ... >= s_n of the named recipe."""
    j = np.arange(1, n + 1, dtype=np.float64)
    if kind == "geometric":        # s_j = 10^(-decades (j-1)/(n-1))
        decades = kw.get("decades", 12.0)
        return 10.0 ** (-decades * (j - 1) / max(n - 1, 1))
    if kind == "fast":             # s_j = beta^((j-1)/(n-1)), beta = 1e-5
        beta = kw.get("beta", 1e-5)
        return beta ** ((j - 1) / max(n - 1, 1))
    if kind == "power":            # s_j = j^-p
        return j ** (-kw.get("p", 2.0))
    if kind == "exp":              # s_j = exp(-j / scale)
        return np.exp(-j / kw.get("scale", 800.0))
    if kind == "gap":              # s_j = 1 (j <= k), lo after
        k = kw.get("k", 1000)
        return np.where(j <= k, 1.0, kw.get("lo", 1e-10))
    if kind == "ones":
        return np.ones(n)
    raise ValueError(f"unknown spectrum {kind!r}")


SPECTRA = ("geometric", "fast", "power", "exp", "gap", "ones")


def _np_rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([int(seed), int(stream)])


def _torch_gen(device, seed: int, stream: int):
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) * 8 + int(stream))
    return g


def _is_cpu(device) -> bool:
    return device is None or str(device) == "cpu"


def gaussian_matrix(m: int, n: int, seed: int = 0, stream: int = 0, device=None):
    """m x n i.i.d. N(0,1), float64, column-major (numpy on CPU, torch else)."""
    if _is_cpu(device):
        return np.asfortranarray(_np_rng(seed, stream).standard_normal((m, n)))
    import torch
    g = _torch_gen(device, seed, stream)
    # column-major storage: draw the transpose and view it back
    return torch.randn((n, m), generator=g, dtype=torch.float64, device=device).t()


def haar(m: int, k: int, seed: int = 0, stream: int = 1, device=None):
    """m x k matrix with orthonormal columns, Haar distributed (k <= m)."""
    if _is_cpu(device):
        G = _np_rng(seed, stream).standard_normal((m, k))
        Q, R = np.linalg.qr(G)
        d = np.sign(np.diag(R))
        d[d == 0] = 1.0
        return np.asfortranarray(Q * d[None, :])
    import torch
    G = gaussian_matrix(m, k, seed, stream, device).contiguous()
    Q, R = torch.linalg.qr(G)
    d = torch.sign(torch.diagonal(R))
    d = torch.where(d == 0, torch.ones_like(d), d)
    Q = Q * d[None, :]
    return Q.t().contiguous().t()  # column-major


def spectral_matrix(m: int, n: int, s, seed: int = 0, noise: float = 0.0, device=None):
    """A = Q1 diag(s) Q2^T (+ noise N(0,1)), Q1 m x n, Q2 n x n (m >= n)."""
    if m < n:
        raise ValueError("spectral_matrix expects m >= n")
    s = np.asarray(s, dtype=np.float64)
    if s.shape != (n,):
        raise ValueError("need n singular values")
    if _is_cpu(device):
        Q1 = haar(m, n, seed, 1)
        Q2 = haar(n, n, seed, 2)
        A = (Q1 * s[None, :]) @ Q2.T
        if noise:
            A = A + noise * _np_rng(seed, 3).standard_normal((m, n))
        return np.asfortranarray(A)
    import torch
    Q1 = haar(m, n, seed, 1, device)
    Q2 = haar(n, n, seed, 2, device)
    st = torch.as_tensor(s, dtype=torch.float64, device=device)
    A = (Q1 * st[None, :]) @ Q2.t()
    if noise:
        A = A + noise * gaussian_matrix(m, n, seed, 3, device)
    return A.t().contiguous().t()


def batch_shapes(count: int, seed: int = 0, nmin: int = 64, nmax: int = 512):
    """Shapes of a batch of small matrices: n ~ U{nmin..nmax}, m ~ U{n..2n}
    (integers, inclusive), drawn from numpy's PCG64 seeded with [seed, 4]."""
    rng = _np_rng(seed, 4)
    ns = rng.integers(nmin, nmax + 1, size=count)
    ms = [int(rng.integers(n, 2 * n + 1)) for n in ns]
    return [(m, int(n)) for m, n in zip(ms, ns)]


def batch_gaussians(shapes, seed: int = 0, device=None):
    """One i.i.d. N(0,1) matrix per shape, column-major with ld = m. On a
    GPU the matrices are views into one buffer (stream 5 of the seed)."""
    if _is_cpu(device):
        rng = _np_rng(seed, 5)
        return [np.asfortranarray(rng.standard_normal((m, n))) for m, n in shapes]
    import torch
    total = sum(m * n for m, n in shapes)
    buf = torch.randn(total, generator=_torch_gen(device, seed, 5), dtype=torch.float64,
                      device=device)
    out, off = [], 0
    for m, n in shapes:
        out.append(buf[off:off + m * n].view(n, m).t())
        off += m * n
    return out


def _spectral_one(m: int, n: int, seed: int, j: int, decades: float) -> np.ndarray:
    rng = np.random.default_rng([int(seed), 6, int(j)])
    q = []
    for r, c in ((m, n), (n, n)):
        Q, R = np.linalg.qr(rng.standard_normal((r, c)))
        d = np.sign(np.diag(R))
        d[d == 0] = 1.0
        q.append(Q * d[None, :])
    s = 10.0 ** (-decades * np.arange(n, dtype=np.float64) / max(n - 1, 1))
    return np.asfortranarray((q[0] * s[None, :]) @ q[1].T)


def batch_spectral(shapes, seed: int = 0, decades: float = 8.0, device=None,
                   workers: int | None = None):
    """A_j = Q1_j diag(s_j) Q2_j^T for each shape (m, n), s_j,i =
    10^(-decades (i-1)/(n-1)), Q1_j (m x n) and Q2_j (n x n) Haar with the
    sign fix of ``haar``, drawn from numpy stream [seed, 6, j]; column-major,
    ld = m. Made on the host (a thread pool, one BLAS thread each) on every
    device, so CPU and GPU get the same matrices; on a GPU they are views
    into one device buffer."""
    import concurrent.futures as cf
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    import contextlib
    workers = workers or min(16, len(__import__("os").sched_getaffinity(0)))
    ctx = threadpool_limits(1) if threadpool_limits else contextlib.nullcontext()
    with ctx, cf.ThreadPoolExecutor(workers) as ex:
        mats = list(ex.map(lambda a: _spectral_one(a[1][0], a[1][1], seed, a[0], decades),
                           enumerate(shapes)))
    if _is_cpu(device):
        return mats
    import torch
    flat = np.concatenate([a.ravel(order="F") for a in mats])
    del mats
    buf = torch.from_numpy(flat).to(device)
    out, off = [], 0
    for m, n in shapes:
        out.append(buf[off:off + m * n].view(n, m).t())
        off += m * n
    return out


def describe(kind: str, **kw) -> str:
    return kind + "(" + ",".join(f"{k}={v}" for k, v in sorted(kw.items())) + ")"
