"""Host-side check of the batched randUTV driver (randutv_batched.hip).

The driver's C++ is compiled with the host compiler against a test double
of its device side (tests/batched_host/mock_kernels.cpp): stubbed HIP
runtime calls and CPU loops with each batched kernel's contract, checking
every access (inside an allocation, no cross-workgroup conflict within a
launch, no read of unwritten device memory). The emulated factorizations
are then held to the oracle like the GPU results: U, V orthogonal,
A = U T V^T, T upper trapezoidal with diagonal blocks, |T| equal to the
oracle's. Cases cover ragged batches, n < b, the narrow tile family of the
autotuner, the column split of tall
panels (twice), T aliasing A, padded lda, and no U / no V. No GPU needed.
"""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import oracle
from oracle import metrics as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST = os.path.join(ROOT, "tests", "batched_host")
CSRC = os.path.join(ROOT, "paper_2106_13402_amd", "csrc")


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    gxx = shutil.which("g++")
    hip_inc = "/opt/rocm/include"
    if not gxx or not os.path.isdir(hip_inc):
        pytest.skip("needs g++ and the HIP headers")
    out = tmp_path_factory.mktemp("planner")
    flags = ["-std=c++17", "-O2", "-D__HIP_PLATFORM_AMD__", f"-I{hip_inc}",
             f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}", "-Wno-attributes"]
    objs = []
    for src, lang in ((os.path.join(CSRC, "randutv_batched.hip"), ["-x", "c++"]),
                      (os.path.join(HOST, "mock_kernels.cpp"), []),
                      (os.path.join(HOST, "harness.cpp"), [])):
        obj = str(out / (os.path.basename(src) + ".o"))
        subprocess.run([gxx, *flags, *lang, "-c", src, "-o", obj], check=True)
        objs.append(obj)
    exe = str(out / "harness")
    subprocess.run([gxx, *objs, "-o", exe, "-pthread"], check=True)
    return exe, out


def _run(harness, shapes, b, q, seed, wu=True, wv=True, inplace=False, pad=0, precision=0,
         graph=False, leaf=0, tile_mask=31):
    exe, out = harness
    rng = np.random.default_rng(len(shapes) * 7 + b + q)
    As = []
    fin, fout = str(out / "in.bin"), str(out / "out.bin")
    with open(fin, "wb") as f:
        f.write(struct.pack("<11q", len(shapes), b, q, seed, int(wu), int(wv), int(inplace),
                            precision, int(graph), leaf, tile_mask))
        for m, n in shapes:
            A = rng.standard_normal((m, n))
            As.append(A)
            lda = m + (0 if inplace else pad)
            Ap = np.zeros((lda, n))
            Ap[:m] = A
            f.write(struct.pack("<3q", m, n, lda))
            f.write(np.asfortranarray(Ap).tobytes(order="F"))
    r = subprocess.run([exe, fin, fout], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "mock_errors=0" in r.stdout, r.stdout + r.stderr[:2000]
    launches = int(r.stdout.split("graph_launches=")[1].split()[0])
    assert (launches > 0) == graph, r.stdout
    raw = np.fromfile(fout)
    off = 0
    for j, (m, n) in enumerate(shapes):
        T = raw[off:off + m * n].reshape((m, n), order="F"); off += m * n
        U = V = None
        if wu:
            U = raw[off:off + m * m].reshape((m, m), order="F"); off += m * m
        if wv:
            V = raw[off:off + n * n].reshape((n, n), order="F"); off += n * n
        A = As[j]
        _, To, _ = oracle.randutv(A, b, q, seed + j, want_u=False, want_v=False)
        nA = M.spec(A)
        if wu:
            assert M.orth_error(U) <= 1e-13
        if wv:
            assert M.orth_error(V) <= 1e-13
        if wu and wv:
            assert M.recon_error(A, U, T, V) <= 1e-13
        assert np.all(np.tril(T, -1) == 0.0)
        for c0 in range(0, n, b):
            c1 = min(c0 + b, n)
            blk = T[c0:c1, c0:c1]
            assert np.all(blk - np.diag(np.diag(blk)) == 0.0)
        if precision == 0:
            np.testing.assert_allclose(np.abs(T), np.abs(To), atol=1e-9 * nA)
        else:  # the bfloat16 sketch changes the trajectory; e_k stays comparable
            ks = list(range(0, n, b))
            eg, eo = M.trailing_norms(T, ks), M.trailing_norms(To, ks)
            assert np.all(eg <= 1.5 * eo + 1e-12 * nA), (eg, eo)


MODES = pytest.mark.parametrize("graph", [False, True], ids=["lockstep", "replay"])


@MODES
def test_planner_ragged_batch(harness, graph):
    _run(harness, [(40, 30), (64, 64), (33, 17), (100, 64), (9, 4), (70, 70), (1, 1), (5, 1)],
         8, 1, 5, graph=graph)


@MODES
def test_planner_no_u_and_narrow(harness, graph):
    _run(harness, [(40, 30), (64, 64), (33, 17), (20, 5), (7, 7)], 16, 0, 5, wu=False,
         graph=graph)
    _run(harness, [(50, 20), (20, 20)], 4, 2, 9, wv=False, pad=3, graph=graph)


@MODES
def test_planner_in_place(harness, graph):
    _run(harness, [(30, 30), (45, 31)], 64, 1, 3, inplace=True, graph=graph)


@MODES
def test_planner_split_panels(harness, graph):
    # b = 64: 300-row panels exceed one workgroup at k = 64 and are split
    # once; b = 32 with 1100 rows is split twice (32 -> 16 -> 8)
    _run(harness, [(300, 200), (130, 64), (64, 10)], 64, 1, 11, graph=graph)
    _run(harness, [(1100, 24), (31, 31)], 32, 0, 2, wv=False, graph=graph)
    # a forced leaf width (the tuner's panel knob): 32-column panels factored
    # as 8-column leaves merged twice, though one workgroup would hold them
    _run(harness, [(120, 70), (64, 33)], 32, 1, 4, graph=graph, leaf=8)


@MODES
def test_planner_slices(harness, graph):
    # 520 matrices: cut into two slices, each on its own stream
    rng = np.random.default_rng(7)
    ns = rng.integers(1, 7, size=520)
    shapes = [(int(rng.integers(n, 2 * n + 1)), int(n)) for n in ns]
    _run(harness, shapes, 4, 1, 13, graph=graph)


@MODES
def test_planner_mixed_sketch(harness, graph):
    # the bfloat16 sketch: its conversions, grouped products and column
    # roundings go through the same bounds, race and padding checks
    _run(harness, [(40, 30), (64, 64), (33, 17), (100, 64), (9, 4), (70, 70)], 8, 1, 5,
         precision=1, graph=graph)
    _run(harness, [(300, 200), (64, 10)], 32, 2, 11, precision=1, graph=graph)


@MODES
def test_planner_narrow_tiles(harness, graph):
    # the autotuner's narrow tile family (128 x 32, 128 x 16; 64 x 64 is
    # always allowed): every product of the plan on those shapes
    narrow = (1 << 2) | (1 << 3)
    _run(harness, [(200, 64), (150, 70), (33, 17), (64, 64)], 32, 1, 3, graph=graph,
         tile_mask=narrow)
    _run(harness, [(90, 40), (16, 16), (70, 33)], 16, 1, 8, graph=graph, tile_mask=narrow)
