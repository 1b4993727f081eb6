"""The batched call's autotuner on the GPU: a hand-written table is looked up
exactly (and only for its architecture and precision), the batched call with
b = 0 follows it (block size, tile family, panel leaf) and stays at oracle
parity; a short tuning run writes a valid cache that the next lookups use."""
import json
import os

import numpy as np
import pytest

from synthetic import batch_shapes, gaussian_matrix

from test_gpu_batched import _check_against_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def restore_default():
    import paper_2106_13402_amd as rrf
    yield
    p = rrf.default_tune_path()
    rrf.batched_tune_load(p if os.path.exists(p) else None)


def _arch():
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def _run_b0(As_host, q, seed, gpu):
    from paper_2106_13402_amd import randutv_batched
    from test_gpu_factorizations import _host, _to_dev
    As = [_to_dev(A, gpu) for A in As_host]
    Us, Ts, Vs = randutv_batched(As, 0, q, seed)
    return [_host(U) for U in Us], [_host(T) for T in Ts], [_host(V) for V in Vs]


def test_table_lookup_and_parity(gpu, tmp_path):
    import paper_2106_13402_amd as rrf
    table = {"format": "rrf-batched-tune-1", "tables": [
        {"arch": _arch(), "precision": 0, "q": 1, "count": 8, "buckets": [
            {"nmin": 1, "nmax": 80, "b": 8, "tile_mask": 13, "leaf": 0},
            {"nmin": 81, "nmax": 200, "b": 64, "tile_mask": 15, "leaf": 16}]},
        {"arch": "gfx000", "precision": 0, "buckets": [
            {"nmin": 201, "nmax": 4096, "b": 4, "tile_mask": 31, "leaf": 0}]}]}
    path = tmp_path / "tune.json"
    path.write_text(json.dumps(table))
    rrf.batched_tune_load(str(path))
    assert rrf.batched_config(70, 60) == {"b": 8, "tile_mask": 13, "leaf": 0, "tuned": True}
    assert rrf.batched_config(150, 100) == {"b": 64, "tile_mask": 15, "leaf": 16, "tuned": True}
    assert rrf.batched_config(100, 150)["b"] == 64          # wide: the transpose's n
    assert rrf.batched_config(600, 300) == {"b": 32, "tile_mask": 31, "leaf": 0, "tuned": False}
    assert rrf.batched_config(70, 60, "bf16_sketch")["tuned"] is False
    shapes = [(70, 60), (150, 100), (90, 81), (300, 200), (45, 45), (130, 250)]
    As = [gaussian_matrix(m, n, seed=i) for i, (m, n) in enumerate(shapes)]
    print("case: tuned table parity", flush=True)
    Us, Ts, Vs = _run_b0(As, 1, 3, gpu)
    wide = [j for j, (m, n) in enumerate(shapes) if m < n]
    tall = [j for j in range(len(shapes)) if j not in wide]
    _check_against_oracle([As[j] for j in tall], [Us[j] for j in tall], [Ts[j] for j in tall],
                          [Vs[j] for j in tall], 0, 1, 3, seeds=[3 + j for j in tall])
    for j in wide:  # a wide matrix equals its transpose's factorization
        import oracle
        b = rrf.batched_config(*shapes[j])["b"]
        _, To, _ = oracle.randutv(As[j], b, 1, 3 + j, want_u=False, want_v=False)
        np.testing.assert_allclose(np.abs(Ts[j]), np.abs(To), atol=1e-9 * np.linalg.norm(As[j], 2))


def test_autotune_short_run(gpu, tmp_path):
    import paper_2106_13402_amd as rrf
    path = str(tmp_path / "tuned.json")
    print("case: autotune count=12 nmax=128", flush=True)
    rrf.batched_autotune("fp64", q=1, count=12, nmax=128, seed=5, path=path)  # synthetic
    tab = json.load(open(path))
    assert tab["format"] == "rrf-batched-tune-1"
    t = [x for x in tab["tables"] if x["arch"] == _arch() and x["precision"] == 0][0]
    assert [(bk["nmin"], bk["nmax"]) for bk in t["buckets"]] == [(1, 64), (65, 128)]
    for bk in t["buckets"]:
        assert bk["b"] in (16, 32, 64) and bk["ms"] > 0 and bk["candidates"] >= 6
        c = rrf.batched_config(2 * bk["nmax"], bk["nmax"])
        assert c == {"b": bk["b"], "tile_mask": bk["tile_mask"], "leaf": bk["leaf"], "tuned": True}
    # the written cache loads back to the same choices
    rrf.batched_tune_load(path)
    shapes = batch_shapes(10, seed=2, nmin=20, nmax=128)
    As = [gaussian_matrix(m, n, seed=40 + i) for i, (m, n) in enumerate(shapes)]
    Us, Ts, Vs = _run_b0(As, 1, 11, gpu)
    _check_against_oracle(As, Us, Ts, Vs, 0, 1, 11)


def test_autotune_on_a_workload(gpu, tmp_path):
    """Tuning on the caller's shapes: only the buckets the batch occupies get
    entries, each one of the candidates, and the batched call follows them."""
    import paper_2106_13402_amd as rrf
    shapes = [(90, 70), (120, 100), (80, 80), (200, 150), (300, 180), (160, 130)] * 4
    path = str(tmp_path / "wl.json")
    print("case: autotune on a 24-matrix workload", flush=True)
    rrf.batched_autotune("fp64", q=1, shapes=shapes, nmax=1024, seed=3, path=path)
    t = [x for x in json.load(open(path))["tables"] if x["arch"] == _arch() and x["precision"] == 0][0]
    assert [(bk["nmin"], bk["nmax"]) for bk in t["buckets"]] == [(65, 128), (129, 192)]
    for bk in t["buckets"]:
        assert bk["b"] in (16, 32, 64) and bk["tile_mask"] in (31, 15, 13) and bk["leaf"] in (0, 16)
    assert rrf.batched_config(150, 130)["tuned"] is True
    assert rrf.batched_config(600, 300)["tuned"] is False   # no entry beyond the workload
    As = [gaussian_matrix(m, n, seed=70 + i) for i, (m, n) in enumerate(shapes[:6])]
    Us, Ts, Vs = _run_b0(As, 1, 11, gpu)
    _check_against_oracle(As, Us, Ts, Vs, 0, 1, 11)
