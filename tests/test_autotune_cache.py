"""The batched call's tuning cache on the host: valid caches load, malformed
ones are rejected whole (-1) and leave the loaded tables as they were, and
without a device every lookup falls back to the built-in rule."""
import json

import pytest

import paper_2106_13402_amd as rrf

GOOD = {"format": "rrf-batched-tune-1", "tables": [
    {"arch": "gfx950", "precision": 0, "q": 1, "count": 64, "buckets": [
        {"nmin": 1, "nmax": 64, "b": 16, "tile_mask": 31, "leaf": 0, "ms": 1.0, "candidates": 6},
        {"nmin": 65, "nmax": 512, "b": 32, "tile_mask": 7, "leaf": 16, "ms": 2.0,
         "candidates": 18}]}]}


@pytest.fixture(autouse=True)
def restore_default():
    yield
    import os
    p = rrf.default_tune_path()
    rrf.batched_tune_load(p if os.path.exists(p) else None)


def _write(tmp_path, obj, name="t.json"):
    p = tmp_path / name
    p.write_text(obj if isinstance(obj, str) else json.dumps(obj))
    return str(p)


def test_valid_cache_loads(tmp_path):
    rrf.batched_tune_load(_write(tmp_path, GOOD))
    rrf.batched_tune_load(None)


@pytest.mark.parametrize("bad", [
    "{",                                                       # truncated
    '{"format": "other", "tables": []}',                       # wrong format tag
    {"format": "rrf-batched-tune-1"},                          # no tables
    {"format": "rrf-batched-tune-1", "tables": [{"arch": "gfx950", "precision": 0,
                                                 "buckets": [{"nmin": 1, "nmax": 64, "b": 0}]}]},
    {"format": "rrf-batched-tune-1", "tables": [{"arch": "gfx950", "precision": 0,
                                                 "buckets": [{"nmin": 9, "nmax": 4, "b": 16}]}]},
    {"format": "rrf-batched-tune-1", "tables": [{"arch": "gfx950", "precision": 0,
                                                 "buckets": [{"nmin": 1, "nmax": 4, "b": 16,
                                                              "tile_mask": 64}]}]},
    '{"format": "rrf-batched-tune-1", "tables": []} trailing',
    # integer fields must hold whole numbers in range (no undefined casts)
    json.dumps(GOOD).replace('"nmin": 65', '"nmin": 1e300'),
    json.dumps(GOOD).replace('"b": 32', '"b": nan'),
    json.dumps(GOOD).replace('"leaf": 16', '"leaf": -inf'),
    json.dumps(GOOD).replace('"b": 32', '"b": 32.5'),
    json.dumps(GOOD).replace('"precision": 0', '"precision": 1e20'),
    json.dumps(GOOD).replace('"candidates": 18', '"candidates": 4294967296'),
])
def test_malformed_cache_rejected(tmp_path, bad):
    with pytest.raises(rrf.RRFError) as e:
        rrf.batched_tune_load(_write(tmp_path, bad))
    assert e.value.status == -1


def test_missing_file_rejected(tmp_path):
    with pytest.raises(rrf.RRFError) as e:
        rrf.batched_tune_load(str(tmp_path / "absent.json"))
    assert e.value.status == -1


def test_lookup_without_device_is_builtin(tmp_path):
    import torch
    if torch.cuda.is_available():
        pytest.skip("host-only check")
    rrf.batched_tune_load(_write(tmp_path, GOOD))
    for m, n, b in ((100, 60, 16), (600, 300, 32), (40, 700, 16), (300, 700, 32)):
        c = rrf.batched_config(m, n)
        assert c == {"b": b, "tile_mask": 31, "leaf": 0, "tuned": False}


def test_config_argument_errors():
    with pytest.raises(rrf.RRFError) as e:
        rrf.batched_config(0, 4)
    assert e.value.status == -1
    import ctypes as C
    from paper_2106_13402_amd import _lib
    cfg = _lib.rrf_batched_cfg()
    assert rrf.lib.rrf_batched_config(4, 4, 2, C.byref(cfg)) == -3  # x3: not batched
    assert rrf.lib.rrf_batched_config(4, 4, 0, None) == -4
    f = rrf.lib.rrf_batched_autotune
    assert f(5, 1, 8, None, None, 64, 0, None, None) == -1
    assert f(0, -1, 8, None, None, 64, 0, None, None) == -2
    assert f(0, 1, 0, None, None, 64, 0, None, None) == -3
    two = (C.c_int64 * 2)(10, 20)
    assert f(0, 1, 2, two, None, 64, 0, None, None) == -4
    bad = (C.c_int64 * 2)(10, 5000)
    assert f(0, 1, 2, two, bad, 64, 0, None, None) == -5
    assert f(0, 1, 8, None, None, 2048, 0, None, None) == -6
    many = (C.c_int64 * 257)(*([64] * 257))
    assert f(0, 1, 257, many, many, 64, 0, None, None) == _lib.RRF_E_NOTSUP  # workload cap
