"""Host C++ under AddressSanitizer, UndefinedBehaviorSanitizer (with
float-cast-overflow) and LeakSanitizer, built with the host compiler; no GPU.

* The batched randUTV driver (randutv_batched.hip) against its test double
  (tests/batched_host/mock_kernels.cpp): the planner cases of
  test_batched_planner.py (lockstep and graph replay, ragged batches, split
  and forced-leaf panels, in place, padded lda, no U or no V, the bfloat16
  sketch, several slices; the slowest, emulated 300-row panels, run only
  unsanitized there), each held to the
  oracle as there, with the driver's resources released at the end so that
  anything it loses shows as a leak.
* The autotuner's search through the library's C ABI (api.hip, autotune.hip
  and the driver against the test double; tests/batched_host/
  api_host.cpp): on a caller's workload of tall and wide matrices and on
  the synthetic buckets, then the cache it writes read back; and the
  batched call through the same ABI with the library-managed workspace,
  with allocation and device failures injected by RRF_TEST_FAIL.
* The tuning-cache reader (autotune.hip) through rrf_batched_tune_load and
  rrf_batched_config (tests/batched_host/tune_host.cpp): a valid cache, the
  malformed ones, numbers that no integer field can hold (1e300, nan, inf,
  fractions, values past 2^31 or 2^53), and seeded mutations of a valid cache
  (every truncation, substituted, deleted and inserted bytes). Every load
  returns 0 or -1, a rejected file leaves the lookups as they were, and no
  sanitizer fires.

Under ThreadSanitizer (a build of its own): the batched driver's direct
mode with four slices, whose rounds run on four host threads; and
allow_dynamic_lds (context.hip, tests/batched_host/context_host.cpp), which
the kernels' launchers call from those threads, hammered from eight threads
on three devices: the attribute is set once per (kernel, device), raised
for a larger request, and a failed request changes nothing.

Each source is copied to a .cpp file first, so the compiler line names no
HIP source; device code is not built.
"""
import json
import os
import shutil
import subprocess

import numpy as np
import pytest

import test_batched_planner as planner

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST = os.path.join(ROOT, "tests", "batched_host")
CSRC = os.path.join(ROOT, "paper_2106_13402_amd", "csrc")

SAN = ["-fsanitize=address,undefined,float-cast-overflow", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer"]
ENV = {"ASAN_OPTIONS": "detect_leaks=1:halt_on_error=1",
       "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}


TSAN = ["-fsanitize=thread", "-fno-omit-frame-pointer"]
TSAN_ENV = {"TSAN_OPTIONS": "halt_on_error=1"}


def _sanitizers_work(gxx, out, san=SAN, env=ENV):
    src = out / "probe.cpp"
    src.write_text("#include <thread>\n#include <vector>\nint main(){std::vector<int> v(3);"
                   "std::thread t([&]{v[0]=1;});t.join();return v[1];}\n")
    exe = str(out / "probe")
    try:
        subprocess.run([gxx, *san, str(src), "-o", exe, "-pthread"], check=True,
                       capture_output=True)
        return subprocess.run([exe], env={**os.environ, **env}).returncode == 0
    except (subprocess.CalledProcessError, OSError):
        return False


def _build(gxx, out, san, sources, links):
    hip_inc = "/opt/rocm/include"
    flags = ["-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", f"-I{hip_inc}",
             f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}", "-Wno-attributes", *san]
    # api.hip's allocation-free entry point declares a device array; on the
    # host it is an ordinary array and its symbol address the array's own
    api_flags = ["-D__align__(x)=alignas(x)", "-DHIP_SYMBOL(x)=((const void*)&(x))"]
    objs = {}
    for name, src in sources:
        cpp = out / f"{name}.cpp"
        shutil.copyfile(src, cpp)
        obj = str(out / f"{name}.o")
        subprocess.run([gxx, *flags, *(api_flags if name == "api" else []), "-c", str(cpp),
                        "-o", obj], check=True)
        objs[name] = obj
    exes = {}
    for exe, names, libs in links:
        path = str(out / exe)
        subprocess.run([gxx, *san, *[objs[n] for n in names], "-o", path, "-pthread", *libs],
                       check=True)
        exes[exe] = path
    return exes


@pytest.fixture(scope="module")
def objects(tmp_path_factory):
    gxx = shutil.which("g++")
    if not gxx or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("needs g++ and the HIP headers")
    out = tmp_path_factory.mktemp("sanitized")
    if not _sanitizers_work(gxx, out):
        pytest.skip("the host compiler's sanitizer runtimes are not available")
    exes = _build(gxx, out, SAN,
                  [("driver", os.path.join(CSRC, "randutv_batched.hip")),
                   ("autotune", os.path.join(CSRC, "autotune.hip")),
                   ("api", os.path.join(CSRC, "api.hip")),
                   ("mock", os.path.join(HOST, "mock_kernels.cpp")),
                   ("harness", os.path.join(HOST, "harness.cpp")),
                   ("tune_host", os.path.join(HOST, "tune_host.cpp")),
                   ("api_host", os.path.join(HOST, "api_host.cpp"))],
                  [("planner", ["driver", "mock", "harness"], []),
                   ("tune", ["autotune", "driver", "mock", "tune_host"], ["-ldl"]),
                   ("api_host", ["api", "autotune", "driver", "mock", "api_host"], ["-ldl"])])
    return {"planner": exes["planner"], "tune": exes["tune"], "api": exes["api_host"],
            "out": out}


@pytest.fixture(scope="module")
def tsan_objects(tmp_path_factory):
    gxx = shutil.which("g++")
    if not gxx or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("needs g++ and the HIP headers")
    out = tmp_path_factory.mktemp("tsan")
    if not _sanitizers_work(gxx, out, TSAN, TSAN_ENV):
        pytest.skip("the host compiler's thread sanitizer runtime is not available")
    exes = _build(gxx, out, TSAN,
                  [("driver", os.path.join(CSRC, "randutv_batched.hip")),
                   ("mock", os.path.join(HOST, "mock_kernels.cpp")),
                   ("harness", os.path.join(HOST, "harness.cpp")),
                   ("context", os.path.join(CSRC, "context.hip")),
                   ("context_host", os.path.join(HOST, "context_host.cpp"))],
                  [("planner", ["driver", "mock", "harness"], []),
                   ("context_host", ["context", "context_host"], [])])
    return {**exes, "out": out}


@pytest.fixture
def sanitizer_env(monkeypatch):
    for k, v in ENV.items():
        monkeypatch.setenv(k, v)


@pytest.mark.parametrize("graph", [False, True], ids=["lockstep", "replay"])
def test_planner_sanitized(objects, sanitizer_env, graph):
    h = (objects["planner"], objects["out"])
    planner._run(h, [(40, 30), (64, 64), (33, 17), (100, 64), (9, 4), (70, 70), (1, 1), (5, 1)],
                 8, 1, 5, graph=graph)
    if not graph:  # 1100-row panels split twice (32 -> 16 -> 8 columns)
        planner._run(h, [(1100, 24), (31, 31)], 32, 0, 2, wv=False, graph=graph)
    planner._run(h, [(30, 30), (45, 31)], 64, 1, 3, inplace=True, graph=graph)
    planner._run(h, [(50, 20), (20, 20)], 4, 2, 9, wu=False, pad=3, graph=graph)
    planner._run(h, [(40, 30), (64, 64), (9, 4)], 8, 1, 5, precision=1, graph=graph)
    planner._run(h, [(120, 70), (64, 33)], 32, 1, 4, graph=graph, leaf=8)


def test_planner_slices_sanitized(objects, sanitizer_env):
    rng = np.random.default_rng(7)
    ns = rng.integers(1, 7, size=520)
    shapes = [(int(rng.integers(n, 2 * n + 1)), int(n)) for n in ns]
    planner._run((objects["planner"], objects["out"]), shapes, 4, 1, 13, graph=True)


GOOD = {"format": "rrf-batched-tune-1", "tables": [
    {"arch": "gfx950", "precision": 0, "q": 1, "count": 64, "buckets": [
        {"nmin": 1, "nmax": 64, "b": 16, "tile_mask": 31, "leaf": 0, "ms": 1.0, "candidates": 6},
        {"nmin": 65, "nmax": 512, "b": 32, "tile_mask": 7, "leaf": 16, "ms": 2.0,
         "candidates": 18}]},
    {"arch": "gfx942", "precision": 0, "buckets": [{"nmin": 1, "nmax": 4096, "b": 64}]}]}
# lookups (n = 1, 40, 64, 65, 300, 512, 4096) with GOOD loaded: its gfx950
# buckets, then the built-in rule for n = 4096 (no bucket holds it)
GOOD_LOOKUPS = ["0:16,31,0,1"] * 3 + ["0:32,7,16,1"] * 3
BUILTIN_4096 = "0:32,31,0,0"


def _tune(objects, args, extra_env=None):
    r = subprocess.run([objects["tune"], *args], capture_output=True, text=True, timeout=300,
                       env={**os.environ, **ENV, "RRF_TUNE_CACHE": "", **(extra_env or {})})
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    lines = r.stdout.splitlines()
    assert len(lines) == len(args), r.stdout[-2000:]
    return [(int(ln.split()[0]), ln.split()[1:]) for ln in lines]


def _write(out, name, text):
    p = out / name
    p.write_bytes(text if isinstance(text, bytes) else text.encode())
    return str(p)


def _bucket_field(field, value):
    g = json.loads(json.dumps(GOOD))
    g["tables"][0]["buckets"][1][field] = "@@"
    return json.dumps(g).replace('"@@"', value)


def test_tune_cache_reader_sanitized(objects):
    out = objects["out"]
    good = _write(out, "good.json", json.dumps(GOOD, indent=1))
    bad = []
    for field in ("nmin", "nmax", "b", "tile_mask", "leaf", "candidates"):
        for v in ("1e300", "-1e300", "nan", "inf", "-inf", "32.5", "9007199254740993",
                  "1e19", '"32"'):
            if field == "nmax" and v == "9007199254740993":
                continue  # 2^53 is a valid upper end of the bucket
            bad.append(_write(out, f"bad_{field}_{len(bad)}.json", _bucket_field(field, v)))
    for field, v in (("precision", "1e20"), ("precision", "nan"), ("precision", "0.5"),
                     ("q", "inf"), ("q", "4294967296"), ("count", "1e300"), ("count", "-nan")):
        g = json.loads(json.dumps(GOOD))
        g["tables"][0][field] = "@@"
        bad.append(_write(out, f"bad_{field}_{len(bad)}.json",
                          json.dumps(g).replace('"@@"', v)))
    for i, text in enumerate(["", "{", "[]", '{"format": "rrf-batched-tune-1"}', "null",
                              '{"format": "rrf-batched-tune-1", "tables": [1]}',
                              '{"format": "rrf-batched-tune-1", "tables": []} x',
                              "[" * 40 + "]" * 40, '{"a": "\\']):
        bad.append(_write(out, f"bad_text_{i}.json", text))
    args = ["NULL", good] + [a for p in bad for a in (p, good)] + ["NULL", good]
    res = _tune(objects, args)
    builtin = res[0][1]
    assert res[0][0] == 0 and builtin[-1] == BUILTIN_4096
    assert all(s.endswith(",0") for s in builtin)  # nothing tuned after an unload
    for k, (rc, look) in enumerate(res[1:], 1):
        if args[k] == good:
            assert rc == 0 and look == GOOD_LOOKUPS + [BUILTIN_4096], (args[k], look)
        elif args[k] == "NULL":
            assert rc == 0 and look == builtin
        else:  # each malformed file is rejected and the GOOD tables stay
            assert rc == -1 and look == res[k - 1][1], args[k]


def test_tune_cache_default_path_sanitized(objects):
    out = objects["out"]
    good = _write(out, "default_good.json", json.dumps(GOOD))
    bad = _write(out, "default_bad.json", _bucket_field("b", "nan"))
    assert _tune(objects, ["--lookup"], {"RRF_TUNE_CACHE": good}) == \
        [(0, GOOD_LOOKUPS + [BUILTIN_4096])]
    (rc, look), = _tune(objects, ["--lookup"], {"RRF_TUNE_CACHE": bad})
    assert rc == 0 and all(s.endswith(",0") for s in look)


def test_tune_cache_mutations_sanitized(objects):
    out = objects["out"]
    text = json.dumps(GOOD, indent=1).encode()
    rng = np.random.default_rng(2106)
    alphabet = b'{}[],:"\\0123456789.-+eEnNaIfltrusx \n\t'
    muts = [text[:i] for i in range(len(text))]
    for _ in range(400):
        i = int(rng.integers(len(text)))
        muts.append(text[:i] + bytes([alphabet[int(rng.integers(len(alphabet)))]]) + text[i + 1:])
    for _ in range(150):
        i = int(rng.integers(len(text)))
        muts.append(text[:i] + text[i + 1 + int(rng.integers(4)):])
    for _ in range(150):
        i = int(rng.integers(len(text)))
        ins = bytes(alphabet[int(j)] for j in rng.integers(len(alphabet), size=int(rng.integers(1, 5))))
        muts.append(text[:i] + ins + text[i:])
    for _ in range(100):  # bytes outside the alphabet, NUL and high bytes included
        i = int(rng.integers(len(text)))
        muts.append(text[:i] + bytes([int(rng.integers(256))]) + text[i + 1:])
    paths = [_write(out, f"mut_{i}.json", m) for i, m in enumerate(muts)]
    res = _tune(objects, ["NULL"] + paths)
    for k, (rc, look) in enumerate(res[1:], 1):
        assert rc in (0, -1), paths[k - 1]
        assert all(s.startswith("0:") for s in look)
        if rc == -1:
            assert look == res[k - 1][1], paths[k - 1]
        else:  # an accepted mutation still yields valid configurations
            for s in look:
                b, mask, leaf, _ = map(int, s[2:].split(","))
                assert 1 <= b <= 64 and 0 <= mask < 32 and 0 <= leaf <= 64, (paths[k - 1], s)
    assert sum(rc == -1 for rc, _ in res[1:]) > len(muts) // 2


def _search(objects, cache, mode, count, hi):
    r = subprocess.run([objects["api"], cache, mode, str(count), str(hi)], capture_output=True,
                       text=True, timeout=600, env={**os.environ, **ENV, "RRF_TUNE_CACHE": ""})
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    lines = r.stdout.splitlines()
    _, rc, errors = lines[0].split()
    return int(rc), int(errors), {ln.split()[0]: ln.split()[1:] for ln in lines[1:]}, lines


# lookups are printed for n = 1..8 and 64
LOOKUP_N = [1, 2, 3, 4, 5, 6, 7, 8, 64]


@pytest.mark.parametrize("mode,count,hi", [("workload", 200, 6), ("buckets", 64, 6)])
def test_tune_search_sanitized(objects, mode, count, hi):
    cache = str(objects["out"] / f"search_{mode}.json")
    rc, errors, look, lines = _search(objects, cache, mode, count, hi)
    assert rc == 0 and errors == 0, lines
    assert look["loaded"] == look["tuned"]  # the written cache reads back the same
    assert all(s.endswith(",0") for s in look["builtin"])
    # the workload's matrices (n <= 6) all fall in the bucket 1-64, which is
    # tuned; the synthetic buckets stop at nmax = 6
    tuned = [s.endswith(",1") for s in look["tuned"]]
    assert tuned == [n <= (64 if mode == "workload" else hi) for n in LOOKUP_N], look["tuned"]
    with open(cache) as f:
        tabs = json.load(f)["tables"]
    assert [t["arch"] for t in tabs] == ["gfx950"] and tabs[0]["count"] == count
    assert tabs[0]["buckets"][0]["nmin"] == 1


def test_tune_search_workload_limit_sanitized(objects):
    rc, errors, _, lines = _search(objects, str(objects["out"] / "limit.json"), "workload", 300, 4)
    assert rc == 3 and errors == 0, lines  # RRF_E_NOTSUP: at most 256 matrices


@pytest.mark.parametrize("inject,status", [("", 0), ("alloc", 2), ("hip", 1)])
def test_batched_abi_fault_injection_sanitized(objects, inject, status):
    # RRF_E_NOMEM / RRF_E_HIP from the injected failure; the next call, with
    # the variable unset, allocates the workspace and runs
    r = subprocess.run([objects["api"], "-", "batched", "40", "9"], capture_output=True,
                       text=True, timeout=600,
                       env={**os.environ, **ENV, "RRF_TUNE_CACHE": "", "RRF_TEST_FAIL": inject})
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    # the b = 0 lookups of the 40 matrices query the device's properties once
    # per process, not once per matrix
    queries = "0" if inject == "hip" else "1"
    assert r.stdout.split() == ["batched", str(status), "0", queries,
                                "batched", "0", "0", "1"], r.stdout


def test_planner_threads_tsan(tsan_objects, monkeypatch):
    # 1100 matrices: four slices, the direct mode runs each on a host thread
    for k, v in TSAN_ENV.items():
        monkeypatch.setenv(k, v)
    rng = np.random.default_rng(11)
    ns = rng.integers(1, 7, size=1100)
    shapes = [(int(rng.integers(n, 2 * n + 1)), int(n)) for n in ns]
    planner._run((tsan_objects["planner"], tsan_objects["out"]), shapes, 4, 1, 13, graph=False)


def test_allow_dynamic_lds_tsan(tsan_objects):
    r = subprocess.run([tsan_objects["context_host"]], capture_output=True, text=True,
                       timeout=300, env={**os.environ, **TSAN_ENV})
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    lines = r.stdout.splitlines()
    assert "unexpected" not in lines
    calls = {}
    for ln in lines:
        parts = ln.split()
        if len(parts) == 3 and parts[0] in ("0", "1"):
            calls.setdefault((int(parts[0]), int(parts[1])), []).append(int(parts[2]))
    assert sorted(calls) == [(k, d) for k in (0, 1) for d in range(3)]
    for seq in calls.values():  # once per (kernel, device), raised only for a larger request
        assert seq == sorted(set(seq)) and seq[-1] == 128 * 1024 and len(seq) <= 2, seq
    assert "failed 1" in lines and "after 0" in lines  # RRF_E_HIP, then RRF_OK
    assert [ln for ln in lines if ln.startswith("2 ")] == ["2 1 102400"]
