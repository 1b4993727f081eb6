"""bench.py's stdout contract on the host: the last line is one short JSON
object carrying the contract's keys, `roofline` and `cpu_baseline`, with the
bulky per-leg arrays left to the full-results file."""
import json
import math

import bench


def _acc(n=51):
    return {"orth_U": 2e-14, "orth_V": 3e-14, "recon": 2.5e-14, "ek_over_sigma_max": 1.11,
            "ek_over_sigma_argmax_k": 256, "ek_over_sigma_min": 0.98,
            "k_grid": list(range(n)), "e_k": [1.0 / (k + 1) for k in range(n)],
            "norm_estimator": "power iteration"}


def _kernels(count=40):
    return {f"kernel_{i}": {"launches": 100, "ms_per_step": 1.0, "tflops": 10.0, "gbs": None}
            for i in range(count)}


def _full_object():
    out = {
        "metric": bench.METRIC, "value": 1.1980123456, "unit": "s", "n_gpus": 1, "steps": 20,
        "warmup": 5, "ms_per_step": 1198.0123456, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "randUTV n=16384 b=128 q=2", "n": 16384, "b": 128, "q": 2,
                   "precision": "fp64", "sketch_seed": 1},
        "roofline": {"bound": "mfma", "kernel": "dgemm_mfma_128x128_TN", "achieved": 49.9123,
                     "peak": 78.6, "unit": "TFLOP/s", "frac": 0.6350123, "traffic": 595841394,
                     "traffic_unit": "bytes per launch", "algorithmic_bytes_per_launch": 5e8,
                     "flops_per_launch": 1.56e10, "avg_launch_ms": 0.313},
        "gemm_all": {"tflops": 45.0, "frac": 0.57, "ms_per_step": 900.0},
        "model_tflops": 39.7, "kernels": _kernels(), "kernels_from": "warmup",
        "accuracy": _acc(),
        "cpu_baseline": {"value": 144.39, "unit": "s", "cores": 16, "kind": "oracle",
                         "sample": "first 8 of 128 steps"},
    }
    for name, prec in (("mixed", "bf16_sketch"), ("mixed_x3", "bf16_x3")):
        out[name] = {"precision": prec, "value": 1.0, "unit": "s", "ms_per_step": 1000.0,
                     "speedup_vs_fp64": 1.19, "model_tflops": 47.0, "kernels": _kernels(),
                     "accuracy": _acc(), "ek_over_fp64_max": 1.01, "ek_gate_pass": True,
                     "ek_gate_k": list(range(11)), "recon_le_1e-6": True}
    out["powerurv"] = {"model_flops": 1e14,
                       "fp64": {"value": 3.0, "unit": "s", "model_tflops": 34.0,
                                "accuracy": _acc()},
                       "bf16_sketch": {"value": 2.5, "unit": "s", "model_tflops": 40.0,
                                       "accuracy": _acc(), "ek_gate_pass": True},
                       "speedup_mixed": 1.2}
    out["gap"] = {"k_grid": list(range(900, 1101, 4)), "modes": {
        mode: {"value": 1.0, "speedup_vs_fp64": 1.0, "recon": 1e-14, "orth_U": 1e-14,
               "orth_V": 1e-14, "e_k": [3e-10] * 51, "ek_over_fp64": [1.0] * 51,
               "e_1000": 2.96e-10, "e_1024": 2.96e-10}
        for mode in ("fp64", "bf16_sketch", "bf16_x3")},
        "fp64_thin_u": {"value": 0.72, "unit": "s", "recon": 1.7e-14}}
    out["boosted"] = {"value": 4.9, "unit": "s", "accuracy": _acc(), "ek_over_basic": [1.0] * 51}
    out["partial"] = {"value": 0.5, "unit": "s", "k": 3712}
    out["rsvd"] = {"value": 0.0259, "unit": "s", "err_over_sigma_l1": 1.085}
    out["batched"] = {"value": 15601.5, "unit": "matrices/s", "ms_per_call": 262.5,
                      "model_tflops": 11.28, "residual_fro_rel": {"max": 6.6e-15},
                      "kernels": _kernels(), "cpu_baseline": {"value": 2.38}}
    out["full_results"] = "results/bench_full.json"
    return out


def test_headline_is_short_and_parseable():
    full = _full_object()
    line = json.dumps(bench.headline(full), separators=(",", ":"))
    assert "\n" not in line
    assert len(line) < 4096, len(line)
    h = json.loads(line)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config"):
        assert k in h
    assert h["roofline"]["frac"] == bench._r(0.6350123)
    assert h["roofline"]["traffic"] == 595841394
    assert h["cpu_baseline"]["cores"] == 16 and h["cpu_baseline"]["kind"] == "oracle"
    assert math.isclose(h["value"], 1.198, rel_tol=1e-3)
    assert h["legs"]["mixed"]["ek_gate_pass"] is True
    assert h["legs"]["batched"]["unit"] == "matrices/s"


def test_headline_without_optional_legs():
    full = _full_object()
    for k in ("mixed", "mixed_x3", "powerurv", "gap", "boosted", "partial", "rsvd", "batched",
              "cpu_baseline", "accuracy"):
        del full[k]
    h = bench.headline(full)
    assert h["legs"] == {} and "cpu_baseline" not in h
