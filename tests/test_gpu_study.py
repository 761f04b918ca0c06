"""The precision and large-graph study drivers at a small scale (R-MAT 12).

Checks that every run the drivers report converges where it must, that the
FP32 and mixed-storage eigenvalues match the FP64-storage solve to 1e-8
relative, that BF16 storage stays within its own accuracy (1e-3), and that
the JSON carries the fields the documented tables are built from.
"""
import argparse
import json

import pytest

pytestmark = pytest.mark.gpu


def run(capsys, fn, **kw):
    fn(argparse.Namespace(**kw))
    out = capsys.readouterr().out.strip().splitlines()
    return json.loads(out[-1])


def test_precision_driver(fe, capsys):
    from paper_1602_01421_amd import study
    d = run(capsys, study.precision, scale=12, block=8, m=64, bf16_restarts=200, spmm_reps=5)
    assert d["n"] == 4096 and len(d["spmm"]) == 2
    for x in d["spmm"]:
        assert x["reps"] == 5 and x["ms_p10"] <= x["ms"] <= x["ms_p90"]
    by = {r["run"]: r for r in d["solves"]}
    assert set(by) == {"f64", "f32", "bf16", "mixed_bf16_f32"}
    assert by["f64"]["status"] == 0 and by["f64"]["max_resid"] <= 1e-9
    for name in ("f32", "mixed_bf16_f32"):
        assert by[name]["status"] == 0 and by[name]["max_resid"] <= 1.5e-6
        assert by[name]["max_eval_rel_err_vs_f64"] <= 1e-8
    assert by["bf16"]["max_eval_rel_err_vs_f64"] <= 1e-3
    assert by["mixed_bf16_f32"]["spmm_calls_bf16"] > 0


def test_large_driver_small_scale(fe, capsys):
    from paper_1602_01421_amd import study
    from paper_1602_01421_amd.learned import DEFAULT_WEIGHTS
    d = run(capsys, study.large, scale=12, configs="4x32,8x48", runs="f64,f32,learned,learned32,mixed",
            max_restarts=500, weights=DEFAULT_WEIGHTS, spmm_reps=3, seeds=1)
    assert [c["block"] for c in d["configs"]] == [4, 8]
    for cfg in d["configs"]:
        by = {r["run"]: r for r in cfg["solves"]}
        assert set(by) == {"f64_reference", "f32_random_start", "learned_start_mixed",
                           "learned_start_f32", "random_start_mixed"}
        for name, r in by.items():
            assert r["status"] == 0, (cfg["block"], name)
            if name != "f64_reference":
                assert r["max_eval_rel_err_vs_f64"] <= 1e-8, (cfg["block"], name)
        assert by["learned_start_f32"]["fallback"] is False
        assert by["learned_start_f32"]["end_to_end_s"] >= by["learned_start_f32"]["seconds"]


def test_gnn_driver_small(fe, capsys):
    from paper_1602_01421_amd import study
    d = run(capsys, study.gnn, log2n=12, mean_deg=16.0, reps=2)
    assert d["n"] == 4096 and d["params"] == 19136
    for mode in ("bf16", "f32"):
        assert all(d[mode][k] > 0 for k in ("forward_ms", "train_step_ms", "adam_ms"))


def test_gathers_driver_small(fe, capsys):
    from paper_1602_01421_amd import study
    d = run(capsys, study.gathers, scale=12, b=16, hub=64, shifts="10,8")
    assert d["n"] == 4096 and d["hub_rows"] > 0 and 0 < d["hub_nonzeros"] < d["nnz"]
    assert [x["columns_per_band"] for x in d["bands"]] == [1024, 256]
    assert d["product_ms"] > 0 and d["gathers_storage_order_ms"] > 0


def test_large_driver_restart_size(fe, capsys):
    from paper_1602_01421_amd import study
    d = run(capsys, study.large, scale=12, configs="8x48k16", runs="f32", max_restarts=500,
            weights=None, spmm_reps=3, seeds=1)
    cfg = d["configs"][0]
    assert (cfg["block"], cfg["m"], cfg["keep"]) == (8, 48, 16)
    assert cfg["solves"][0]["status"] == 0
