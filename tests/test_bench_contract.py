"""bench.py's one-line JSON contract, checked on the CPU: the GPU paths are
replaced by a stand-in that returns fixed timings, so only the assembly of
the line, the refusal of several GPUs and the oracle baseline's record are
exercised here."""
import contextlib
import io
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2605_05543_amd import bunch  # noqa: E402


def _fake_path(wl, r, u, precision, guess, *args):
    return {"precision": ["fp64", "mixed"][precision], "guess": bench.GUESS_NAMES[guess],
            "pair_evals_per_s": [1.2e11, 1.3e11][precision], "ms_per_step": [35.7, 32.9][precision],
            "pair_kernel_ms": 35.5, "flops_per_pair": 182.9}


def _run_main(monkeypatch, argv):
    import torch

    monkeypatch.setattr(torch.cuda, "is_available", lambda: True)
    monkeypatch.setattr(bench, "run_path", _fake_path)
    monkeypatch.setattr(sys, "argv", ["bench.py", *argv])
    buf = io.StringIO()
    with contextlib.redirect_stdout(buf):
        bench.main()
    lines = [x for x in buf.getvalue().splitlines() if x.strip()]
    assert len(lines) == 1
    return json.loads(lines[0])


def test_line_has_the_contract_fields(monkeypatch):
    d = _run_main(monkeypatch, ["--no-cpu", "--paths", "fp64:bisect,mixed:mlp/12"])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["higher_is_better"] is True and d["vs_baseline"] is None
    assert d["config"]["workload"] == bunch.C3.name
    assert d["value"] == 1.3e11  # the FP32 + surrogate path is the headline
    assert abs(d["speedup_vs_plain_fp64"] - 1.3 / 1.2) < 1e-12
    rf = d["roofline"]
    for key in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert key in rf, key
    assert rf["bound"] == "alu" and rf["unit"] == "TFLOP/s" and rf["peak"] == 78.6
    n = bunch.C3.bunch.n
    assert abs(rf["achieved"] - 182.9 * n * (n - 1) / 35.5e-3 / 1e12) < 1e-9
    assert abs(rf["frac"] - rf["achieved"] / 78.6) < 1e-12
    # traffic comes from the committed counters while the kernel sources match them
    if rf["traffic"] is not None:
        assert rf["hbm_bytes_per_pair"] == rf["traffic"] / (n * (n - 1))


def test_several_gpus_are_refused(monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as ei:
        bench.main()
    assert ei.value.code == 2


def test_cpu_baseline_record():
    wl = bunch.C1
    r, u = bunch.gaussian_bunch(wl.bunch)
    rec = bench.cpu_baseline(wl, r, u, target_seconds=0.2)
    assert rec["kind"] == "oracle" and rec["unit"] == "pair-evals/s"
    assert rec["value"] > 0 and rec["single_core_value"] > 0 and rec["cores"] >= 1
    assert "targets" in rec["sample"] and "one thread" in rec["single_core_sample"]
