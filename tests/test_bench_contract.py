"""bench.py's one-line JSON contract, checked on the CPU: the GPU paths are
replaced by a stand-in that returns fixed timings, so only the assembly of
the line, the refusal of several GPUs and the oracle baseline's record are
exercised here."""
import contextlib
import io
import json
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2605_05543_amd import bunch  # noqa: E402


def _fake_path(wl, r, u, precision, guess, steps, warmup, train_epochs=2, group_log2=0, keep_fields=False,
               stage2=None, start=None):
    spec = f"{['fp64', 'mixed'][precision]}:{bench.GUESS_NAMES[guess]}" + (f"/{group_log2}" if group_log2 else "")
    rate = {"fp64:bisect": 1.2e11, "fp64:ballistic": 1.35e11}.get(spec, 1.3e11)
    out = {"precision": ["fp64", "mixed"][precision], "guess": bench.GUESS_NAMES[guess], "spec": spec,
           "pair_evals_per_s": rate, "ms_per_step": 35.7, "pair_kernel_ms": 35.5, "flops_per_pair": 182.9,
           "probes_per_pair": 10.0 if guess == 0 else 7.0}
    if keep_fields:
        n = wl.bunch.n
        out["_fields"] = (np.ones((3, n)), np.ones((3, n)))
    return out


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
    d = _run_main(monkeypatch, ["--no-cpu", "--paths", "fp64:bisect,mixed:mlp/12,fp64:ballistic"])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["higher_is_better"] is True and d["vs_baseline"] is None
    assert d["config"]["workload"] == bunch.C3.name
    assert d["value"] == 1.3e11  # the FP32 + surrogate path is the headline
    assert abs(d["speedup_vs_plain_fp64"] - 1.3 / 1.2) < 1e-12
    assert abs(d["speedup_vs_ballistic"] - 1.3 / 1.35) < 1e-12
    assert d["config"]["search"] == "mixed:mlp/12"
    rf = d["roofline"]
    for key in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert key in rf, key
    assert rf["bound"] == "alu" and rf["unit"] == "TFLOP/s" and rf["peak"] == 78.6
    n = bunch.C3.bunch.n
    # the plan's algorithmic work per pair, over the plain kernel's launch time
    assert rf["flops_per_pair"] == 220.0 and rf["counted_flops_per_pair"] == 182.9
    assert abs(rf["achieved"] - 220.0 * n * (n - 1) / 35.5e-3 / 1e12) < 1e-9
    assert abs(rf["frac"] - rf["achieved"] / 78.6) < 1e-12
    # traffic comes from the committed counters while the kernel sources match them
    if rf["traffic"] is not None:
        assert rf["hbm_bytes_per_pair"] == rf["traffic"] / (n * (n - 1))


def test_line_without_the_plain_path(monkeypatch):
    # no plain FP64 path among those run: no speedup over it is claimed, and
    # the roofline names the kernel it was taken from
    d = _run_main(monkeypatch, ["--no-cpu", "--paths", "mixed:mlp/12,fp64:ballistic"])
    assert d["value"] == 1.3e11 and d["speedup_vs_plain_fp64"] is None
    assert d["roofline"]["kernel"] == "pair kernel of the mixed:mlp/12 path"
    d = _run_main(monkeypatch, ["--no-cpu", "--paths", "fp64:ballistic,fp64:bisect"])
    # without a mixed path the plain one is the headline
    assert d["roofline"]["kernel"].startswith("pair_fp64_kernel (plain")
    assert d["value"] == 1.2e11 and d["speedup_vs_plain_fp64"] == 1.0
    assert abs(d["speedup_vs_ballistic"] - 1.2 / 1.35) < 1e-12


def test_several_gpus_are_refused(monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as ei:
        bench.main()
    assert ei.value.code == 2


def test_cpu_baseline_record():
    wl = bunch.C1
    r, u = bunch.gaussian_bunch(wl.bunch)
    rec, (sub, E, B, SE, SB) = bench.cpu_baseline(wl, r, u, target_seconds=0.2)
    assert rec["kind"] == "oracle" and rec["unit"] == "pair-evals/s"
    assert rec["value"] > 0 and rec["single_core_value"] > 0 and rec["cores"] >= 1
    assert "targets" in rec["sample"] and "one thread" in rec["single_core_sample"]
    assert E.shape == (3, len(sub)) and np.all(SE > 0)
    # a path's error against those oracle fields: zero for the oracle's own
    full = (np.zeros((3, wl.bunch.n)), np.zeros((3, wl.bunch.n)))
    full[0][:, sub], full[1][:, sub] = E, B
    err = bench.error_vs_oracle(full, (sub, E, B, SE, SB))
    assert err["E_max_over_rms"] == 0.0 and err["B_max_over_S"] == 0.0 and err["targets"] == len(sub)


def test_headline_error_reported(monkeypatch):
    """With the oracle leg, the line carries each kept path's field error
    against the oracle's fields at the baseline's targets."""
    monkeypatch.setattr(bench, "cpu_baseline", lambda wl, r, u, **kw: (
        {"value": 1.0, "unit": "pair-evals/s", "cores": 1, "kind": "oracle", "sample": "s"},
        (np.arange(4), np.ones((3, 4)), np.ones((3, 4)), np.ones(4), np.ones(4))))
    d = _run_main(monkeypatch, ["--paths", "fp64:bisect,mixed:mlp/12"])
    assert set(d["error_vs_oracle"]) == {"fp64:bisect", "mixed:mlp/12"}
    assert d["error_vs_oracle"]["mixed:mlp/12"]["E_max_over_rms"] == 0.0
    assert "_fields" not in json.dumps(d)


def test_gyrating_workload_line(monkeypatch):
    """The gyrating workload's line: its config, the stored start and each
    path's sign tests against the bisection's."""
    monkeypatch.setattr(bench, "gyrating_start", lambda wl, r, u, epochs=2: {
        "spin_up_steps": wl.depth + 20, "training": {"steps": 1}})
    d = _run_main(monkeypatch, ["--no-cpu", "--workload", "c3g", "--paths", "fp64:bisect,mixed:mlp/12"])
    assert d["config"]["workload"] == bunch.C3G.name
    assert d["gyrating_start"]["spin_up_steps"] == bunch.C3G.depth + 20
    assert [x["probes_vs_bisect"] for x in d["paths"]] == [1.0, 0.7]


def test_cpu_baseline_from_a_stored_history():
    """From a stored history (the gyrating workload's start) the oracle leg
    uses that history and its newest positions as targets: given the
    straight-line history it reproduces the default leg's fields."""
    import oracle

    wl = bunch.C1
    r, u = bunch.gaussian_bunch(wl.bunch)
    T, w, v = oracle.get().init_straight(r, u, wl.depth, wl.dt)
    _, (sub, E, B, _, _) = bench.cpu_baseline(wl, r, u, target_seconds=0.2)
    _, (sub2, E2, B2, _, _) = bench.cpu_baseline(wl, None, None, target_seconds=0.2,
                                                 start={"T": T, "w": w, "v": v})
    common, i1, i2 = np.intersect1d(sub, sub2, return_indices=True)
    assert len(common) > 0
    assert np.array_equal(E[:, i1], E2[:, i2]) and np.array_equal(B[:, i1], B2[:, i2])
