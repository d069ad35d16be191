"""Throughput of the EM-PP Lienard-Wiechert hot path on one MI355X.

A step is one pass of the whole hot path over the bunch: the all-pairs
retarded-time search + LW field sum (pair kernel) and the Higuera-Cary
push with the history update (push kernel).  Inputs are resident in HBM
before the timed region.  Prints ONE JSON line on stdout; progress goes to
stderr.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload c3] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2605_05543_amd import bunch  # noqa: E402

PEAK_FP64_VECTOR_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
PEAK_BF16_TFLOPS = 2500.0  # dense matrix-core peak
# one evaluation of the 10 -> 128 -> 128 -> 1 network: 2 x 17792 multiply-adds
MLP_FLOP_EVAL = 2 * (10 * 128 + 128 * 128 + 128)

# Algorithmic FP64 operations of one (target, source) pair, counted from the
# method's steps (add, sub, mul = 1; sqrt, div = 1; compare = 0):
#   sign test of one stored sample (Sec. 2.2):      9 per probe
#   root of Eq. (dt) incl. coefficients:           32
#   reconstruction Eq. (linear) / (linear2):       20 / 6
#   LW E and B, Eqs. (LW_E), (LW_B):               69 / 48 (a = 0 out of history)
#   accumulation of E and B:                        6
FLOP_PROBE = 9
GUESS_NAMES = ["bisect", "mlp", "ballistic", None, "previous"]
# The roofline's algorithmic work per pair: the plain path's estimate of the
# measurement plan (about 10 sign tests of 11 flops, 33 for the quadratic,
# 22 for the reconstruction, 80 for the LW terms, 6 for the sum, in history;
# 2 sign tests and no acceleration terms before it; the workload's mix).
ROOFLINE_FLOP_PER_PAIR = 220.0
FLOP_INRING = 32 + 20 + 69 + 6
FLOP_BEFORE = 32 + 6 + 48 + 6


def measured_traffic():
    """HBM bytes per launch of the pair kernels from the committed rocprofv3
    FETCH_SIZE/WRITE_SIZE summary, {path: bytes}, or {} when the kernel
    sources have changed since those counters were taken."""
    import re

    prof = os.path.join(ROOT, "profiles", "pair_kernels_c3_traffic.md")
    try:
        text = open(prof).read()
    except OSError:
        return {}
    m_h = re.search(r"sources: " + " ".join(KERNEL_SOURCES) + r" sha256 ([0-9a-f]+)", text)
    if not m_h or not kernel_sources_sha().startswith(m_h.group(1)):
        return {}
    return {m.group(1): float(m.group(2)) for m in re.finditer(r"traffic_bytes_per_launch\[([a-z0-9:/]+)\]:\s*([0-9.eE+]+)",
                                                              text)}


# the sources the pair kernels are compiled from (traffic counters are
# valid while they are unchanged)
KERNEL_SOURCES = ("pair_fp64.hip", "pair_mixed.hip", "pair_kernel.h", "pair_common.h", "empp_dev.h")


def kernel_sources_sha():
    import hashlib

    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2605_05543_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_flops(counters):
    return (FLOP_PROBE * counters["probes"] + FLOP_INRING * (counters["pairs"] - counters["before"])
            + FLOP_BEFORE * counters["before"])


SURROGATE_SAMPLES = 50_000_000  # training pairs, half from a C2 bunch, half from this workload's


def train_surrogate(ctx, wl, r, epochs=2):
    """Train the context's surrogate network on pairs drawn from a C2 bunch
    and from this workload's bunch (4 steps in), before any timing."""
    from paper_2605_05543_amd import surrogate

    half = SURROGATE_SAMPLES // 2
    s2 = surrogate.draw_samples(bunch.C2, half, seed=21)
    ctx.step(4)
    ctx.surrogate_set(bunch.surrogate_init(0), bunch.sigma_ref_of(r))
    s3 = ctx.surrogate_samples_torch(half, seed=23)
    batch = 8192
    rep = surrogate.train(ctx, [s2, s3], batch=batch, steps=epochs * (SURROGATE_SAMPLES // batch))
    rep["batch"] = batch
    del s2, s3
    log(f"  surrogate trained on {SURROGATE_SAMPLES:.1e} pairs: loss {rep['loss_first']:.3e} -> "
        f"{rep['loss_last']:.3e} in {rep['steps']} steps, {rep['seconds']:.2f} s")
    return rep


def gyrating_start(wl, r, u, epochs=2):
    """The gyrating workload's starting state: the bunch stepped (FP64, the
    paper's bisection) for depth + 20 steps from its straight history, so
    that every stored slot lies on the curving paths, and the surrogate
    trained on 2^23 pairs of that state.  Returns the history, proper
    velocities and network."""
    from paper_2605_05543_amd import surrogate
    from paper_2605_05543_amd._lib import Context

    ctx = Context(n=wl.bunch.n, depth=wl.depth, q=-bunch.E_CHARGE, m=bunch.M_ELECTRON, dt=wl.dt,
                  ext_field=wl.ext_field, dipole_b0=wl.dipole_b0, dipole_re=wl.dipole_re)
    ctx.init_bunch(r, u, 0.0)
    ctx.init_history_straight()
    spin = wl.depth + 20
    done = 0
    while done < spin:
        k = min(128, spin - done)
        ctx.step(k)
        done += k
        ctx.sync()
        log(f"  spin-up: {done} of {spin} steps")
    rn, un, _, _ = ctx.state()
    sig = bunch.sigma_ref_of(rn)
    ctx.surrogate_set(bunch.surrogate_init(0), sig)
    count = 1 << 23
    X, y = ctx.surrogate_samples_torch(count, seed=31)
    rep = surrogate.train(ctx, [(X, y)], batch=8192, steps=epochs * (count // 8192))
    rep["batch"] = 8192
    log(f"  surrogate trained on {count} pairs of the gyrating state: loss {rep['loss_first']:.3e} -> "
        f"{rep['loss_last']:.3e} in {rep['steps']} steps, {rep['seconds']:.2f} s")
    T, w, v = ctx.history()
    start = {"T": T, "w": w, "v": v, "u": un, "params": ctx.surrogate_get(), "sigma_ref": sig, "training": rep,
             "spin_up_steps": spin}
    ctx.close()
    return start


def run_path(wl, r, u, precision, guess, steps, warmup, train_epochs=2, group_log2=0, keep_fields=False,
             stage2=None, start=None):
    """Time one search mode on the workload: ``steps`` steps after
    ``warmup``, kernel times from HIP events.  With ``keep_fields`` the
    path's step fields at the initial state (all particles) are returned
    too, for the error check against the oracle; with ``stage2`` (c5) the
    run continues with the handoff and Stage-II transport; ``start`` (the
    gyrating workload) is a stored state and trained network to begin from."""
    import torch

    from paper_2605_05543_amd._lib import Context

    n = wl.bunch.n
    spec = f"{['fp64', 'mixed'][precision]}:{GUESS_NAMES[guess]}" + (f"/{group_log2}" if group_log2 else "")
    ctx = Context(n=n, depth=wl.depth, q=-bunch.E_CHARGE, m=bunch.M_ELECTRON, dt=wl.dt, ext_field=wl.ext_field,
                  dipole_b0=wl.dipole_b0, dipole_re=wl.dipole_re, precision=precision,
                  guess=4 if guess == 4 else 0, guess_group_log2=group_log2)

    def initial_state():
        if start:
            ctx.set_history(start["T"], start["w"], start["v"], start["u"])
        else:
            ctx.init_bunch(r, u, 0.0)
            ctx.init_history_straight()

    initial_state()
    train_rep = None
    if guess == 1 and start:
        ctx.surrogate_set(start["params"], start["sigma_ref"])
    elif guess == 1:
        train_rep = train_surrogate(ctx, wl, r, train_epochs)
    ctx.set_mode(precision, guess)
    if guess == 4:
        ctx.step(1)  # the first step bisects and fills the bracket cache
    # one counting step (untimed) for the algorithmic work per launch
    ctx.set_counting(True)
    ctx.step(1)
    cnt = ctx.counters()
    ctx.set_counting(False)
    if warmup:
        ctx.step(warmup)
    ctx.sync()
    d0 = ctx.diag()
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:  # progress every 100 steps on long runs
        k = min(100, steps - done)
        ctx.step(k)
        done += k
        if steps > 100:
            ctx.sync()
            log(f"    {spec}: {done} steps")
    ctx.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tim = ctx.timing()
    ctx.set_timing(False)
    d = ctx.diag()
    pairs = n * (n - 1)
    pair_ms = tim["pair_ms"] / max(1, tim["pair_launches"])
    flops = algorithmic_flops(cnt)
    out = {
        "precision": ["fp64", "mixed"][precision], "guess": GUESS_NAMES[guess], "spec": spec,
        "pair_evals_per_s": pairs * steps / elapsed, "ms_per_step": 1e3 * elapsed / steps,
        "pair_kernel_ms": pair_ms, "push_kernel_ms": tim["push_ms"] / max(1, tim["push_launches"]),
        "probes_per_pair": cnt["probes"] / cnt["pairs"], "before_history_fraction": cnt["before"] / cnt["pairs"],
        "fallbacks": cnt["fallbacks"], "flops_per_pair": flops / cnt["pairs"],
        "achieved_tflops": flops / (pair_ms * 1e-3) / 1e12, "sigma_after": d["sigma"],
        "guess_kernel_ms": tim["guess_ms"] / max(1, tim["guess_launches"]) if tim["guess_launches"] else 0.0,
        "rescues_per_pair": cnt["rescues"] / cnt["pairs"],
    }
    if guess == 1:
        # the network on the matrix cores: evaluations per launch x its BF16
        # operations, over the measured guess-kernel time
        tpg = 1 << (group_log2 or 6)
        evals = -(-n // tpg) * n
        out["targets_per_guess"] = tpg
        if out["guess_kernel_ms"] > 0:
            tf = evals * MLP_FLOP_EVAL / (out["guess_kernel_ms"] * 1e-3) / 1e12
            out["guess_bf16_tflops"] = tf
            out["guess_mfma_frac"] = tf / PEAK_BF16_TFLOPS
    if train_rep:
        # forward plus input and weight gradients: about three forward passes
        train_rep["bf16_tflops"] = (train_rep["steps"] * train_rep["batch"] * 3 * MLP_FLOP_EVAL
                                    / train_rep["seconds"] / 1e12)
        out["surrogate_training"] = train_rep
    if stage2:
        # Stage I -> II (Sec. 2.7): handoff, then transport in the dipole
        sig1 = d["sigma"]
        ctx.handoff()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        left = stage2["steps"]
        while left > 0:
            k = min(20000, left)
            ctx.transport(stage2["dt_max"], stage2["gyro_fraction"], k)
            left -= k
            log(f"    transport: {stage2['steps'] - left} steps, t = {ctx.state()[2]:.4e} s")
        el2 = time.perf_counter() - t1
        d2 = ctx.diag()
        out["stage2"] = {"steps": stage2["steps"], "dt_max": stage2["dt_max"], "gyro_fraction": stage2["gyro_fraction"],
                         "seconds": el2, "steps_per_s": stage2["steps"] / el2, "t_end": d2["t"],
                         "sigma_stage1_start": d0["sigma"], "sigma_handoff": sig1, "sigma_end": d2["sigma"],
                         "sigma_growth_stage1": [b / a for a, b in zip(d0["sigma"], sig1)],
                         "sigma_growth_stage2": [b / a for a, b in zip(sig1, d2["sigma"])]}
        ctx.close()
        ctx = None
    if keep_fields and ctx is not None:
        # the path's step fields at the initial state, in the timed launch shape
        if start:
            initial_state()
        else:
            ctx.init_history_straight()
        ctx.step(1)
        out["_fields"] = ctx.fields()
    if ctx is not None:
        ctx.close()
    log(f"  {spec}: {out['pair_evals_per_s']:.3e} pair-evals/s, {out['ms_per_step']:.2f} ms/step, pair kernel "
        f"{pair_ms:.2f} ms, {out['probes_per_pair']:.2f} probes/pair")
    return out


def cpu_baseline(wl, r, u, target_seconds=15.0, start=None):
    """The oracle's rate on a bounded sample of the workload (fields at
    seeded targets x all sources at the initial state: the straight-line
    history, or the stored state of the gyrating workload), on all host
    threads and on one.  Returns the record and the oracle's fields at the
    sample's targets (for the GPU paths' error)."""
    import oracle

    orc = oracle.get()
    n = wl.bunch.n
    if start:
        T, w, v = start["T"], start["w"], start["v"]
        r = np.ascontiguousarray(w[-1])
    else:
        T, w, v = orc.init_straight(r, u, wl.depth, wl.dt)
    threads = orc.max_threads()
    probe = bunch.target_subset(n, 4 * threads, 1001)  # every thread busy in the rate probe
    t0 = time.perf_counter()
    orc.fields(T, w, v, -bunch.E_CHARGE, T[-1], r[:, probe], probe)
    rate = len(probe) / (time.perf_counter() - t0)
    m = int(max(8, min(n, rate * target_seconds)))
    sub = bunch.target_subset(n, m, 1002)
    t0 = time.perf_counter()
    E, B, SE, SB = orc.fields(T, w, v, -bunch.E_CHARGE, T[-1], r[:, sub], sub, want_abs=True)
    el = time.perf_counter() - t0
    value = m * (n - 1) / el
    log(f"  cpu oracle: {m} targets x {n - 1} sources in {el:.1f} s on {threads} threads: {value:.3e} pair-evals/s")
    # the same scan on one thread, over a short sample (about 4 s)
    m1 = int(max(2, min(n, 4.0 * value / threads / (n - 1))))
    sub1 = bunch.target_subset(n, m1, 1003)
    t0 = time.perf_counter()
    orc.fields(T, w, v, -bunch.E_CHARGE, T[-1], r[:, sub1], sub1, nthreads=1)
    el1 = time.perf_counter() - t0
    value1 = m1 * (n - 1) / el1
    log(f"  cpu oracle, one thread: {m1} targets in {el1:.1f} s: {value1:.3e} pair-evals/s")
    rec = {"value": value, "unit": "pair-evals/s", "cores": threads, "kind": "oracle",
           "sample": f"fields at {m} seeded targets x {n - 1} sources, one step of {wl.name} "
                     f"(FP64 C oracle, linear history scan), {el:.1f} s",
           "single_core_value": value1,
           "single_core_sample": f"{m1} seeded targets x {n - 1} sources on one thread, {el1:.1f} s"}
    return rec, (sub, E, B, SE, SB)


def field_error(got, ref, S):
    """max_i |d_i| / rms_k |ref_k| and max_i |d_i| / S_i for [3, m] arrays."""
    d = np.linalg.norm(got - ref, axis=0)
    rms = np.sqrt(np.mean(np.sum(ref * ref, axis=0)))
    return float(d.max() / rms), float(np.max(d / S))


def error_vs_oracle(fields, ref):
    sub, E0, B0, SE, SB = ref
    E, B = fields
    e_rms, e_s = field_error(E[:, sub], E0, SE)
    b_rms, b_s = field_error(B[:, sub], B0, SB)
    return {"targets": int(len(sub)), "E_max_over_rms": e_rms, "B_max_over_rms": b_rms, "E_max_over_S": e_s,
            "B_max_over_S": b_s}


def c5_error(fields):
    """Error of step fields against the stored oracle values at 1024 seeded
    targets of the N = 262144 workload (tests/golden/c5_subset.json)."""
    import json

    doc = json.load(open(os.path.join(ROOT, "tests", "golden", "c5_subset.json")))
    sub = np.asarray(doc["targets"], dtype=np.int64)
    ref = (sub, np.asarray(doc["E"]), np.asarray(doc["B"]), np.asarray(doc["SE"]), np.asarray(doc["SB"]))
    return error_vs_oracle(fields, ref)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3", "c5", "c3g"],
                    help="c3g: the C3 bunch gyrating in a 0.5 T field, timed from a curved history")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--train-epochs", type=int, default=2, help="passes over the surrogate's training pairs")
    ap.add_argument("--paths", default=None,
                    help="precision:search[/k], k = log2 of the targets per surrogate evaluation (c3 default: "
                         "fp64:bisect,mixed:mlp/12,mixed:mlp,mixed:bisect,mixed:ballistic,fp64:ballistic,"
                         "fp64:previous; c5: fp64:bisect,mixed:mlp/12)")
    ap.add_argument("--transport-steps", type=int, default=100000, help="c5: Stage-II steps after the handoff")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (scale for the FETCH_SIZE/WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch

        src = torch.ones(2**27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copied 3 x 1 GiB")
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the pair sum would shard by "
              "targets, each GPU holding a replica of the history ring). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    wl = {"c1": bunch.C1, "c2": bunch.C2, "c3": bunch.C3, "c5": bunch.C5, "c3g": bunch.C3G}[args.workload]
    c5 = wl is bunch.C5
    gyro = wl is bunch.C3G
    paths = args.paths or ("fp64:bisect,mixed:mlp/12" if c5 else
                           "fp64:bisect,mixed:mlp/12,mixed:mlp,fp64:mlp/12,fp64:mlp,mixed:ballistic,fp64:ballistic"
                           if gyro else
                           "fp64:bisect,mixed:mlp/12,mixed:mlp,mixed:bisect,mixed:ballistic,fp64:ballistic,"
                           "fp64:previous")
    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    r, u = bunch.gyrating_bunch(wl) if gyro else bunch.gaussian_bunch(wl.bunch)
    log(f"workload {wl.name}: N={wl.bunch.n} D={wl.depth} dt={wl.dt} steps={args.steps} warmup={args.warmup}")
    start = gyrating_start(wl, r, u, args.train_epochs) if gyro else None
    pmap = {"fp64": 0, "mixed": 1}
    gmap = {name: k for k, name in enumerate(GUESS_NAMES) if name}
    results = []
    for k, spec in enumerate(paths.split(",")):
        p, g = spec.split(":")
        g, _, lg = g.partition("/")
        head_candidate = p == "mixed" and g == "mlp"
        st2 = ({"steps": args.transport_steps, "dt_max": 1e-7, "gyro_fraction": 1 / 32}
               if c5 and head_candidate else None)
        results.append(run_path(wl, r, u, pmap[p], gmap[g], args.steps, args.warmup, args.train_epochs, int(lg or 0),
                                keep_fields=(k == 0 or spec == "fp64:bisect" or head_candidate or gyro) and not st2, stage2=st2, start=start))
    # the plain FP64 path (the paper's bisection) when it was run; the
    # roofline then describes its kernel, else the first path's
    plain = next((x for x in results if x["spec"] == "fp64:bisect"), None)
    ref = plain or results[0]
    # headline: the mixed-precision surrogate-guided path when it was run,
    # else the first mixed path, else the plain FP64 path
    mixed = [x for x in results if x["precision"] == "mixed"]
    head = next((x for x in mixed if x["guess"] == "mlp"), mixed[0] if mixed else ref)
    ball = next((x for x in results if x["spec"] == "fp64:ballistic"), None)
    n = wl.bunch.n
    pairs = n * (n - 1)
    achieved = ROOFLINE_FLOP_PER_PAIR * pairs / (ref["pair_kernel_ms"] * 1e-3) / 1e12
    traffic = measured_traffic() if wl is bunch.C3 else {}
    for x in results:
        tb = traffic.get(x["spec"])
        x["hbm_bytes_per_launch"] = tb
        x["hbm_bytes_per_pair"] = tb / pairs if tb else None
    tplain = traffic.get(ref["spec"])
    line = {
        "metric": "LW pair-evals/s at N=65536 (FP32+surrogate vs FP64 plain, <=1e-5 rel err)",
        "value": head["pair_evals_per_s"],
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head["precision"] == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "n": n, "depth": wl.depth, "dt": wl.dt, "ext_field": wl.ext_field,
                   "precision": head["precision"], "search": head["spec"]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_VECTOR_TFLOPS, "traffic": tplain,
                     "kernel": ("pair_fp64_kernel (plain FP64 path, the paper's bisection)" if plain else
                                f"pair kernel of the {ref['spec']} path"),
                     "flops_per_pair": ROOFLINE_FLOP_PER_PAIR, "counted_flops_per_pair": ref["flops_per_pair"],
                     "launch_ms": ref["pair_kernel_ms"],
                     # counted HBM bytes over the measured launch time, against 8 TB/s
                     "hbm_gbs": tplain / (ref["pair_kernel_ms"] * 1e-3) / 1e9 if tplain else None,
                     "hbm_frac": tplain / (ref["pair_kernel_ms"] * 1e-3) / 1e9 / PEAK_HBM_GBS if tplain else None,
                     "hbm_bytes_per_pair": tplain / pairs if tplain else None},
        # the metric's comparison: FP32 + surrogate over the plain FP64 path,
        # and over the FP64 path with the closed-form straight-line guess
        "speedup_vs_plain_fp64": head["pair_evals_per_s"] / plain["pair_evals_per_s"] if plain else None,
        "speedup_vs_ballistic": head["pair_evals_per_s"] / ball["pair_evals_per_s"] if ball else None,
        "paths": results,
    }
    if c5 and plain and "_fields" in plain:
        line["error_vs_oracle"] = {"plain": c5_error(plain["_fields"])}
    if c5 and "stage2" in head:
        line["stage2"] = head.pop("stage2")
    if gyro:
        line["gyrating_start"] = {"spin_up_steps": start["spin_up_steps"], "surrogate_training": start["training"]}
        # sign tests per pair of each path over the bisection's: what each
        # guess saves in searching the curved histories
        for x in results:
            x["probes_vs_bisect"] = x["probes_per_pair"] / plain["probes_per_pair"] if plain else None
    if not args.no_cpu and not c5:
        rec, ref = cpu_baseline(wl, r, u, target_seconds=8.0 if gyro else 15.0, start=start)
        line["cpu_baseline"] = rec
        line["error_vs_oracle"] = {x["spec"]: error_vs_oracle(x["_fields"], ref) for x in results if "_fields" in x}
        log(f"  errors vs the oracle: {line['error_vs_oracle']}")
    for x in results:
        x.pop("_fields", None)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
