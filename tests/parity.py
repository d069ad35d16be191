"""Comparison helpers for GPU-vs-oracle parity tests."""
import numpy as np

# FP64 field tolerance: per target |dE_i| <= TOL * S_i (S_i = sum_j |E_ij|)
# and max_i |dE_i| / rms_k |E_k| <= TOL.
FP64_TOL = 1e-12


def field_errors(got, ref, S):
    """(max_i |d_i| / S_i, max_i |d_i| / rms_k |ref_k|) for [3, m] arrays."""
    d = np.linalg.norm(got - ref, axis=0)
    rms = np.sqrt(np.mean(np.sum(ref * ref, axis=0)))
    return float(np.max(d / S)), float(np.max(d) / rms)


def assert_fields(tag, got_E, got_B, ref_E, ref_B, SE, SB, tol=FP64_TOL):
    e1, e2 = field_errors(got_E, ref_E, SE)
    b1, b2 = field_errors(got_B, ref_B, SB)
    print(f"{tag}: E err/S {e1:.2e} err/rms {e2:.2e}; B err/S {b1:.2e} err/rms {b2:.2e}", flush=True)
    assert e1 <= tol and e2 <= tol and b1 <= tol and b2 <= tol, (e1, e2, b1, b2)


def assert_kstar(tag, got, ref):
    bad = np.argwhere(got != ref)
    print(f"{tag}: k* pairs {got.size}, mismatches {len(bad)}, before-history {np.mean(ref < 0):.3f}", flush=True)
    assert len(bad) == 0, [(tuple(b), int(got[tuple(b)]), int(ref[tuple(b)])) for b in bad[:5]]


# Mixed precision: max_i |dE_i| / rms_k |E_k| <= 1e-5 (and the same for B).
MIXED_TOL = 1e-5


def mixed_report(tag, got_E, got_B, ref_E, ref_B, SE, SB):
    """Primary criterion plus the spread of per-target errors (stated)."""
    out = {}
    for name, g, r, S in (("E", got_E, ref_E, SE), ("B", got_B, ref_B, SB)):
        d = np.linalg.norm(g - r, axis=0)
        rms = np.sqrt(np.mean(np.sum(r * r, axis=0)))
        rel = d / np.maximum(np.linalg.norm(r, axis=0), 1e-300)
        out[name] = {"max_over_rms": float(d.max() / rms), "per_S_max": float(np.max(d / S)),
                     "rel_p50": float(np.percentile(rel, 50)), "rel_p99": float(np.percentile(rel, 99)),
                     "rel_max": float(rel.max())}
    print(f"{tag}: " + "; ".join(f"{k} max/rms {v['max_over_rms']:.2e} max/S {v['per_S_max']:.2e} "
                                f"rel p50 {v['rel_p50']:.1e} p99 {v['rel_p99']:.1e} max {v['rel_max']:.1e}"
                                for k, v in out.items()), flush=True)
    return out


def assert_mixed(tag, got_E, got_B, ref_E, ref_B, SE, SB, tol=MIXED_TOL):
    out = mixed_report(tag, got_E, got_B, ref_E, ref_B, SE, SB)
    assert out["E"]["max_over_rms"] <= tol and out["B"]["max_over_rms"] <= tol, out
    return out


def bracket_checksums(kstar):
    """Per target of a [m, N] k* array: sum_j (k*_aj + 2) and
    sum_j (j + 1)(k*_aj + 2), exact in int64 (a wrong bracket on any one
    pair changes the second sum)."""
    k = np.asarray(kstar).astype(np.int64) + 2
    j = np.arange(1, k.shape[1] + 1, dtype=np.int64)
    return k.sum(axis=1), (k * j).sum(axis=1)


def load_c5_subset():
    """The stored oracle reference at 1024 targets of the N=262144, D=1024
    workload (written by tests/golden/make_c5_subset.py)."""
    import json
    import os

    doc = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c5_subset.json")))
    out = {k: np.asarray(doc[k]) for k in ("targets", "E", "B", "SE", "SB", "kstar_sum", "kstar_weighted_sum")}
    out["targets"] = out["targets"].astype(np.int64)
    out["before_history_fraction"] = doc["before_history_fraction"]
    return out
