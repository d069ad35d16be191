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
    """The GPU's bracket of every pair equals the oracle's.  On a near tie of
    the oracle's light-cone test (``ref.alt`` differs from ``ref`` there) the
    bracket of the other decision is accepted as well; the number of near
    ties is printed (none are expected on the workloads: the band is about
    1e-13 of the light distance)."""
    got = np.asarray(got)
    k = np.asarray(ref)
    alt = getattr(ref, "alt", None)
    wrong = got != k
    ties = 0
    if alt is not None:
        ties = int(np.count_nonzero(alt != k))
        wrong &= got != alt
    bad = np.argwhere(wrong)
    print(f"{tag}: k* pairs {got.size}, mismatches {len(bad)}, near ties {ties}, "
          f"before-history {np.mean(k < 0):.3f}", flush=True)
    assert len(bad) == 0, [(tuple(b), int(got[tuple(b)]), int(k[tuple(b)])) for b in bad[:5]]


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


def bracket_row_hashes(kstar):
    """Per target of a [m, N] k* array: the SHA-256 of its row as
    little-endian int32 (a different bracket on any pair changes it)."""
    import hashlib

    k = np.ascontiguousarray(np.asarray(kstar), dtype="<i4")
    return [hashlib.sha256(row.tobytes()).hexdigest() for row in k]


def near_tie_list(ref):
    """[(target, source, k*, alt)] of the oracle's near ties."""
    k = np.asarray(ref)
    alt = getattr(ref, "alt", None)
    if alt is None:
        return []
    return [(int(a), int(j), int(k[a, j]), int(alt[a, j])) for a, j in np.argwhere(alt != k)]


def assert_kstar_hashes(tag, got, hashes, ties):
    """The GPU's k* rows against stored per-row hashes of the oracle's; on
    the stored near ties the other decision's bracket is mapped back to the
    oracle's before hashing."""
    got = np.array(got, dtype=np.int32, copy=True)
    for a, j, k, alt in ties:
        if got[a, j] == alt:
            got[a, j] = k
    mine = bracket_row_hashes(got)
    bad = [a for a, (h1, h2) in enumerate(zip(mine, hashes)) if h1 != h2]
    print(f"{tag}: k* rows {len(hashes)} x {got.shape[1]} pairs, rows differing {len(bad)}, near ties {len(ties)}",
          flush=True)
    assert not bad, bad[:5]


def load_c5_subset():
    """The stored oracle reference at 1024 targets of the N=262144, D=1024
    workload (written by tests/golden/make_c5_subset.py)."""
    import json
    import os

    doc = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c5_subset.json")))
    out = {k: np.asarray(doc[k]) for k in ("targets", "E", "B", "SE", "SB")}
    out["targets"] = out["targets"].astype(np.int64)
    out["kstar_sha256"] = list(doc["kstar_sha256"])
    out["near_ties"] = [tuple(t) for t in doc["near_ties"]]
    out["before_history_fraction"] = doc["before_history_fraction"]
    return out


def load_c2_steps():
    """The oracle's free run of the N=8192, D=512 workload at steps 1 and 10
    (written by tests/golden/make_c2_steps.py)."""
    import json
    import os

    doc = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_steps.json")))
    out = {"targets": np.asarray(doc["targets"], dtype=np.int64), "steps": {}}
    for s, d in doc["steps"].items():
        e = {k: np.asarray(d[k]) for k in ("y", "u", "E", "B", "SE", "SB", "sigma")}
        e["t"] = float(d["t"])
        e["kstar_sha256"] = list(d["kstar_sha256"])
        e["near_ties"] = [tuple(t) for t in d["near_ties"]]
        e["before_history_fraction"] = d["before_history_fraction"]
        out["steps"][int(s)] = e
    return out
