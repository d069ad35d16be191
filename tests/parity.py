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
