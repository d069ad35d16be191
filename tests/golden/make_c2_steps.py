"""Write c2_steps.json: the oracle's own free run of the N = 8192, D = 512
workload (2 MeV bunch, sigma = (0.5, 0.5, 2) mm, dt = 5e-14 s, no external
field, straight-line prior history) to step 10, and at steps 1 and 10 the
positions of the 64 seeded targets (seed 102), the self-fields at them
(the fields the next step's kick uses), their sums of magnitudes and one
SHA-256 per target of its k* row, with the near ties of the light-cone
test.  The reference for the GPU's free run of the same workload.

Only the oracle computes these values (test infrastructure); the file
records the sha256 of the oracle's C source.  Run from the repository root
(a few minutes on 8 cores):

    python tests/golden/make_c2_steps.py
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2605_05543_amd import bunch  # noqa: E402
from parity import bracket_row_hashes, near_tie_list  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_steps.json")
TARGETS, SEED, CHECK_STEPS = 64, 102, (1, 10)


def oracle_source_sha():
    return hashlib.sha256(open(os.path.join(ROOT, "oracle", "empp_oracle.c"), "rb").read()).hexdigest()


def main():
    wl = bunch.C2
    n = wl.bunch.n
    r, u = bunch.gaussian_bunch(wl.bunch)
    sub = bunch.target_subset(n, TARGETS, SEED)
    orc = oracle.get()
    q = -bunch.E_CHARGE
    run = oracle.OracleRun(orc, r, u, D=wl.depth, dt=wl.dt, q=q, mass=bunch.M_ELECTRON)
    t0 = time.time()
    doc = {"what": "oracle free run of the N=8192, D=512 workload; see make_c2_steps.py",
           "oracle_sha256": oracle_source_sha(), "targets": sub.tolist(), "steps": {}}
    done = 0
    for s in CHECK_STEPS:
        run.step(s - done)
        done = s
        y = run.y
        E, B, k, SE, SB = orc.fields(run.T, run.w, run.v, q, run.t, y[:, sub], sub, want_kstar=True, want_abs=True)
        doc["steps"][str(s)] = {
            "t": run.t, "y": y[:, sub].tolist(), "u": run.u[:, sub].tolist(),
            "E": E.tolist(), "B": B.tolist(), "SE": SE.tolist(), "SB": SB.tolist(),
            "kstar_sha256": bracket_row_hashes(k), "near_ties": near_tie_list(k),
            "before_history_fraction": float((np.asarray(k) < 0).mean()),
            "sigma": run.diag()[:3].tolist(),
        }
        print(f"step {s}: t = {run.t:.6e} s, {time.time() - t0:.0f} s elapsed", flush=True)
    with open(OUT, "w") as f:
        json.dump(doc, f)
    print(f"wrote {OUT} in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
