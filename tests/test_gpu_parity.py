"""GPU (HIP, through the C ABI) against the CPU oracle, FP64 path.

k* must match bit for bit; fields within 1e-12 of the per-target sum of
magnitudes and of the rms field.  Inputs come from the seeded generators
(paper_2605_05543_amd.bunch) or from the oracle's own stepping."""
import numpy as np
import pytest

import oracle
from paper_2605_05543_amd import bunch
from parity import (FP64_TOL, MIXED_TOL, assert_fields, assert_kstar, assert_kstar_hashes, assert_mixed,
                    field_errors, load_c2_steps, load_c5_subset)

pytestmark = pytest.mark.gpu

Q, ME = -bunch.E_CHARGE, bunch.M_ELECTRON


def _ctx(n, depth, dt, guess=0, precision=0, **kw):
    from paper_2605_05543_amd._lib import Context

    return Context(n=n, depth=depth, q=Q, m=ME, dt=dt, guess=guess, precision=precision, **kw)


@pytest.fixture(scope="module")
def orc():
    return oracle.get()


@pytest.mark.parametrize("guess", [0, 2])
@pytest.mark.parametrize("n,depth,m", [(48, 64, 300), (61, 37, 129), (300, 128, 257), (40, 600, 70), (40, 1500, 70),
                                       (24, 2500, 70), (24, 4064, 70)])
def test_fields_at_wiggly(orc, n, depth, m, guess):
    """Curving sources (non-zero acceleration in history), external
    targets spanning several LDS tiles and ragged tails.  The depths cover
    every LDS layout: four, three and one source per double-buffered tile
    (D <= 512, D = 600, 1024 < D <= 2048) and one buffer sized to the
    history (D > 2048, up to the largest supported depth)."""
    print(f"case wiggly n={n} D={depth} m={m} guess={guess}", flush=True)
    dt = 1e-13
    T, w, v = bunch.wiggly_history(n, depth, dt, beta=0.9, accel_rel=0.1, seed=n + depth)
    rng = np.random.default_rng(m)
    x = 1.5e-3 * rng.standard_normal((3, m))
    u = np.zeros((3, n))
    E0, B0, k0, SE, SB = orc.fields(T, w, v, Q, T[-1], x, want_kstar=True, want_abs=True)
    with _ctx(n, depth, dt, guess=guess) as ctx:
        ctx.set_history(T, w, v, u)
        E, B, k = ctx.fields_at(T[-1], x, want_kstar=True)
    assert_kstar("wiggly", k, k0)
    assert_fields("wiggly", E, B, E0, B0, SE, SB)


@pytest.mark.parametrize("precision", [0, 1])
def test_unrolled_bisection_every_halving_count(orc, precision):
    """The fields launch (no bracket output) runs the bisection unrolled in a
    kernel per number of halvings, ceil(log2(D - 1)) = 1 ... 11 for the
    double-buffered depths; the bracket-output launch runs the halving loop.
    Both must give bit-identical fields, within the tolerance of the
    oracle's, at a depth of every halving count."""
    dt = 1e-13
    for depth in (3, 4, 6, 10, 18, 34, 66, 130, 258, 514, 1026, 2048):
        n, m = 24, 70
        print(f"case unrolled bisection D={depth} precision={precision}", flush=True)
        # sources and targets spread over a third of the history's light
        # distance: about a third of the pairs fall inside the history
        L = bunch.C_LIGHT * dt * (depth - 1)
        T, w, v = bunch.wiggly_history(n, depth, dt, beta=0.9, sigma=0.3 * L, accel_rel=0.1, seed=5 + depth)
        rng = np.random.default_rng(depth)
        x = w[-1][:, rng.integers(0, n, m)] + 0.3 * L * rng.standard_normal((3, m))
        u = np.zeros((3, n))
        E0, B0, k0, SE, SB = orc.fields(T, w, v, Q, T[-1], x, want_kstar=True, want_abs=True)
        with _ctx(n, depth, dt, precision=precision) as ctx:
            ctx.set_history(T, w, v, u)
            E1, B1 = ctx.fields_at(T[-1], x)
            E2, B2, k = ctx.fields_at(T[-1], x, want_kstar=True)
        assert (k0 > 0).sum() > m * n // 4 and k0.max() == depth - 1
        assert_kstar(f"D={depth}", k, k0)
        assert np.array_equal(E1, E2) and np.array_equal(B1, B2), f"D={depth}: unrolled and looped bisection differ"
        if precision == 0:
            assert_fields(f"D={depth}", E1, B1, E0, B0, SE, SB)
        else:
            assert_mixed(f"D={depth} (mixed)", E1, B1, E0, B0, SE, SB)


@pytest.mark.parametrize("guess", [0, 2])
def test_c1_initial_all_targets(orc, guess):
    wl = bunch.C1
    print(f"case C1 initial all targets guess={guess}", flush=True)
    r, u = bunch.gaussian_bunch(wl.bunch)
    n = wl.bunch.n
    T, w, v = orc.init_straight(r, u, wl.depth, wl.dt)
    E0, B0, k0, SE, SB = orc.fields(T, w, v, Q, T[-1], r, np.arange(n), want_kstar=True, want_abs=True)
    with _ctx(n, wl.depth, wl.dt, guess=guess) as ctx:
        ctx.init_bunch(r, u, 0.0)
        ctx.init_history_straight()
        Tg, wg, vg = ctx.history()
        assert np.array_equal(Tg, T) and np.array_equal(wg, w) and np.array_equal(vg, v)
        E, B, k = ctx.fields_at(0.0, r, np.arange(n), want_kstar=True)
        ctx.step(1)
        Es, Bs = ctx.fields()
    assert_kstar("C1 init", k, k0)
    assert_fields("C1 init fields_at", E, B, E0, B0, SE, SB)
    assert_fields("C1 init step", Es, Bs, E0, B0, SE, SB)


def test_c1_synchronised_steps(orc):
    """C1 for 200 steps in the oracle; at several steps the GPU is given the
    oracle's state, takes one step, and must reproduce the oracle's fields
    (1e-12), k* (exact) and next state."""
    wl = bunch.C1
    r, u = bunch.gaussian_bunch(wl.bunch)
    n = wl.bunch.n
    run = oracle.OracleRun(orc, r, u, D=wl.depth, dt=wl.dt, q=Q, mass=ME)
    check_at = {0, 1, 7, 50, 120, 199}
    with _ctx(n, wl.depth, wl.dt) as ctx:
        for step in range(wl.steps):
            if step in check_at:
                print(f"case C1 synchronised step {step}", flush=True)
                T, w, v, uu = run.T.copy(), run.w.copy(), run.v.copy(), run.u.copy()
                E0, B0, k0, SE, SB = orc.fields(T, w, v, Q, T[-1], w[-1], np.arange(n), want_kstar=True,
                                                want_abs=True)
                ctx.set_history(T, w, v, uu)
                _, _, k = ctx.fields_at(T[-1], w[-1], np.arange(n), want_kstar=True)
                ctx.step(1)
                Eg, Bg = ctx.fields()
                rg, ug, tg, _ = ctx.state()
                run.step(1)
                assert_kstar(f"C1 step {step}", k, k0)
                assert_fields(f"C1 step {step}", Eg, Bg, E0, B0, SE, SB)
                dy = np.max(np.abs(rg - run.y))
                du = np.max(np.abs(ug - run.u)) / np.max(np.abs(run.u))
                print(f"   next state: max|dy| {dy:.2e} m, max|du|/|u| {du:.2e}, t {tg} vs {run.t}", flush=True)
                assert dy < 1e-16 and du < 1e-15 and tg == run.t
            else:
                run.step(1)


def test_c1_free_running(orc):
    """Both sides run C1's 200 steps from the same initial bunch; the
    trajectories may only drift apart by rounding."""
    wl = bunch.C1
    print("case C1 free running 200 steps", flush=True)
    r, u = bunch.gaussian_bunch(wl.bunch)
    n = wl.bunch.n
    run = oracle.OracleRun(orc, r, u, D=wl.depth, dt=wl.dt, q=Q, mass=ME)
    run.step(wl.steps)
    with _ctx(n, wl.depth, wl.dt) as ctx:
        ctx.init_bunch(r, u, 0.0)
        ctx.init_history_straight()
        ctx.step(wl.steps)
        rg, ug, tg, sg = ctx.state()
        Eg, Bg = ctx.fields()
        diag = ctx.diag()
    sig = np.std(r, axis=1).mean()
    dy = np.max(np.abs(rg - run.y)) / sig
    du = np.max(np.abs(ug - run.u)) / np.max(np.abs(run.u))
    dE = np.max(np.linalg.norm(Eg - run.E, axis=0)) / np.sqrt(np.mean(np.sum(run.E**2, 0)))
    print(f"C1 200 steps: max|dy|/sigma {dy:.2e}, max|du|/|u| {du:.2e}, last-step field err/rms {dE:.2e}", flush=True)
    assert sg == wl.steps and tg == run.t
    assert dy < 1e-12 and du < 1e-13 and dE < 1e-10
    od = run.diag()
    for k in range(3):
        assert abs(diag["sigma"][k] / od[k] - 1) < 1e-9
    assert abs(diag["mean_kinetic"] / od[7] - 1) < 1e-12


def test_c2_subset_and_invariants(orc):
    """C2 size (N=8192, D=512): 64 seeded targets against the oracle at the
    initial state (the launch shape the step uses), then 1000 GPU steps with
    the history invariants checked at the end."""
    wl = bunch.C2
    print("case C2 subset", flush=True)
    r, u = bunch.gaussian_bunch(wl.bunch)
    n = wl.bunch.n
    sub = bunch.target_subset(n, 64, 102)
    T, w, v = orc.init_straight(r, u, wl.depth, wl.dt)
    E0, B0, k0, SE, SB = orc.fields(T, w, v, Q, T[-1], r[:, sub], sub, want_kstar=True, want_abs=True)
    with _ctx(n, wl.depth, wl.dt) as ctx:
        ctx.init_bunch(r, u, 0.0)
        ctx.init_history_straight()
        _, _, k = ctx.fields_at(0.0, r[:, sub], sub, want_kstar=True)
        ctx.step(1)
        Es, Bs = ctx.fields()
        assert_kstar("C2 subset", k, k0)
        assert_fields("C2 subset (step launch)", Es[:, sub], Bs[:, sub], E0, B0, SE, SB)
        print("case C2 1000 steps", flush=True)
        ctx.step(wl.steps - 1)
        Tg, wg, vg = ctx.history()
        rg, ug, tg, sg = ctx.state()
    assert sg == wl.steps
    seg = np.max(np.abs(wg[1:] - (wg[:-1] + vg[:-1] * np.diff(Tg)[:, None, None])))
    g = np.sqrt(1 + (ug**2).sum(0) / bunch.C_LIGHT**2)
    print(f"C2 after 1000 steps: segment invariant {seg:.2e} m, newest v vs u/gamma "
          f"{np.max(np.abs(vg[-1] - ug / g)):.2e}", flush=True)
    assert seg < 1e-17 and np.max(np.abs(vg[-1] - ug / g)) < 1e-6
    assert np.all(np.isfinite(wg))


def test_c2_free_run_against_the_oracles():
    """C2 (N=8192, D=512, 2 MeV): the GPU's free run from the seeded bunch
    against the oracle's own free run, stored at steps 1 and 10 for the 64
    seeded targets (tests/golden/c2_steps.json, written by an oracle-only
    script).  Step 1: positions to rounding, k* of the 64 targets exact
    (one hash per target row), fields within 1e-12.  Step 10: the
    divergence of positions and fields is stated, and bounded by 1e-12 of
    sigma and 1e-10 of the rms field."""
    wl = bunch.C2
    ref = load_c2_steps()
    r, u = bunch.gaussian_bunch(wl.bunch)
    n = wl.bunch.n
    sub = ref["targets"]
    done = 0
    with _ctx(n, wl.depth, wl.dt) as ctx:
        ctx.init_bunch(r, u, 0.0)
        ctx.init_history_straight()
        for s in sorted(ref["steps"]):
            print(f"case C2 free run, step {s}", flush=True)
            ctx.step(s - done)
            done = s
            rg, ug, t, _ = ctx.state()
            e = ref["steps"][s]
            assert t == e["t"]
            E, B, k = ctx.fields_at(t, rg[:, sub], sub, want_kstar=True)
            sig = float(np.mean(e["sigma"]))
            dy = float(np.max(np.abs(rg[:, sub] - e["y"]))) / sig
            du = float(np.max(np.abs(ug[:, sub] - e["u"]) / np.max(np.abs(e["u"]))))
            e1, e2 = field_errors(E, e["E"], e["SE"])
            print(f"   step {s}: max|dy|/sigma {dy:.2e}, max|du|/|u| {du:.2e}, fields err/S {e1:.2e}, "
                  f"err/rms {e2:.2e}", flush=True)
            if s == 1:
                assert dy < 1e-15 and du < 1e-15
                assert_kstar_hashes(f"C2 step {s}", k, e["kstar_sha256"], e["near_ties"])
                assert_fields(f"C2 step {s}", E, B, e["E"], e["B"], e["SE"], e["SB"])
            else:
                assert dy < 1e-12 and du < 1e-12 and e2 < 1e-10


def test_c3_full_size_sampled(orc):
    """C3 size (N=65536, D=512, dipole at 3 R_E): the step's fields at 1024
    seeded targets against the oracle, and k* of those targets (6.7e7
    pairs)."""
    wl = bunch.C3
    print("case C3 full size sampled, 1024 targets", flush=True)
    r, u = bunch.gaussian_bunch(wl.bunch)
    n = wl.bunch.n
    sub = bunch.target_subset(n, 1024, 103)
    T, w, v = orc.init_straight(r, u, wl.depth, wl.dt)
    E0, B0, k0, SE, SB = orc.fields(T, w, v, Q, T[-1], r[:, sub], sub, want_kstar=True, want_abs=True)
    with _ctx(n, wl.depth, wl.dt, ext_field=1, dipole_b0=wl.dipole_b0, dipole_re=wl.dipole_re) as ctx:
        ctx.init_bunch(r, u, 0.0)
        ctx.init_history_straight()
        _, _, k = ctx.fields_at(0.0, r[:, sub], sub, want_kstar=True)
        ctx.step(1)
        Es, Bs = ctx.fields()
    assert_kstar("C3 subset", k, k0)
    assert_fields("C3 subset (step launch)", Es[:, sub], Bs[:, sub], E0, B0, SE, SB)


def test_errors_are_reported(orc):
    """Host-checked and device-latched errors come back as statuses."""
    from paper_2605_05543_amd._lib import EMPP_EINVAL, EMPP_ENUMERIC, EMPP_ESTATE, EmppError

    print("case error paths", flush=True)
    T, w, v = bunch.wiggly_history(8, 16, 1e-13, seed=3)
    u = np.zeros((3, 8))
    with _ctx(8, 16, 1e-13) as ctx:
        with pytest.raises(EmppError) as ei:
            ctx.step(1)
        assert ei.value.status == EMPP_ESTATE
        vbad = v.copy()
        vbad[3, 2, 5] = 1.01 * bunch.C_LIGHT
        with pytest.raises(EmppError) as ei:
            ctx.set_history(T, w, vbad, u)
        assert ei.value.status == EMPP_EINVAL
        ctx.set_history(T, w, v, u)
        with pytest.raises(EmppError) as ei:
            ctx.fields_at(T[-1] + 1e-15, np.zeros((3, 1)))
        assert ei.value.status == EMPP_EINVAL
        # a target sitting exactly on source 4's newest position: eta = 0
        x = w[-1][:, 4:5].copy()
        with pytest.raises(EmppError) as ei:
            ctx.fields_at(T[-1], x)
        assert ei.value.status == EMPP_ENUMERIC and "source 4" in str(ei.value)
        # the same target with source 4 excluded is fine
        E, B = ctx.fields_at(T[-1], x, np.array([4]))
        assert np.all(np.isfinite(E))


def test_step_error_reaches_every_getter():
    """Two particles on one position: the step's pair kernels latch the
    coincident pair; the next synchronising call reports ENUMERIC naming
    both particles, whichever it is (state, diag, fields, history, fields_at
    after a step, handoff), and the error is cleared once reported."""
    from paper_2605_05543_amd._lib import EMPP_ENUMERIC, EmppError

    print("case step error reaches the getters", flush=True)
    n, depth, dt = 16, 8, 1e-13
    r, u = bunch.gaussian_bunch(bunch.BunchSpec(n, (1e-3, 1e-3, 1e-3), 1.0, seed=21))
    r[:, 7] = r[:, 3]
    getters = {"state": lambda c: c.state(), "diag": lambda c: c.diag(), "fields": lambda c: c.fields(),
               "history": lambda c: c.history(), "fields_at": lambda c: c.fields_at(c.state_t, r[:, :1] + 1e-3),
               "handoff": lambda c: c.handoff()}
    for name, call in getters.items():
        with _ctx(n, depth, dt) as ctx:
            ctx.init_bunch(r, u, 0.0)
            ctx.init_history_straight()
            ctx.step(1)
            ctx.state_t = dt
            with pytest.raises(EmppError) as ei:
                call(ctx)
            print(f"   {name}: {ei.value}", flush=True)
            assert ei.value.status == EMPP_ENUMERIC
            assert "source 3" in str(ei.value) or "source 7" in str(ei.value)
            ctx.sync()  # reported once, then cleared


@pytest.mark.parametrize("n,depth,m", [(48, 64, 300), (300, 128, 257)])
def test_midpoint_ablation_matches_oracle(orc, n, depth, m):
    """The midpoint reconstruction of Eq. (mid) (an accuracy ablation) on
    accelerating sources: same k*, fields to 1e-12, as the oracle in the same
    mode."""
    print(f"case midpoint ablation n={n} depth={depth} m={m}", flush=True)
    dt = 1e-13
    T, w, v = bunch.wiggly_history(n, depth, dt, seed=n + 5)
    rng = np.random.default_rng(m)
    x = 2e-3 * rng.standard_normal((3, m))
    try:
        orc.set_reconstruction(1)
        E0, B0, k0, SE, SB = orc.fields(T, w, v, Q, T[-1], x, None, want_kstar=True, want_abs=True)
    finally:
        orc.set_reconstruction(0)
    El, Bl = orc.fields(T, w, v, Q, T[-1], x, None)
    g = 1 / np.sqrt(1 - (v[-1] ** 2).sum(0) / bunch.C_LIGHT**2)
    with _ctx(n, depth, dt, recon=1) as ctx:
        ctx.set_history(T, w, v, v[-1] * g)
        E, B, k = ctx.fields_at(T[-1], x, want_kstar=True)
    assert_kstar("midpoint", k, k0)
    assert_fields("midpoint", E, B, E0, B0, SE, SB)
    diff = np.max(np.linalg.norm(E0 - El, axis=0)) / np.sqrt(np.mean((El**2).sum(0)))
    print(f"   midpoint vs linear reconstruction: max |dE| / rms E = {diff:.2e}", flush=True)
    assert diff > 1e-9  # the ablation changes the fields


def test_c5_full_size_subset():
    """C5 size (N=262144, D=1024, dipole at 3 R_E, 17 GB history ring): the
    step's fields at 1024 seeded targets against the stored oracle values,
    and a SHA-256 of each target's k* row (2.7e8 pairs)."""
    wl = bunch.C5
    print("case C5 full size, 1024 stored targets", flush=True)
    ref = load_c5_subset()
    r, u = bunch.gaussian_bunch(wl.bunch)
    n = wl.bunch.n
    sub = ref["targets"]
    with _ctx(n, wl.depth, wl.dt, ext_field=1, dipole_b0=wl.dipole_b0, dipole_re=wl.dipole_re) as ctx:
        ctx.init_bunch(r, u, 0.0)
        ctx.init_history_straight()
        _, _, k = ctx.fields_at(0.0, r[:, sub], sub, want_kstar=True)
        ctx.step(1)
        Es, Bs = ctx.fields()
    print(f"   before-history fraction {float((k < 0).mean()):.3f} (oracle {ref['before_history_fraction']:.3f})",
          flush=True)
    assert_kstar_hashes("C5 subset", k, ref["kstar_sha256"], ref["near_ties"])
    assert_fields("C5 subset (step launch)", Es[:, sub], Bs[:, sub], ref["E"], ref["B"], ref["SE"], ref["SB"])


def test_c3_size_accelerating_history(orc):
    """C3 size (N=65536, D=512) on curving histories (acceleration in every
    segment, pairs in and before the history): the step's fields at 128
    seeded targets and their k* against the oracle."""
    print("case C3 size, accelerating history", flush=True)
    n, depth, dt = 65536, 512, 1e-13
    T, w, v = bunch.wiggly_history(n, depth, dt, beta=0.9, sigma=1e-3, accel_rel=0.05, seed=33)
    g = 1 / np.sqrt(1 - (v[-1] ** 2).sum(0) / bunch.C_LIGHT**2)
    sub = bunch.target_subset(n, 128, 104)
    E0, B0, k0, SE, SB = orc.fields(T, w, v, Q, T[-1], w[-1][:, sub], sub, want_kstar=True, want_abs=True)
    with _ctx(n, depth, dt) as ctx:
        ctx.set_history(T, w, v, v[-1] * g)
        _, _, k = ctx.fields_at(T[-1], w[-1][:, sub], sub, want_kstar=True)
        ctx.step(1)
        Es, Bs = ctx.fields()
    print(f"   before-history fraction {float((k0 < 0).mean()):.3f}", flush=True)
    assert_kstar("C3 accelerating", k, k0)
    assert_fields("C3 accelerating (step launch)", Es[:, sub], Bs[:, sub], E0, B0, SE, SB)


@pytest.mark.parametrize("splits", [48, 7, 1])
def test_source_chunks_of_any_size(orc, splits):
    """Source chunks from one source each (a chunk shorter than a staged
    tile) to one chunk of all sources: k* and fields against the oracle."""
    print(f"case source chunks: {splits} chunks of 48 sources", flush=True)
    n, depth, m, dt = 48, 64, 100, 1e-13
    T, w, v = bunch.wiggly_history(n, depth, dt, beta=0.9, accel_rel=0.1, seed=77)
    rng = np.random.default_rng(78)
    x = 1.5e-3 * rng.standard_normal((3, m))
    E0, B0, k0, SE, SB = orc.fields(T, w, v, Q, T[-1], x, want_kstar=True, want_abs=True)
    with _ctx(n, depth, dt, source_splits=splits) as ctx:
        ctx.set_history(T, w, v, np.zeros((3, n)))
        E, B, k = ctx.fields_at(T[-1], x, want_kstar=True)
    assert_kstar("chunks", k, k0)
    assert_fields("chunks", E, B, E0, B0, SE, SB)


@pytest.mark.parametrize("precision", [0, 1])
def test_smallest_and_empty_inputs(orc, precision):
    """The smallest sizes the method allows: two or three sources, a history
    of two or three slots (one or two segments), one target, more targets
    than sources (chunked), and no targets at all.  Targets sit microns
    from source 0, so its pairs fall inside the short history while the
    millimetre-distant sources' pairs fall before it."""
    for n, depth, m in ((2, 2, 5), (2, 3, 3), (3, 2, 1)):
        print(f"case smallest inputs n={n} D={depth} m={m} precision={precision}", flush=True)
        dt = 1e-13
        T, w, v = bunch.wiggly_history(n, depth, dt, beta=0.9, accel_rel=0.1, seed=11 + n + depth)
        rng = np.random.default_rng(12 + m)
        x = w[-1][:, :1] + 4e-6 * rng.standard_normal((3, m))
        g = 1 / np.sqrt(1 - (v[-1] ** 2).sum(0) / bunch.C_LIGHT**2)
        E0, B0, k0, SE, SB = orc.fields(T, w, v, Q, T[-1], x, want_kstar=True, want_abs=True)
        assert (k0 > 0).any() and (k0 < 0).any()
        with _ctx(n, depth, dt, precision=precision) as ctx:
            ctx.set_history(T, w, v, v[-1] * g)
            E, B, k = ctx.fields_at(T[-1], x, want_kstar=True)
            Ee, Be = ctx.fields_at(T[-1], np.zeros((3, 0)))
        assert Ee.shape == (3, 0) and Be.shape == (3, 0)
        assert_kstar("smallest", k, k0)
        if precision == 0:
            assert_fields("smallest", E, B, E0, B0, SE, SB)
        else:
            assert_mixed("smallest (mixed)", E, B, E0, B0, SE, SB)


def test_exact_tie_goes_older(orc):
    """A sample exactly on the target's past light cone (light distance
    2^-12 m, whose square is a double) belongs to the older side: k* = 9
    for a tie 8 slots back, on the GPU as in the oracle, in both precisions
    and with the bisection and the straight-line guess."""
    from pins import _exact_light_delay

    print("case exact tie", flush=True)
    ns, dt = 16, 1e-13
    r0 = np.array([[0.0, 1e-3], [0.0, 0.0], [0.0, 0.0]])
    T, w, v = bunch.uniform_history(ns, dt, r0, np.zeros((3, 2)))
    t = T[-1]
    L0 = 2.0**-12
    s = ns - 1 - 8
    T[s] = t - _exact_light_delay(L0)
    assert bunch.C_LIGHT * (t - T[s]) == L0
    x = np.array([[L0], [0.0], [0.0]])
    E0, B0, k0, SE, SB = orc.fields(T, w, v, Q, t, x, want_kstar=True, want_abs=True)
    assert k0[0, 0] == 9
    for precision in (0, 1):
        for guess in (0, 2):
            with _ctx(2, ns, dt, guess=guess, precision=precision) as ctx:
                ctx.set_history(T, w, v, np.zeros((3, 2)))
                E, B, k = ctx.fields_at(t, x, want_kstar=True)
            assert_kstar(f"tie precision={precision} guess={guess}", k, k0)
            # sources at rest on the target's axis: E along it, B exactly 0
            e1, e2 = field_errors(E, E0, SE)
            print(f"   E err/S {e1:.2e}, err/|E| {e2:.2e}; max |B| {np.abs(B).max():.1e}", flush=True)
            assert e2 <= (FP64_TOL if precision == 0 else MIXED_TOL)
            assert np.all(B == 0) and np.all(B0 == 0)
