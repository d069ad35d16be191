"""Mixed-precision path against the FP64 oracle.  Every light-cone sign
test stays FP64 (the bracket search is the FP64 path's); the root, the
reconstruction and the LW terms run in FP32 around FP64 quadratic
coefficients, with two-sum accumulation, and an FP32 root that fails its
residual test is recomputed in FP64 (a rescue).

k* must equal the oracle's (either bracket only on a flagged near tie).
Fields: max_i |dE_i| / rms_k |E_k| <= 1e-5 (same for B); the spread of
per-target relative errors is printed."""
import numpy as np
import pytest

import oracle
from paper_2605_05543_amd import bunch
from parity import assert_kstar, assert_mixed, assert_kstar_hashes, load_c5_subset

pytestmark = pytest.mark.gpu

Q, ME = -bunch.E_CHARGE, bunch.M_ELECTRON


def _ctx(n, depth, dt, guess=0, **kw):
    from paper_2605_05543_amd._lib import EMPP_MIXED, Context

    return Context(n=n, depth=depth, q=Q, m=ME, dt=dt, guess=guess, precision=EMPP_MIXED, **kw)


@pytest.fixture(scope="module")
def orc():
    return oracle.get()


@pytest.mark.parametrize("guess", [0, 2])
@pytest.mark.parametrize("n,depth,m", [(48, 64, 300), (300, 128, 257), (24, 2500, 70)])
def test_mixed_fields_at_wiggly(orc, n, depth, m, guess):
    print(f"case mixed wiggly n={n} D={depth} m={m} guess={guess}", flush=True)
    dt = 1e-13
    T, w, v = bunch.wiggly_history(n, depth, dt, beta=0.9, accel_rel=0.1, seed=n + depth)
    rng = np.random.default_rng(m)
    x = 1.5e-3 * rng.standard_normal((3, m))
    E0, B0, k0, SE, SB = orc.fields(T, w, v, Q, T[-1], x, want_kstar=True, want_abs=True)
    with _ctx(n, depth, dt, guess=guess) as ctx:
        ctx.set_history(T, w, v, np.zeros((3, n)))
        ctx.set_counting(True)
        E, B, k = ctx.fields_at(T[-1], x, want_kstar=True)
        cnt = ctx.counters()
    print(f"   rescues {cnt['rescues']} of {cnt['pairs']} pairs", flush=True)
    assert_kstar("mixed wiggly", k, k0)
    assert_mixed("mixed wiggly", E, B, E0, B0, SE, SB)


def test_mixed_c1_initial(orc):
    wl = bunch.C1
    print("case mixed C1 initial", flush=True)
    r, u = bunch.gaussian_bunch(wl.bunch)
    n = wl.bunch.n
    T, w, v = orc.init_straight(r, u, wl.depth, wl.dt)
    E0, B0, k0, SE, SB = orc.fields(T, w, v, Q, T[-1], r, np.arange(n), want_kstar=True, want_abs=True)
    with _ctx(n, wl.depth, wl.dt) as ctx:
        ctx.init_bunch(r, u, 0.0)
        ctx.init_history_straight()
        _, _, k = ctx.fields_at(0.0, r, np.arange(n), want_kstar=True)
        ctx.step(1)
        Es, Bs = ctx.fields()
    assert_kstar("mixed C1", k, k0)
    assert_mixed("mixed C1 step", Es, Bs, E0, B0, SE, SB)


@pytest.mark.parametrize("guess", [0, 2])
def test_mixed_c3_full_size_sampled(orc, guess):
    """The headline workload (N=65536, D=512, dipole at 3 R_E) in the launch
    shape the bench times: the step's fields at 128 seeded targets."""
    wl = bunch.C3
    print(f"case mixed C3 sampled guess={guess}", flush=True)
    r, u = bunch.gaussian_bunch(wl.bunch)
    n = wl.bunch.n
    sub = bunch.target_subset(n, 128, 103)
    T, w, v = orc.init_straight(r, u, wl.depth, wl.dt)
    E0, B0, k0, SE, SB = orc.fields(T, w, v, Q, T[-1], r[:, sub], sub, want_kstar=True, want_abs=True)
    with _ctx(n, wl.depth, wl.dt, guess=guess, ext_field=1, dipole_b0=wl.dipole_b0, dipole_re=wl.dipole_re) as ctx:
        ctx.init_bunch(r, u, 0.0)
        ctx.init_history_straight()
        _, _, k = ctx.fields_at(0.0, r[:, sub], sub, want_kstar=True)
        ctx.set_counting(True)
        ctx.step(1)
        cnt = ctx.counters()
        Es, Bs = ctx.fields()
    print(f"   rescues per pair {cnt['rescues'] / cnt['pairs']:.2e}, probes per pair {cnt['probes'] / cnt['pairs']:.2f}",
          flush=True)
    assert_kstar("mixed C3", k, k0)
    assert_mixed("mixed C3 (step launch)", Es[:, sub], Bs[:, sub], E0, B0, SE, SB)


def test_mixed_c5_full_size_subset():
    """C5 size (N=262144, D=1024, 5 MeV: gamma = 10.8, so forward pairs have
    1 - eta_hat.beta down to 0.004): the mixed step's fields at 1024 seeded
    targets against the stored oracle values, and the per-target hashes of k*."""
    wl = bunch.C5
    print("case mixed C5, 1024 stored targets", flush=True)
    ref = load_c5_subset()
    r, u = bunch.gaussian_bunch(wl.bunch)
    n = wl.bunch.n
    sub = ref["targets"]
    with _ctx(n, wl.depth, wl.dt, guess=2, ext_field=1, dipole_b0=wl.dipole_b0, dipole_re=wl.dipole_re) as ctx:
        ctx.init_bunch(r, u, 0.0)
        ctx.init_history_straight()
        _, _, k = ctx.fields_at(0.0, r[:, sub], sub, want_kstar=True)
        ctx.step(1)
        Es, Bs = ctx.fields()
    assert_kstar_hashes("C5 subset", k, ref["kstar_sha256"], ref["near_ties"])
    assert_mixed("mixed C5 (step launch)", Es[:, sub], Bs[:, sub], ref["E"], ref["B"], ref["SE"], ref["SB"])


def test_mixed_c1_free_running_position_error(orc):
    """C1's 200 steps in mixed precision against the FP64 oracle: the
    position error is stated as a number (max |dy| / sigma)."""
    wl = bunch.C1
    print("case mixed C1 200 steps", flush=True)
    r, u = bunch.gaussian_bunch(wl.bunch)
    n = wl.bunch.n
    run = oracle.OracleRun(orc, r, u, D=wl.depth, dt=wl.dt, q=Q, mass=ME)
    run.step(wl.steps)
    with _ctx(n, wl.depth, wl.dt) as ctx:
        ctx.init_bunch(r, u, 0.0)
        ctx.init_history_straight()
        ctx.step(wl.steps)
        rg, ug, _, _ = ctx.state()
    sig = np.std(r, axis=1).mean()
    dy = np.max(np.abs(rg - run.y)) / sig
    du = np.max(np.abs(ug - run.u)) / np.max(np.abs(run.u))
    print(f"mixed C1 200 steps: max|dy|/sigma {dy:.2e}, max|du|/|u| {du:.2e}", flush=True)
    assert dy < 1e-9 and du < 1e-9


def test_mixed_c3_size_accelerating_history(orc):
    """Mixed precision at C3 size on curving histories (every segment
    accelerates): k* exact, fields within 1e-5 of the rms field."""
    print("case mixed C3 size, accelerating history", flush=True)
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
    assert_kstar("mixed C3 accelerating", k, k0)
    assert_mixed("mixed C3 accelerating (step launch)", Es[:, sub], Bs[:, sub], E0, B0, SE, SB)
