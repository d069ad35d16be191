"""Adaptive step of Sec. 2.4 through the C ABI: the step the GPU takes
(from the eta_min / v_max reductions fused into the pair pass) against the
oracle's scan of the same history, and a run of adaptive steps against the
oracle's adaptive stepper."""
import numpy as np
import pytest

import oracle
from paper_2605_05543_amd import bunch

pytestmark = pytest.mark.gpu

Q, ME, C = -bunch.E_CHARGE, bunch.M_ELECTRON, bunch.C_LIGHT


@pytest.fixture(scope="module")
def orc():
    return oracle.get()


def _ctx(n, depth, dt, **kw):
    from paper_2605_05543_amd._lib import Context

    return Context(n=n, depth=depth, q=Q, m=ME, dt=dt, adaptive=True, **kw)


@pytest.mark.parametrize("guess", [0, 2, 4])
@pytest.mark.parametrize("allow_q", [0.0, 0.3])
def test_adaptive_step_matches_oracle_scan(orc, guess, allow_q):
    """Accelerating sources (in and before the history): the first step's
    dt equals c_dt eta_min / v_max of the oracle's scan to 1e-13."""
    print(f"case adaptive scan guess={guess} allow quantile={allow_q}", flush=True)
    n, depth, dt = 300, 128, 1e-13
    T, w, v = bunch.wiggly_history(n, depth, dt, beta=0.9, accel_rel=0.1, seed=21)
    g = 1 / np.sqrt(1 - (v[-1] ** 2).sum(0) / C**2)
    u = v[-1] * g
    pos = w[-1]
    d = np.linalg.norm(pos[:, :, None] - pos[:, None, :], axis=0)
    allow = float(np.quantile(d[d > 0], allow_q)) if allow_q > 0 else 0.0
    em, vm = orc.adaptive_scan(T, w, v, T[-1], pos, np.arange(n), v[-1], allow)
    want = 0.05 * em / vm
    with _ctx(n, depth, dt, guess=guess, dt_min=1e-30, dt_max=1.0, eta_allow=allow) as ctx:
        ctx.set_history(T, w, v, u)
        ctx.step(1)
        got = ctx.diag()["dt_last"]
        t1 = ctx.state()[2]
    print(f"   eta_min {em:.6e} m, v_max {vm:.6e} m/s: dt {got:.6e} vs {want:.6e} (rel {abs(got / want - 1):.1e})",
          flush=True)
    assert abs(got / want - 1) < 1e-13
    assert t1 == T[-1] + got


def test_adaptive_run_matches_oracle(orc):
    """A wide-angle bunch (the rule is live, between the clamps) for 25
    adaptive steps on both sides from the same initial state: the step
    sequences agree to 1e-12 and the states to rounding."""
    print("case adaptive run 25 steps", flush=True)
    spec = bunch.BunchSpec(96, (1e-3, 1e-3, 1e-3), 1.0, angle_spread=1.0, seed=22)
    r, u = bunch.gaussian_bunch(spec)
    D, dt = 32, 1e-13
    T0, w0, v0 = orc.init_straight(r, u, D, dt)
    To, wo, vo, uo, dto = orc.step_adaptive(T0, w0, v0, u, 25, q=Q, mass=ME, c_dt=0.05, dt_min=1e-16, dt_max=1e-12)
    dtg = []
    with _ctx(96, D, dt, dt_min=1e-16, dt_max=1e-12) as ctx:
        ctx.init_bunch(r, u, 0.0)
        ctx.init_history_straight()
        for _ in range(25):
            ctx.step(1)
            dtg.append(ctx.diag()["dt_last"])
        rg, ug, tg, _ = ctx.state()
        Tg, wg, vg = ctx.history()
    dtg = np.array(dtg)
    rel = np.max(np.abs(dtg / dto - 1))
    dy = np.max(np.abs(rg - wo[-1])) / 1e-3
    du = np.max(np.abs(ug - uo)) / np.max(np.abs(uo))
    print(f"   steps {dto[:3]} ... {dto[-1]:.3e}; GPU vs oracle: dt {rel:.1e}, max|dy|/sigma {dy:.1e}, "
          f"max|du|/|u| {du:.1e}, t {tg:.6e} vs {To[-1]:.6e}", flush=True)
    assert np.all(dto < 1e-12) and np.all(dto > 1e-16)
    assert rel < 1e-12 and dy < 1e-12 and du < 1e-12 and abs(tg / To[-1] - 1) < 1e-12
    assert np.allclose(Tg, To, rtol=1e-12, atol=0)
    seg = np.max(np.abs(wg[1:] - (wg[:-1] + vg[:-1] * np.diff(Tg)[:, None, None])))
    assert seg < 1e-17


def test_adaptive_rejected_where_unsupported():
    from paper_2605_05543_amd._lib import EMPP_EINVAL, EMPP_EUNSUPPORTED, EmppError

    print("case adaptive options", flush=True)
    for kw, status in ((dict(precision=1), EMPP_EUNSUPPORTED), (dict(guess=1), EMPP_EUNSUPPORTED),
                       (dict(dt_min=0.0), EMPP_EINVAL), (dict(c_dt=-1.0), EMPP_EINVAL)):
        with pytest.raises(EmppError) as ei:
            _ctx(8, 8, 1e-13, **kw)
        assert ei.value.status == status
