"""Warm-started bracket search (guess mode PREVIOUS) through the C ABI.

The search starts from each pair's bracket of the previous step and must
reach exactly the bracket the paper's bisection reaches (Sec. 2.2): the
whole state and the fields after many steps are compared bit for bit with
a bisection run (which the parity tests hold against the oracle), on a
field-free bunch where brackets hardly move and on a bunch gyrating in a
strong field where they move every step."""
import numpy as np
import pytest

from paper_2605_05543_amd import bunch

pytestmark = pytest.mark.gpu

Q, ME = -bunch.E_CHARGE, bunch.M_ELECTRON


def _run(r, u, depth, dt, steps, guess, count_at=None, **kw):
    from paper_2605_05543_amd._lib import Context

    n = r.shape[1]
    counts = None
    with Context(n=n, depth=depth, q=Q, m=ME, dt=dt, guess=guess, **kw) as ctx:
        ctx.init_bunch(r, u, 0.0)
        ctx.init_history_straight()
        for s in range(steps):
            if s == count_at:
                ctx.set_counting(True)
                ctx.step(1)
                counts = ctx.counters()
                ctx.set_counting(False)
            else:
                ctx.step(1)
        T, w, v = ctx.history()
        rr, uu, t, st = ctx.state()
        E, B = ctx.fields()
    return (T, w, v, rr, uu, E, B), counts


def _same(a, b):
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_warm_start_c1_bit_identical():
    wl = bunch.C1
    print("case warm start C1 60 steps", flush=True)
    r, u = bunch.gaussian_bunch(wl.bunch)
    ref, _ = _run(r, u, wl.depth, wl.dt, 60, guess=0)
    got, cnt = _run(r, u, wl.depth, wl.dt, 60, guess=4, count_at=30)
    _same(ref, got)
    ppp = cnt["probes"] / cnt["pairs"]
    print(f"   warm step: {ppp:.3f} sign tests per pair, {cnt['fallbacks']} gallops", flush=True)
    assert ppp < 2.05


def test_warm_start_strong_field_bit_identical():
    """Electrons at 1 MeV crossing a 10 T field (the dipole's equatorial
    value at 1 m): gyration radius about 0.5 mm, 0.06 rad per step, so
    brackets of close pairs move between steps and the gallop runs."""
    n, depth, dt = 256, 128, 1e-13
    print("case warm start strong field 40 steps", flush=True)
    rng = np.random.default_rng(11)
    r = 1e-3 * rng.standard_normal((3, n))
    r[0] += 1.0
    g = bunch.gamma_of_kinetic(1.0 * bunch.MEV)
    umag = bunch.C_LIGHT * np.sqrt(g * g - 1.0)
    u = np.zeros((3, n))
    u[1] = umag  # across the equatorial field (along -z there)
    kw = dict(ext_field=1, dipole_b0=10.0, dipole_re=1.0)
    ref, _ = _run(r, u, depth, dt, 40, guess=0, **kw)
    got, cnt = _run(r, u, depth, dt, 40, guess=4, count_at=25, **kw)
    _same(ref, got)
    ppp = cnt["probes"] / cnt["pairs"]
    print(f"   warm step: {ppp:.3f} sign tests per pair, {cnt['fallbacks']} fallbacks", flush=True)
    assert ppp > 2.0  # brackets moved: the gallop from the old bracket ran


def test_warm_start_needs_its_cache():
    from paper_2605_05543_amd._lib import EMPP_EUNSUPPORTED, Context, EmppError

    print("case warm start mode switch", flush=True)
    with Context(n=8, depth=16, q=Q, m=ME, dt=1e-13, guess=0) as ctx:
        with pytest.raises(EmppError) as ei:
            ctx.set_mode(0, 4)
        assert ei.value.status == EMPP_EUNSUPPORTED
    with Context(n=8, depth=16, q=Q, m=ME, dt=1e-13, guess=4) as ctx:
        ctx.set_mode(0, 0)
        ctx.set_mode(0, 4)
