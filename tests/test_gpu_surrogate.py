"""The surrogate network on the GPU (BF16 matrix-core kernels) against the
FP64 oracle of oracle/mlp.py, and the guarantee that a guess never changes
a result.

Tolerances: features 1e-6 (float32 rounding of FP64 quantities); forward
and gradient 1e-2 relative (BF16 activations on the GPU, FP64 activations
in the oracle; the figure reached is printed); Adam 1e-6."""
import numpy as np
import pytest

import oracle
from oracle import mlp as omlp
from paper_2605_05543_amd import bunch

pytestmark = pytest.mark.gpu

Q, ME, C = -bunch.E_CHARGE, bunch.M_ELECTRON, bunch.C_LIGHT


def _ctx(n, depth, dt, guess=0, precision=0):
    from paper_2605_05543_amd._lib import Context

    return Context(n=n, depth=depth, q=Q, m=ME, dt=dt, guess=guess, precision=precision)


@pytest.fixture(scope="module")
def orc():
    return oracle.get()


def test_samples_match_oracle(orc):
    """Features and exact normalised delays of given pairs."""
    print("case surrogate samples", flush=True)
    n, D, dt = 48, 64, 1e-13
    T, w, v = bunch.wiggly_history(n, D, dt, beta=0.9, accel_rel=0.1, seed=5)
    sig = 1e-3
    rng = np.random.default_rng(6)
    tgt = rng.integers(0, n, 500)
    src = (tgt + rng.integers(1, n, 500)) % n
    with _ctx(n, D, dt) as ctx:
        ctx.set_history(T, w, v, np.zeros((3, n)))
        ctx.surrogate_set(bunch.surrogate_init(1), sig)
        X, y = ctx.surrogate_samples(500, tgt=tgt, src=src)
    Xo = omlp.features(w[-1][:, tgt], w[-1][:, src], v[-1][:, src], w[-5][:, src], T[-1], T[-5], T[-1], dt, sig)
    ret = orc.retarded(T, w, v, T[-1], w[-1], np.arange(n))
    tr = ret["tr"][tgt, src]
    yo = np.log(C * (T[-1] - tr) / omlp.straight_line_lookback(w[-1][:, tgt], w[-1][:, src], v[-1][:, src]))
    ex = np.max(np.abs(X - Xo) / np.maximum(np.abs(Xo), 1.0))
    ey = np.max(np.abs(y - yo))
    print(f"   features max err {ex:.2e}, log-delay max err {ey:.2e}, delay / straight-line delay "
          f"{np.exp(yo).min():.4f}..{np.exp(yo).max():.4f}", flush=True)
    assert ex < 1e-6 and ey < 1e-6


def test_forward_and_gradient_match_oracle():
    print("case surrogate forward/backward", flush=True)
    rng = np.random.default_rng(7)
    P = bunch.surrogate_init(2)
    X = rng.standard_normal((1000, 10)).astype(np.float32)
    X[:, 3:9] *= 0.5
    y = rng.standard_normal(1000).astype(np.float32)
    with _ctx(8, 8, 1e-13) as ctx:
        ctx.surrogate_set(P, 1e-3)
        z = ctx.surrogate_forward(X)
        loss, g = ctx.surrogate_loss_grad(X, y)
    zo, _ = omlp.forward(P.astype(np.float64), X.astype(np.float64))
    lo, go = omlp.loss_and_grad(P.astype(np.float64), X.astype(np.float64), y.astype(np.float64))
    ez = np.max(np.abs(z - zo)) / np.max(np.abs(zo))
    el = abs(loss - lo) / lo
    eg = np.linalg.norm(g - go) / np.linalg.norm(go)
    blocks = {name: np.linalg.norm(g[o:o + k] - go[o:o + k]) / np.linalg.norm(go[o:o + k])
              for name, o, k in (("W1", 0, 1280), ("b1", 1280, 128), ("W2", 1408, 16384), ("b2", 17792, 128),
                                 ("W3", 17920, 128), ("b3", 18048, 1))}
    print(f"   forward max rel err {ez:.2e}; loss rel err {el:.2e}; gradient rel L2 err {eg:.2e}; "
          + ", ".join(f"{k} {v:.1e}" for k, v in blocks.items()), flush=True)
    assert ez < 1e-2 and el < 1e-2 and eg < 1e-2
    assert all(v < 3e-2 for v in blocks.values())


def test_adam_step_matches_oracle():
    print("case surrogate adam", flush=True)
    rng = np.random.default_rng(8)
    P = bunch.surrogate_init(3)
    X = rng.standard_normal((256, 10)).astype(np.float32)
    y = rng.standard_normal(256).astype(np.float32)
    import torch

    with _ctx(8, 8, 1e-13) as ctx:
        ctx.surrogate_set(P, 1e-3)
        _, g = ctx.surrogate_loss_grad(X, y)
        Xt = torch.tensor(X, device="cuda")
        yt = torch.tensor(y, device="cuda")
        ctx.surrogate_train_torch(Xt, yt, steps=1, batch=256, lr=1e-3, lr_final=1e-3)
        P1 = ctx.surrogate_get()
    Po, _, _ = omlp.adam_step(P.astype(np.float64), 0.0, 0.0, g.astype(np.float64), 1, 1e-3)
    err = np.max(np.abs(P1 - Po))
    print(f"   adam max abs err {err:.2e}", flush=True)
    assert err < 1e-6


def test_training_reduces_loss():
    """Training pairs drawn from a C1 bunch's straight history; the loss of
    the log-delay falls by more than 10x."""
    print("case surrogate training", flush=True)
    wl = bunch.C1
    r, u = bunch.gaussian_bunch(wl.bunch)
    with _ctx(wl.bunch.n, wl.depth, wl.dt) as ctx:
        ctx.init_bunch(r, u, 0.0)
        ctx.init_history_straight()
        ctx.surrogate_set(bunch.surrogate_init(4), bunch.sigma_ref_of(r))
        X, y = ctx.surrogate_samples_torch(1 << 16, seed=11)
        rep = ctx.surrogate_train_torch(X, y, steps=600, batch=1024, lr=3e-3, lr_final=1e-4)
    print(f"   loss {rep['loss_first']:.3e} -> {rep['loss_last']:.3e} in {rep['steps']} steps, "
          f"{rep['seconds']:.2f} s", flush=True)
    assert rep["loss_last"] < 0.1 * rep["loss_first"]


def test_training_is_deterministic():
    """Training sums its block partials in a fixed order: the same run of
    300 steps (two launches of the persistent training kernel) twice from the
    same parameters gives bit-identical parameters and losses."""
    print("case surrogate training determinism", flush=True)
    wl = bunch.C1
    r, u = bunch.gaussian_bunch(wl.bunch)
    out = []
    with _ctx(wl.bunch.n, wl.depth, wl.dt) as ctx:
        ctx.init_bunch(r, u, 0.0)
        ctx.init_history_straight()
        ctx.surrogate_set(bunch.surrogate_init(4), bunch.sigma_ref_of(r))
        X, y = ctx.surrogate_samples_torch(1 << 15, seed=12)
        for _ in range(2):
            ctx.surrogate_set(bunch.surrogate_init(4), bunch.sigma_ref_of(r))
            rep = ctx.surrogate_train_torch(X, y, steps=300, batch=1024, lr=3e-3, lr_final=1e-4)
            out.append((ctx.surrogate_get(), rep))
    (p0, r0), (p1, r1) = out
    print(f"   loss {r0['loss_first']:.4e} -> {r0['loss_last']:.4e}; rerun {r1['loss_first']:.4e} -> "
          f"{r1['loss_last']:.4e}", flush=True)
    assert np.array_equal(p0, p1)
    assert r0["loss_first"] == r1["loss_first"] and r0["loss_last"] == r1["loss_last"]
    assert r0["loss_last"] < 0.5 * r0["loss_first"]


@pytest.mark.parametrize("precision", [0, 1])
def test_guess_never_changes_results(precision):
    """k* and the fields are bit-identical with the paper's bisection, the
    ballistic guess, a trained and an untrained network, and a network
    whose guesses are garbage (non-finite)."""
    print(f"case guess invariance precision={precision}", flush=True)
    n, D, dt = 300, 128, 1e-13
    T, w, v = bunch.wiggly_history(n, D, dt, beta=0.9, accel_rel=0.1, seed=9)
    rng = np.random.default_rng(10)
    x = 1.5e-3 * rng.standard_normal((3, 257))
    outs = {}
    with _ctx(n, D, dt, precision=precision) as ctx:
        ctx.set_history(T, w, v, np.zeros((3, n)))
        ctx.surrogate_set(bunch.surrogate_init(5), 1e-3)
        Xs, ys = ctx.surrogate_samples_torch(1 << 14, seed=3)
        for name, guess, params in (("bisect", 0, None), ("ballistic", 2, None), ("untrained", 1, None),
                                    ("trained", 1, "train"), ("garbage", 1, "garbage")):
            if params == "train":
                ctx.surrogate_train_torch(Xs, ys, steps=200, batch=1024, lr=3e-3, lr_final=1e-4)
            elif params == "garbage":
                ctx.surrogate_set(np.full(18049, 1e30, np.float32), 1e-3)
            ctx.set_mode(precision, guess)
            ctx.set_counting(True)
            E, B, k = ctx.fields_at(T[-1], x, want_kstar=True)
            outs[name] = (E, B, k, ctx.counters())
    ref = outs["bisect"]
    for name, (E, B, k, cnt) in outs.items():
        print(f"   {name}: probes/pair {cnt['probes'] / cnt['pairs']:.2f}, fallbacks {cnt['fallbacks']}", flush=True)
        assert np.array_equal(k, ref[2]), name
        assert np.array_equal(E, ref[0]) and np.array_equal(B, ref[1]), name
    assert outs["garbage"][3]["fallbacks"] > 0


def test_what_the_network_gains():
    """C3 workload (N=65536, D=512, dipole): the network trained on pairs from
    C2 and C3 bunches against the method without it and against the
    straight-line control.  Iterations (sign
    tests per pair) over 1024 seeded targets x all sources for the paper's
    bisection, the network evaluated per pair, the network amortised over
    groups of 64 targets (its correction to the straight-line delay at the
    group centroid applied to each target's straight-line delay), and the
    straight-line (ballistic) guess alone, which is the model with z = 0;
    k* and fields are identical in all four."""
    from paper_2605_05543_amd import surrogate
    from paper_2605_05543_amd._lib import EMPP_GUESS_BALLISTIC, EMPP_GUESS_BISECT, EMPP_GUESS_MLP, EMPP_GUESS_MLP_PAIR

    print("case surrogate gain on C3", flush=True)
    wl = bunch.C3
    r, u = bunch.gaussian_bunch(wl.bunch)
    n = wl.bunch.n
    sX2, sy2 = surrogate.draw_samples(bunch.C2, 1 << 21, seed=21)
    with _ctx(n, wl.depth, wl.dt) as ctx:
        ctx.init_bunch(r, u, 0.0)
        ctx.init_history_straight()
        ctx.step(4)
        ctx.surrogate_set(bunch.surrogate_init(0), bunch.sigma_ref_of(r))
        sX3, sy3 = ctx.surrogate_samples_torch(1 << 21, seed=23)
        rep = surrogate.train(ctx, [(sX2, sy2), (sX3, sy3)], batch=8192, steps=1536)
        print(f"   training: loss {rep['loss_first']:.3e} -> {rep['loss_last']:.3e}, {rep['steps']} steps, "
              f"{rep['seconds']:.2f} s", flush=True)
        sub = bunch.target_subset(n, 1024, 103)
        rg, _, t, _ = ctx.state()
        x = rg[:, sub]
        out = {}
        for name, g in (("bisect", EMPP_GUESS_BISECT), ("mlp-pair", EMPP_GUESS_MLP_PAIR),
                        ("mlp-group", EMPP_GUESS_MLP), ("ballistic", EMPP_GUESS_BALLISTIC)):
            ctx.set_mode(0, g)
            ctx.set_counting(True)
            E, B, k = ctx.fields_at(t, x, sub, want_kstar=True)
            c = ctx.counters()
            out[name] = (E, B, k, c["probes"] / c["pairs"], c["fallbacks"] / c["pairs"])
            print(f"   {name}: {out[name][3]:.2f} sign tests per pair, fallbacks per pair {out[name][4]:.2e}",
                  flush=True)
    for name in out:
        assert np.array_equal(out[name][2], out["bisect"][2]), name
        assert np.array_equal(out[name][0], out["bisect"][0]) and np.array_equal(out[name][1], out["bisect"][1])
    assert rep["loss_last"] < 0.05 * rep["loss_first"]
    assert out["mlp-pair"][3] < 0.5 * out["bisect"][3]
    assert out["mlp-group"][3] < 0.5 * out["bisect"][3]
    # against the straight-line control (the model with z = 0): the C3
    # histories are straight to within a slot, so the closed form already
    # places the bracket and the network can only match it, not beat it
    for name in ("mlp-pair", "mlp-group"):
        ratio = out[name][3] / out["ballistic"][3]
        print(f"   {name} / straight line: {ratio:.4f} sign tests", flush=True)
        assert 0.98 < ratio < 1.02, (name, ratio)


@pytest.mark.parametrize("group_log2", [6, 10])
def test_group_size_keeps_results(group_log2):
    """Stepping with the network evaluated once per 64 or per 1024 targets:
    the state after 6 steps is bit-identical to the bisection run."""
    from paper_2605_05543_amd._lib import EMPP_GUESS_BISECT, EMPP_GUESS_MLP, Context

    print(f"case surrogate group 2^{group_log2}", flush=True)
    wl = bunch.C1
    spec = bunch.BunchSpec(4096, (1e-3, 1e-3, 1e-3), 1.0, seed=31)
    r, u = bunch.gaussian_bunch(spec)
    out = {}
    for guess in (EMPP_GUESS_BISECT, EMPP_GUESS_MLP):
        with Context(n=4096, depth=wl.depth, q=Q, m=ME, dt=wl.dt, guess=guess, guess_group_log2=group_log2) as ctx:
            ctx.init_bunch(r, u, 0.0)
            ctx.init_history_straight()
            ctx.surrogate_set(bunch.surrogate_init(7), bunch.sigma_ref_of(r))
            ctx.step(5)
            ctx.set_counting(True)
            ctx.step(1)
            c = ctx.counters()
            out[guess] = (ctx.state(), ctx.fields(), c["probes"] / c["pairs"])
    print(f"   sign tests per pair: bisection {out[EMPP_GUESS_BISECT][2]:.2f}, "
          f"network per 2^{group_log2} targets {out[EMPP_GUESS_MLP][2]:.2f}", flush=True)
    a, b = out[EMPP_GUESS_BISECT], out[EMPP_GUESS_MLP]
    for x, y in zip(a[0] + a[1], b[0] + b[1]):
        assert np.array_equal(np.asarray(x), np.asarray(y))
    assert b[2] < a[2]


def test_network_corrects_curving_histories():
    """A bunch gyrating in a 0.5 T field (1 MeV: radius 9.5 mm, 2.9 mrad per
    step; 0.74 rad over the 256 stored steps): the straight-line term misses
    long look-backs by several slots.  The network, trained on pairs of this
    state, corrects it from the features (the 4-step slope differs from the
    newest velocity by the acceleration): fewer sign tests per pair than the
    straight-line guess, with identical k* and fields."""
    from paper_2605_05543_amd._lib import EMPP_GUESS_BALLISTIC, EMPP_GUESS_BISECT, EMPP_GUESS_MLP_PAIR, Context

    print("case surrogate on gyrating histories", flush=True)
    n, D, dt = 2048, 256, 1e-13
    rng = np.random.default_rng(41)
    r = 1e-3 * rng.standard_normal((3, n))
    r[0] += 1.0
    g = bunch.gamma_of_kinetic(bunch.MEV)
    u = np.zeros((3, n))
    u[1] = C * np.sqrt(g * g - 1.0)  # across the equatorial field
    out = {}
    with Context(n=n, depth=D, q=Q, m=ME, dt=dt, ext_field=1, dipole_b0=0.5, dipole_re=1.0) as ctx:
        ctx.init_bunch(r, u, 0.0)
        ctx.init_history_straight()
        ctx.step(D + 20)  # every stored slot on the gyrating path
        rg, _, t, _ = ctx.state()
        ctx.surrogate_set(bunch.surrogate_init(8), bunch.sigma_ref_of(rg))
        Xs, ys = ctx.surrogate_samples_torch(1 << 20, seed=5)
        rep = ctx.surrogate_train_torch(Xs, ys, steps=1500, batch=8192, lr=3e-3, lr_final=3e-5)
        print(f"   training: loss {rep['loss_first']:.3e} -> {rep['loss_last']:.3e}", flush=True)
        for name, gm in (("bisect", EMPP_GUESS_BISECT), ("straight line", EMPP_GUESS_BALLISTIC),
                         ("network per pair", EMPP_GUESS_MLP_PAIR)):
            ctx.set_mode(0, gm)
            ctx.set_counting(True)
            E, B, k = ctx.fields_at(t, rg, np.arange(n), want_kstar=True)
            c = ctx.counters()
            out[name] = (E, B, k, c["probes"] / c["pairs"])
            print(f"   {name}: {out[name][3]:.3f} sign tests per pair", flush=True)
    for name in out:
        assert np.array_equal(out[name][2], out["bisect"][2])
        assert np.array_equal(out[name][0], out["bisect"][0]) and np.array_equal(out[name][1], out["bisect"][1])
    assert out["straight line"][3] > 4.0  # the straight-line term misses
    assert out["network per pair"][3] < 0.7 * out["straight line"][3]
