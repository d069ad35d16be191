"""Surrogate-network oracle against finite differences and library routines."""
import numpy as np
import torch

from oracle import mlp


def _params(seed=0, scale=0.3):
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal(mlp.N_PARAMS)


def test_param_count():
    assert mlp.N_PARAMS == 18049


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-5, 5, 5000),
                        [1.0, 1.0 + 2**-8, 1.0 + 3 * 2**-8, -0.0, 65504.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(x), ref)


def test_forward_matches_torch():
    flat = _params(2)
    X = np.random.default_rng(3).standard_normal((64, 10))
    z, _ = mlp.forward(flat, X, round_bf16=False)
    p = {k: torch.tensor(v) for k, v in mlp.unpack(flat).items()}
    h = torch.nn.functional.silu(torch.tensor(X) @ p["W1"].T + p["b1"])
    h = torch.nn.functional.silu(h @ p["W2"].T + p["b2"])
    zt = (h @ p["W3"].T + p["b3"])[:, 0].numpy()
    assert np.max(np.abs(z - zt)) < 1e-12


def test_backward_vs_finite_differences():
    flat = _params(4)
    rng = np.random.default_rng(5)
    X = rng.standard_normal((32, 10))
    y = rng.standard_normal(32)
    loss, g = mlp.loss_and_grad(flat, X, y, round_bf16=False)
    idx = rng.choice(mlp.N_PARAMS, 200, replace=False)
    h = 1e-6
    worst = 0.0
    for i in idx:
        e = np.zeros_like(flat)
        e[i] = h
        lp, _ = mlp.loss_and_grad(flat + e, X, y, round_bf16=False)
        lm, _ = mlp.loss_and_grad(flat - e, X, y, round_bf16=False)
        fd = (lp - lm) / (2 * h)
        worst = max(worst, abs(fd - g[i]) / max(abs(g).max() * 1e-3, abs(fd)))
    assert worst < 1e-6, worst


def test_backward_matches_autograd():
    flat = _params(6)
    rng = np.random.default_rng(7)
    X = rng.standard_normal((48, 10))
    y = rng.standard_normal(48)
    loss, g = mlp.loss_and_grad(flat, X, y, round_bf16=False)
    ft = torch.tensor(flat, requires_grad=True)
    p, o = {}, 0
    for name, shape in mlp.SHAPES:
        k = int(np.prod(shape))
        p[name] = ft[o:o + k].reshape(shape)
        o += k
    h = torch.nn.functional.silu(torch.tensor(X) @ p["W1"].T + p["b1"])
    h = torch.nn.functional.silu(h @ p["W2"].T + p["b2"])
    z = (h @ p["W3"].T + p["b3"])[:, 0]
    lt = ((z - torch.tensor(y)) ** 2).mean()
    lt.backward()
    assert abs(lt.item() - loss) < 1e-12
    assert np.max(np.abs(ft.grad.numpy() - g)) < 1e-12 * max(1.0, np.abs(g).max())


def test_adam_matches_torch():
    flat = _params(8)
    rng = np.random.default_rng(9)
    pt = torch.tensor(flat.copy(), requires_grad=True)
    opt = torch.optim.Adam([pt], lr=1e-3)
    m = np.zeros_like(flat)
    v = np.zeros_like(flat)
    cur = flat.copy()
    for step in range(1, 6):
        grad = rng.standard_normal(flat.size)
        opt.zero_grad()
        pt.grad = torch.tensor(grad)
        opt.step()
        cur, m, v = mlp.adam_step(cur, m, v, grad, step, 1e-3)
    assert np.max(np.abs(cur - pt.detach().numpy())) < 1e-14


def test_straight_line_lookback_closed_forms():
    """A source at rest: the look-back is the distance.  A source heading
    straight at the target at speed beta c: d / (1 - beta).  Receding:
    d / (1 + beta).  Moving across the line of sight: d / sqrt(1 - beta^2)."""
    C = mlp.C_LIGHT
    d, beta = 2.5e-3, 0.94
    y = np.array([[d, d, d, 0.0], [0.0, 0.0, 0.0, d], [0.0, 0.0, 0.0, 0.0]])
    w = np.zeros((3, 4))
    v = np.array([[0.0, beta * C, -beta * C, beta * C], [0.0, 0.0, 0.0, 0.0], [0.0, 0.0, 0.0, 0.0]])
    s = mlp.straight_line_lookback(y, w, v)
    want = np.array([d, d / (1 - beta), d / (1 + beta), d / np.sqrt(1 - beta * beta)])
    assert np.allclose(s, want, rtol=1e-14, atol=0)


def test_straight_line_lookback_matches_retarded_solve():
    """On histories of uniform motion the exact retarded solve of the
    oracle (bracket and segment root inside the history, straight
    extrapolation before it) lands on the straight-line look-back."""
    import oracle
    from paper_2605_05543_amd import bunch

    n, D, dt = 24, 64, 1e-13
    T, w, v = bunch.wiggly_history(n, D, dt, beta=0.9, accel_rel=0.0, seed=4)
    rng = np.random.default_rng(5)
    x = 1.5e-3 * rng.standard_normal((3, 40))
    ret = oracle.get().retarded(T, w, v, T[-1], x)
    look = mlp.C_LIGHT * (T[-1] - ret["tr"])  # [40, n]
    assert 0.05 < (ret["kstar"] >= 0).mean() < 0.95  # both cases present
    for j in range(n):
        s = mlp.straight_line_lookback(x, w[-1][:, j:j + 1], v[-1][:, j:j + 1])
        assert np.allclose(look[:, j], s, rtol=1e-11, atol=0)
