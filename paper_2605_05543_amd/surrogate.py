"""Training of the retarded-delay surrogate network on pairs drawn from the
histories of running bunches (all work on the GPU through the C ABI: pair
sampling with the exact search, BF16 matrix-core forward/backward, Adam).

The network only seeds the bracket search; results never depend on it.
"""
from __future__ import annotations

from . import bunch
from ._lib import Context


def draw_samples(workload, count, seed, steps_before=4, params=None, sigma_ref=None):
    """(X, y) torch tensors of ``count`` pairs drawn from ``workload``'s bunch
    after ``steps_before`` FP64 steps.  sigma_ref defaults to the bunch's."""
    r, u = bunch.gaussian_bunch(workload.bunch)
    sig = sigma_ref or bunch.sigma_ref_of(r)
    with Context(n=workload.bunch.n, depth=workload.depth, q=-bunch.E_CHARGE, m=bunch.M_ELECTRON, dt=workload.dt,
                 ext_field=workload.ext_field, dipole_b0=workload.dipole_b0, dipole_re=workload.dipole_re) as ctx:
        ctx.init_bunch(r, u, 0.0)
        ctx.init_history_straight()
        if steps_before:
            ctx.step(steps_before)
        ctx.surrogate_set(bunch.surrogate_init(0) if params is None else params, sig)
        X, y = ctx.surrogate_samples_torch(count, seed)
        ctx.sync()
        return X, y


def train(ctx: Context, samples, *, steps=None, batch=8192, lr=3e-3, lr_final=3e-5, seed=4):
    """Train ``ctx``'s network from initial parameters on the concatenated
    sample sets (one pass over them unless ``steps`` is given)."""
    import torch

    X = torch.cat([s[0] for s in samples]).contiguous()
    y = torch.cat([s[1] for s in samples]).contiguous()
    # interleave the sets so every batch mixes them
    perm = torch.randperm(X.shape[0], generator=torch.Generator().manual_seed(seed)).to(X.device)
    X = X[perm].contiguous()
    y = y[perm].contiguous()
    steps = steps or max(1, X.shape[0] // batch)
    return ctx.surrogate_train_torch(X, y, steps=steps, batch=batch, lr=lr, lr_final=lr_final)
