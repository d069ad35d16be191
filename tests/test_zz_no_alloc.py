"""The allocation-free fields call (empp_fields_at_dev_noalloc) through the
C ABI against empp_fields_at_dev on the same context: k* and fields
bit-identical, for two calls in a row, the second with fewer targets, in
both precisions; a call beyond the scratch array's maximum is refused."""
import numpy as np
import pytest

from paper_2605_05543_amd import bunch

pytestmark = pytest.mark.gpu

Q, ME = -bunch.E_CHARGE, bunch.M_ELECTRON


def _fields(fn, ctx, t, x, self_index, want_kstar=True):
    import torch

    m = x.shape[1]
    n = ctx.n
    xd = torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")
    sd = torch.tensor(self_index, dtype=torch.int64, device="cuda")
    Ed = torch.full((3, m), float("nan"), dtype=torch.float64, device="cuda")
    Bd = torch.full((3, m), float("nan"), dtype=torch.float64, device="cuda")
    kd = torch.full((m, n), -7, dtype=torch.int32, device="cuda") if want_kstar else None
    torch.cuda.synchronize()
    fn(ctx.h, t, m, xd.data_ptr(), sd.data_ptr(), Ed.data_ptr(), Bd.data_ptr(), kd.data_ptr() if want_kstar else None)
    ctx.sync()
    return Ed.cpu().numpy(), Bd.cpu().numpy(), (kd.cpu().numpy() if want_kstar else None)


@pytest.mark.parametrize("precision,guess", [(0, 0), (1, 0), (0, 2)])
def test_noalloc_matches_fields_at_dev(precision, guess):
    from paper_2605_05543_amd import _lib

    print(f"case no-alloc fields precision={precision} guess={guess}", flush=True)
    n, depth, dt = 300, 128, 1e-13
    T, w, v = bunch.wiggly_history(n, depth, dt, beta=0.9, accel_rel=0.1, seed=17)
    rng = np.random.default_rng(18)
    with _lib.Context(n=n, depth=depth, q=Q, m=ME, dt=dt, precision=precision, guess=guess) as ctx:
        ctx.set_history(T, w, v, np.zeros((3, n)))
        for m in (700, 129):
            x = 1.5e-3 * rng.standard_normal((3, m))
            x[:, :5] = w[-1][:, 10:15]  # targets on sources 10..14, excluded
            si = np.full(m, -1, np.int64)
            si[:5] = np.arange(10, 15)
            E1, B1, k1 = _fields(_lib.empp_fields_at_dev, ctx, T[-1], x, si)
            E2, B2, k2 = _fields(_lib.empp_fields_at_dev_noalloc, ctx, T[-1], x, si)
            d = float(np.max(np.abs(E2 - E1)) / np.max(np.abs(E1)))
            print(f"   m={m}: k* equal {np.array_equal(k1, k2)}, fields equal {np.array_equal(E1, E2)} "
                  f"and {np.array_equal(B1, B2)} (max |dE| / max |E| {d:.1e})", flush=True)
            assert np.all(np.isfinite(E1)) and np.all(np.isfinite(E2))
            assert np.array_equal(k1, k2)
            assert np.array_equal(E1, E2) and np.array_equal(B1, B2)


def test_noalloc_refuses_more_targets_than_its_scratch():
    from paper_2605_05543_amd import _lib

    print("case no-alloc size limit", flush=True)
    n, depth, dt = 65536, 8, 1e-13
    r, u = bunch.gaussian_bunch(bunch.BunchSpec(n, (1e-3, 1e-3, 1e-3), 1.0, seed=3))
    with _lib.Context(n=n, depth=depth, q=Q, m=ME, dt=dt) as ctx:
        ctx.init_bunch(r, u, 0.0)
        ctx.init_history_straight()
        import torch

        m = 20000  # 128 chunks x 96 B per target: at most 10922 fit 128 MiB
        xd = torch.zeros((3, m), dtype=torch.float64, device="cuda")
        Ed = torch.zeros((3, m), dtype=torch.float64, device="cuda")
        with pytest.raises(_lib.EmppError) as ei:
            _lib.empp_fields_at_dev_noalloc(ctx.h, 0.0, m, xd.data_ptr(), None, Ed.data_ptr(), Ed.data_ptr())
        assert ei.value.status == _lib.EMPP_EINVAL and "maximum" in str(ei.value)
