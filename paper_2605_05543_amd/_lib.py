"""ctypes binding of libempp.so (the C ABI in include/empp.h).

Argument marshalling only: every step of the hot path runs in the HIP
library.  The functions keep the C names; ``Context`` is a small
convenience wrapper that owns one ``empp_ctx``.  If the library is
missing the import of this module fails loudly -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libempp.so")

EMPP_OK, EMPP_EINVAL, EMPP_ENOMEM, EMPP_EDEVICE, EMPP_ESTATE, EMPP_ENUMERIC, EMPP_EUNSUPPORTED = range(7)
STATUS_NAMES = ["OK", "EINVAL", "ENOMEM", "EDEVICE", "ESTATE", "ENUMERIC", "EUNSUPPORTED"]
EMPP_FP64, EMPP_MIXED = 0, 1
EMPP_GUESS_BISECT, EMPP_GUESS_MLP, EMPP_GUESS_BALLISTIC, EMPP_GUESS_MLP_PAIR, EMPP_GUESS_PREVIOUS = 0, 1, 2, 3, 4

# Functions declared in include/empp.h (tests check that each is exported).
EXPORTS = [
    "empp_workspace_size", "empp_create", "empp_destroy", "empp_last_error", "empp_init_bunch",
    "empp_init_history_straight", "empp_set_history", "empp_step", "empp_fields_at", "empp_fields_at_dev",
    "empp_fields_at_dev_noalloc",
    "empp_get_state", "empp_get_history", "empp_get_fields", "empp_get_diag", "empp_set_counting",
    "empp_get_counters", "empp_sync", "empp_set_mode", "empp_set_timing", "empp_get_timing",
    "empp_surrogate_set", "empp_surrogate_get", "empp_surrogate_samples", "empp_surrogate_samples_dev",
    "empp_surrogate_forward", "empp_surrogate_loss_grad", "empp_surrogate_train", "empp_step_until_switch",
    "empp_handoff", "empp_transport", "empp_save", "empp_load",
]
N_PARAMS = 18049


class EmppError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"EMPP_{name}: {message}")


class Config(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("depth", ctypes.c_int32), ("ext_field", ctypes.c_int32),
        ("q", ctypes.c_double), ("m", ctypes.c_double), ("dt", ctypes.c_double),
        ("dipole_b0", ctypes.c_double), ("dipole_re", ctypes.c_double),
        ("precision", ctypes.c_int32), ("guess", ctypes.c_int32), ("device", ctypes.c_int32),
        ("source_splits", ctypes.c_int32), ("stream", ctypes.c_void_p), ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_uint64), ("adaptive", ctypes.c_int32), ("c_dt", ctypes.c_double),
        ("dt_min", ctypes.c_double), ("dt_max", ctypes.c_double), ("eta_allow", ctypes.c_double),
        ("recon", ctypes.c_int32), ("guess_group_log2", ctypes.c_int32),
    ]


class Diag(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_double * 3), ("sigma_xy", ctypes.c_double), ("centroid", ctypes.c_double * 3),
                ("mean_kinetic", ctypes.c_double), ("t", ctypes.c_double), ("step", ctypes.c_int64),
                ("dt_last", ctypes.c_double)]


class Counters(ctypes.Structure):
    _fields_ = [("pairs", ctypes.c_uint64), ("before", ctypes.c_uint64), ("probes", ctypes.c_uint64),
                ("rescues", ctypes.c_uint64), ("fallbacks", ctypes.c_uint64)]


class Timing(ctypes.Structure):
    _fields_ = [("pair_ms", ctypes.c_double), ("pair_launches", ctypes.c_int64), ("push_ms", ctypes.c_double),
                ("push_launches", ctypes.c_int64), ("guess_ms", ctypes.c_double), ("guess_launches", ctypes.c_int64)]


class TrainCfg(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("lr_final", ctypes.c_float)]


class TrainReport(ctypes.Structure):
    _fields_ = [("loss_first", ctypes.c_double), ("loss_last", ctypes.c_double), ("steps", ctypes.c_int64),
                ("seconds", ctypes.c_double)]


_P = ctypes.c_void_p
_D = ctypes.c_double
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64


def _load():
    # PyTorch brings its own HIP runtime.  Importing it first makes
    # libempp.so bind to that same runtime (same soname), so torch's streams
    # and device pointers are valid in the library and only one runtime is
    # loaded in the process.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build() (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "empp_workspace_size": [ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_uint64)],
        "empp_create": [ctypes.POINTER(Config), ctypes.POINTER(_P)],
        "empp_init_bunch": [_P, _P, _P, _D],
        "empp_init_history_straight": [_P],
        "empp_set_history": [_P, _I32, _P, _P, _P, _P],
        "empp_step": [_P, _I64],
        "empp_fields_at": [_P, _D, _I64, _P, _P, _P, _P, _P],
        "empp_fields_at_dev": [_P, _D, _I64, _P, _P, _P, _P, _P],
        "empp_fields_at_dev_noalloc": [_P, _D, _I64, _P, _P, _P, _P, _P],
        "empp_get_state": [_P, _P, _P, ctypes.POINTER(_D), ctypes.POINTER(_I64)],
        "empp_get_history": [_P, _P, _P, _P],
        "empp_get_fields": [_P, _P, _P],
        "empp_get_diag": [_P, ctypes.POINTER(Diag)],
        "empp_set_counting": [_P, _I32],
        "empp_get_counters": [_P, ctypes.POINTER(Counters)],
        "empp_sync": [_P],
        "empp_set_mode": [_P, _I32, _I32],
        "empp_set_timing": [_P, _I32],
        "empp_get_timing": [_P, ctypes.POINTER(Timing)],
        "empp_surrogate_set": [_P, _P, _I64, _D],
        "empp_surrogate_get": [_P, _P, _I64],
        "empp_surrogate_samples": [_P, _I64, ctypes.c_uint64, _P, _P, _P, _P],
        "empp_surrogate_samples_dev": [_P, _I64, ctypes.c_uint64, _P, _P],
        "empp_surrogate_forward": [_P, _P, _I64, _P],
        "empp_surrogate_loss_grad": [_P, _P, _P, _I64, ctypes.POINTER(_D), _P],
        "empp_surrogate_train": [_P, _P, _P, _I64, ctypes.POINTER(TrainCfg), ctypes.POINTER(TrainReport)],
        "empp_step_until_switch": [_P, _D, _I64, _I64, ctypes.POINTER(_I64), ctypes.POINTER(_D),
                                   ctypes.POINTER(_I32)],
        "empp_handoff": [_P],
        "empp_transport": [_P, _D, _D, _I64],
        "empp_save": [_P, ctypes.c_char_p],
        "empp_load": [_P, ctypes.c_char_p],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.empp_destroy.argtypes = [_P]
    L.empp_destroy.restype = None
    L.empp_last_error.argtypes = []
    L.empp_last_error.restype = ctypes.c_char_p
    return L


lib = _load()


def _check(status: int):
    if status != EMPP_OK:
        raise EmppError(status, lib.empp_last_error().decode(errors="replace"))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_P)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# -- thin wrappers with the C names -------------------------------------------------

def empp_workspace_size(cfg: Config) -> int:
    out = ctypes.c_uint64()
    _check(lib.empp_workspace_size(ctypes.byref(cfg), ctypes.byref(out)))
    return out.value


def empp_create(cfg: Config):
    h = _P()
    _check(lib.empp_create(ctypes.byref(cfg), ctypes.byref(h)))
    return h


def empp_destroy(h):
    lib.empp_destroy(h)


def empp_init_bunch(h, r, u, t0=0.0):
    _check(lib.empp_init_bunch(h, _ptr(_f64(r)), _ptr(_f64(u)), float(t0)))


def empp_init_history_straight(h):
    _check(lib.empp_init_history_straight(h))


def empp_set_history(h, T, w, v, u):
    T, w, v, u = _f64(T), _f64(w), _f64(v), _f64(u)
    _check(lib.empp_set_history(h, int(T.shape[0]), _ptr(T), _ptr(w), _ptr(v), _ptr(u)))


def empp_step(h, nsteps=1):
    _check(lib.empp_step(h, int(nsteps)))


def empp_fields_at(h, t, x, n_src, self_index=None, want_kstar=False):
    x = _f64(x)
    m = x.shape[1]
    si = None if self_index is None else np.ascontiguousarray(self_index, dtype=np.int64)
    E = np.zeros((3, m))
    B = np.zeros((3, m))
    ks = np.zeros((m, n_src), np.int32) if want_kstar else None
    _check(lib.empp_fields_at(h, float(t), m, _ptr(x), _ptr(si), _ptr(E), _ptr(B), _ptr(ks)))
    return (E, B, ks) if want_kstar else (E, B)


def empp_fields_at_dev(h, t, m, x_ptr, self_ptr, E_ptr, B_ptr, kstar_ptr=None):
    _check(lib.empp_fields_at_dev(h, float(t), int(m), x_ptr, self_ptr, E_ptr, B_ptr, kstar_ptr))


def empp_fields_at_dev_noalloc(h, t, m, x_ptr, self_ptr, E_ptr, B_ptr, kstar_ptr=None):
    _check(lib.empp_fields_at_dev_noalloc(h, float(t), int(m), x_ptr, self_ptr, E_ptr, B_ptr, kstar_ptr))


def empp_get_state(h, n):
    r = np.zeros((3, n))
    u = np.zeros((3, n))
    t = _D()
    s = _I64()
    _check(lib.empp_get_state(h, _ptr(r), _ptr(u), ctypes.byref(t), ctypes.byref(s)))
    return r, u, t.value, s.value


def empp_get_history(h, n, depth):
    T = np.zeros(depth)
    w = np.zeros((depth, 3, n))
    v = np.zeros((depth, 3, n))
    _check(lib.empp_get_history(h, _ptr(T), _ptr(w), _ptr(v)))
    return T, w, v


def empp_get_fields(h, n):
    E = np.zeros((3, n))
    B = np.zeros((3, n))
    _check(lib.empp_get_fields(h, _ptr(E), _ptr(B)))
    return E, B


def empp_get_diag(h):
    d = Diag()
    _check(lib.empp_get_diag(h, ctypes.byref(d)))
    return {"sigma": list(d.sigma), "sigma_xy": d.sigma_xy, "centroid": list(d.centroid),
            "mean_kinetic": d.mean_kinetic, "t": d.t, "step": d.step, "dt_last": d.dt_last}


def empp_set_counting(h, enable=True):
    _check(lib.empp_set_counting(h, 1 if enable else 0))


def empp_get_counters(h):
    c = Counters()
    _check(lib.empp_get_counters(h, ctypes.byref(c)))
    return {"pairs": c.pairs, "before": c.before, "probes": c.probes, "rescues": c.rescues,
            "fallbacks": c.fallbacks}


def empp_set_timing(h, enable=True):
    _check(lib.empp_set_timing(h, 1 if enable else 0))


def empp_get_timing(h):
    t = Timing()
    _check(lib.empp_get_timing(h, ctypes.byref(t)))
    return {"pair_ms": t.pair_ms, "pair_launches": t.pair_launches, "push_ms": t.push_ms,
            "push_launches": t.push_launches, "guess_ms": t.guess_ms, "guess_launches": t.guess_launches}


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def empp_surrogate_set(h, params, sigma_ref):
    params = _f32(params)
    _check(lib.empp_surrogate_set(h, _ptr(params), params.size, float(sigma_ref)))


def empp_surrogate_get(h):
    out = np.zeros(N_PARAMS, np.float32)
    _check(lib.empp_surrogate_get(h, _ptr(out), N_PARAMS))
    return out


def empp_surrogate_samples(h, count, seed=0, tgt=None, src=None):
    X = np.zeros((count, 10), np.float32)
    y = np.zeros(count, np.float32)
    t = None if tgt is None else np.ascontiguousarray(tgt, dtype=np.int64)
    s_ = None if src is None else np.ascontiguousarray(src, dtype=np.int64)
    _check(lib.empp_surrogate_samples(h, int(count), int(seed), _ptr(t), _ptr(s_), _ptr(X), _ptr(y)))
    return X, y


def empp_surrogate_samples_dev(h, count, seed, X_ptr, y_ptr):
    _check(lib.empp_surrogate_samples_dev(h, int(count), int(seed), X_ptr, y_ptr))


def empp_surrogate_forward(h, X):
    X = _f32(X)
    z = np.zeros(X.shape[0], np.float32)
    _check(lib.empp_surrogate_forward(h, _ptr(X), X.shape[0], _ptr(z)))
    return z


def empp_surrogate_loss_grad(h, X, y):
    X, y = _f32(X), _f32(y)
    g = np.zeros(N_PARAMS, np.float32)
    loss = _D()
    _check(lib.empp_surrogate_loss_grad(h, _ptr(X), _ptr(y), X.shape[0], ctypes.byref(loss), _ptr(g)))
    return loss.value, g


def empp_surrogate_train(h, X_ptr, y_ptr, count, steps, batch, lr, lr_final):
    cfg = TrainCfg(steps=int(steps), batch=int(batch), lr=float(lr), lr_final=float(lr_final))
    rep = TrainReport()
    _check(lib.empp_surrogate_train(h, X_ptr, y_ptr, int(count), ctypes.byref(cfg), ctypes.byref(rep)))
    return {"loss_first": rep.loss_first, "loss_last": rep.loss_last, "steps": rep.steps, "seconds": rep.seconds}


def empp_sync(h):
    _check(lib.empp_sync(h))


def empp_set_mode(h, precision, guess):
    _check(lib.empp_set_mode(h, int(precision), int(guess)))


def empp_step_until_switch(h, eps_E, check_every, max_steps):
    steps, t_sw, sw = _I64(), _D(), _I32()
    _check(lib.empp_step_until_switch(h, float(eps_E), int(check_every), int(max_steps), ctypes.byref(steps),
                                      ctypes.byref(t_sw), ctypes.byref(sw)))
    return steps.value, t_sw.value, bool(sw.value)


def empp_handoff(h):
    _check(lib.empp_handoff(h))


def empp_transport(h, dt_max, gyro_fraction, nsteps):
    _check(lib.empp_transport(h, float(dt_max), float(gyro_fraction), int(nsteps)))


def empp_save(h, path):
    _check(lib.empp_save(h, os.fsencode(path)))


def empp_load(h, path):
    _check(lib.empp_load(h, os.fsencode(path)))


class Context:
    """One empp_ctx.  Device memory comes from a torch tensor (PyTorch is
    the allocator and stream provider); kernels run on torch's current
    stream of ``device``."""

    def __init__(self, *, n, depth, q, m, dt, ext_field=0, dipole_b0=0.0, dipole_re=0.0,
                 precision=EMPP_FP64, guess=EMPP_GUESS_BISECT, device=0, source_splits=0, use_torch=True,
                 adaptive=False, c_dt=0.05, dt_min=1e-15, dt_max=1e-12, eta_allow=0.0, recon=0,
                 guess_group_log2=0):
        self.n, self.depth = int(n), int(depth)
        cfg = Config(n=self.n, depth=self.depth, ext_field=int(ext_field), q=float(q), m=float(m), dt=float(dt),
                     dipole_b0=float(dipole_b0), dipole_re=float(dipole_re), precision=int(precision),
                     guess=int(guess), device=int(device), source_splits=int(source_splits),
                     adaptive=int(bool(adaptive)), c_dt=float(c_dt), dt_min=float(dt_min), dt_max=float(dt_max),
                     eta_allow=float(eta_allow), recon=int(recon), guess_group_log2=int(guess_group_log2))
        self._ws = None
        self.stream_handle = None
        if use_torch:
            import torch

            dev = torch.device("cuda", device)
            nbytes = empp_workspace_size(cfg)
            self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
            base = self._ws.data_ptr()
            aligned = (base + 255) // 256 * 256
            cfg.workspace = aligned
            cfg.workspace_bytes = nbytes
            self.stream_handle = torch.cuda.current_stream(dev).cuda_stream
            cfg.stream = self.stream_handle
        self.cfg = cfg
        self.h = empp_create(cfg)

    def close(self):
        if self.h:
            empp_destroy(self.h)
            self.h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def init_bunch(self, r, u, t0=0.0):
        empp_init_bunch(self.h, r, u, t0)

    def init_history_straight(self):
        empp_init_history_straight(self.h)

    def set_history(self, T, w, v, u):
        empp_set_history(self.h, T, w, v, u)

    def step(self, nsteps=1):
        empp_step(self.h, nsteps)

    def fields_at(self, t, x, self_index=None, want_kstar=False):
        return empp_fields_at(self.h, t, x, self.n, self_index, want_kstar)

    def state(self):
        return empp_get_state(self.h, self.n)

    def history(self):
        return empp_get_history(self.h, self.n, self.depth)

    def fields(self):
        return empp_get_fields(self.h, self.n)

    def diag(self):
        return empp_get_diag(self.h)

    def set_counting(self, enable=True):
        empp_set_counting(self.h, enable)

    def counters(self):
        return empp_get_counters(self.h)

    def sync(self):
        empp_sync(self.h)

    def set_timing(self, enable=True):
        empp_set_timing(self.h, enable)

    def timing(self):
        return empp_get_timing(self.h)

    # -- surrogate network ---------------------------------------------------
    def surrogate_set(self, params, sigma_ref):
        empp_surrogate_set(self.h, params, sigma_ref)

    def surrogate_get(self):
        return empp_surrogate_get(self.h)

    def surrogate_samples(self, count, seed=0, tgt=None, src=None):
        return empp_surrogate_samples(self.h, count, seed, tgt, src)

    def surrogate_forward(self, X):
        return empp_surrogate_forward(self.h, X)

    def surrogate_loss_grad(self, X, y):
        return empp_surrogate_loss_grad(self.h, X, y)

    def surrogate_train_torch(self, X, y, steps, batch, lr=1e-3, lr_final=1e-5):
        """Train on torch device tensors X [count, 10], y [count] (float32)."""
        assert X.is_cuda and X.dtype.itemsize == 4 and X.is_contiguous() and y.is_contiguous()
        return empp_surrogate_train(self.h, X.data_ptr(), y.data_ptr(), X.shape[0], steps, batch, lr, lr_final)

    def surrogate_samples_torch(self, count, seed):
        """Drawn training pairs of the present state as torch device tensors."""
        import torch

        X = torch.empty((count, 10), dtype=torch.float32, device=self._ws.device)
        y = torch.empty(count, dtype=torch.float32, device=self._ws.device)
        empp_surrogate_samples_dev(self.h, count, seed, X.data_ptr(), y.data_ptr())
        self.sync()
        return X, y

    def set_mode(self, precision, guess):
        empp_set_mode(self.h, precision, guess)

    def step_until_switch(self, eps_E, check_every, max_steps):
        """Stage I until |d(mean kinetic energy)/dt| < eps_E (J/s) over a
        window of check_every steps: (steps taken, t_sw, switched)."""
        return empp_step_until_switch(self.h, eps_E, check_every, max_steps)

    def handoff(self):
        empp_handoff(self.h)

    def transport(self, dt_max, gyro_fraction, nsteps):
        empp_transport(self.h, dt_max, gyro_fraction, nsteps)

    def save(self, path):
        empp_save(self.h, path)

    def load(self, path):
        empp_load(self.h, path)
