"""FP64 CPU oracle of the EM-PP hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may import this package.  The product path (the HIP
library and its Python binding) never touches it.

The arithmetic lives in ``empp_oracle.c`` (plain C, IEEE double, no FMA
contraction, OpenMP over targets) and, for the surrogate network, in
``mlp.py`` (numpy float64).  This module only compiles the C file and
marshals numpy arrays into it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "empp_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

OR_OK, OR_EINVAL, OR_ENUMERIC, OR_ECHECK = 0, 1, 2, 3

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared"]


class OracleError(RuntimeError):
    def __init__(self, status, bad=None):
        self.status = status
        self.bad = bad
        super().__init__(f"oracle status {status} bad={bad}")


def build(out: str = LIB, defines=()) -> str:
    """Compile the oracle (optionally with -D mutation flags) into ``out``."""
    cmd = ["gcc", *CFLAGS, *[f"-D{d}" for d in defines], "-o", out + ".tmp", SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build_mutant(name: str, workdir: str | None = None) -> str:
    workdir = workdir or tempfile.mkdtemp(prefix="oracle_mut_")
    return build(os.path.join(workdir, f"liboracle_{name}.so"), defines=[name])


_D = ctypes.c_double
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_P = ctypes.c_void_p


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_P)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Brackets(np.ndarray):
    """The oracle's bracket index k* of every (target, source) pair (int32
    [m, N]: slots back from the newest of the bracket's older end, -1 before
    the history, 0 for an excluded pair), with ``alt``: the same array
    except on near ties of the light-cone test, where it holds the bracket
    the other decision gives.  Views and slices drop ``alt``."""

    def __new__(cls, kstar, alt):
        obj = np.asarray(kstar).view(cls)
        obj.alt = alt
        return obj

    def __array_finalize__(self, obj):
        self.alt = None

    @property
    def near_ties(self) -> int:
        return 0 if self.alt is None else int(np.count_nonzero(self.alt != np.asarray(self)))


class Oracle:
    """ctypes view of one compiled oracle library."""

    def __init__(self, path: str = LIB):
        if not os.path.exists(path):
            build(path)
        self.path = path
        L = ctypes.CDLL(path)
        L.oracle_constants.argtypes = [_P]
        L.oracle_retarded.argtypes = [_I64, _I32, _P, _P, _P, _D, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _P]
        L.oracle_fields.argtypes = [_I64, _I32, _P, _P, _P, _D, _D, _I64, _P, _P, _P, _P, _P, ctypes.c_int, _P]
        L.oracle_fields_abs.argtypes = [_I64, _I32, _P, _P, _P, _D, _D, _I64, _P, _P, _P, _P, _P, _P, _P, _P,
                                        ctypes.c_int, _P]
        L.oracle_dipole.argtypes = [_D, _D, _I64, _P, _P]
        L.oracle_dipole.restype = None
        L.oracle_hc.argtypes = [_D, _D, _D, _I64, _P, _P, _P]
        L.oracle_hc.restype = None
        L.oracle_init_straight.argtypes = [_I64, _I32, _D, _D, _P, _P, _P, _P, _P]
        L.oracle_step.argtypes = [_I64, _I32, _D, _D, _D, _D, _P, _I32, _D, _D, _P, _P, _P, _P, _P, _P, _I64,
                                  ctypes.c_int, _P]
        L.oracle_diag.argtypes = [_I64, _P, _P, _D, _P]
        L.oracle_diag.restype = None
        L.oracle_set_reconstruction.argtypes = [ctypes.c_int]
        L.oracle_set_reconstruction.restype = None
        L.oracle_transport.argtypes = [_I64, _D, _D, _I32, _D, _D, _D, _D, _P, _P, _P, _I64, _P]
        L.oracle_transport.restype = ctypes.c_int
        L.oracle_adaptive_scan.argtypes = [_I64, _I32, _P, _P, _P, _D, _I64, _P, _P, _P, _D, _P]
        L.oracle_adaptive_scan.restype = ctypes.c_int
        L.oracle_adaptive_dt.argtypes = [_D, _D, _D, _D, _D]
        L.oracle_adaptive_dt.restype = ctypes.c_double
        L.oracle_step_adaptive.argtypes = [_I64, _I32, _D, _D, _D, _D, _D, _D, _I32, _D, _D, _P, _P, _P, _P, _P,
                                           _I64, ctypes.c_int, _P]
        L.oracle_step_adaptive.restype = ctypes.c_int
        L.oracle_max_threads.argtypes = []
        self.L = L
        c = np.zeros(6)
        L.oracle_constants(_ptr(c))
        self.c, self.e, self.me, self.mu0, self.eps0, self.kC = (float(x) for x in c)

    def max_threads(self) -> int:
        return int(self.L.oracle_max_threads())

    # -- Sec. 2.2 inspection ---------------------------------------------------
    def retarded(self, T, w, v, t, x, self_index=None):
        T, w, v, x = _f64(T), _f64(w), _f64(v), _f64(x)
        ns, _, N = w.shape
        m = x.shape[1]
        si = None if self_index is None else np.ascontiguousarray(self_index, dtype=np.int64)
        kstar = np.zeros((m, N), np.int32)
        kalt = np.zeros((m, N), np.int32)
        dt_root = np.zeros((m, N))
        tr = np.zeros((m, N))
        wr = np.zeros((m, N, 3))
        vr = np.zeros((m, N, 3))
        ar = np.zeros((m, N, 3))
        st = self.L.oracle_retarded(N, ns, _ptr(T), _ptr(w), _ptr(v), float(t), m, _ptr(x), _ptr(si),
                                    _ptr(kstar), _ptr(kalt), _ptr(dt_root), _ptr(tr), _ptr(wr), _ptr(vr), _ptr(ar))
        if st != OR_OK:
            raise OracleError(st)
        return dict(kstar=Brackets(kstar, kalt), kalt=kalt, dt_root=dt_root, tr=tr, wr=wr, vr=vr, ar=ar)

    # -- Sec. 2.1 fields ---------------------------------------------------------
    def fields(self, T, w, v, q, t, x, self_index=None, want_kstar=False, nthreads=None, want_abs=False):
        T, w, v, x = _f64(T), _f64(w), _f64(v), _f64(x)
        ns, _, N = w.shape
        m = x.shape[1]
        si = None if self_index is None else np.ascontiguousarray(self_index, dtype=np.int64)
        E = np.zeros((3, m))
        B = np.zeros((3, m))
        kstar = np.zeros((m, N), np.int32) if want_kstar else None
        kalt = np.zeros((m, N), np.int32) if want_kstar else None
        SE = np.zeros(m) if want_abs else None
        SB = np.zeros(m) if want_abs else None
        bad = np.full(2, -1, np.int64)
        nt = nthreads or self.max_threads()
        st = self.L.oracle_fields_abs(N, ns, _ptr(T), _ptr(w), _ptr(v), float(q), float(t), m, _ptr(x), _ptr(si),
                                      _ptr(E), _ptr(B), _ptr(kstar), _ptr(kalt), _ptr(SE), _ptr(SB), int(nt),
                                      _ptr(bad))
        if st != OR_OK:
            raise OracleError(st, tuple(bad))
        out = (E, B)
        if want_kstar:
            out = out + (Brackets(kstar, kalt),)
        if want_abs:
            out = out + (SE, SB)
        return out

    def dipole(self, b0, re, x):
        x = _f64(x)
        B = np.zeros_like(x)
        self.L.oracle_dipole(float(b0), float(re), x.shape[1], _ptr(x), _ptr(B))
        return B

    def hc(self, q, mass, dt, u, E, B):
        u = _f64(u).copy()
        self.L.oracle_hc(float(q), float(mass), float(dt), u.shape[1], _ptr(u), _ptr(_f64(E)), _ptr(_f64(B)))
        return u

    def init_straight(self, r, u, D, dt, t0=0.0):
        r, u = _f64(r), _f64(u)
        N = r.shape[1]
        T = np.zeros(D)
        w = np.zeros((D, 3, N))
        v = np.zeros((D, 3, N))
        st = self.L.oracle_init_straight(N, D, float(dt), float(t0), _ptr(r), _ptr(u), _ptr(T), _ptr(w), _ptr(v))
        if st != OR_OK:
            raise OracleError(st)
        return T, w, v

    def set_reconstruction(self, mode):
        """0: the local linear reconstruction (Eq. linear); 1: the midpoint
        values of Eq. (mid), for the accuracy ablation."""
        self.L.oracle_set_reconstruction(int(mode))

    def transport(self, y, u, t, *, q, mass, dt_max, frac, nsteps, ext_field=0, b0=0.0, re=0.0):
        """Stage II (E = 0, B = B_geo): returns (y, u, t, last dt)."""
        y, u = _f64(y).copy(), _f64(u).copy()
        tt = np.array([float(t)])
        dl = np.zeros(1)
        st = self.L.oracle_transport(y.shape[1], float(q), float(mass), int(ext_field), float(b0), float(re),
                                     float(dt_max), float(frac), _ptr(y), _ptr(u), _ptr(tt), int(nsteps), _ptr(dl))
        if st != OR_OK:
            raise OracleError(st)
        return y, u, float(tt[0]), float(dl[0])

    def adaptive_scan(self, T, w, v, t, x, self_index, vt, eta_allow):
        """Sec. 2.4: (eta_min, v_max) over the pairs of targets x[3][m] with
        present velocities vt[3][m] against the history."""
        T, w, v, x, vt = _f64(T), _f64(w), _f64(v), _f64(x), _f64(vt)
        si = None if self_index is None else np.ascontiguousarray(self_index, dtype=np.int64)
        out = np.zeros(2)
        st = self.L.oracle_adaptive_scan(w.shape[2], len(T), _ptr(T), _ptr(w), _ptr(v), float(t), x.shape[1],
                                         _ptr(x), _ptr(si), _ptr(vt), float(eta_allow), _ptr(out))
        if st != OR_OK:
            raise OracleError(st)
        return float(out[0]), float(out[1])

    def adaptive_dt(self, eta_min, v_max, c_dt=0.05, dt_min=1e-15, dt_max=1e-12):
        return float(self.L.oracle_adaptive_dt(float(eta_min), float(v_max), float(c_dt), float(dt_min),
                                               float(dt_max)))

    def step_adaptive(self, T, w, v, u, nsteps, *, q, mass, c_dt=0.05, dt_min=1e-15, dt_max=1e-12, eta_allow=0.0,
                      ext_field=0, b0=0.0, re=0.0, nthreads=None):
        """Adaptive-step EM-PP (in place on copies): returns (T, w, v, u, dts)."""
        T, w, v, u = _f64(T).copy(), _f64(w).copy(), _f64(v).copy(), _f64(u).copy()
        dts = np.zeros(max(int(nsteps), 1))
        bad = np.zeros(2, dtype=np.int64)
        nt = nthreads or self.L.oracle_max_threads()
        st = self.L.oracle_step_adaptive(w.shape[2], len(T), float(q), float(mass), float(c_dt), float(dt_min),
                                         float(dt_max), float(eta_allow), int(ext_field), float(b0), float(re),
                                         _ptr(T), _ptr(w), _ptr(v), _ptr(u), _ptr(dts), int(nsteps), int(nt),
                                         _ptr(bad))
        if st != OR_OK:
            raise OracleError(st)
        return T, w, v, u, dts[:nsteps]

    def diag(self, y, u, mass):
        out = np.zeros(8)
        y, u = _f64(y), _f64(u)
        self.L.oracle_diag(y.shape[1], _ptr(y), _ptr(u), float(mass), _ptr(out))
        return out


class OracleRun:
    """A stepping oracle simulation (state held in numpy arrays)."""

    def __init__(self, orc: Oracle, r, u, *, D, dt, q, mass, t0=0.0, ext_field=0, b0=0.0, re=0.0, nthreads=None):
        self.o = orc
        self.N = r.shape[1]
        self.D, self.dt, self.q, self.mass, self.t0 = D, dt, q, mass, t0
        self.ext_field, self.b0, self.re = ext_field, b0, re
        self.T, self.w, self.v = orc.init_straight(r, u, D, dt, t0)
        self.u = _f64(u).copy()
        self.n = np.zeros(1, np.int64)
        self.E = np.zeros((3, self.N))
        self.B = np.zeros((3, self.N))
        self.nthreads = nthreads or orc.max_threads()

    @property
    def y(self):
        return self.w[-1]

    @property
    def t(self):
        return float(self.T[-1])

    def step(self, nsteps=1):
        bad = np.full(2, -1, np.int64)
        st = self.o.L.oracle_step(self.N, self.D, float(self.q), float(self.mass), float(self.dt), float(self.t0),
                                  _ptr(self.n), int(self.ext_field), float(self.b0), float(self.re), _ptr(self.T),
                                  _ptr(self.w), _ptr(self.v), _ptr(self.u), _ptr(self.E), _ptr(self.B),
                                  int(nsteps), int(self.nthreads), _ptr(bad))
        if st != OR_OK:
            raise OracleError(st, tuple(bad))

    def diag(self):
        return self.o.diag(self.y, self.u, self.mass)


_default = None


def get() -> Oracle:
    """The default oracle build (compiled on first use)."""
    global _default
    if _default is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(LIB)
        _default = Oracle(LIB)
    return _default
