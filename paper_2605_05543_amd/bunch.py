"""Seeded synthetic inputs: electron bunches, workload configurations and
test histories.

This module only *draws* inputs.  It holds none of the method's arithmetic
(no retarded-time search, no field evaluation, no push); both the HIP
library and the CPU oracle take what it produces as plain arrays.

Units are SI.  Arrays are component-major: ``r[3, N]``, ``u[3, N]`` with
``u`` the proper velocity gamma * v (m/s).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# CODATA 2018 values used only to turn a kinetic energy into a momentum.
C_LIGHT = 299792458.0
E_CHARGE = 1.602176634e-19
M_ELECTRON = 9.1093837015e-31
MEV = 1e6 * E_CHARGE
R_EARTH = 6.371e6


def gamma_of_kinetic(kin_joule):
    """Lorentz factor of an electron with kinetic energy ``kin_joule``
    (Sec. 2.5: gamma = 1 + E / (m_e c^2))."""
    return 1.0 + np.asarray(kin_joule) / (M_ELECTRON * C_LIGHT**2)


@dataclasses.dataclass(frozen=True)
class BunchSpec:
    """Gaussian bunch: positions N(center, sigma^2) per axis; kinetic energy
    K0 (1 + rel_spread * xi); direction (theta_x, theta_y, 1) normalised with
    theta ~ N(0, angle_spread^2) about +z."""

    n: int
    sigma: tuple  # (sx, sy, sz) metres
    kinetic_mev: float
    rel_energy_spread: float = 1e-3
    angle_spread: float = 1e-3
    center: tuple = (0.0, 0.0, 0.0)
    seed: int = 1


def gaussian_bunch(spec: BunchSpec):
    """Draw (r, u) for ``spec`` with numpy's PCG64 generator."""
    rng = np.random.default_rng(spec.seed)
    n = spec.n
    r = np.empty((3, n))
    for c in range(3):
        r[c] = spec.center[c] + spec.sigma[c] * rng.standard_normal(n)
    kin = spec.kinetic_mev * MEV * (1.0 + spec.rel_energy_spread * rng.standard_normal(n))
    gam = gamma_of_kinetic(kin)
    umag = C_LIGHT * np.sqrt(gam * gam - 1.0)
    th = spec.angle_spread * rng.standard_normal((2, n))
    dirn = np.stack([th[0], th[1], np.ones(n)])
    dirn /= np.linalg.norm(dirn, axis=0)
    u = dirn * umag
    return r, u


def paper_beam(n, *, e0_mev=1.0, delta_e=0.01, emittance=1e-6, r_perp=2e-3, r_par=2e-3, seed=0):
    """The beam-frame sampling of Sec. 2.5 (Eqs. space-sampling,
    vel-sampling, rel-vz): x, y ~ N(0, r_perp^2), z ~ N(0, r_par^2);
    v_x, v_y ~ N(0, sigma_perp^2) with sigma_perp = eps_r v0 / r_perp;
    E ~ N(E0, (delta_E E0)^2) -> v_z(E); the sample mean of v_z is shifted
    back to v0.  Returns (r, u) with u = gamma(v) v."""
    rng = np.random.default_rng(seed)
    g0 = gamma_of_kinetic(e0_mev * MEV)
    v0 = C_LIGHT * math.sqrt(1.0 - 1.0 / (g0 * g0))
    r = np.stack([r_perp * rng.standard_normal(n), r_perp * rng.standard_normal(n), r_par * rng.standard_normal(n)])
    sig_perp = emittance * v0 / r_perp
    vx = sig_perp * rng.standard_normal(n)
    vy = sig_perp * rng.standard_normal(n)
    en = e0_mev * MEV * (1.0 + delta_e * rng.standard_normal(n))
    ge = gamma_of_kinetic(en)
    vz = C_LIGHT * np.sqrt(1.0 - 1.0 / (ge * ge))
    vz = vz - (vz.mean() - v0)
    vel = np.stack([vx, vy, vz])
    g = 1.0 / np.sqrt(1.0 - (vel * vel).sum(0) / C_LIGHT**2)
    return r, vel * g


def beam_rotation(theta, phi):
    """R(theta, phi) = R_z(phi) R_y(theta) of Sec. 2.5: takes the beam axis
    (+z of the beam frame) to polar angle theta and azimuth phi in the
    laboratory frame."""
    ct, st, cp, sp = math.cos(theta), math.sin(theta), math.cos(phi), math.sin(phi)
    Ry = np.array([[ct, 0.0, st], [0.0, 1.0, 0.0], [-st, 0.0, ct]])
    Rz = np.array([[cp, -sp, 0.0], [sp, cp, 0.0], [0.0, 0.0, 1.0]])
    return Rz @ Ry


def rotate_to_lab(r, u, theta, phi, center=(0.0, 0.0, 0.0)):
    """Beam-frame positions and proper velocities [3, N] -> laboratory frame
    (Sec. 2.5: x_lab = R x_beam, v_lab = R v_beam; u = gamma v rotates the
    same way), the rotated bunch then centred on ``center``."""
    R = beam_rotation(theta, phi)
    return R @ np.asarray(r) + np.asarray(center, dtype=np.float64).reshape(3, 1), R @ np.asarray(u)


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic workload: bunch, history depth, step, steps, field."""

    name: str
    bunch: BunchSpec
    depth: int
    dt: float
    steps: int
    ext_field: int = 0  # 0 none, 1 centred dipole along +z
    dipole_b0: float = 3.12e-5
    dipole_re: float = R_EARTH


# The five workloads of the measurement plan.  Electrons (charge -e, mass
# m_e, weight 1), momenta along +z.
C1 = Workload("c1_n256_d256", BunchSpec(256, (1e-3, 1e-3, 1e-3), 1.0, seed=1), 256, 1e-13, 200)
C2 = Workload("c2_n8192_d512", BunchSpec(8192, (0.5e-3, 0.5e-3, 2e-3), 2.0, seed=2), 512, 5e-14, 1000)
C3 = Workload("c3_n65536_d512_dipole",
              BunchSpec(65536, (1e-3, 1e-3, 1e-3), 1.0, center=(3 * R_EARTH, 0.0, 0.0), seed=3),
              512, 1e-13, 500, ext_field=1)
C5 = Workload("c5_n262144_d1024_dipole",
              BunchSpec(262144, (2e-3, 2e-3, 5e-3), 5.0, center=(3 * R_EARTH, 0.0, 0.0), seed=5),
              1024, 1e-13, 2000, ext_field=1)
# C3's bunch (N = 65536, sigma = 1 mm, 1 MeV) moving across a uniform-looking
# 0.5 T field: a dipole of equatorial field 0.5 T at 1 m, the bunch centred
# there with its momenta along +y (gyro-radius 9.5 mm, 2.9 mrad of turn per
# 0.1 ps step).  Its history curves by 1.5 rad over the 512 stored steps once
# stepping has refilled the ring (depth + 20 steps from the straight start).
C3G = Workload("c3g_n65536_d512_gyrating_0.5T", BunchSpec(65536, (1e-3, 1e-3, 1e-3), 1.0, seed=3),
               512, 1e-13, 500, ext_field=1, dipole_b0=0.5, dipole_re=1.0)
WORKLOADS = {w.name: w for w in (C1, C2, C3, C5, C3G)}


def gyrating_bunch(wl=C3G):
    """(r, u) of the gyrating workload: the seeded bunch about +z turned so
    that it moves along +y, centred at (dipole_re, 0, 0)."""
    r, u = gaussian_bunch(wl.bunch)
    return rotate_to_lab(r, u, math.pi / 2, math.pi / 2, center=(wl.dipole_re, 0.0, 0.0))


def target_subset(n, count, seed):
    """Seeded subset of target indices (sorted, without repetition)."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=min(count, n), replace=False)).astype(np.int64)


# -- synthetic histories for fields_at tests -----------------------------------
#
# A history is (T[ns], w[ns, 3, N], v[ns, 3, N]), oldest slot first.  The
# generators below integrate a prescribed velocity sequence with
# w[k+1] = w[k] + v[k] (T[k+1] - T[k]) so that, like the histories the
# stepping code writes, every stored segment moves at the stored velocity.


def wiggly_history(n, ns, dt, *, beta=0.9, sigma=1e-3, accel_rel=0.05, seed=7, t_now=0.0):
    """Sources on smoothly curving paths: speed ``beta`` c along a random
    mean direction plus a slowly rotating transverse velocity of relative
    size ``accel_rel``.  Returns (T, w, v) with the newest slot at t_now."""
    rng = np.random.default_rng(seed)
    T = t_now + dt * np.arange(-(ns - 1), 1, dtype=np.float64)
    base = rng.standard_normal((3, n))
    base /= np.linalg.norm(base, axis=0)
    perp1 = np.cross(base.T, rng.standard_normal((n, 3))).T
    perp1 /= np.linalg.norm(perp1, axis=0)
    perp2 = np.cross(base.T, perp1.T).T
    omega = rng.uniform(0.5, 2.0, n) * 2 * math.pi / (ns * dt) * 3.0
    phase = rng.uniform(0, 2 * math.pi, n)
    v = np.empty((ns, 3, n))
    for k in range(ns):
        ang = omega * T[k] + phase
        d = base + accel_rel * (np.cos(ang) * perp1 + np.sin(ang) * perp2)
        d /= np.linalg.norm(d, axis=0)
        v[k] = beta * C_LIGHT * d
    w = np.empty((ns, 3, n))
    w[ns - 1] = sigma * rng.standard_normal((3, n))
    for k in range(ns - 2, -1, -1):
        w[k] = w[k + 1] - v[k] * (T[k + 1] - T[k])
    return T, w, v


def circular_history(ns, dt, *, radius, omega, t_now=0.0, exact_velocity=True):
    """One source on the circle radius*(cos wt, sin wt, 0).  With
    ``exact_velocity`` the stored v is the analytic velocity at T_k (the
    positions are then exact samples of the orbit); otherwise v is the chord
    velocity (w[k+1]-w[k])/dt."""
    T = t_now + dt * np.arange(-(ns - 1), 1, dtype=np.float64)
    ph = omega * T
    w = np.zeros((ns, 3, 1))
    w[:, 0, 0] = radius * np.cos(ph)
    w[:, 1, 0] = radius * np.sin(ph)
    v = np.zeros((ns, 3, 1))
    if exact_velocity:
        v[:, 0, 0] = -radius * omega * np.sin(ph)
        v[:, 1, 0] = radius * omega * np.cos(ph)
    else:
        v[:-1] = (w[1:] - w[:-1]) / dt
        v[-1] = v[-2]
    return T, w, v


def uniform_history(ns, dt, w_now, vel, t_now=0.0):
    """Sources in uniform motion: w_k = w_now + vel (T_k - t_now)."""
    w_now = np.asarray(w_now, dtype=np.float64).reshape(3, -1)
    vel = np.asarray(vel, dtype=np.float64).reshape(3, -1)
    T = t_now + dt * np.arange(-(ns - 1), 1, dtype=np.float64)
    w = w_now[None] + vel[None] * (T - t_now)[:, None, None]
    v = np.broadcast_to(vel[None], w.shape).copy()
    return T, w, v


def surrogate_init(seed=4):
    """Initial parameters of the 10 -> 128 -> 128 -> 1 surrogate network in
    its flat layout (W1[128][10], b1, W2[128][128], b2, W3[128], b3): weights
    uniform in +-1/sqrt(fan_in), biases zero; float32."""
    rng = np.random.default_rng(seed)
    parts = [rng.uniform(-1, 1, 128 * 10) / np.sqrt(10.0), np.zeros(128),
             rng.uniform(-1, 1, 128 * 128) / np.sqrt(128.0), np.zeros(128),
             rng.uniform(-1, 1, 128) / np.sqrt(128.0), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


def sigma_ref_of(r):
    """Reference length (sigma_x sigma_y sigma_z)^(1/3) of a bunch r[3, N]."""
    s = r.std(axis=1)
    return float(np.prod(s) ** (1.0 / 3.0))
