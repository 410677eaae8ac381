"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no part of the method's arithmetic: it only draws particle
sets.  Every generator returns ``(pos [N,3], vel [N,3], mass [N])`` as numpy
float64 arrays with body 0 the massive object (black hole) and bodies
1..N-1 the stars.

* :func:`plummer_bh` -- Plummer sphere of equal-mass stars (total star mass 1,
  scale radius 1, G = 1) sampled with the Aarseth-Henon-Wielen (1974) recipe,
  truncated at ``rmax``, recentred to zero mass-weighted position and velocity,
  plus a black hole at rest at the origin.  The paper's own experiments use no
  public dataset; this is the synthetic stand-in for the clusters it describes.
* :func:`cold_sphere_bh` -- the paper's test model (Sec. 4): stars uniform in
  the shell 1 < r < 10, all at rest, mass 1/N_stars each, black hole of mass
  100 m at the origin.  The paper draws from a linear congruential generator
  whose constants it does not give; a PCG64 stream stands in for it.
* :func:`random_cluster` -- small random configurations for physics checks.
"""
from __future__ import annotations

import numpy as np


def _isotropic(rng: np.random.Generator, n: int) -> np.ndarray:
    """n unit vectors uniform on the sphere."""
    z = 1.0 - 2.0 * rng.random(n)
    phi = 2.0 * np.pi * rng.random(n)
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)


def plummer_stars(n: int, seed: int, rmax: float = 10.0):
    """n Plummer-sphere stars (G = 1, total mass 1, a = 1): (pos, vel, mass)."""
    rng = np.random.default_rng(seed)
    radii = np.empty(0)
    while radii.size < n:
        x1 = rng.random(2 * n + 16)
        x1 = x1[x1 > 0.0]
        r = 1.0 / np.sqrt(x1 ** (-2.0 / 3.0) - 1.0)
        radii = np.concatenate([radii, r[r <= rmax]])
    r = radii[:n]
    pos = r[:, None] * _isotropic(rng, n)
    # speed fraction q from g(q) = q^2 (1 - q^2)^(7/2) by rejection
    q = np.empty(0)
    while q.size < n:
        x4 = rng.random(4 * n + 16)
        x5 = rng.random(4 * n + 16)
        ok = 0.1 * x5 < x4 * x4 * (1.0 - x4 * x4) ** 3.5
        q = np.concatenate([q, x4[ok]])
    q = q[:n]
    speed = q * np.sqrt(2.0) * (1.0 + r * r) ** (-0.25)
    vel = speed[:, None] * _isotropic(rng, n)
    mass = np.full(n, 1.0 / n)
    pos -= (mass[:, None] * pos).sum(0) / mass.sum()
    vel -= (mass[:, None] * vel).sum(0) / mass.sum()
    return pos, vel, mass


def plummer_bh(N: int, M_bh: float, seed: int, rmax: float = 10.0):
    """N bodies: black hole of mass M_bh at rest at the origin + N-1 Plummer stars."""
    if N < 2:
        raise ValueError("N counts the black hole and needs at least one star")
    ps, vs, ms = plummer_stars(N - 1, seed, rmax)
    pos = np.zeros((N, 3))
    vel = np.zeros((N, 3))
    mass = np.empty(N)
    pos[1:], vel[1:], mass[1:] = ps, vs, ms
    mass[0] = M_bh
    return pos, vel, mass


def cold_sphere_bh(n_stars: int = 10000, seed: int = 0, r_in: float = 1.0,
                   r_out: float = 10.0, bh_over_m: float = 100.0):
    """The paper's cold-collapse test model: stars at rest, uniform in r_in < r < r_out."""
    rng = np.random.default_rng(seed)
    u = rng.random(n_stars)
    r = (r_in ** 3 + u * (r_out ** 3 - r_in ** 3)) ** (1.0 / 3.0)
    N = n_stars + 1
    pos = np.zeros((N, 3))
    pos[1:] = r[:, None] * _isotropic(rng, n_stars)
    vel = np.zeros((N, 3))
    m = 1.0 / n_stars
    mass = np.full(N, m)
    mass[0] = bh_over_m * m
    return pos, vel, mass


def random_cluster(n_stars: int, seed: int, M: float = 1.0, m_star: float = 1e-3,
                   r_scale: float = 1.0, v_scale: float = 0.3, zero_momentum: bool = True):
    """Small random cluster: stars in a unit-ish ball with random velocities.

    With ``zero_momentum`` the black hole gets v_0 = -P/M so the total
    Newtonian momentum vanishes.
    """
    rng = np.random.default_rng(seed)
    N = n_stars + 1
    pos = np.zeros((N, 3))
    vel = np.zeros((N, 3))
    pos[1:] = r_scale * (0.3 + 0.7 * rng.random(n_stars))[:, None] * _isotropic(rng, n_stars)
    vel[1:] = v_scale * rng.standard_normal((n_stars, 3))
    pos[0] = 0.05 * r_scale * rng.standard_normal(3)
    mass = np.full(N, m_star)
    mass[0] = M
    if zero_momentum:
        vel[0] = -(mass[1:, None] * vel[1:]).sum(0) / M
    return pos, vel, mass


# Workloads of the benchmark and the parity tests (sizes, masses, light speed,
# softening, step).  N counts the black hole.
WORKLOADS = {
    "plummer_n1024_fp64": dict(N=1024, M_bh=0.1, c=50.0, eps=1e-4, dt=1e-4, steps=100,
                               seed=1, precision="fp64"),
    "plummer_n16384_fp64": dict(N=16384, M_bh=0.05, c=30.0, eps=1e-4, dt=1e-4, steps=1000,
                                seed=2, precision="fp64"),
    "plummer_n65536_mixed": dict(N=65536, M_bh=0.1, c=30.0, eps=1e-4, dt=1e-4, steps=1000,
                                 seed=3, precision="mixed"),
    "plummer_n262144_mixed": dict(N=262144, M_bh=0.1, c=30.0, eps=1e-4, dt=1e-4, steps=100,
                                  seed=5, precision="mixed"),
}


def ensemble(n_sys: int = 256, seed: int = 4, n_lo: int = 1024, n_hi: int = 16384):
    """Batched-ensemble workload: per-system (N, M_bh, c, seed) with N ~ U{n_lo..n_hi},
    M_bh ~ U[0.01, 0.1], c ~ U[20, 100]; system b uses seed 10000 + b."""
    rng = np.random.default_rng(seed)
    Ns = rng.integers(n_lo, n_hi + 1, size=n_sys)
    Ms = rng.uniform(0.01, 0.1, size=n_sys)
    cs = rng.uniform(20.0, 100.0, size=n_sys)
    return [dict(N=int(Ns[b]), M_bh=float(Ms[b]), c=float(cs[b]), eps=1e-4, dt=1e-4,
                 seed=10000 + b) for b in range(n_sys)]
