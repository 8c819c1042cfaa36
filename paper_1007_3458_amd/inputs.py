"""Seeded synthetic planetary systems for tests, examples and the benchmark.

This module only *draws* initial conditions: orbital elements from seeded
numpy PCG64 streams, converted to heliocentric Cartesian positions and
barycentric velocities.  It holds none of the integrator's arithmetic and is
the one module that both the HIP path and the CPU oracle are fed from.

Recipes (G = 1, central mass m0 = 1; angles Omega, omega and the mean anomaly
uniform on [0, 2 pi)).  The paper profiles "four massive planets inside a
debris disk" (Sec. 4) without giving the initial conditions, so these disks
stand in for it:

* ``small``   4 planets (m = 1e-3, 3e-4, 4.4e-5, 5.1e-5; a = 5.2, 9.5, 19.2,
  30.1; e ~ U[0, 0.05]; i ~ U[0, 0.02]) + 100 planetesimals (m = 1e-9,
  a ~ U[20, 35], e ~ U[0, 0.1], i ~ U[0, 0.05]); seed 1.
* ``disk16k`` the 4 planets + 16384 planetesimals (m = 1e-8, a ~ U[15, 40],
  e ~ Rayleigh(0.05), i ~ Rayleigh(0.025)); seed 2.
* ``disk128k`` the 4 planets + 131072 planetesimals (m = 2e-9, same
  distributions); seed 3.
* ``batch``   independent systems with N ~ log-U[64, 4096] bodies: one planet
  (m = 1e-3, a = 5.2, e ~ U[0, 0.05], i ~ U[0, 0.02]) + N - 1 planetesimals
  (m = 1e-8, a ~ U[3, 10], e ~ U[0, 0.1], i ~ U[0, 0.05]); system k uses
  seed 4_000_000 + k.
* ``kepler_test`` massless bodies (a ~ U[0.5, 50], e ~ U[0, 0.9],
  i ~ U[0, 0.1]); seed 6.
* ``kepler_train`` training solves for the learned Kepler starting value:
  a ~ U[0.5, 50], e ~ U[0, 0.9], isotropic orientation, steps
  dt ~ log-U[0.005, 0.5]; seed 5.
* ``learned_workload`` 1,048,576 ``kepler_test`` bodies (seed 6) after a
  65,536-planetesimal disk with the 4 planets (disk16k distributions, seed 6).
* ``guess_init`` Glorot-uniform starting weights of the 4-32-32-1 network,
  zero biases, rounded to float32; seed 7.
* ``two_planet_encounter`` two Jupiter-mass planets on circular orbits at
  5.2 and 5.45 (inside three mutual Hill radii) with small bodies
  (m = 1e-9, a ~ U[4, 7], e ~ U[0, 0.05], i ~ U[0, 0.02]) around them.

Positions are heliocentric; velocities are barycentric, i.e. the heliocentric
velocity minus sum_j m_j u_j / (m0 + sum_j m_j) (the democratic-heliocentric
change of variables of Sec. 2).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

PLANET_M = np.array([1e-3, 3e-4, 4.4e-5, 5.1e-5])
PLANET_A = np.array([5.2, 9.5, 19.2, 30.1])


@dataclass
class System:
    """One planetary system in the integrator's variables.

    q, v: (n, 3) float64 heliocentric positions / barycentric velocities;
    m: (n,) masses; h: (n,) Hill factors cbrt(m / (3 m0)), computed here once
    so that both implementations use identical bits.
    """

    name: str
    G: float
    m0: float
    m: np.ndarray
    q: np.ndarray
    v: np.ndarray
    h: np.ndarray = field(default=None)  # type: ignore[assignment]

    def __post_init__(self):
        self.m = np.ascontiguousarray(self.m, dtype=np.float64)
        self.q = np.ascontiguousarray(self.q, dtype=np.float64).reshape(-1, 3)
        self.v = np.ascontiguousarray(self.v, dtype=np.float64).reshape(-1, 3)
        if self.h is None:
            self.h = np.cbrt(self.m / (3.0 * self.m0))
        self.h = np.ascontiguousarray(self.h, dtype=np.float64)

    @property
    def n(self) -> int:
        return int(self.m.shape[0])

    def copy(self) -> "System":
        return System(self.name, self.G, self.m0, self.m.copy(), self.q.copy(), self.v.copy(),
                      self.h.copy())

    def permuted(self, perm: np.ndarray) -> "System":
        return System(self.name + "-perm", self.G, self.m0, self.m[perm], self.q[perm],
                      self.v[perm], self.h[perm])


def _solve_eccentric_anomaly(M: np.ndarray, e: np.ndarray) -> np.ndarray:
    """E - e sin E = M for 0 <= e < 1 (Newton, started at M + e sin M)."""
    E = M + e * np.sin(M)
    for _ in range(60):
        d = (E - e * np.sin(E) - M) / (1.0 - e * np.cos(E))
        E = E - d
        if d.size == 0 or np.max(np.abs(d)) < 1e-15:
            break
    return E


def elements_to_cartesian(mu, a, e, inc, Om, om, M):
    """Heliocentric position/velocity of bound orbits from classical elements."""
    a, e, inc, Om, om, M = (np.asarray(x, dtype=np.float64) for x in (a, e, inc, Om, om, M))
    E = _solve_eccentric_anomaly(np.mod(M, 2 * np.pi), e)
    cE, sE = np.cos(E), np.sin(E)
    b = np.sqrt(1.0 - e * e)
    xp = a * (cE - e)
    yp = a * b * sE
    r = a * (1.0 - e * cE)
    n = np.sqrt(mu / a ** 3)
    vxp = -a * n * sE / (1.0 - e * cE)
    vyp = a * n * b * cE / (1.0 - e * cE)
    cO, sO, co, so, ci, si = np.cos(Om), np.sin(Om), np.cos(om), np.sin(om), np.cos(inc), np.sin(inc)
    # rotation perifocal -> reference frame: Rz(Om) Rx(i) Rz(om)
    P = np.stack([cO * co - sO * so * ci, sO * co + cO * so * ci, so * si], axis=-1)
    Q = np.stack([-cO * so - sO * co * ci, -sO * so + cO * co * ci, co * si], axis=-1)
    pos = xp[..., None] * P + yp[..., None] * Q
    vel = vxp[..., None] * P + vyp[..., None] * Q
    del r
    return pos, vel


def _to_barycentric(m0, m, u):
    return u - (m[:, None] * u).sum(axis=0) / (m0 + m.sum())


def _draw_planets(rng, masses, axes, emax=0.05, imax=0.02):
    k = len(masses)
    e = rng.uniform(0.0, emax, k)
    inc = rng.uniform(0.0, imax, k)
    ang = rng.uniform(0.0, 2 * np.pi, (3, k))
    return np.asarray(masses, float), np.asarray(axes, float), e, inc, ang


def make_disk(name, seed, n_disk, m_disk, a_lo, a_hi, e_dist, i_dist, e_par, i_par,
              planets=True, G=1.0, m0=1.0) -> System:
    rng = np.random.Generator(np.random.PCG64(seed))
    mu = G * m0
    ms, as_, es, is_, angs = [], [], [], [], []
    if planets:
        pm, pa, pe, pi, pang = _draw_planets(rng, PLANET_M, PLANET_A)
        ms.append(pm); as_.append(pa); es.append(pe); is_.append(pi); angs.append(pang)
    a = rng.uniform(a_lo, a_hi, n_disk)
    if e_dist == "uniform":
        e = rng.uniform(0.0, e_par, n_disk)
    else:
        e = np.minimum(rng.rayleigh(e_par, n_disk), 0.9)
    if i_dist == "uniform":
        inc = rng.uniform(0.0, i_par, n_disk)
    else:
        inc = np.minimum(rng.rayleigh(i_par, n_disk), 0.5)
    ang = rng.uniform(0.0, 2 * np.pi, (3, n_disk))
    ms.append(np.full(n_disk, m_disk)); as_.append(a); es.append(e); is_.append(inc); angs.append(ang)
    m = np.concatenate(ms)
    A = np.concatenate(as_)
    e = np.concatenate(es)
    inc = np.concatenate(is_)
    ang = np.concatenate(angs, axis=1)
    q, u = elements_to_cartesian(mu, A, e, inc, ang[0], ang[1], ang[2])
    v = _to_barycentric(m0, m, u)
    return System(name, G, m0, m, q, v)


def enhanced_outer(seed: int, scale: float = 50.0, G: float = 1.0, m0: float = 1.0) -> System:
    """The four giant planets with their masses multiplied by ``scale`` (an
    unstable configuration with planet-planet encounters), at a = 5.2, 9.5,
    19.2, 30.1 with e ~ U[0, 0.05], i ~ U[0, 0.02] and uniform angles (seeded
    elements stand in for the unpublished epoch elements)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m, a, e, inc, ang = _draw_planets(rng, PLANET_M * scale, PLANET_A)
    q, u = elements_to_cartesian(G * m0, a, e, inc, ang[0], ang[1], ang[2])
    return System(f"outer_x{scale:g}_s{seed}", G, m0, m, q, _to_barycentric(m0, m, u))


def small(seed: int = 1) -> System:
    """4 planets + 100 planetesimals (the oracle-sized case)."""
    return make_disk("small", seed, 100, 1e-9, 20.0, 35.0, "uniform", "uniform", 0.1, 0.05)


def disk16k(seed: int = 2, n_disk: int = 16384) -> System:
    """4 planets + 16384 planetesimals of 1e-8 (the plain FP64 benchmark disk)."""
    return make_disk("disk16k", seed, n_disk, 1e-8, 15.0, 40.0, "rayleigh", "rayleigh", 0.05, 0.025)


def disk128k(seed: int = 3, n_disk: int = 131072) -> System:
    """4 planets + 131072 planetesimals of 2e-9 (the precision-form disk)."""
    return make_disk("disk128k", seed, n_disk, 2e-9, 15.0, 40.0, "rayleigh", "rayleigh", 0.05, 0.025)


def scaled_disk(n_disk: int, seed: int, m_disk: float = 1e-8) -> System:
    """The disk16k recipe at another planetesimal count (parity sizes)."""
    return make_disk(f"disk{n_disk}", seed, n_disk, m_disk, 15.0, 40.0, "rayleigh", "rayleigh",
                     0.05, 0.025)


def batch_sizes(nsys: int = 512, lo: int = 64, hi: int = 4096, seed: int = 4) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi), nsys))).astype(np.int64)


def batch_system(k: int, n: int, G: float = 1.0, m0: float = 1.0) -> System:
    """System k of the batched workload: 1 Jupiter-mass planet + n-1 planetesimals."""
    rng = np.random.Generator(np.random.PCG64(4_000_000 + k))
    mu = G * m0
    pm, pa, pe, pi, pang = _draw_planets(rng, [1e-3], [5.2])
    nd = n - 1
    a = rng.uniform(3.0, 10.0, nd)
    e = rng.uniform(0.0, 0.1, nd)
    inc = rng.uniform(0.0, 0.05, nd)
    ang = rng.uniform(0.0, 2 * np.pi, (3, nd))
    m = np.concatenate([pm, np.full(nd, 1e-8)])
    A = np.concatenate([pa, a]); E = np.concatenate([pe, e]); I = np.concatenate([pi, inc])
    ang = np.concatenate([pang, ang], axis=1)
    q, u = elements_to_cartesian(mu, A, E, I, ang[0], ang[1], ang[2])
    return System(f"batch{k}", G, m0, m, q, _to_barycentric(m0, m, u))


def batch(nsys: int = 512, lo: int = 64, hi: int = 4096) -> list[System]:
    return [batch_system(k, int(n)) for k, n in enumerate(batch_sizes(nsys, lo, hi))]


def kepler_test(n: int, seed: int = 6, a_lo=0.5, a_hi=50.0, e_hi=0.9, i_hi=0.1,
                G: float = 1.0, m0: float = 1.0) -> System:
    """Massless bodies on bound orbits (Kepler solver workload)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.uniform(a_lo, a_hi, n)
    e = rng.uniform(0.0, e_hi, n)
    inc = rng.uniform(0.0, i_hi, n)
    ang = rng.uniform(0.0, 2 * np.pi, (3, n))
    q, u = elements_to_cartesian(G * m0, a, e, inc, ang[0], ang[1], ang[2])
    return System("kepler_test", G, m0, np.zeros(n), q, u)


def random_unit(rng, n):
    x = rng.normal(size=(n, 3))
    return x / np.linalg.norm(x, axis=1, keepdims=True)


def kepler_train(n: int = 1_000_000, seed: int = 5, a_lo=0.5, a_hi=50.0, e_hi=0.9,
                 dt_lo=0.005, dt_hi=0.5, mu: float = 1.0):
    """Bound orbits with isotropic orientation and log-uniform steps:
    returns q (n, 3), u (n, 3), dt (n,)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.uniform(a_lo, a_hi, n)
    e = rng.uniform(0.0, e_hi, n)
    inc = np.arccos(rng.uniform(-1.0, 1.0, n))
    ang = rng.uniform(0.0, 2 * np.pi, (3, n))
    q, u = elements_to_cartesian(mu, a, e, inc, ang[0], ang[1], ang[2])
    dt = np.exp(rng.uniform(np.log(dt_lo), np.log(dt_hi), n))
    return q, u, dt


def learned_workload(n_test: int = 1_048_576, n_disk: int = 65_536, seed: int = 6) -> System:
    """Massless test bodies behind a planetesimal disk with four planets."""
    disk = make_disk("disk64k", seed, n_disk, 1e-8, 15.0, 40.0, "rayleigh", "rayleigh",
                     0.05, 0.025)
    tp = kepler_test(n_test, seed)
    m = np.concatenate([disk.m, tp.m])
    q = np.concatenate([disk.q, tp.q])
    u = np.concatenate([disk.v, tp.v])
    return System("learned", disk.G, disk.m0, m, q, u)


# (size, fan_in, fan_out) of W1, b1, W2, b2, W3, b3; fan_in 0 marks a bias
GUESS_BLOCKS = ((128, 4, 32), (32, 0, 0), (1024, 32, 32), (32, 0, 0), (32, 32, 1), (1, 0, 0))


def guess_init(seed: int = 7) -> np.ndarray:
    """1249 starting parameters (W1, b1, W2, b2, W3, b3 in that order, weight
    matrices row-major with one row per output unit), float32-exact."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for size, fan_in, fan_out in GUESS_BLOCKS:
        if fan_in:
            lim = np.sqrt(6.0 / (fan_in + fan_out))
            parts.append(rng.uniform(-lim, lim, size))
        else:
            parts.append(np.zeros(size))
    w = np.concatenate(parts).astype(np.float32).astype(np.float64)
    assert w.size == 1249
    return w


def two_planet_encounter(n_small: int = 8, seed: int = 3, G: float = 1.0,
                         m0: float = 1.0) -> System:
    rng = np.random.Generator(np.random.PCG64(seed))
    m = np.concatenate([[1e-3, 1e-3], np.full(n_small, 1e-9)])
    a = np.concatenate([[5.2, 5.45], rng.uniform(4.0, 7.0, n_small)])
    e = np.concatenate([[0.0, 0.0], rng.uniform(0, 0.05, n_small)])
    inc = np.concatenate([[0.0, 0.001], rng.uniform(0, 0.02, n_small)])
    ang = rng.uniform(0, 2 * np.pi, (3, n_small + 2))
    ang[:, 0] = 0.0
    ang[:, 1] = [0.0, 0.0, 0.02]
    q, u = elements_to_cartesian(G * m0, a, e, inc, ang[0], ang[1], ang[2])
    return System("two_planets", G, m0, m, q, _to_barycentric(m0, m, u))
