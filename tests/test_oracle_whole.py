"""Pins of the whole-system Hermite rule (Sec. 2.3, after the steps): when a
set of an encounter holds two planets, the step integrates every body with
the Hermite.  Reading: one set of all bodies with an infinite r_crit, so
K = 0 and W = 1 for every pair; the corrections take back both half kicks
and the step becomes E_Dft(τ/2) Φ(τ) E_Dft(τ/2) with Φ the Hermite flow of
H_Kep + H_Int (all pairs, star fixed).  Pinned by: when the rule fires and
when it does not, and agreement of the step with an independent RK4
integration of the same equations between the two drifts."""
import numpy as np
import pytest

from paper_1007_3458_amd import inputs


def _two_planet_system(n_small=8, seed=3):
    s = inputs.two_planet_encounter(n_small, seed)
    return s.m, s.h, s.q, s.v


def test_rule_fires_only_for_two_planets_in_one_set(orc):
    m, h, q, v = _two_planet_system()
    p_on = orc.make_params(planet_mass=1e-4)
    q1, v1, r = orc.step(p_on, 0.05, m, h, q, v)
    st = r.stats
    assert st["n_encounters"] > 0 and st["whole_system"] == 1
    assert st["n_sets"] == 1 and np.all(r.label == 0)
    # planets lighter than the threshold: the ordinary hybrid step
    q2, v2, r2 = orc.step(orc.make_params(planet_mass=2e-3), 0.05, m, h, q, v)
    assert r2.stats["whole_system"] == 0
    q3, v3, r3 = orc.step(orc.make_params(), 0.05, m, h, q, v)
    assert np.array_equal(q2, q3) and np.array_equal(v2, v3)
    # a single planet among planetesimals never triggers it
    s = inputs.make_disk("crowd", 5, 60, 1e-6, 4.5, 6.0, "uniform", "uniform", 0.05, 0.01)
    pm = orc.make_params(planet_mass=5e-4)   # only the first planet (1e-3) qualifies
    _, _, r4 = orc.step(pm, 0.05, s.m, s.h, s.q, s.v)
    assert r4.stats["n_encounters"] > 0 and r4.stats["whole_system"] == 0


def _rhs(mu, m, q, v):
    d = q[None, :, :] - q[:, None, :]          # d[i, j] = q_j - q_i
    r2 = (d ** 2).sum(-1) + 1e-16              # the Hermite's in-set softening eps_H = 1e-8
    np.fill_diagonal(r2, 1.0)
    f = m[None, :, None] * d / r2[:, :, None] ** 1.5
    for i in range(len(m)):
        f[i, i] = 0.0
    r = np.linalg.norm(q, axis=1)
    acc = -mu * q / r[:, None] ** 3 + f.sum(1)
    return v, acc


def _rk4(mu, m, q, v, T, nsteps):
    h = T / nsteps
    for _ in range(nsteps):
        k1q, k1v = _rhs(mu, m, q, v)
        k2q, k2v = _rhs(mu, m, q + h / 2 * k1q, v + h / 2 * k1v)
        k3q, k3v = _rhs(mu, m, q + h / 2 * k2q, v + h / 2 * k2v)
        k4q, k4v = _rhs(mu, m, q + h * k3q, v + h * k3v)
        q = q + h / 6 * (k1q + 2 * k2q + 2 * k3q + k4q)
        v = v + h / 6 * (k1v + 2 * k2v + 2 * k3v + k4v)
    return q, v


def test_whole_system_step_is_drift_hermite_drift(orc):
    """E_Dft(tau/2), then the full Newtonian flow (star fixed, W = 1 for all
    pairs) over tau, then E_Dft(tau/2): RK4 with 4000 substeps reproduces
    the step to the Hermite's truncation error."""
    m, h, q, v = _two_planet_system()
    tau = 0.05
    p = orc.make_params(planet_mass=1e-4)
    q1, v1, r = orc.step(p, tau, m, h, q, v)
    assert r.stats["whole_system"] == 1
    qm = orc.drift(1.0, m, q, v, tau / 2)
    qe, ve = _rk4(1.0, m, qm, v, tau, 4000)
    qe = orc.drift(1.0, m, qe, ve, tau / 2)
    assert np.max(np.linalg.norm(q1 - qe, axis=1) / np.linalg.norm(qe, axis=1)) < 1e-9
    assert np.max(np.linalg.norm(v1 - ve, axis=1) / np.linalg.norm(ve, axis=1)) < 1e-8
    # the ordinary hybrid step differs from that flow by far more
    q2, v2, _ = orc.step(orc.make_params(), tau, m, h, q, v)
    assert np.max(np.linalg.norm(q2 - qe, axis=1)) > 100 * np.max(np.linalg.norm(q1 - qe, axis=1))


def test_whole_system_energy_across_planet_encounter(orc):
    """Over a close planet-planet passage the whole-system step keeps the
    energy error below that of the ordinary hybrid step."""
    m, h, q, v = _two_planet_system(4, seed=7)
    G, m0 = 1.0, 1.0
    E0 = orc.energy(G, m0, m, q, v)
    worst = {}
    for pm in (0.0, 1e-4):
        p = orc.make_params(planet_mass=pm)
        qq, vv = q, v
        w = 0.0
        for _ in range(60):
            qq, vv, _ = orc.step(p, 0.05, m, h, qq, vv)
            w = max(w, abs(orc.energy(G, m0, m, qq, vv) / E0 - 1))
        worst[pm] = w
    assert worst[1e-4] < 0.01 * worst[0.0]
