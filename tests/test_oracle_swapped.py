"""Pins of the oracle's encounter-free step with the Keplerian and interaction
operators swapped (Sec. 2, after the second-order composition):
E_Dft(τ/2) E_Kep(τ/2) E_Int(τ) E_Kep(τ/2) E_Dft(τ/2).  What fixes it: exact
Kepler motion when every mass is zero, time reversibility and second order
of a symmetric composition, conservation of angular momentum (every operator
conserves it), agreement with the standard ordering to O(τ²) over a fixed
span, and invariance under reordering the bodies."""
import numpy as np

from paper_1007_3458_amd import inputs


def test_massless_system_is_exact_kepler(orc):
    mu = 1.0
    rng = np.random.Generator(np.random.PCG64(18))
    n = 12
    a = rng.uniform(1.0, 30.0, n); e = rng.uniform(0, 0.6, n); inc = rng.uniform(0, 0.3, n)
    ang = rng.uniform(0, 2 * np.pi, (3, n))
    q, v = inputs.elements_to_cartesian(mu, a, e, inc, ang[0], ang[1], ang[2])
    p = orc.make_params()
    tau, ns = 0.05, 1000
    q1, v1, fails, _ = orc.step_swapped(p, tau, np.zeros(n), q, v, ns)
    assert fails == 0
    qe, ve = inputs.elements_to_cartesian(mu, a, e, inc, ang[0], ang[1],
                                          ang[2] + np.sqrt(mu / a ** 3) * tau * ns)
    assert np.max(np.linalg.norm(q1 - qe, axis=1) / np.linalg.norm(qe, axis=1)) < 1e-12
    assert np.max(np.linalg.norm(v1 - ve, axis=1) / np.linalg.norm(ve, axis=1)) < 1e-12


def test_reversibility(orc):
    s = inputs.small()
    p = orc.make_params()
    q, v, _, _ = orc.step_swapped(p, 0.05, s.m, s.q, s.v, 20)
    q, v, _, _ = orc.step_swapped(p, -0.05, s.m, q, v, 20)
    assert np.max(np.abs(q - s.q)) < 1e-12 * np.max(np.abs(s.q))
    assert np.max(np.abs(v - s.v)) < 1e-12 * np.max(np.abs(s.v))


def test_angular_momentum_conserved(orc):
    s = inputs.make_disk("crowd", 5, 92, 1e-6, 4.5, 6.0, "uniform", "uniform", 0.05, 0.01)
    p = orc.make_params()
    L0 = orc.angmom(s.m, s.q, s.v)
    q, v, _, _ = orc.step_swapped(p, 0.05, s.m, s.q, s.v, 40)
    assert np.linalg.norm(orc.angmom(s.m, q, v) - L0) < 1e-14 * np.linalg.norm(L0)


def _max_de(orc, s, tau, T):
    p = orc.make_params()
    E0 = orc.energy(s.G, s.m0, s.m, s.q, s.v)
    q, v = s.q, s.v
    worst = 0.0
    for _ in range(int(round(T / tau))):
        q, v, _, _ = orc.step_swapped(p, tau, s.m, q, v)
        worst = max(worst, abs(orc.energy(s.G, s.m0, s.m, q, v) / E0 - 1))
    return worst


def test_energy_error_scales_as_tau_squared(orc):
    s = inputs.small()
    e1 = _max_de(orc, s, 0.2, 40.0)
    e2 = _max_de(orc, s, 0.1, 40.0)
    slope = np.log2(e1 / e2)
    assert 1.7 < slope < 2.3, (e1, e2, slope)


def test_agrees_with_standard_ordering_to_second_order(orc):
    """Both orderings are second-order approximations of the same flow, so
    their difference over a fixed span shrinks as tau^2."""
    s = inputs.small()
    p_std = orc.make_params(aE=0.0)     # no encounters: the plain DH step
    p = orc.make_params()
    diffs = []
    for tau in (0.2, 0.1):
        ns = int(round(20.0 / tau))
        q1, v1, _, _ = orc.step_swapped(p, tau, s.m, s.q, s.v, ns)
        q2, v2 = s.q, s.v
        for _ in range(ns):
            q2, v2, r = orc.step(p_std, tau, s.m, s.h, q2, v2)
            assert r.stats["n_encounters"] == 0
        diffs.append(np.max(np.linalg.norm(q1 - q2, axis=1)))
    slope = np.log2(diffs[0] / diffs[1])
    assert 1.7 < slope < 2.3, (diffs, slope)


def test_permutation_invariance(orc):
    s = inputs.make_disk("crowd", 2, 60, 1e-6, 4.5, 6.0, "uniform", "uniform", 0.05, 0.01)
    perm = np.random.Generator(np.random.PCG64(4)).permutation(s.n)
    sp = s.permuted(perm)
    p = orc.make_params()
    q, v, _, _ = orc.step_swapped(p, 0.05, s.m, s.q, s.v, 3)
    qp, vp, _, _ = orc.step_swapped(p, 0.05, sp.m, sp.q, sp.v, 3)
    assert np.max(np.abs(qp - q[perm])) < 1e-13 * np.max(np.abs(q))
    assert np.max(np.abs(vp - v[perm])) < 1e-13 * np.max(np.abs(v))
