"""Pins of the oracle's whole hybrid step (Sec. 2.3) through properties the
method fixes: exact Kepler motion of test particles, time reversibility of
the symmetric composition (Sec. 2, eq. for the second-order operator
product) with encounters off, angular-momentum conservation, the τ² scaling
of the energy error (Sec. 3), invariance under reordering the bodies (Sec. 2,
DH coordinates do not depend on the particle order) and the bounded energy
error of the small disk; and convergence to the exact N-body flow (an
independent high-accuracy integration of Newton's equations) at the
method's order while an encounter set is active.

The composite step itself has no worked numeric example in the paper; these
properties are its pins."""
import numpy as np
import pytest

from paper_1007_3458_amd import inputs


def test_massless_system_step_is_exact_kepler(orc):
    """All masses zero: drift and kick vanish and no pair can be an encounter,
    so 1000 steps equal the closed-form orbits from the elements."""
    mu = 1.0
    rng = np.random.Generator(np.random.PCG64(8))
    n = 12
    a = rng.uniform(1.0, 30.0, n); e = rng.uniform(0, 0.6, n); inc = rng.uniform(0, 0.3, n)
    ang = rng.uniform(0, 2 * np.pi, (3, n))
    q, v = inputs.elements_to_cartesian(mu, a, e, inc, ang[0], ang[1], ang[2])
    m = np.zeros(n); h = np.zeros(n)
    p = orc.make_params()
    tau, ns = 0.05, 1000
    for _ in range(ns):
        q, v, r = orc.step(p, tau, m, h, q, v)
        assert r.stats["n_encounters"] == 0
    qe, ve = inputs.elements_to_cartesian(mu, a, e, inc, ang[0], ang[1],
                                          ang[2] + np.sqrt(mu / a ** 3) * tau * ns)
    assert np.max(np.linalg.norm(q - qe, axis=1) / np.linalg.norm(qe, axis=1)) < 1e-12
    assert np.max(np.linalg.norm(v - ve, axis=1) / np.linalg.norm(ve, axis=1)) < 1e-12


def test_reversibility_without_encounters(orc):
    s = inputs.small()
    p = orc.make_params(aE=0.0)
    q, v = s.q, s.v
    for _ in range(20):
        q, v, r = orc.step(p, 0.05, s.m, s.h, q, v)
        assert r.stats["n_encounters"] == 0
    for _ in range(20):
        q, v, _ = orc.step(p, -0.05, s.m, s.h, q, v)
    assert np.max(np.abs(q - s.q)) < 1e-12 * np.max(np.abs(s.q))
    assert np.max(np.abs(v - s.v)) < 1e-12 * np.max(np.abs(s.v))


def test_angular_momentum_conserved_with_encounters(orc):
    s = _crowded(96, 5)
    p = orc.make_params()
    L0 = orc.angmom(s.m, s.q, s.v)
    q, v = s.q, s.v
    nenc = 0
    for _ in range(40):
        q, v, r = orc.step(p, 0.05, s.m, s.h, q, v)
        nenc += r.stats["n_encounters"]
    L1 = orc.angmom(s.m, q, v)
    assert nenc > 0
    # the Hermite conserves L to truncation error only; the rest to rounding
    assert np.linalg.norm(L1 - L0) < 1e-9 * np.linalg.norm(L0)
    p0 = orc.make_params(aE=0.0)
    q, v = s.q, s.v
    for _ in range(40):
        q, v, _ = orc.step(p0, 0.05, s.m, s.h, q, v)
    assert np.linalg.norm(orc.angmom(s.m, q, v) - L0) < 1e-14 * np.linalg.norm(L0)


def _crowded(n, seed):
    return inputs.make_disk("crowd", seed, n - 4, 1e-6, 4.5, 6.0, "uniform", "uniform", 0.05, 0.01)


def _max_de(orc, s, p, tau, T):
    E0 = orc.energy(s.G, s.m0, s.m, s.q, s.v)
    q, v = s.q, s.v
    worst = 0.0
    for _ in range(int(round(T / tau))):
        q, v, _ = orc.step(p, tau, s.m, s.h, q, v)
        worst = max(worst, abs(orc.energy(s.G, s.m0, s.m, q, v) / E0 - 1))
    return worst


def test_energy_error_scales_as_tau_squared(orc):
    """Sec. 3: smaller steps conserve energy better, the method being second
    order (over a fixed span the maximum error ~ tau^2)."""
    s = inputs.small()
    p = orc.make_params()
    e1 = _max_de(orc, s, p, 0.2, 40.0)
    e2 = _max_de(orc, s, p, 0.1, 40.0)
    slope = np.log2(e1 / e2)
    assert 1.7 < slope < 2.3, (e1, e2, slope)


def test_permutation_invariance_of_step(orc):
    s = _crowded(64, 2)
    p = orc.make_params()
    perm = np.random.Generator(np.random.PCG64(3)).permutation(s.n)
    sp = s.permuted(perm)
    q, v, r = orc.step(p, 0.05, s.m, s.h, s.q, s.v)
    qp, vp, rp = orc.step(p, 0.05, sp.m, sp.h, sp.q, sp.v)
    assert r.stats["n_encounters"] > 0
    assert np.max(np.abs(qp - q[perm])) < 1e-13 * np.max(np.abs(q))
    assert np.max(np.abs(vp - v[perm])) < 1e-13 * np.max(np.abs(v))


def test_small_disk_energy_bounded(orc):
    s = inputs.small()
    assert _max_de(orc, s, orc.make_params(), 0.05, 50.0) < 1e-8


def _newton_flow(m0, m, q, v, T, G=1.0):
    """The exact flow of the N-body problem over T from a DH state
    (heliocentric positions, barycentric velocities; Sec. 2): Newton's
    equations of all bodies and the star in the barycentric frame, integrated
    by scipy's DOP853 at tolerances far below the step's errors, mapped back
    to DH coordinates."""
    from scipy.integrate import solve_ivp
    mm = np.concatenate([[m0], m])
    x0 = -(m[:, None] * q).sum(0) / mm.sum()
    X = np.vstack([x0, x0 + q])
    U = np.vstack([-(m[:, None] * v).sum(0) / m0, v])
    nb = len(mm)

    def rhs(t, y):
        X = y[:3 * nb].reshape(-1, 3)
        A = np.zeros_like(X)
        for i in range(nb):
            d = np.delete(X, i, 0) - X[i]
            r3 = ((d * d).sum(1)) ** 1.5
            A[i] = (G * np.delete(mm, i)[:, None] * d / r3[:, None]).sum(0)
        return np.concatenate([y[3 * nb:], A.ravel()])

    sol = solve_ivp(rhs, (0.0, T), np.concatenate([X.ravel(), U.ravel()]), method="DOP853",
                    rtol=1e-13, atol=1e-16)
    y = sol.y[:, -1]
    X, U = y[:3 * nb].reshape(-1, 3), y[3 * nb:].reshape(-1, 3)
    return X[1:] - X[0], U[1:]


def test_step_converges_to_newton_flow_through_an_encounter(orc):
    """Two bodies of 1e-4 solar masses 0.015 apart (inside r_crit: the
    transition's ramp, Sec. 2.1) form one encounter set, so a step runs the
    corrections and the Hermite (Sec. 2.3 steps 5-7).  Against the exact
    flow its one-step error falls as tau^3 in the velocities and faster in
    the positions (a second-order method), which a wrong sign or a dropped
    term in the corrections, the weights or the Hermite would turn into
    O(tau) or O(tau^2); and it is below the error of the same step with the
    encounter switch off (the close pair then split between the kick and
    the Kepler drift)."""
    m0 = 1.0
    m = np.array([1e-4, 1e-4])
    h = np.cbrt(m / (3.0 * m0))
    q = np.array([[1.0, 0.0, 0.0], [1.0, 0.015, 0.002]])
    v = np.array([[0.0, 1.0, 0.0], [0.004, 1.0, 0.0]])
    p = orc.make_params()
    p_off = orc.make_params(aE=1e-9)
    dq, dv = [], []
    for T in (0.04, 0.02, 0.01):
        qe, ve = _newton_flow(m0, m, q, v, T)
        qo, vo, r = orc.step(p, T, m, h, q, v)
        assert r.rc == 0 and r.stats["n_encounters"] == 1 and r.stats["max_set"] == 2
        qf, vf, rf = orc.step(p_off, T, m, h, q, v)
        assert rf.stats["n_encounters"] == 0
        dq.append(np.abs(qo - qe).max())
        dv.append(np.abs(vo - ve).max())
        assert dv[-1] < 0.5 * np.abs(vf - ve).max()
    for k in range(2):
        assert 6.0 < dv[k] / dv[k + 1] < 11.0, dv
        assert dq[k] / dq[k + 1] > 8.0, dq
