"""Pins of the transition function (Sec. 2.1), the Hermite force/jerk and
integrator (Sec. 2.2) and the interaction corrections (Sec. 2.3 steps 5, 7):
finite differences of the modified Hamiltonians, 4th-order convergence to the
closed-form Kepler orbit, conservation of H'_Kep and angular momentum."""
import math

import numpy as np
import pytest

from paper_1007_3458_amd import inputs


def test_transition_values_and_derivatives(orc):
    rc = 0.7
    assert orc.transition(0.0, rc)[0] == 0.0
    assert orc.transition(0.1 * rc / 1.1 * 0.999, rc) == (0.0, 0.0, 0.0)
    assert orc.transition(rc * 1.0001, rc) == (1.0, 0.0, 0.0)
    s = (0.5 + 0.1) * rc / 1.1  # y = 0.5
    assert orc.transition(s, rc)[0] == pytest.approx(math.sin(math.pi / 4), rel=1e-15)
    h = 1e-6
    for s in np.linspace(0.12 * rc, 0.98 * rc, 17):
        K, Kp, Kpp = orc.transition(s, rc)
        Kph = (orc.transition(s + h, rc)[0] - orc.transition(s - h, rc)[0]) / (2 * h)
        Kpph = (orc.transition(s + h, rc)[1] - orc.transition(s - h, rc)[1]) / (2 * h)
        assert Kp == pytest.approx(Kph, rel=1e-7, abs=1e-9)
        assert Kpp == pytest.approx(Kpph, rel=1e-6, abs=1e-7)


def _set_in_transition_zone(seed, n=5, rc=0.3):
    """n bodies spread so that pair separations fall inside (0.1, 1) r_crit."""
    rng = np.random.Generator(np.random.PCG64(seed))
    base = np.array([5.0, 0.2, 0.0])
    x = base + rng.normal(size=(n, 3)) * 0.12
    u = rng.normal(size=(n, 3)) * 0.1 + np.array([0.0, 0.44, 0.0])
    m = rng.uniform(0.2, 1.0, n) * 1e-3
    return m, x, u, rc


def _hkep_pot(G, mu, m, x, rc, eps, orc):
    """Potential part of H'_Kep (star fixed): -sum mu m/r - sum G m m (1-K(s))/s."""
    E = -np.sum(mu * m / np.linalg.norm(x, axis=1))
    for a in range(len(m)):
        for b in range(a + 1, len(m)):
            s = math.sqrt(np.sum((x[b] - x[a]) ** 2) + eps * eps)
            K = orc.transition(s, rc)[0]
            E -= G * m[a] * m[b] * (1.0 - K) / s
    return E


@pytest.mark.parametrize("eps", [0.0, 1e-3])
def test_hermite_acc_is_gradient_of_hkep(orc, eps):
    G, mu = 1.0, 1.0
    m, x, u, rc = _set_in_transition_zone(1)
    a, _ = orc.hermite_force(m, x, u, G, mu, rc, eps)
    h = 1e-6
    for i in range(len(m)):
        for k in range(3):
            xp = x.copy(); xp[i, k] += h
            xm = x.copy(); xm[i, k] -= h
            dV = (_hkep_pot(G, mu, m, xp, rc, eps, orc) - _hkep_pot(G, mu, m, xm, rc, eps, orc)) / (2 * h)
            assert m[i] * a[i, k] == pytest.approx(-dV, rel=2e-7, abs=1e-12)


def test_hermite_jerk_is_time_derivative_of_acc(orc):
    G, mu, eps = 1.0, 1.0, 1e-4
    m, x, u, rc = _set_in_transition_zone(2)
    _, j = orc.hermite_force(m, x, u, G, mu, rc, eps)
    d = 1e-6
    ap, _ = orc.hermite_force(m, x + d * u, u, G, mu, rc, eps)
    am, _ = orc.hermite_force(m, x - d * u, u, G, mu, rc, eps)
    jfd = (ap - am) / (2 * d)
    assert np.allclose(j, jfd, rtol=1e-6, atol=1e-9 * np.abs(j).max())


def test_hermite_pure_kepler_fourth_order(orc):
    """With r_crit -> 0 every pair has K = 1, W = 0: the Hermite must follow
    the closed-form Kepler orbit, with error ~ h^4 (eta ~ h^2)."""
    mu = 1.0
    a = np.array([1.0, 1.3]); e = np.array([0.3, 0.1])
    ang = np.array([[0.1, 2.0], [0.5, 1.0], [0.2, 3.0]])
    q0, v0 = inputs.elements_to_cartesian(mu, a, e, np.zeros(2), ang[0], ang[1], ang[2])
    T = 2.0
    qe, ve = inputs.elements_to_cartesian(mu, a, e, np.zeros(2), ang[0], ang[1],
                                          ang[2] + np.sqrt(mu / a ** 3) * T)
    m = np.array([1e-3, 1e-3])
    errs = []
    for eta in (0.02, 0.005):
        p = orc.make_params(eta=eta, eta_s=0.01, epsH=0.0)
        q1, v1, ns = orc.hermite_set([0, 1], m, q0, v0, p, 1e-12, T)
        assert ns > 0
        errs.append(np.max(np.linalg.norm(q1 - qe, axis=1)))
    ratio = errs[0] / errs[1]
    # eta -> eta/4 halves h: 4th order => error / 16 (allow 10..24)
    assert 10.0 < ratio < 24.0, (errs, ratio)


def _pair_encounter(dy, rel):
    m = np.array([1e-3, 1e-3])
    rH = 5.0 * np.cbrt(1e-3 / 3)
    q0 = np.array([[5.0, 0.0, 0.0], [5.0 + 0.6 * rH, dy, 0.0]])
    vc = math.sqrt(1.0 / 5.0)
    v0 = np.array([[0.0, vc, 0.0], [0.0, vc + rel, 0.0]])
    return m, q0, v0, rH


def test_hermite_conserves_hkep_inside_transition_zone(orc):
    """Sec. 2.2 claim: H'_Kep is conserved through a close approach.  While
    the pair stays inside 0 < y < 1 the force is smooth: the error is small at
    eta = 0.02 and falls at 4th order (eta ~ h^2) when eta is tightened."""
    m, q0, v0, rH = _pair_encounter(-0.05, 0.2)
    errs = []
    for eta in (0.02, 0.005):
        p = orc.make_params(eta=eta, eta_s=eta / 2, epsH=1e-8)
        E0 = orc.hkep_set([0, 1], m, q0, v0, p, rH)
        L0 = orc.angmom(m, q0, v0)
        q1, v1, ns = orc.hermite_set([0, 1], m, q0, v0, p, rH, 0.5)
        for q in (q0, q1):
            y = 1.1 * np.linalg.norm(q[1] - q[0]) / rH - 0.1
            assert 0.0 < y < 1.0
        errs.append(abs(orc.hkep_set([0, 1], m, q1, v1, p, rH) / E0 - 1))
        L1 = orc.angmom(m, q1, v1)
        assert ns >= 5
        assert np.linalg.norm(L1 - L0) < 1e-9 * np.linalg.norm(L0)  # truncation-level
    assert errs[0] < 2e-8
    assert errs[0] / errs[1] > 10.0, errs


def test_hermite_energy_through_r_crit_converges(orc):
    """Crossing s = r_crit (y = 1) the jerk of the paper's sine transition
    jumps (K'' is discontinuous there), so the local order drops; the H'_Kep
    and angular-momentum errors must still fall as the accuracy parameters
    are tightened."""
    m, q0, v0, rH = _pair_encounter(-0.8, 0.6)
    errs, lerrs = [], []
    for eta in (0.02, 0.00125):
        p = orc.make_params(eta=eta, eta_s=eta / 2, epsH=1e-8)
        E0 = orc.hkep_set([0, 1], m, q0, v0, p, rH)
        q1, v1, ns = orc.hermite_set([0, 1], m, q0, v0, p, rH, 3.0)
        errs.append(abs(orc.hkep_set([0, 1], m, q1, v1, p, rH) / E0 - 1))
        L0, L1 = orc.angmom(m, q0, v0), orc.angmom(m, q1, v1)
        lerrs.append(np.linalg.norm(L1 - L0) / np.linalg.norm(L0))
    assert errs[1] < errs[0] / 8, errs
    assert lerrs[1] < lerrs[0] / 8, lerrs


def test_correction_leaves_hprime_int_force(orc):
    """Sec. 2.3 steps 5 and 7: full kick minus the W-weighted correction equals
    the force of H'_Int (finite differences of its potential)."""
    G = 1.0
    m, x, u, rc = _set_in_transition_zone(3, n=6)
    mem = np.array([0, 2, 3, 5], np.int32)  # 1 and 4 are not members
    a_full = orc.accel(G, m, x)
    dv = orc.correct_set(mem, m, x, np.zeros_like(x), G, rc, 1.0)  # = -sum W-weighted
    a_int = a_full + dv
    inset = np.zeros(len(m), bool); inset[mem] = True

    def hint_prime(xx):
        E = 0.0
        for i in range(len(m)):
            for j in range(i + 1, len(m)):
                q = np.linalg.norm(xx[j] - xx[i])
                K = orc.transition(q, rc)[0] if (inset[i] and inset[j]) else 1.0
                E -= G * m[i] * m[j] * K / q
        return E

    h = 1e-6
    for i in range(len(m)):
        for k in range(3):
            xp = x.copy(); xp[i, k] += h
            xm = x.copy(); xm[i, k] -= h
            dV = (hint_prime(xp) - hint_prime(xm)) / (2 * h)
            assert m[i] * a_int[i, k] == pytest.approx(-dV, rel=1e-6, abs=1e-13)
