"""Pins of the oracle's drift, kick and energy (Sec. 2, eqs. for H_Dft, H_Kep,
H_Int) against closed forms, finite differences of the Hamiltonian and
physical invariants."""
import numpy as np
import pytest

from paper_1007_3458_amd import inputs


def _rand_system(n, seed, spread=3.0, mass=1e-3):
    rng = np.random.Generator(np.random.PCG64(seed))
    q = rng.normal(size=(n, 3)) * spread + np.array([10.0, 0, 0])
    v = rng.normal(size=(n, 3)) * 0.2
    m = rng.uniform(0.1, 1.0, n) * mass
    return m, q, v


def test_drift_closed_form(orc):
    m, q, v = _rand_system(17, 1)
    P = (m[:, None] * v).sum(0)
    q1 = orc.drift(1.7, m, q, v, 0.3)
    assert np.allclose(q1, q + 0.3 * P / 1.7, rtol=0, atol=1e-15)
    # zero total momentum -> no motion
    v0 = v - P / m.sum()
    q2 = orc.drift(1.7, m, q, v0 * 0 + (v0 - (m[:, None] * v0).sum(0) / m.sum()), 0.3)
    assert np.allclose(q2, q, rtol=0, atol=1e-15)


def test_drift_preserves_angular_momentum(orc):
    m, q, v = _rand_system(40, 2)
    L0 = orc.angmom(m, q, v)
    q1 = orc.drift(1.0, m, q, v, 0.77)
    L1 = orc.angmom(m, q1, v)
    assert np.linalg.norm(L1 - L0) <= 1e-15 * np.linalg.norm(L0) * 10


def test_accel_two_body_closed_form(orc):
    q = np.array([[1.0, 2.0, 3.0], [4.0, 6.0, 3.0]])  # separation (3,4,0), |d| = 5
    m = np.array([2.0, 3.0])
    a = orc.accel(0.5, m, q)
    assert np.allclose(a[0], 0.5 * 3.0 * np.array([3.0, 4.0, 0.0]) / 125.0, rtol=1e-15)
    assert np.allclose(a[1], -0.5 * 2.0 * np.array([3.0, 4.0, 0.0]) / 125.0, rtol=1e-15)


def _hint(G, m, q):
    """H_Int = -sum_{i<j} G m_i m_j / |Q_i - Q_j| (numpy, pairwise)."""
    d = q[:, None, :] - q[None, :, :]
    r = np.sqrt((d ** 2).sum(-1))
    iu = np.triu_indices(len(m), 1)
    return -G * np.sum(m[iu[0]] * m[iu[1]] / r[iu])


def test_accel_is_minus_gradient_of_hint(orc):
    """m_i a_i = -dH_Int/dQ_i (central finite differences, 4th order)."""
    m, q, v = _rand_system(12, 3, spread=1.0, mass=1.0)
    G = 1.0
    a = orc.accel(G, m, q)
    h = 1e-4
    for i in range(len(m)):
        for k in range(3):
            qs = []
            for s in (-2, -1, 1, 2):
                qq = q.copy()
                qq[i, k] += s * h
                qs.append(_hint(G, m, qq))
            dH = (qs[0] - 8 * qs[1] + 8 * qs[2] - qs[3]) / (12 * h)
            assert abs(m[i] * a[i, k] + dH) <= 1e-8 * max(1.0, abs(dH))


def test_kick_momentum_angular_momentum_and_zero_separation(orc):
    m, q, v = _rand_system(64, 4)
    a = orc.accel(1.0, m, q)
    F = m[:, None] * a
    assert np.linalg.norm(F.sum(0)) <= 1e-15 * np.abs(F).sum() * 10
    L0 = orc.angmom(m, q, v)
    v1 = orc.kick(1.0, m, q, v, 0.5)
    L1 = orc.angmom(m, q, v1)
    assert np.linalg.norm(L1 - L0) <= 1e-14 * np.linalg.norm(L0)
    # a coincident pair contributes nothing (degenerate input)
    q2 = q.copy()
    q2[1] = q2[0]
    a2 = orc.accel(1.0, m, q2)
    assert np.all(np.isfinite(a2))


def test_accel_permutation_invariance(orc):
    m, q, v = _rand_system(50, 5)
    perm = np.random.Generator(np.random.PCG64(9)).permutation(50)
    a = orc.accel(1.0, m, q)
    ap = orc.accel(1.0, m[perm], q[perm])
    assert np.max(np.abs(ap - a[perm])) <= 1e-14 * np.max(np.abs(a))


def test_energy_equals_inertial_newtonian_energy(orc):
    """The DH Hamiltonian equals the barycentric-frame Newtonian energy of the
    star + bodies system rebuilt in inertial coordinates."""
    s = inputs.small()
    G, m0 = s.G, s.m0
    E = orc.energy(G, m0, s.m, s.q, s.v)
    Mtot = m0 + s.m.sum()
    x0 = -(s.m[:, None] * s.q).sum(0) / Mtot   # star position (centre of mass at 0)
    u0 = -(s.m[:, None] * s.v).sum(0) / m0      # star velocity (zero total momentum)
    X = np.vstack([x0, s.q + x0])
    U = np.vstack([u0, s.v])
    M = np.concatenate([[m0], s.m])
    assert np.allclose((M[:, None] * X).sum(0), 0, atol=1e-15)
    kin = 0.5 * np.sum(M * np.sum(U ** 2, 1))
    d = X[:, None, :] - X[None, :, :]
    r = np.sqrt((d ** 2).sum(-1))
    iu = np.triu_indices(len(M), 1)
    pot = -G * np.sum(M[iu[0]] * M[iu[1]] / r[iu])
    assert abs(E - (kin + pot)) <= 1e-14 * abs(E)


def test_energy_two_body_value(orc):
    q = np.array([[2.0, 0.0, 0.0]])
    v = np.array([[0.0, 0.5, 0.0]])
    m = np.array([0.25])
    E = orc.energy(1.0, 1.0, m, q, v)
    assert E == pytest.approx(0.5 * 0.25 * 0.25 + (0.25 * 0.5) ** 2 / 2.0 - 0.25 / 2.0, rel=1e-15)


def test_prepass_semimajor_axis_and_escape_speed(orc):
    mu = 1.0
    a = np.array([5.2, 9.5, 30.1])
    e = np.array([0.0, 0.3, 0.8])
    q, u = inputs.elements_to_cartesian(mu, a, e, np.zeros(3), np.zeros(3), np.zeros(3),
                                        np.array([0.3, 1.0, 2.0]))
    A, ve = orc.prepass(mu, q, u)
    assert np.allclose(A, a, rtol=1e-13)
    assert np.allclose(ve, np.sqrt(2 * mu / np.linalg.norm(q, axis=1)), rtol=1e-15)
    # unbound: A falls back to r
    qh = np.array([[1.0, 0, 0]])
    vh = np.array([[0, 2.0, 0]])
    A2, _ = orc.prepass(mu, qh, vh)
    assert A2[0] == 1.0


def test_accel_rows_equals_full_accel(orc):
    m, q, v = _rand_system(40, 6)
    rows = np.array([0, 7, 39, 7], np.int64)
    assert np.array_equal(orc.accel_rows(1.0, m, q, rows), orc.accel(1.0, m, q)[rows])
