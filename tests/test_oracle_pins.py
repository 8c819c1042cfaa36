"""Pins of oracle parts that the other pin files reach only indirectly:

* r_crit of each encounter set (Sec. 2.2, the equation for r_crit: a_H times
  the largest Hill radius h_i a_i in the set), checked against the semi-major
  axes the orbits were drawn with, not against the oracle's own pre-pass;
* the angular-momentum checker L = sum m_i Q_i x v_i against hand-computed
  values and the two-body closed form sqrt(mu a (1 - e^2)) along the orbit
  normal;
* the crude sweep of Sec. 2.4 against brute force: the fine test over every
  pair finds no encounter the two-stage sweep misses, on the small disk, the
  16k-body disk (all pairs) and the 131k-body disk (every pair of sampled
  rows); and, independently of the predicate's formula, every pair whose
  straight-line relative motion comes within a_E mutual Hill radii during the
  step is a candidate.
"""
import numpy as np
import pytest

from paper_1007_3458_amd import inputs

MU = 1.0


def _mirrored(m, a, e, inc, Om, om, M):
    """Bodies from elements, each followed by its point reflection (-Q, -v):
    the reflection is an orbit with the same a and e, and the barycentric
    momentum of every pair is exactly zero, so the first drift of a step
    moves nothing and the step's Hill radii see the drawn orbits."""
    q, u = inputs.elements_to_cartesian(MU, a, e, inc, Om, om, M)
    n = len(m)
    Q = np.empty((2 * n, 3)); V = np.empty((2 * n, 3))
    Q[0::2] = q; Q[1::2] = -q
    V[0::2] = u; V[1::2] = -u
    mm = np.repeat(np.asarray(m, float), 2)
    aa = np.repeat(np.asarray(a, float), 2)
    return mm, Q, V, aa


def test_rcrit_per_set_from_drawn_elements(orc):
    """Two encounter sets of unequal masses and semi-major axes, placed at the
    pericentres of their orbits a few tenths apart.  In set A the largest
    h_i a_i belongs to the lightest body (largest a); in set B to the
    heaviest.  r_crit must equal a_H max h_i a_i with the drawn a_i: using
    h_i alone, the minimum, or a_E in place of a_H fails."""
    # set A near angle 0 (r = 5), set B near angle 2 (r = 12), two lone bodies
    m = np.array([1e-4, 1e-6, 3e-5, 2e-5, 4e-7, 1e-8, 1e-8])
    a = np.array([5.0, 30.0, 8.0, 12.0, 20.0, 25.0, 40.0])
    e = 1.0 - np.array([5.0, 5.0, 5.0, 12.0, 12.0, 25.0, 40.0]) / a  # pericentre distances
    om = np.array([0.0, 0.05, -0.05, 2.0, 2.02, 4.0, 1.0])
    zeros = np.zeros(7)
    mm, Q, V, aa = _mirrored(m, a, e, zeros, zeros, om, zeros)
    h = np.cbrt(mm / 3.0)
    aE, aH = 3.0, 1.7
    p = orc.make_params(aE=aE, aH=aH)
    tau = 0.05
    _, _, r = orc.step(p, tau, mm, h, Q, V)
    # body k of the list is index 2k, its mirror 2k + 1
    setA, setB = [0, 2, 4], [6, 8]
    want_sets = [setA, [x + 1 for x in setA], setB, [x + 1 for x in setB]]
    lab = r.label
    for sset in want_sets:
        assert np.all(lab[sset] == min(sset)), (sset, lab)
    assert np.all(lab[10:] == -1)
    assert r.stats["n_sets"] == 4
    hA = np.cbrt(m / 3.0) * a
    want_A = aH * max(hA[0], hA[1], hA[2])
    want_B = aH * max(hA[3], hA[4])
    assert np.argmax(hA[:3]) == 1 and np.argmax(hA[3:5]) == 0
    want = np.array([want_A, want_A, want_B, want_B])
    assert np.allclose(r.rcrit, want, rtol=1e-12, atol=0.0), (r.rcrit, want)
    # the mirrored sets see the same orbits, bit for bit
    assert r.rcrit[0] == r.rcrit[1] and r.rcrit[2] == r.rcrit[3]
    # the alternatives a wrong r_crit would produce are far from it
    for wrong in (aH * np.cbrt(m[:3] / 3.0).max(), aH * hA[:3].min(), aE * hA[:3].max()):
        assert abs(wrong / want_A - 1.0) > 0.05


def test_rcrit_is_infinite_for_whole_system_sets(orc):
    """Sec. 2.3, after the steps: two planets in one set make the whole system
    one set whose r_crit is infinite (every pair at full weight)."""
    s = inputs.two_planet_encounter(6)
    p = orc.make_params(planet_mass=1e-4)
    _, _, r = orc.step(p, 0.05, s.m, s.h, s.q, s.v)
    assert r.stats["whole_system"] == 1
    assert r.rcrit.shape == (1,) and np.isinf(r.rcrit[0])


def test_angmom_hand_values(orc):
    m = np.array([2.0, 3.0])
    q = np.array([[1.0, 0.0, 0.0], [0.0, 2.0, 0.0]])
    v = np.array([[0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    # 2 (x x y) + 3 (2y x z) = 2 z + 6 x
    assert np.array_equal(orc.angmom(m, q, v), np.array([6.0, 0.0, 2.0]))
    # every component at once: (1,2,3) x (4,5,6) = (-3, 6, -3)
    L = orc.angmom(np.array([0.5]), np.array([[1.0, 2.0, 3.0]]), np.array([[4.0, 5.0, 6.0]]))
    assert np.array_equal(L, np.array([-1.5, 3.0, -1.5]))
    # a massless body carries none
    assert np.array_equal(orc.angmom(np.zeros(1), q[:1], v[:1]), np.zeros(3))


def test_angmom_two_body_closed_form(orc):
    """Each orbit's specific angular momentum is sqrt(mu a (1 - e^2)) along
    (sin i sin Om, -sin i cos Om, cos i), whatever the anomaly."""
    rng = np.random.Generator(np.random.PCG64(21))
    n = 50
    a = rng.uniform(0.5, 40.0, n); e = rng.uniform(0.0, 0.9, n); inc = rng.uniform(0.0, 3.0, n)
    Om, om, M = rng.uniform(0, 2 * np.pi, (3, n))
    m = rng.uniform(1e-9, 1e-3, n)
    q, u = inputs.elements_to_cartesian(MU, a, e, inc, Om, om, M)
    nhat = np.stack([np.sin(inc) * np.sin(Om), -np.sin(inc) * np.cos(Om), np.cos(inc)], 1)
    Lk = (m * np.sqrt(MU * a * (1 - e * e)))[:, None] * nhat
    for k in range(n):
        Lo = orc.angmom(m[k:k + 1], q[k:k + 1], u[k:k + 1])
        assert np.allclose(Lo, Lk[k], rtol=0, atol=1e-13 * np.linalg.norm(Lk[k]))
    assert np.allclose(orc.angmom(m, q, u), Lk.sum(0), rtol=0, atol=1e-13 * np.abs(Lk).sum())


def _sweep_states(orc, s, tau, kick=True):
    """(q0, v0, q1, v1, A, ve) of the step's encounter search: drift tau/2,
    Hill terms at the drifted state, the first half kick (skipped on request:
    the comparison below holds for any state), Kepler over tau."""
    q = orc.drift(s.m0, s.m, s.q, s.v, tau / 2)
    A, ve = orc.prepass(s.G * s.m0, q, s.v)
    v0 = orc.kick(s.G, s.m, q, s.v, tau / 2) if kick else s.v
    q1, v1, _, fails = orc.kepler(s.G * s.m0, q, v0, tau, 0)
    assert fails == 0
    return q, v0, q1, v1, A, ve


def _check_brute_in_crude(orc, s, tau, rows, kick, min_pairs):
    p = orc.make_params()
    q0, v0, q1, v1, A, ve = _sweep_states(orc, s, tau, kick)
    cand = orc.crude(p, tau, q0, s.h, A, ve)
    brute = orc.fine_brute(p, tau, s.m, s.h, A, q0, v0, q1, v1, rows)
    cset = {tuple(x) for x in cand}
    missed = [tuple(x) for x in brute if tuple(x) not in cset]
    assert not missed, missed[:10]
    assert len(brute) >= min_pairs
    # and the two-stage sweep flags exactly those pairs among the rows
    fc, _, _ = orc.fine(p, tau, cand, s.m, s.h, A, q0, v0, q1, v1)
    sel = cand[fc]
    if rows is not None:
        rs = set(int(x) for x in rows)
        sel = np.array([x for x in sel if int(x[0]) in rs or int(x[1]) in rs]).reshape(-1, 2)
    assert {tuple(x) for x in sel} == {tuple(x) for x in brute}
    return len(brute), len(cand)


def test_brute_force_inside_crude_small(orc):
    """The 104-body disk over 30 steps (its few encounters come and go)."""
    s = inputs.small()
    p = orc.make_params()
    q, v = s.q, s.v
    total = 0
    for _ in range(30):
        st = inputs.System("small", s.G, s.m0, s.m, q, v, s.h)
        nb, _ = _check_brute_in_crude(orc, st, 0.05, None, True, 0)
        total += nb
        q, v, _ = orc.step(p, 0.05, s.m, s.h, q, v)
    assert total > 0


def test_brute_force_inside_crude_disk16k(orc):
    """Every pair of the 16388-body benchmark disk."""
    nb, nc = _check_brute_in_crude(orc, inputs.disk16k(), 0.05, None, True, 100)
    assert nc >= nb


def test_brute_force_inside_crude_disk128k_rows(orc):
    """Every pair that involves one of 2048 sampled bodies of the 131076-body
    disk (the planets included); the first half kick is left out, which the
    comparison does not need."""
    s = inputs.disk128k()
    rng = np.random.Generator(np.random.PCG64(11))
    rows = np.unique(np.concatenate([np.arange(4), rng.choice(s.n, 2044, replace=False)]))
    _check_brute_in_crude(orc, s, 0.05, rows, False, 20)


def test_crude_contains_straight_line_approaches(orc):
    """Conservativeness of the crude sweep without its formula: bodies on bound
    orbits move slower than their escape speed, so a pair whose straight-line
    relative motion from (Q, v) comes within a_E times the mutual Hill radius
    (computed here from the masses and the drawn semi-major axes) during the
    step must be a candidate."""
    rng = np.random.Generator(np.random.PCG64(13))
    aE, tau = 3.0, 0.05
    p = orc.make_params(aE=aE)
    hits = 0
    for trial in range(40):
        n = 400
        a = rng.uniform(4.8, 5.2, n); e = rng.uniform(0, 0.1, n); inc = rng.uniform(0, 0.01, n)
        Om, om, M = rng.uniform(0, 2 * np.pi, (3, n))
        M = rng.uniform(0, 0.2, n)   # crowd them into one arc
        m = 10.0 ** rng.uniform(-9, -5, n)
        q, u = inputs.elements_to_cartesian(MU, a, e, inc, Om * 0, om * 0, M)
        # each body exactly on its own Kepler orbit: A = a, speed < escape speed
        A, ve = orc.prepass(MU, q, u)
        assert np.allclose(A, a, rtol=1e-12)
        cand = {tuple(x) for x in orc.crude(p, tau, q, np.cbrt(m / 3.0), A, ve)}
        iu, ju = np.triu_indices(n, 1)
        d = q[ju] - q[iu]; w = u[ju] - u[iu]
        t = np.clip(-(d * w).sum(1) / np.maximum((w * w).sum(1), 1e-300), 0.0, tau)
        dmin = np.linalg.norm(d + t[:, None] * w, axis=1)
        RMH = np.cbrt((m[iu] + m[ju]) / 3.0) * (a[iu] + a[ju]) / 2.0
        close = dmin < aE * RMH
        hits += int(close.sum())
        for i, j in zip(iu[close], ju[close]):
            assert (int(i), int(j)) in cand
    assert hits > 100
