"""Pins of the oracle's encounter identification (Sec. 2.4) and set partition
(Sec. 2.3 step 4): exact straight-line minimum, dense sampling of the cubic,
brute force over all pairs on small N, and a breadth-first search."""
import numpy as np
import pytest

from paper_1007_3458_amd import inputs


def test_fine_min_is_exact_for_straight_lines(orc):
    """Relative motion on a straight line: D(s) is quadratic and the cubic
    interpolant reproduces it, so the minimum is |a x b|^2/|b|^2."""
    p = orc.make_params(hill_mode=1, aE=1.0)
    rng = np.random.Generator(np.random.PCG64(3))
    tau = 0.7
    for _ in range(200):
        qi = rng.normal(size=3)
        vi = rng.normal(size=3)
        d0 = rng.normal(size=3)
        w = rng.normal(size=3)
        # pick a closest-approach time strictly inside the step
        tc = rng.uniform(0.1, 0.9) * tau
        d0 = d0 - (d0 @ w) / (w @ w) * w - tc * w  # makes (d0 + t w) closest at t = tc
        q0 = np.array([qi, qi + d0])
        v0 = np.array([vi, vi + w])
        q1 = q0 + tau * v0
        dmin2 = np.sum(np.cross(d0, w) ** 2) / (w @ w)
        m = np.array([1e-3, 1e-3]); h = np.array([1.0, 1.0]); A = np.array([1.0, 1.0])
        _, lhs, _ = orc.fine(p, tau, np.array([[0, 1]]), m, h, A, q0, v0, q1, v0)
        assert abs(lhs[0] - dmin2) <= 1e-12 * max(dmin2, 1e-300) + 1e-15 * (d0 @ d0)


def _cubic_min_sampled(D0, D1, d0, d1, ns=100001):
    s = np.linspace(0, 1, ns)
    c2 = 3 * (D1 - D0) - 2 * d0 - d1
    c3 = 2 * (D0 - D1) + d0 + d1
    return np.min(D0 + d0 * s + c2 * s ** 2 + c3 * s ** 3)


def test_fine_min_matches_dense_sampling(orc):
    p = orc.make_params(hill_mode=1, aE=1.0)
    rng = np.random.Generator(np.random.PCG64(4))
    tau = 0.3
    for _ in range(300):
        q0 = rng.normal(size=(2, 3)); v0 = rng.normal(size=(2, 3))
        q1 = q0 + tau * v0 + rng.normal(size=(2, 3)) * 0.05
        v1 = v0 + rng.normal(size=(2, 3)) * 0.3
        a0 = q0[1] - q0[0]; b0 = v0[1] - v0[0]; a1 = q1[1] - q1[0]; b1 = v1[1] - v1[0]
        D0, D1 = a0 @ a0, a1 @ a1
        d0, d1 = 2 * tau * a0 @ b0, 2 * tau * a1 @ b1
        ref = max(0.0, _cubic_min_sampled(D0, D1, d0, d1))
        m = np.ones(2); h = np.ones(2); A = np.ones(2)
        _, lhs, _ = orc.fine(p, tau, np.array([[0, 1]]), m, h, A, q0, v0, q1, v1)
        assert lhs[0] <= ref + 1e-12 * max(D0, D1)
        assert ref - lhs[0] <= 1e-8 * max(D0, D1)


def test_fine_threshold_is_aE_mutual_hill_radius(orc):
    """Two bodies at rest relative to each other at separation d: marked iff
    d < a_E ((m_i+m_j)/(3 m0))^(1/3) (a_i+a_j)/2 (computed directly)."""
    p = orc.make_params(aE=3.0)
    m = np.array([1e-3, 1e-8]); h = np.cbrt(m / 3.0); A = np.array([5.0, 5.5])
    RMH = np.cbrt((m[0] + m[1]) / 3.0) * (A[0] + A[1]) / 2.0
    for d in (0.9, 0.999, 1.001, 1.1):
        q0 = np.array([[5.0, 0, 0], [5.0 + d * 3.0 * RMH, 0, 0]])
        v0 = np.zeros((2, 3))
        f, _, _ = orc.fine(p, 0.1, np.array([[0, 1]]), m, h, A, q0, v0, q0, v0)
        assert bool(f[0]) == (d < 1.0)


def _close_system(n, seed):
    """n bodies with several planets and crowded planetesimals (forces encounters)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = inputs.make_disk("crowd", seed, n - 4, 1e-6, 4.5, 6.0, "uniform", "uniform", 0.05, 0.01)
    return s


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_two_stage_sweep_equals_brute_force(orc, seed):
    """Sec. 2.4: the crude sweep must lose no encounter: fine test over ALL
    pairs == fine test over the crude candidates."""
    s = _close_system(64, seed)
    p = orc.make_params()
    tau = 0.05
    mu = 1.0
    q = orc.drift(s.m0, s.m, s.q, s.v, tau / 2)
    A, ve = orc.prepass(mu, q, s.v)
    cand = orc.crude(p, tau, q, s.h, A, ve)
    v0 = orc.kick(1.0, s.m, q, s.v, tau / 2)
    q1, v1, _, _ = orc.kepler(mu, q, v0, tau, 0)
    iu = np.triu_indices(s.n, 1)
    allp = np.stack(iu, 1).astype(np.int32)
    fa, _, _ = orc.fine(p, tau, allp, s.m, s.h, A, q, v0, q1, v1)
    fc, _, _ = orc.fine(p, tau, cand, s.m, s.h, A, q, v0, q1, v1)
    brute = {tuple(x) for x in allp[fa]}
    two = {tuple(x) for x in cand[fc]}
    assert len(brute) > 0
    assert brute == two
    # candidate list is lexicographic with i < j
    assert np.all(cand[:, 0] < cand[:, 1])
    keys = cand[:, 0].astype(np.int64) * s.n + cand[:, 1]
    assert np.all(np.diff(keys) > 0)


def test_crude_predicate_reading(orc):
    """States the reading taken of the garbled crude predicate of Sec. 2.4
    (symmetric, conservative: |dq|^2 < (c_s (R_up + tau (ve_i + ve_j)))^2 with
    R_up = a_E (h_i + h_j)(A_i + A_j)/2).  This documents the reading and
    keeps it from drifting; what pins the predicate to the method is that it
    loses no encounter: brute force over all pairs on the 104- and 16k-body
    disks and sampled rows of the 131k-body disk, and every straight-line
    approach within a_E mutual Hill radii (test_oracle_pins.py)."""
    s = _close_system(48, 7)
    p = orc.make_params()
    A, ve = orc.prepass(1.0, s.q, s.v)
    cand = orc.crude(p, 0.05, s.q, s.h, A, ve)
    got = {tuple(x) for x in cand}
    ref = set()
    for i in range(s.n):
        for j in range(i + 1, s.n):
            r2 = np.sum((s.q[j] - s.q[i]) ** 2)
            R = 3.0 * (s.h[i] + s.h[j]) * (A[i] + A[j]) / 2
            lim = 1.1 * (R + 0.05 * (ve[i] + ve[j]))
            if r2 < lim * lim:
                ref.add((i, j))
    assert got == ref


def _bfs_labels(n, pairs):
    adj = {i: [] for i in range(n)}
    for a, b in pairs:
        adj[a].append(b); adj[b].append(a)
    lab = -np.ones(n, np.int32)
    for s in range(n):
        if lab[s] >= 0 or not adj[s]:
            continue
        comp, stack = [s], [s]
        lab[s] = s
        while stack:
            u = stack.pop()
            for w in adj[u]:
                if lab[w] < 0:
                    lab[w] = s; comp.append(w); stack.append(w)
        lab[comp] = min(comp)
    return lab


@pytest.mark.parametrize("seed", range(5))
def test_sets_equal_bfs_components(orc, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    n = 200
    k = int(rng.integers(1, 150))
    a = rng.integers(0, n, k); b = rng.integers(0, n, k)
    keep = a != b
    pairs = np.stack([np.minimum(a, b), np.maximum(a, b)], 1)[keep].astype(np.int32)
    lab, ns = orc.sets(n, pairs)
    ref = _bfs_labels(n, pairs)
    assert np.array_equal(lab, ref)
    assert ns == len({x for x in ref if x >= 0})


def test_encounter_set_is_permutation_invariant(orc):
    s = _close_system(64, 2)
    p = orc.make_params()
    perm = np.random.Generator(np.random.PCG64(1)).permutation(s.n)
    sp = s.permuted(perm)
    _, _, r = orc.step(p, 0.05, s.m, s.h, s.q, s.v)
    _, _, rp = orc.step(p, 0.05, sp.m, sp.h, sp.q, sp.v)
    got = {tuple(sorted((perm[a], perm[b]))) for a, b in rp.pairs}
    ref = {tuple(x) for x in r.pairs}
    assert len(ref) > 0 and got == ref
