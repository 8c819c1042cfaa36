"""No encounter pair is dropped (Sec. 2.4: the sweeps count their pairs before
recording them, so the lists have no fixed length).  Through the C ABI,
against the FP64 oracle:

* a system with more than 4096 encounter pairs in one step (beyond the
  on-chip set partition) is partitioned in global memory and steps in
  lockstep with the oracle: positions and velocities to 1e-12, encounter
  list, set ids and r_crit exact, clean status;
* a candidate list too short for the crude sweep's pairs makes the fine test
  run over all pairs, with the same result;
* a system with more encounter pairs than its segment holds (4 per body
  + 64) leaves the state of every system exactly as it was at the start of
  that step, reports QSYM_EOVERFLOW, and a new state steps normally again.
"""
import sys

import numpy as np
import pytest

from paper_1007_3458_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def Q():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_1007_3458_amd import qsym
    qsym.lib()
    return qsym


def per_body_rel(a, b):
    na = np.linalg.norm(a - b, axis=1)
    nb = np.maximum(np.linalg.norm(b, axis=1), 1e-300)
    return np.max(na / nb)


def crowded(n, seed, m):
    return inputs.make_disk(f"crowd{n}", seed, n - 4, m, 4.5, 6.0, "uniform", "uniform", 0.05, 0.01)


def _want_sid(label):
    roots = sorted({x for x in label if x >= 0})
    rank = {r: k for k, r in enumerate(roots)}
    return np.array([rank[x] if x >= 0 else -1 for x in label], np.int32)


def _lockstep_big(Q, orc, s, nsteps, cand_cap=None, **kw):
    """Lockstep steps with every output compared; returns the GPU stats."""
    p = orc.make_params()
    ctx = Q.Context(s, **kw)
    q, v = s.q.copy(), s.v.copy()
    for k in range(nsteps):
        ctx.set_state(s.m, s.h, q, v)
        ctx.step(0.05, 1)
        ctx.sync()
        qg, vg = ctx.get_state()
        pg, sid = ctx.encounters()
        st = ctx.stats()
        qo, vo, r = orc.step(p, 0.05, s.m, s.h, q, v, cand_cap=cand_cap or 64 * s.n)
        say(f"  step {k}: {len(r.pairs)} pairs, {r.stats['n_sets']} sets, largest "
            f"{r.stats['max_set']}, candidates {r.stats['n_candidates']}")
        assert r.rc == 0
        assert st["status"] == 0
        assert st["n_encounters"] == len(r.pairs)
        assert np.array_equal(pg, r.pairs)
        assert np.array_equal(sid, _want_sid(r.label))
        assert np.array_equal(ctx.set_rcrit(), r.rcrit)
        assert per_body_rel(qg, qo) < 1e-12, per_body_rel(qg, qo)
        assert per_body_rel(vg, vo) < 1e-12, per_body_rel(vg, vo)
        q, v = qo, vo
    ctx.close()
    return st


def test_more_than_4096_pairs_lockstep(Q, orc):
    """A crowded 10004-body disk: about 5900 encounter pairs per step (sets up
    to ~640 members) -- the global-memory partition and the grid Hermite."""
    s = crowded(10004, 41, 5e-8)
    say("more than 4096 pairs", s.n)
    st = _lockstep_big(Q, orc, s, 2)
    assert st["global_sets"] == 2
    assert st["n_encounters"] > 4096
    assert st["fallbacks"] == 0 and st["overflows"] == 0


def test_candidate_list_overflow_lockstep(Q, orc):
    """The same disk with heavier bodies: ~91k crude candidates against a list
    of 8n + 1024 = 81056, ~8800 encounter pairs; the fine test runs over all
    pairs and the step equals the oracle's (given room for every
    candidate)."""
    s = crowded(10004, 41, 1e-7)
    say("candidate list overflow", s.n)
    st = _lockstep_big(Q, orc, s, 1)
    assert st["fallbacks"] == 1
    assert st["n_candidates"] > 8 * s.n + 1024
    assert st["global_sets"] == 1


def test_global_partition_with_the_whole_system_rule(Q, orc):
    """More than 4096 pairs in a system where an encounter set also holds two
    planets: the global partition applies the whole-system rule of Sec. 2.3
    (one set of every body, r_crit infinite), as the oracle does."""
    base = inputs.make_disk("crowd_wp", 43, 1500, 1e-6, 5.0, 5.3, "uniform", "uniform", 0.02,
                            0.005, planets=False)
    # two Jupiters side by side inside the crowd
    a = np.array([5.15, 5.16]); zero = np.zeros(2)
    qp, up = inputs.elements_to_cartesian(1.0, a, zero, zero, zero, zero, np.array([0.0, 0.004]))
    s = inputs.System("crowd_wp", 1.0, 1.0, np.concatenate([base.m, [1e-3, 1e-3]]),
                      np.vstack([base.q, qp]), np.vstack([base.v, up]))
    p = orc.make_params(planet_mass=1e-4)
    qo, vo, r = orc.step(p, 0.05, s.m, s.h, s.q, s.v, cand_cap=64 * s.n)
    say("whole-system rule in the global partition", s.n, r.stats)
    assert r.rc == 0 and r.stats["whole_system"] == 1
    assert r.stats["n_encounters"] > 4096
    ctx = Q.Context(s, planet_mass=1e-4)
    ctx.step(0.05, 1)
    ctx.sync()
    qg, vg = ctx.get_state()
    pg, sid = ctx.encounters()
    st = ctx.stats()
    assert st["status"] == 0 and st["whole_system"] == 1 and st["global_sets"] == 1
    assert np.array_equal(pg, r.pairs)
    assert np.array_equal(sid, np.zeros(s.n, np.int32))
    assert np.isinf(ctx.set_rcrit()).all() and len(ctx.set_rcrit()) == 1
    assert per_body_rel(qg, qo) < 1e-12 and per_body_rel(vg, vo) < 1e-12
    ctx.close()


def _clump(n, seed):
    """n bodies a thousandth apart on neighbouring circular orbits: every
    pair is an encounter, n (n - 1) / 2 of them."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = 5.0 + rng.uniform(0, 1e-3, n)
    M = rng.uniform(0, 2e-4, n)
    z = np.zeros(n)
    q, u = inputs.elements_to_cartesian(1.0, a, z, z, z, z, M)
    return inputs.System("clump", 1.0, 1.0, np.full(n, 1e-6), q, u)


def test_encounter_overflow_leaves_the_state_unchanged(Q, orc):
    """A 20-body clump has 190 encounter pairs, more than its segment's 144:
    the step is left undone for every system of the context (here with an
    ordinary system beside it), QSYM_EOVERFLOW is reported, the state stays
    bit for bit at the start of that step through later steps, and a new
    state steps as the oracle does."""
    clump = _clump(20, 5)
    other = inputs.batch_system(3, 300)
    say("encounter overflow")
    ctx = Q.Context([clump, other])
    q0 = np.vstack([clump.q, other.q]); v0 = np.vstack([clump.v, other.v])
    ctx.step(0.05, 3)
    with pytest.raises(Q.QsymError) as e:
        ctx.sync()
    assert e.value.code == -6
    st = ctx.stats()
    assert st["overflows"] == 3 and st["steps"] == 0
    qg, vg = ctx.get_state(check=False)
    assert np.array_equal(qg, q0) and np.array_equal(vg, v0)
    # a new state clears the status: the ordinary system alone steps normally
    ctx.close()
    ctx = Q.Context([other])
    ctx.step(0.05, 1)
    ctx.sync()
    qg, vg = ctx.get_state()
    qo, vo, r = orc.step(orc.make_params(), 0.05, other.m, other.h, other.q, other.v)
    assert per_body_rel(qg, qo) < 1e-12 and per_body_rel(vg, vo) < 1e-12
    ctx.close()


def test_new_state_after_an_overflow_steps_again(Q, orc):
    """After an overflow, set_state with a state that fits clears the status
    and the same context steps like the oracle."""
    clump = _clump(20, 6)
    ctx = Q.Context(clump)
    ctx.step(0.05, 1)
    with pytest.raises(Q.QsymError):
        ctx.sync()
    sparse = _clump(20, 6)
    sparse.q = sparse.q * np.linspace(1.0, 3.0, 20)[:, None]   # spread the clump out
    sparse.v = sparse.v / np.sqrt(np.linspace(1.0, 3.0, 20))[:, None]
    ctx.set_state(sparse.m, sparse.h, sparse.q, sparse.v)
    ctx.step(0.05, 2)
    ctx.sync()
    qg, vg = ctx.get_state()
    q, v = sparse.q, sparse.v
    for _ in range(2):
        q, v, r = orc.step(orc.make_params(), 0.05, sparse.m, sparse.h, q, v)
        assert r.rc == 0
    assert per_body_rel(qg, q) < 1e-12 and per_body_rel(vg, v) < 1e-12
    assert ctx.stats()["status"] == 0
    ctx.close()
