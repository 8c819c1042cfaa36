"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Operator by operator on identical inputs, then whole steps in lockstep
(both sides start every step from the same state).  Tolerances:
  * accelerations / velocities / positions: 1e-13 relative per operator,
    1e-12 relative per whole step (the oracle's rounding order differs);
  * encounter flags: bit-exact, except pairs within 1e-12 of the threshold
    (lockstep runs count those and expect none);
  * integer outputs (candidate sets, sets, labels): exact.
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


def crowded(n, seed, m=1e-6):
    """Planets + planetesimals packed near a = 5 (forces encounters)."""
    return inputs.make_disk(f"crowd{n}", seed, n - 4, m, 4.5, 6.0, "uniform", "uniform", 0.05, 0.01)


def rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def per_body_rel(a, b):
    na = np.linalg.norm(a - b, axis=1)
    nb = np.maximum(np.linalg.norm(b, axis=1), 1e-300)
    return np.max(na / nb)


SYSTEMS = {
    "small": lambda: inputs.small(),
    "ragged1029": lambda: inputs.scaled_disk(1025, seed=12),
    "crowd300": lambda: crowded(300, 3),
}

SHAPES = [dict(ipl=1, block=128, jchunk=128, remap=0), dict(ipl=2, block=256, jchunk=256, remap=1),
          dict(ipl=4, block=256, jchunk=512, remap=1), dict(ipl=2, block=128, jchunk=384, remap=1),
          # symmetric kick: each unordered pair once, reaction on j (one or two i per lane)
          dict(ipl=1, block=128, jchunk=128, remap=0, sym=1),
          dict(ipl=2, block=128, jchunk=256, remap=1, sym=2),
          dict(ipl=1, block=256, jchunk=1024, remap=1, sym=1),
          dict(ipl=2, block=256, jchunk=512, remap=0, sym=1),
          dict(ipl=1, block=128, jchunk=512, remap=0, sym=4),
          dict(ipl=2, block=128, jchunk=512, remap=3, sym=1),
          dict(ipl=1, block=256, jchunk=256, remap=2, sym=2),
          # balanced rows: every row cut along j into items of equal pair count
          dict(ipl=1, block=256, jchunk=256, remap=0, sym=16),
          dict(ipl=2, block=256, jchunk=512, remap=0, sym=16),
          dict(ipl=1, block=128, jchunk=128, remap=0, sym=16)]


@pytest.mark.parametrize("name", list(SYSTEMS))
@pytest.mark.parametrize("shape", range(len(SHAPES)))
def test_kick_parity(Q, orc, name, shape):
    s = SYSTEMS[name]()
    s.v[:] = 0.0  # v1 = dt * a exactly: no cancellation in the comparison
    say("kick parity", name, SHAPES[shape], s.n)
    ctx = Q.Context(s)
    sh = dict(SHAPES[shape])
    ctx.set_kick_shape(**sh)
    ctx.apply_kick(1.0)
    _, v1 = ctx.get_state()
    a_gpu = v1 - s.v
    a_orc = orc.accel(s.G, s.m, s.q)
    assert per_body_rel(a_gpu, a_orc) < 1e-13
    ctx.close()


@pytest.mark.parametrize("name", list(SYSTEMS))
@pytest.mark.parametrize("shape", [None, 4, 6])
def test_crude_candidates_match(Q, orc, name, shape):
    s = SYSTEMS[name]()
    say("crude candidates", name, shape)
    p = orc.make_params()
    tau = 0.05
    ctx = Q.Context(s)
    if shape is not None:
        ctx.set_kick_shape(**SHAPES[shape])
    ctx.apply_kick(0.0, crude_tau=tau)
    got = {tuple(x) for x in ctx.candidates()}
    A, ve = orc.prepass(1.0, s.q, s.v)
    ref = {tuple(x) for x in orc.crude(p, tau, s.q, s.h, A, ve)}
    # identical inputs: the pairs under the tile bound take the exact test of
    # the definition with the oracle's operands and order -> identical sets
    assert got == ref
    assert len(ref) > 0
    ctx.close()


def test_drift_parity(Q, orc):
    s = crowded(300, 4)
    say("drift parity")
    ctx = Q.Context(s)
    ctx.apply_drift(0.37)
    q1, v1 = ctx.get_state()
    qo = orc.drift(s.m0, s.m, s.q, s.v, 0.37)
    assert rel(q1, qo) < 1e-15
    assert np.array_equal(v1, s.v)
    ctx.close()


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("dt", [0.05, 0.5, -0.3])
def test_kepler_parity(Q, orc, mode, dt):
    s = inputs.kepler_test(5003, seed=31)
    say("kepler parity", mode, dt)
    ctx = Q.Context(s, kepler_mode=mode)
    ctx.apply_kepler(dt)
    q1, v1 = ctx.get_state()
    qo, vo, it, fails = orc.kepler(1.0, s.q, s.v, dt, mode)
    assert fails == 0
    assert per_body_rel(q1, qo) < 1e-13
    assert per_body_rel(v1, vo) < 1e-13
    st = ctx.stats()
    assert sum(st["kepler_hist"]) == s.n
    # same iteration counts up to convergence-threshold ties
    hist_o = np.bincount(it, minlength=32)[:32]
    assert np.abs(np.array(st["kepler_hist"]) - hist_o).sum() <= 0.01 * s.n
    # the statistics are kept in striped copies (79 workgroups over 64
    # copies here) and added up on the host: total and largest agree with
    # the histogram, and a second pass adds to all three
    h = np.array(st["kepler_hist"])
    assert h[-1] == 0
    assert st["kepler_iters"] == int((np.arange(32) * h).sum())
    assert st["kepler_max"] == int(np.nonzero(h)[0].max())
    ctx.apply_kepler(dt)
    st2 = ctx.stats()
    assert sum(st2["kepler_hist"]) == 2 * s.n
    assert st2["kepler_iters"] == int((np.arange(32) * np.array(st2["kepler_hist"])).sum())
    assert st2["kepler_max"] >= st["kepler_max"]
    ctx.close()


def test_fine_flags_bit_exact(Q, orc):
    """Identical inputs -> identical comparison operands and flags, including
    pairs placed within rounding of the threshold."""
    say("fine bit exact")
    rng = np.random.Generator(np.random.PCG64(17))
    n = 400
    q0 = rng.normal(size=(n, 3)) * 0.2 + np.array([5.0, 0.0, 0.0])
    v0 = rng.normal(size=(n, 3)) * 0.05
    q1 = q0 + 0.05 * v0 + rng.normal(size=(n, 3)) * 1e-4
    v1 = v0 + rng.normal(size=(n, 3)) * 1e-3
    m = rng.uniform(1e-9, 1e-3, n)
    h = np.cbrt(m / 3.0)
    A = rng.uniform(4.0, 6.0, n)
    pairs = np.array([(i, j) for i in range(0, n, 3) for j in range(i + 1, n, 7)], np.int32)
    for hill_mode in (0, 1):
        for aE in (3.0, 0.7):
            p_o = orc.make_params(aE=aE, hill_mode=hill_mode)
            p_g = Q.make_params(aE=aE, hill_mode=hill_mode)
            fo, lo, ro = orc.fine(p_o, 0.05, pairs, m, h, A, q0, v0, q1, v1)
            fg, lg, rg = Q.fine_test(p_g, 1.0, 0.05, m, h, A, q0, v0, q1, v1, pairs)
            assert np.array_equal(fo, fg)
            assert np.array_equal(lo, lg) and np.array_equal(ro, rg)
            assert 0 < fo.sum() < len(fo)


def _lockstep(Q, orc, s, nsteps, tau=0.05, **kw):
    p_o = orc.make_params(**{k: v for k, v in kw.items() if k in orc.DEFAULTS})
    ctx = Q.Context(s, **kw)
    q, v = s.q.copy(), s.v.copy()
    tot_enc = 0
    border = 0
    for k in range(nsteps):
        ctx.set_state(s.m, s.h, q, v)
        ctx.step(tau, 1)
        ctx.sync()
        qg, vg = ctx.get_state()
        pg, sid = ctx.encounters()
        qo, vo, r = orc.step(p_o, tau, s.m, s.h, q, v)
        assert r.rc == 0
        eo = {tuple(x) for x in r.pairs}
        eg = {tuple(x) for x in pg}
        if eo != eg:
            border += len(eo ^ eg)
        assert np.array_equal(pg, np.array(sorted(eg), np.int32).reshape(-1, 2))
        tot_enc += len(eo)
        assert per_body_rel(qg, qo) < 1e-12, (k, per_body_rel(qg, qo))
        assert per_body_rel(vg, vo) < 1e-12, (k, per_body_rel(vg, vo))
        # set labels: GPU set ids ordered by smallest member, oracle labels = smallest member
        lab = r.label
        roots = sorted({x for x in lab if x >= 0})
        want = np.array([roots.index(x) if x >= 0 else -1 for x in lab])
        if not border:
            assert np.array_equal(sid, want)
            # r_crit of every set (Sec. 2.2): the same operations on the same
            # inputs, so the same bits
            assert np.array_equal(ctx.set_rcrit(), r.rcrit), (k, ctx.set_rcrit(), r.rcrit)
        q, v = qo, vo
    ctx.close()
    return tot_enc, border


@pytest.mark.parametrize("name,nsteps", [("small", 20), ("crowd300", 20), ("ragged1029", 4)])
def test_step_lockstep(Q, orc, name, nsteps):
    s = SYSTEMS[name]()
    say("lockstep", name, nsteps)
    enc, border = _lockstep(Q, orc, s, nsteps)
    assert border == 0
    if name != "ragged1029":
        assert enc > 0


def test_step_lockstep_large_workgroup_set(Q, orc):
    """A 217-member set on one workgroup (two lanes a member, up to 109
    pairs a lane): each lane marks its pairs inside r_crit in several
    32-pair passes before taking them."""
    s = inputs.make_disk("crowd220", 3, 216, 1e-4, 4.9, 5.1, "uniform", "uniform", 0.05, 0.01)
    _, _, r = orc.step(orc.make_params(), 0.05, s.m, s.h, s.q, s.v)
    assert r.rc == 0
    assert 128 < np.bincount(r.label[r.label >= 0]).max() <= 256
    say("lockstep 217-member set")
    enc, border = _lockstep(Q, orc, s, 3)
    assert enc > 0 and border == 0


def test_step_lockstep_hermite_heavy(Q, orc):
    """Massive crowded bodies: many Hermite substeps per set."""
    s = crowded(120, 9, m=3e-5)
    say("lockstep hermite heavy")
    enc, border = _lockstep(Q, orc, s, 10)
    assert enc > 0 and border == 0


def test_energy_parity(Q, orc):
    for s in (inputs.small(), crowded(300, 5), inputs.scaled_disk(1029, seed=3)):
        say("energy", s.name)
        ctx = Q.Context(s)
        E = ctx.energy()[0]
        Eo = orc.energy(s.G, s.m0, s.m, s.q, s.v)
        assert abs(E - Eo) <= 1e-13 * abs(Eo)
        ctx.close()


def test_energy_full_size_batch_and_coincident(Q, orc):
    """The energy (Sec. 2, H) of the 16388-body disk and of a batch of uneven
    systems (ragged pair tiles, systems of one and two bodies, an empty one)
    to 1e-13; and of a system holding two coincident bodies, whose pair the
    definition leaves out (r = 0), as the oracle does."""
    s = inputs.disk16k()
    say("energy disk16k")
    ctx = Q.Context(s)
    E = ctx.energy()[0]
    ctx.close()
    assert abs(E / orc.energy(s.G, s.m0, s.m, s.q, s.v) - 1.0) <= 1e-13
    sizes = [64, 1, 300, 0, 2, 777, 65, 130]
    systems = [inputs.batch_system(k, n) if n > 0 else inputs.System("empty", 1.0, 1.0,
               np.zeros(0), np.zeros((0, 3)), np.zeros((0, 3))) for k, n in enumerate(sizes)]
    say("energy batch", sizes)
    ctx = Q.Context(systems)
    E = ctx.energy()
    ctx.close()
    for k, b in enumerate(systems):
        Eo = orc.energy(b.G, b.m0, b.m, b.q, b.v) if b.n else 0.0
        assert abs(E[k] - Eo) <= 1e-13 * abs(Eo), (k, E[k], Eo)
    c = crowded(300, 8).copy()
    c.q[17] = c.q[201]
    say("energy with a coincident pair")
    ctx = Q.Context(c)
    E = ctx.energy()[0]
    ctx.close()
    Eo = orc.energy(c.G, c.m0, c.m, c.q, c.v)
    assert np.isfinite(E) and abs(E / Eo - 1.0) <= 1e-13


def test_full_size_step_disk16k(Q, orc):
    """Full plain-FP64 workload size: one whole step of 16388 bodies against
    the oracle, every output compared."""
    s = inputs.disk16k()
    say("full size disk16k")
    ctx = Q.Context(s)
    ctx.step(0.05, 1)
    ctx.sync()
    qg, vg = ctx.get_state()
    pg, sid = ctx.encounters()
    qo, vo, r = orc.step(orc.make_params(), 0.05, s.m, s.h, s.q, s.v)
    assert per_body_rel(qg, qo) < 1e-12
    assert per_body_rel(vg, vo) < 1e-12
    assert np.array_equal(pg, r.pairs)
    st = ctx.stats()
    assert st["n_encounters"] == r.stats["n_encounters"] > 0
    assert st["n_sets"] == r.stats["n_sets"]
    roots = sorted({x for x in r.label if x >= 0})
    assert np.array_equal(sid, np.array([roots.index(x) if x >= 0 else -1 for x in r.label]))
    assert np.array_equal(ctx.set_rcrit(), r.rcrit)
    ctx.close()


def test_batched_equals_single(Q, orc):
    sizes = [64, 300, 1, 2, 777, 130]
    systems = [inputs.batch_system(k, n) for k, n in enumerate(sizes)]
    say("batched", sizes)
    ctx = Q.Context(systems)
    ctx.step(0.05, 3)
    ctx.sync()
    qg, vg = ctx.get_state()
    E = ctx.energy()
    off = ctx.offsets
    p = orc.make_params()
    pg, _ = ctx.encounters()
    want = []
    for k, s in enumerate(systems):
        q, v = s.q, s.v
        for _ in range(3):
            q, v, r = orc.step(p, 0.05, s.m, s.h, q, v)
        sl = slice(off[k], off[k + 1])
        assert per_body_rel(qg[sl], q) < 1e-12
        assert per_body_rel(vg[sl], v) < 1e-12
        assert abs(E[k] - orc.energy(s.G, s.m0, s.m, q, v)) <= 1e-12 * abs(E[k])
        want += [(int(a) + off[k], int(b) + off[k]) for a, b in r.pairs]
    # the last step's encounter pairs of every system, in global indices
    assert len(want) > 0
    assert np.array_equal(pg, np.array(sorted(want), np.int32).reshape(-1, 2))
    ctx.close()


def test_determinism_graph_eager_and_resume(Q):
    s = crowded(300, 6)
    say("determinism")
    a = Q.Context(s)
    a.step(0.05, 6)
    qa, va = a.get_state()
    b = Q.Context(s)
    b.profile(True)            # eager launches, no graph
    b.step(0.05, 6)
    qb, vb = b.get_state()
    assert np.array_equal(qa, qb) and np.array_equal(va, vb)
    c = Q.Context(s)
    c.step(0.05, 2)
    qc, vc = c.get_state()
    c.close()
    d = Q.Context(s)
    d.set_state(s.m, s.h, qc, vc)
    d.step(0.05, 4)
    qd, vd = d.get_state()
    assert np.array_equal(qa, qd) and np.array_equal(va, vd)
    for x in (a, b, d):
        x.close()


def test_autotune_keeps_results(Q, orc):
    s = inputs.scaled_disk(2049, seed=5)
    say("autotune")
    s.v[:] = 0.0
    ctx = Q.Context(s)
    us = ctx.autotune(0.05)
    assert min(us) > 0
    ctx.apply_kick(1.0)
    _, v1 = ctx.get_state()
    assert per_body_rel(v1 - s.v, orc.accel(s.G, s.m, s.q)) < 1e-13
    ctx.close()


def test_candidate_overflow_loses_no_encounter(Q, orc):
    """A candidate list of 2 pairs: the sweep finds hundreds, the fine test
    then runs over all pairs, and the step equals the oracle's (encounter
    list, sets and r_crit exact) with a clean status."""
    s = crowded(300, 7)
    say("candidate overflow path")
    ctx = Q.Context(s, pair_capacity=2)
    ctx.step(0.05, 1)
    ctx.sync()
    qg, vg = ctx.get_state()
    pg, sid = ctx.encounters()
    st = ctx.stats()
    assert st["status"] == 0 and st["fallbacks"] == 1 and st["n_candidates"] > 2
    with pytest.raises(Q.QsymError) as e:
        ctx.candidates(cap=10)   # the list itself was cut short
    assert e.value.code == -6
    qo, vo, r = orc.step(orc.make_params(), 0.05, s.m, s.h, s.q, s.v)
    assert r.rc == 0 and len(r.pairs) > 0
    assert np.array_equal(pg, r.pairs)
    assert per_body_rel(qg, qo) < 1e-12 and per_body_rel(vg, vo) < 1e-12
    assert np.array_equal(ctx.set_rcrit(), r.rcrit)
    ctx.close()


def test_nonfinite_state_is_reported(Q):
    """A NaN coordinate propagates through the step (no kernel drops it) and
    the step reports QSYM_ENONFINITE at the next synchronisation."""
    s = inputs.small().copy()
    s.q[5, 1] = np.nan
    say("non-finite state")
    ctx = Q.Context(s)
    ctx.step(0.05, 1)
    with pytest.raises(Q.QsymError) as e:
        ctx.sync()
    assert e.value.code == -4
    with pytest.raises(Q.QsymError) as e:   # latched: every synchronising call reports it
        ctx.get_state()
    assert e.value.code == -4
    # a new state clears the status
    c = inputs.small()
    ctx.set_state(c.m, c.h, c.q, c.v)
    ctx.step(0.05, 1)
    ctx.sync()
    qg, vg = ctx.get_state()
    assert np.isfinite(qg).all() and np.isfinite(vg).all()
    ctx.close()


def test_edge_sizes(Q, orc):
    for n in (1, 2, 3, 255, 256, 257):
        s = inputs.scaled_disk(max(n - 4, 1), seed=40 + n) if n > 4 else crowded(5, n).copy()
        if n <= 4:
            s = inputs.System("tiny", 1.0, 1.0, s.m[:n], s.q[:n], s.v[:n])
        say("edge size", s.n)
        ctx = Q.Context(s)
        ctx.step(0.05, 2)
        ctx.sync()
        qg, vg = ctx.get_state()
        q, v = s.q, s.v
        for _ in range(2):
            q, v, _ = orc.step(orc.make_params(), 0.05, s.m, s.h, q, v)
        assert per_body_rel(qg, q) < 1e-12 and per_body_rel(vg, v) < 1e-12
        ctx.close()


def test_time_reversal_without_encounters(Q, orc):
    """With the encounter switch off (a_E = 0) the step is the symmetric
    composition of exact flows (Sec. 2): tau steps forward and then -tau
    steps back return to the start to rounding, and a backward step equals
    the oracle's; a zero step leaves the state unchanged."""
    s = inputs.scaled_disk(1025, seed=14)
    say("time reversal", s.n)
    ctx = Q.Context(s, Q.make_params(aE=0.0))
    ctx.step(0.05, 20)
    ctx.sync()
    assert ctx.stats()["n_encounters"] == 0
    ctx.step(-0.05, 20)
    ctx.sync()
    qg, vg = ctx.get_state()
    assert np.max(np.abs(qg - s.q)) < 1e-12 * np.max(np.abs(s.q))
    assert np.max(np.abs(vg - s.v)) < 1e-12 * np.max(np.abs(s.v))
    ctx.set_state(s.m, s.h, s.q, s.v)
    ctx.step(-0.05, 1)
    ctx.sync()
    qg, vg = ctx.get_state()
    qo, vo, r = orc.step(orc.make_params(aE=0.0), -0.05, s.m, s.h, s.q, s.v)
    assert r.rc == 0 and r.stats["n_encounters"] == 0
    assert per_body_rel(qg, qo) < 1e-12 and per_body_rel(vg, vo) < 1e-12
    ctx.set_state(s.m, s.h, s.q, s.v)
    ctx.step(0.0, 1)
    ctx.sync()
    qg, vg = ctx.get_state()
    assert np.max(np.abs(qg - s.q)) <= 1e-15 * np.max(np.abs(s.q))
    assert np.max(np.abs(vg - s.v)) <= 1e-15 * np.max(np.abs(s.v))
    ctx.close()


def test_empty_systems(Q, orc):
    """Offsets need only be non-decreasing: empty systems in a batch stay
    empty with zero energy while the others step exactly as alone, and a
    context whose only system is empty steps as a no-op."""
    empty = inputs.System("empty", 1.0, 1.0, np.zeros(0), np.zeros((0, 3)), np.zeros((0, 3)))
    a, b = inputs.batch_system(0, 64), inputs.batch_system(1, 130)
    say("empty systems in a batch")
    ctx = Q.Context([a, empty, b, empty])
    ctx.step(0.05, 3)
    ctx.sync()
    qg, vg = ctx.get_state()
    off = ctx.offsets
    E = ctx.energy()
    st = ctx.stats()
    ctx.close()
    assert st["status"] == 0 and E[1] == 0.0 and E[3] == 0.0
    for k, s in ((0, a), (2, b)):
        q, v = s.q, s.v
        for _ in range(3):
            q, v, r = orc.step(orc.make_params(), 0.05, s.m, s.h, q, v)
            assert r.rc == 0
        assert per_body_rel(qg[off[k]:off[k + 1]], q) < 1e-12
        assert per_body_rel(vg[off[k]:off[k + 1]], v) < 1e-12
    say("only an empty system")
    ctx = Q.Context([empty])
    ctx.step(0.05, 2)
    ctx.sync()
    assert ctx.energy()[0] == 0.0 and ctx.stats()["status"] == 0
    ctx.close()


def test_fp32_form_accuracy_and_step(Q, orc):
    """Precision form: m r^-3 in FP32 on FP64 separations, FP64 sums.  Per-body
    acceleration error against the oracle at the FP32 level; the whole step
    stays close to the oracle step and keeps the encounter list."""
    s = inputs.scaled_disk(4096, seed=14)
    say("fp32 form")
    s0 = s.copy()
    s0.v[:] = 0.0
    ctx = Q.Context(s0, precision=1)
    ctx.set_kick_shape(2, 256, 512, 1)
    ctx.apply_kick(1.0)
    _, a = ctx.get_state()
    ao = orc.accel(s.G, s.m, s.q)
    rel = np.linalg.norm(a - ao, axis=1) / np.linalg.norm(ao, axis=1)
    print("fp32 form accel rel err max %.3e rms %.3e" % (rel.max(), np.sqrt(np.mean(rel ** 2))))
    assert rel.max() < 2e-6 and np.sqrt(np.mean(rel ** 2)) < 3e-7
    ctx.close()
    ctx = Q.Context(s, precision=1)
    ctx.step(0.05, 1)
    ctx.sync()
    qg, vg = ctx.get_state()
    pg, _ = ctx.encounters()
    po = orc.make_params()
    qo, vo, r = orc.step(po, 0.05, s.m, s.h, s.q, s.v)
    assert per_body_rel(qg, qo) < 1e-9 and per_body_rel(vg, vo) < 1e-7
    # the encounter list is the FP64 one but for pairs within the FP32
    # form's error of the threshold (Dm^3 vs T^6 M^2 within 1e-5)
    eg, eo = {tuple(x) for x in pg}, {tuple(x) for x in r.pairs}
    assert len(eo) > 0
    diff = np.array(sorted(eg ^ eo), np.int32).reshape(-1, 2)
    if len(diff):
        q0 = orc.drift(s.m0, s.m, s.q, s.v, 0.025)
        A, _ = orc.prepass(1.0, q0, s.v)
        v0 = orc.kick(1.0, s.m, q0, s.v, 0.025)
        q1, v1, _, _ = orc.kepler(1.0, q0, v0, 0.05, 0)
        _, lhs, rhs = orc.fine(po, 0.05, diff, s.m, s.h, A, q0, v0, q1, v1)
        assert np.all(np.abs(lhs / rhs - 1.0) < 1e-5), (diff, lhs / rhs)
    print("fp32 form step: %d encounter pairs, %d within the FP32 margin differ" % (len(eo), len(diff)))
    ctx.close()


def _components(pairs, n):
    """Set id per body from the encounter pairs: connected components (plain
    union-find), numbered in the order of their smallest member; -1 for a
    body in no pair."""
    parent = list(range(n))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for i, j in pairs:
        ri, rj = find(int(i)), find(int(j))
        if ri != rj:
            parent[max(ri, rj)] = min(ri, rj)
    members = sorted({int(x) for p in pairs for x in p})
    roots = sorted({find(x) for x in members})
    rank = {r: k for k, r in enumerate(roots)}
    want = np.full(n, -1, np.int32)
    for x in members:
        want[x] = rank[find(x)]
    return want


def test_sets_of_a_system_beyond_the_bitmap(Q, orc):
    """The set partition ranks the bodies in encounters through a bitmap of
    the system for up to 262144 bodies and by sorting beyond that.  A
    266004-body disk takes the sorting path: its sets must be the connected
    components of the step's encounter pairs, numbered by smallest member."""
    s = inputs.make_disk("disk266k", 11, 266000, 1e-10, 15.0, 40.0, "rayleigh", "rayleigh", 0.05,
                         0.025)
    assert s.n > 262144
    say("sets beyond the bitmap", s.n)
    ctx = Q.Context(s)
    ctx.step(0.05, 1)
    ctx.sync()
    st = ctx.stats()
    assert st["status"] == 0
    pg, sid = ctx.encounters()
    assert 0 < len(pg) <= 4096
    assert st["n_sets"] == int(sid.max()) + 1
    assert np.array_equal(sid, _components(pg, s.n))
    # the oracle's partition of the same pairs (labels = smallest member)
    lab, ns = orc.sets(s.n, pg)
    roots = sorted({int(x) for x in lab if x >= 0})
    rank = {r: k for k, r in enumerate(roots)}
    assert ns == st["n_sets"]
    assert np.array_equal(sid, np.array([rank[int(x)] if x >= 0 else -1 for x in lab]))
    ctx.close()


def _wide_with_parabolic(seed, n_disk):
    """A disk of planetesimals plus one body on a nearly parabolic orbit, whose
    huge osculating semi-major axis (hence Hill radius) pulls every body into
    its encounter set."""
    base = inputs.make_disk("wide%d" % seed, seed, n_disk, 1e-9, 4.5, 6.0, "uniform", "uniform", 0.05,
                            0.01, planets=False)
    r = np.array([5.0, 0.1, 0.0])
    v = np.array([0.0, 0.99995 * np.sqrt(2.0 / np.linalg.norm(r)), 0.0])
    return inputs.System("bigset%d" % seed, 1.0, 1.0, np.concatenate([base.m, [1e-6]]),
                         np.vstack([base.q, r]), np.vstack([base.v, v]))


def test_two_sets_on_the_grid_in_one_step(Q, orc):
    """Two systems in one batch, each with a set of more than 256 members:
    both sets run on the whole grid in one launch, one after the other, so
    the grid barrier's phases carry over from the first set to the second.
    Each system equals its own oracle step."""
    systems = [_wide_with_parabolic(21, 420), _wide_with_parabolic(22, 300)]
    say("two grid sets", [s.n for s in systems])
    ctx = Q.Context(systems)
    ctx.step(0.05, 1)
    ctx.sync()
    st = ctx.stats()
    assert st["status"] == 0
    qg, vg = ctx.get_state()
    off = ctx.offsets
    sizes = []
    for k, s in enumerate(systems):
        qo, vo, res = orc.step(orc.make_params(), 0.05, s.m, s.h, s.q, s.v)
        assert res.rc == 0
        sizes.append(res.stats["max_set"])
        a, b = off[k], off[k + 1]
        assert per_body_rel(qg[a:b], qo) < 1e-12 and per_body_rel(vg[a:b], vo) < 1e-12
    assert min(sizes) > 256
    assert st["max_set"] == max(sizes)
    ctx.close()


def _with_parabolic(nbase, seed=21):
    """A disk of nbase light bodies plus one on a nearly parabolic orbit: its
    huge osculating semi-major axis gives it a huge Hill radius, so the disk
    bodies join its encounter set."""
    base = inputs.make_disk("wide", seed, nbase, 1e-9, 4.5, 6.0, "uniform", "uniform", 0.05, 0.01,
                            planets=False)
    r = np.array([5.0, 0.1, 0.0])
    vesc = np.sqrt(2.0 / np.linalg.norm(r))
    v = np.array([0.0, 0.99995 * vesc, 0.0])
    m = np.concatenate([base.m, [1e-6]])
    q = np.vstack([base.q, r])
    vv = np.vstack([base.v, v])
    return inputs.System(f"parabolic{nbase}", 1.0, 1.0, m, q, vv)


@pytest.mark.parametrize("nbase", [40, 100, 150, 230])
def test_workgroup_set_sizes(Q, orc, nbase):
    """Sets of 17-256 members run on one workgroup, staged in LDS in tiles of
    64: one set of one to four tiles, ragged, a whole step against the
    oracle."""
    s = _with_parabolic(nbase)
    say("workgroup set", s.n)
    ctx = Q.Context(s)
    ctx.step(0.05, 1)
    ctx.sync()
    st = ctx.stats()
    qg, vg = ctx.get_state()
    qo, vo, res = orc.step(orc.make_params(), 0.05, s.m, s.h, s.q, s.v)
    ctx.close()
    assert res.rc == 0 and res.stats["max_set"] == st["max_set"]
    assert 16 < st["max_set"] <= 256 and st["max_set"] > 0.6 * s.n
    assert per_body_rel(qg, qo) < 1e-12 and per_body_rel(vg, vo) < 1e-12


def test_set_larger_than_lds_stage(Q, orc):
    """A set of more than 1024 members (every body joins the nearly parabolic
    body's set) is integrated from the global staging path."""
    s = _with_parabolic(1300)
    say("big set", s.n)
    ctx = Q.Context(s)
    ctx.step(0.05, 1)
    ctx.sync()
    st = ctx.stats()
    assert st["max_set"] > 1024
    qg, vg = ctx.get_state()
    qo, vo, res = orc.step(orc.make_params(), 0.05, s.m, s.h, s.q, s.v)
    assert res.stats["max_set"] == st["max_set"]
    assert per_body_rel(qg, qo) < 1e-12 and per_body_rel(vg, vo) < 1e-12
    ctx.close()


@pytest.mark.parametrize("sym", [1, 2, 16])
def test_symmetric_kick_lockstep_steps(Q, orc, sym):
    """Whole hybrid steps with the symmetric kick for both kicks equal the
    oracle steps (the step never depends on the kick shape beyond rounding)."""
    s = crowded(300, 3)
    say("symmetric kick steps", sym)
    ctx = Q.Context(s)
    with pytest.raises(Q.QsymError):   # the symmetric kick takes one or two i per lane
        ctx.set_kick_shape(4, 128, 512, 1, sym=sym)
    ctx.set_kick_shape(2, 128, 256, 1, sym=sym)
    p = orc.make_params()
    q, v = s.q, s.v
    for k in range(3):
        ctx.set_state(s.m, s.h, q, v)
        ctx.step(0.05, 1)
        qg, vg = ctx.get_state()
        pg, _ = ctx.encounters()
        q, v, r = orc.step(p, 0.05, s.m, s.h, q, v)
        assert per_body_rel(qg, q) < 1e-12 and per_body_rel(vg, v) < 1e-12
        assert {tuple(x) for x in pg} == {tuple(x) for x in r.pairs}
    ctx.close()


def test_symmetric_kick_full_size_and_batched(Q, orc):
    s = inputs.disk16k()
    say("symmetric kick disk16k")
    s0 = s.copy()
    s0.v[:] = 0.0
    rows = np.arange(0, s.n, 97)
    ao = orc.accel_rows(s.G, s.m, s.q, rows)
    for sh in (dict(ipl=2, block=256, jchunk=1024, remap=1, sym=1),
               dict(ipl=1, block=256, jchunk=512, remap=0, sym=16),
               dict(ipl=2, block=256, jchunk=512, remap=0, sym=16)):
        ctx = Q.Context(s0)
        ctx.set_kick_shape(**sh)
        ctx.apply_kick(1.0)
        _, a = ctx.get_state()
        assert per_body_rel(a[rows], ao) < 1e-13, sh
        ctx.close()
    sizes = [64, 300, 1, 2, 777, 130]
    systems = [inputs.batch_system(k, n) for k, n in enumerate(sizes)]
    for b in systems:
        b.v[:] = 0.0
    for sym in (2, 16):
        ctx = Q.Context(systems)
        ctx.set_kick_shape(1, 128, 128, 0, sym=sym)
        ctx.apply_kick(1.0)
        _, a = ctx.get_state()
        off = ctx.offsets
        for k, b in enumerate(systems):
            sl = slice(off[k], off[k + 1])
            assert per_body_rel(a[sl], orc.accel(b.G, b.m, b.q)) < 1e-13, (sym, k)
        ctx.close()
