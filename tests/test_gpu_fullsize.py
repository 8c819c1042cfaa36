"""Parity at the benchmark workloads' full sizes, in the launch configuration
the benchmark uses (the tuned kick shapes), through the C ABI: sampled
outputs the oracle computes one by one (accelerations of sampled bodies over
all bodies, Kepler solves of sampled bodies), and a property of the whole step
that holds at any size (total angular momentum, conserved by every operator
of the splitting: the kicks' pair forces are central and antisymmetric, the
drift moves every body by the same vector parallel to the total momentum,
and the Kepler flow and the Hermite's forces are central)."""
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
    return np.max(np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-300))


def angular_momentum(m, q, v):
    return (m[:, None] * np.cross(q, v)).sum(axis=0)


@pytest.fixture(scope="module")
def disk128k():
    return inputs.disk128k()


def test_small_1000_steps_free_run(Q, orc):
    """The 104-body system (4 planets + 100 planetesimals) run freely for its
    1000 steps of tau = 0.05 on both sides from the same initial conditions,
    the energy taken every 100 steps: the energy errors (the method's,
    ~1e-10) agree with the oracle's to 1e-6 of themselves + 1e-14, the same
    encounter pairs and Hermite substeps are counted over the run, and the
    final positions agree to 1e-12 per body (the per-step tolerance; about
    4e-16 is measured).  The two sides differ only in rounding order, which
    this quiet system amplifies little over 1000 steps."""
    b = inputs.small()
    p = orc.make_params(G=b.G, m0=b.m0)
    q, v = b.q, b.v
    E0 = orc.energy(b.G, b.m0, b.m, q, v)
    dE_o, enc, sub = [], 0, 0
    for k in range(1000):
        q, v, r = orc.step(p, 0.05, b.m, b.h, q, v)
        assert r.rc == 0
        enc += len(r.pairs)
        sub += int(r.stats["substeps"])
        if (k + 1) % 100 == 0:
            dE_o.append(orc.energy(b.G, b.m0, b.m, q, v) / E0 - 1.0)
    say("small 1000 steps: oracle", enc, "encounter pairs,", sub, "substeps")
    ctx = Q.Context(b)
    G0 = ctx.energy()[0]
    dE = []
    for _ in range(10):
        ctx.step(0.05, 100)
        dE.append(ctx.energy()[0] / G0 - 1.0)
    qg, _ = ctx.get_state()
    st = ctx.stats()
    ctx.close()
    dE, dE_o = np.array(dE), np.array(dE_o)
    say(f"  energy errors gpu {dE.max():.3e} oracle {dE_o.max():.3e}; max diff {np.abs(dE - dE_o).max():.2e};"
        f" final positions {per_body_rel(qg, q):.2e}")
    assert st["status"] == 0 and st["steps"] == 1000
    assert st["total_encounters"] == enc and st["total_substeps"] == sub
    assert np.all(np.abs(dE - dE_o) <= 1e-6 * np.abs(dE_o) + 1e-14)
    assert per_body_rel(qg, q) < 1e-12


def test_disk128k_kick_sampled(Q, orc, disk128k):
    """FP64 kick of the 131076-body disk (tuned shape) at 510 sampled bodies."""
    s = disk128k
    say("disk128k kick", s.n)
    s0 = s.copy()
    s0.v[:] = 0.0
    ctx = Q.Context(s0)
    ctx.apply_kick(1.0)
    _, a = ctx.get_state()
    ctx.close()
    rows = np.arange(0, s.n, 257)
    ao = orc.accel_rows(s.G, s.m, s.q, rows)
    assert per_body_rel(a[rows], ao) < 1e-13


def test_disk128k_fp32_form_kick_sampled(Q, orc, disk128k):
    """FP32 pair terms on the 131076-body disk: the form's error bounds at
    510 sampled bodies."""
    s = disk128k
    say("disk128k fp32 kick", s.n)
    s0 = s.copy()
    s0.v[:] = 0.0
    ctx = Q.Context(s0, precision=1)
    ctx.apply_kick(1.0)
    _, a = ctx.get_state()
    ctx.close()
    rows = np.arange(0, s.n, 257)
    ao = orc.accel_rows(s.G, s.m, s.q, rows)
    rel = np.linalg.norm(a[rows] - ao, axis=1) / np.linalg.norm(ao, axis=1)
    say("fp32 form rel err max %.3e rms %.3e" % (rel.max(), np.sqrt(np.mean(rel ** 2))))
    assert rel.max() < 2e-6 and np.sqrt(np.mean(rel ** 2)) < 3e-7


def test_disk128k_kepler_sampled(Q, orc, disk128k):
    """Kepler drift of all 131076 bodies; 510 sampled bodies solved by the
    oracle one by one."""
    s = disk128k
    say("disk128k kepler", s.n)
    ctx = Q.Context(s)
    ctx.apply_kepler(0.05)
    q1, v1 = ctx.get_state()
    ctx.close()
    rows = np.arange(0, s.n, 257)
    qo, vo, _, fails = orc.kepler(s.G * s.m0, s.q[rows], s.v[rows], 0.05, 0)
    assert fails == 0
    assert per_body_rel(q1[rows], qo) < 1e-13
    assert per_body_rel(v1[rows], vo) < 1e-13


def test_disk128k_step_conserves_angular_momentum(Q, disk128k):
    """One whole hybrid step of the 131076-body disk, encounters and all:
    total angular momentum conserved to rounding, energy error at the
    integrator's level."""
    s = disk128k
    say("disk128k step", s.n)
    ctx = Q.Context(s)
    E0 = ctx.energy()[0]
    L0 = angular_momentum(s.m, s.q, s.v)
    ctx.step(0.05, 1)
    ctx.sync()
    q1, v1 = ctx.get_state()
    E1 = ctx.energy()[0]
    st = ctx.stats()
    ctx.close()
    assert st["status"] == 0 and st["n_encounters"] > 0
    L1 = angular_momentum(s.m, q1, v1)
    assert np.linalg.norm(L1 - L0) <= 1e-12 * np.linalg.norm(L0)
    assert abs(E1 / E0 - 1.0) < 1e-9


@pytest.fixture(scope="module")
def disk128k_oracle_step(orc, disk128k):
    """The oracle's hybrid step of the 131076-body disk (all host cores)."""
    s = disk128k
    say("oracle step of disk128k (host cores: %d)" % orc.num_threads())
    return orc.step(orc.make_params(), 0.05, s.m, s.h, s.q, s.v)


def _sid_from_labels(label):
    roots = sorted({int(x) for x in label if x >= 0})
    rank = {r: k for k, r in enumerate(roots)}
    return np.array([rank[int(x)] if x >= 0 else -1 for x in label], np.int32)


def test_disk128k_step_lockstep(Q, disk128k, disk128k_oracle_step):
    """One whole hybrid step of the 131076-body disk in the benchmark's launch
    configuration against the oracle's: every position and velocity to
    1e-12, the encounter list, set ids and r_crit exact."""
    s = disk128k
    qo, vo, r = disk128k_oracle_step
    say("disk128k lockstep", s.n, len(r.pairs), "pairs")
    ctx = Q.Context(s)
    ctx.step(0.05, 1)
    ctx.sync()
    qg, vg = ctx.get_state()
    pg, sid = ctx.encounters()
    rc = ctx.set_rcrit()
    st = ctx.stats()
    ctx.close()
    assert r.rc == 0 and st["status"] == 0 and len(r.pairs) > 1000
    assert np.array_equal(pg, r.pairs)
    assert np.array_equal(sid, _sid_from_labels(r.label))
    assert np.array_equal(rc, r.rcrit)
    assert per_body_rel(qg, qo) < 1e-12
    assert per_body_rel(vg, vo) < 1e-12


def test_disk128k_fp32_form_step(Q, orc, disk128k, disk128k_oracle_step):
    """The FP32 form's step of the same disk: within the form's bounds of the
    FP64 oracle step, and the FP64 encounter list but for pairs within the
    form's error of the threshold."""
    s = disk128k
    qo, vo, r = disk128k_oracle_step
    say("disk128k fp32 form step", s.n)
    ctx = Q.Context(s, precision=1)
    ctx.step(0.05, 1)
    ctx.sync()
    qg, vg = ctx.get_state()
    pg, _ = ctx.encounters()
    ctx.close()
    assert per_body_rel(qg, qo) < 1e-9 and per_body_rel(vg, vo) < 1e-7
    eg, eo = {tuple(x) for x in pg}, {tuple(x) for x in r.pairs}
    diff = np.array(sorted(eg ^ eo), np.int32).reshape(-1, 2)
    say("  %d pairs, %d differ" % (len(eo), len(diff)))
    assert len(diff) <= max(3, len(eo) // 100)
    if len(diff):
        po = orc.make_params()
        q0 = orc.drift(s.m0, s.m, s.q, s.v, 0.025)
        A, _ = orc.prepass(1.0, q0, s.v)
        # v0 of the differing pairs' bodies only: their accelerations over all bodies
        rows = np.unique(diff.ravel())
        v0 = s.v.copy()
        v0[rows] += 0.025 * orc.accel_rows(s.G, s.m, q0, rows)
        q1, v1, _, _ = orc.kepler(1.0, q0[rows], v0[rows], 0.05, 0)
        loc = {int(b): k for k, b in enumerate(rows)}
        dl = np.array([[loc[int(a)], loc[int(b)]] for a, b in diff], np.int32)
        _, lhs, rhs = orc.fine(po, 0.05, dl, s.m[rows], s.h[rows], A[rows], q0[rows], v0[rows], q1,
                               v1)
        assert np.all(np.abs(lhs / rhs - 1.0) < 1e-5), lhs / rhs


def test_disk128k_runs_its_100_steps(Q, disk128k):
    """The precision form's workload for its stated 100 steps (FP64): a clean
    status, no step left undone, energy error at the integrator's level."""
    s = disk128k
    say("disk128k 100 steps")
    ctx = Q.Context(s)
    E0 = ctx.energy()[0]
    for k in range(10):
        ctx.step(0.05, 10)
        ctx.sync()
        st = ctx.stats()
        say("  after %d steps: %d pairs, largest set %d" % (10 * (k + 1), st["n_encounters"],
                                                            st["max_set"]))
    E1 = ctx.energy()[0]
    st = ctx.stats()
    ctx.close()
    assert st["status"] == 0 and st["steps"] == 100 and st["overflows"] == 0
    assert abs(E1 / E0 - 1.0) < 1e-9


def test_batch_step_per_system(Q, orc):
    """One hybrid step of the 512-system batch (launch shapes of the benchmark):
    20 systems -- the largest, every system with a set above 256 members (the
    grid Hermite), and seeded others -- each equal to its own oracle step:
    positions and velocities to 1e-12, encounter pairs exact."""
    systems = inputs.batch()
    say("batch step", len(systems))
    ctx = Q.Context(systems)
    ctx.step(0.05, 1)
    ctx.sync()
    qg, vg = ctx.get_state()
    pg, sid = ctx.encounters()
    st = ctx.stats()
    off = ctx.offsets
    ctx.close()
    assert st["status"] == 0
    sizes = np.array([b.n for b in systems])
    pick = {int(np.argmax(sizes))}
    for k in range(len(systems)):
        ids = sid[off[k]:off[k + 1]]
        ids = ids[ids >= 0]
        if len(ids) and np.bincount(ids - ids.min()).max() > 256:
            pick.add(k)
    say("  systems with a set above 256 members:", sorted(pick))
    rng = np.random.Generator(np.random.PCG64(17))
    for k in rng.permutation(len(systems)):
        if len(pick) >= 20:
            break
        pick.add(int(k))
    p = orc.make_params()
    for k in sorted(pick):
        b = systems[k]
        qo, vo, r = orc.step(p, 0.05, b.m, b.h, b.q, b.v)
        sl = slice(off[k], off[k + 1])
        assert r.rc == 0
        assert per_body_rel(qg[sl], qo) < 1e-12, k
        assert per_body_rel(vg[sl], vo) < 1e-12, k
        mine = pg[(pg[:, 0] >= off[k]) & (pg[:, 0] < off[k + 1])] - off[k]
        assert np.array_equal(mine, r.pairs), k


def test_batch_energy_error_matches_oracle(Q):
    """The 512-system batch over the benchmark's protocol (tau = 0.05, 10
    steps, then 100 steps with the energy every 10 against the energy after
    the first 10): every system's largest relative energy error equals the
    oracle's, integrated system by system (tests/golden/
    batch_energy_oracle.json, written by make_batch_energy.py beside it).
    The two integrate the same initial conditions with the same arithmetic
    up to rounding order, so the energy errors, which range over 2.4e-13 ..
    3.4e-7 between systems, agree to a small fraction of themselves; the
    bound 1e-3 relative + 1e-12 absolute leaves room for rounding amplified
    through close encounters over 110 steps, and is far below the spread
    between systems, so the worst system and its error are reproduced."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                    "batch_energy_oracle.json")))
    dE_o = np.array([float.fromhex(x) for x in g["dE_max"]])
    systems = inputs.batch()
    assert [b.n for b in systems] == g["n"]
    say("batch energy", len(systems))
    ctx = Q.Context(systems)
    ctx.step(g["tau"], g["warmup_steps"])
    E0 = ctx.energy()
    dE = np.zeros(len(systems))
    for _ in range(g["steps"] // g["energy_every"]):
        ctx.step(g["tau"], g["energy_every"])
        dE = np.maximum(dE, np.abs(ctx.energy() / E0 - 1.0))
    st = ctx.stats()
    ctx.close()
    assert st["status"] == 0 and st["overflows"] == 0
    diff = np.abs(dE - dE_o)
    worst = int(np.argmax(diff / (1e-3 * dE_o + 1e-12)))
    say(f"  worst system gpu {int(np.argmax(dE))} ({dE.max():.4e}), oracle "
        f"{int(np.argmax(dE_o))} ({dE_o.max():.4e}); largest disagreement system {worst}: "
        f"{dE[worst]:.6e} vs {dE_o[worst]:.6e}")
    assert np.all(diff <= 1e-3 * dE_o + 1e-12), worst
    assert int(np.argmax(dE)) == int(np.argmax(dE_o))


def test_batch_load_balance_records(Q):
    """Workgroup records (profiling with records) on a 64-system slice of the
    batch: the symmetric kick's recording variant gives the same state bit
    for bit as the captured step, and the busy figures are consistent: at
    most the device's compute units, mean <= max, and the busiest unit's
    time within the launch's event time."""
    import torch
    systems = inputs.batch()[:64]
    a = Q.Context(systems)
    b = Q.Context(systems)
    for c in (a, b):   # the batch's tuned shape: the symmetric kick, which records
        c.set_kick_shape(2, 128, 256, remap=0, which=-1, sym=1)
    a.step(0.05, 3)
    b.profile(True, records=True)
    b.step(0.05, 3)
    st = b.stats()
    b.profile(False)
    qa, va = a.get_state()
    qb, vb = b.get_state()
    a.close()
    b.close()
    assert np.array_equal(qa, qb) and np.array_equal(va, vb)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    say("  busy units", st["busy_units"], "of", cus)
    assert 0 < st["busy_units"] <= cus
    for ph in (1, 5, 6):   # kick + crude sweep, Hermite, second kick
        n = st["busy_calls"][ph]
        assert n == 3, (ph, n)
        mx, mean = st["busy_max_us"][ph], st["busy_mean_us"][ph]
        say(f"  phase {ph}: max {mx / n:.1f} us mean {mean / n:.1f} us, event "
            f"{st['phase_us'][ph] / st['phase_calls'][ph]:.1f} us")
        assert 0 < mean <= mx <= 1.05 * st["phase_us"][ph] + 5.0 * n


def test_batch_kick_sampled(Q, orc):
    """FP64 kick of the 512-system batch (551,375 bodies, tuned shape): the
    first, middle and last body of every system."""
    systems = inputs.batch()
    say("batch kick", len(systems), sum(b.n for b in systems))
    zeroed = []
    for b in systems:
        b0 = b.copy()
        b0.v[:] = 0.0
        zeroed.append(b0)
    ctx = Q.Context(zeroed)
    ctx.apply_kick(1.0)
    _, a = ctx.get_state()
    off = ctx.offsets
    ctx.close()
    worst = 0.0
    for k, b in enumerate(systems):
        rows = np.unique([0, b.n // 2, b.n - 1])
        ao = orc.accel_rows(b.G, b.m, b.q, rows)
        worst = max(worst, per_body_rel(a[off[k] + rows], ao))
    assert worst < 1e-13


def test_learned_workload_kepler_sampled(Q, orc):
    """Kepler solve of the learned-start workload (1,114,116 bodies) from the
    packaged learned start: 1092 sampled bodies solved by the oracle (from
    its own start; the root is the same to the solve's tolerance)."""
    from paper_1007_3458_amd import learned_guess
    s = inputs.learned_workload()
    say("learned workload kepler", s.n)
    ctx = Q.Context([s], Q.make_params(kepler_mode=2), guess=learned_guess.load())
    ctx.apply_kepler(0.05)
    q1, v1 = ctx.get_state()
    st = ctx.stats()
    ctx.close()
    assert st["status"] == 0
    assert sum(st["kepler_hist"]) == s.n
    rows = np.arange(0, s.n, 1021)
    qo, vo, _, fails = orc.kepler(s.G * s.m0, s.q[rows], s.v[rows], 0.05, 1)
    assert fails == 0
    assert per_body_rel(q1[rows], qo) < 1e-12
    assert per_body_rel(v1[rows], vo) < 1e-12
