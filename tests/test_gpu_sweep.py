"""Crude sweep on the hashed grid (qsym_params.sweep = 1, Sec. 2.4 first
sweep with a sub-quadratic search) on the GPU, through the C ABI.  Every
pair is decided by the exact test of the definition, so the candidate sets
equal the oracle's brute-force sets exactly (and the fused sweep's): dense
and ragged disks, a clump that overflows its hash bucket, unbound and
nearly parabolic bodies (the large list), both Hill modes, batched systems,
the full 16388-body disk; whole steps equal the oracle's."""
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


def crowded(n, seed, m=1e-6):
    return inputs.make_disk(f"crowd{n}", seed, n - 4, m, 4.5, 6.0, "uniform", "uniform", 0.05, 0.01)


def clumped():
    """A disk with 60 bodies inside one tiny box: more than a hash bucket holds."""
    s = inputs.scaled_disk(500, seed=21).copy()
    rng = np.random.Generator(np.random.PCG64(22))
    k = np.arange(10, 70)
    s.q[k] = s.q[10] + 1e-6 * rng.uniform(-1, 1, (len(k), 3))
    return s


def unbound():
    """A disk with hyperbolic and nearly parabolic bodies (huge or r-valued a)."""
    s = inputs.scaled_disk(600, seed=23).copy()
    r = np.linalg.norm(s.q, axis=1)
    vesc = np.sqrt(2.0 / r)
    for k, f in ((20, 1.5), (21, 1.2), (22, 0.99999), (23, 0.9999999)):
        s.v[k] *= f * vesc[k] / np.linalg.norm(s.v[k])
    return s


SYSTEMS = {
    "small": lambda: inputs.small(),
    "crowd300": lambda: crowded(300, 3),
    "ragged1029": lambda: inputs.scaled_disk(1025, seed=12),
    "clump": clumped,
    "unbound": unbound,
}


@pytest.mark.parametrize("hill_mode", [0, 1])
@pytest.mark.parametrize("name", list(SYSTEMS))
def test_grid_candidates_equal_oracle(Q, orc, name, hill_mode):
    s = SYSTEMS[name]()
    say("grid sweep", name, "hill_mode", hill_mode)
    tau = 0.05
    ctx = Q.Context(s, Q.make_params(sweep=1, hill_mode=hill_mode))
    ctx.apply_kick(0.0, crude_tau=tau)
    got = ctx.candidates()
    st = ctx.stats()
    ctx.close()
    A, ve = orc.prepass(1.0, s.q, s.v)
    ref = {tuple(x) for x in orc.crude(orc.make_params(hill_mode=hill_mode), tau, s.q, s.h, A, ve)}
    assert len(got) == len(set(map(tuple, got)))       # no pair twice
    assert {tuple(x) for x in got} == ref and len(ref) > 0
    assert st["n_candidates"] == len(ref)
    # the fused sweep finds the same set
    ctx = Q.Context(s, Q.make_params(sweep=0, hill_mode=hill_mode))
    ctx.apply_kick(0.0, crude_tau=tau)
    assert {tuple(x) for x in ctx.candidates()} == ref
    ctx.close()


def test_grid_candidates_full_disk_and_batch(Q, orc):
    s = inputs.disk16k()
    say("grid sweep disk16k")
    ctx = Q.Context(s, Q.make_params(sweep=1))
    ctx.apply_kick(0.0, crude_tau=0.05)
    got = {tuple(x) for x in ctx.candidates()}
    ctx.close()
    A, ve = orc.prepass(1.0, s.q, s.v)
    assert got == {tuple(x) for x in orc.crude(orc.make_params(), 0.05, s.q, s.h, A, ve)}
    sizes = [64, 300, 1, 2, 777, 130]
    systems = [inputs.batch_system(k, n) for k, n in enumerate(sizes)]
    say("grid sweep batched", sizes)
    ctx = Q.Context(systems, Q.make_params(sweep=1))
    ctx.apply_kick(0.0, crude_tau=0.05)
    got = {tuple(x) for x in ctx.candidates()}
    off = ctx.offsets
    ctx.close()
    ref = set()
    for k, b in enumerate(systems):
        A, ve = orc.prepass(1.0, b.q, b.v)
        ref |= {(int(i) + off[k], int(j) + off[k]) for i, j in orc.crude(orc.make_params(), 0.05, b.q, b.h, A, ve)}
    assert got == ref and len(ref) > 0


def test_grid_sweep_whole_steps(Q, orc):
    s = crowded(300, 3)
    say("grid sweep lockstep steps")
    ctx = Q.Context(s, Q.make_params(sweep=1))
    p = orc.make_params()
    q, v = s.q, s.v
    for k in range(3):
        ctx.set_state(s.m, s.h, q, v)
        ctx.step(0.05, 1)
        qg, vg = ctx.get_state()
        pg, _ = ctx.encounters()
        q, v, r = orc.step(p, 0.05, s.m, s.h, q, v)
        assert per_body_rel(qg, q) < 1e-12 and per_body_rel(vg, v) < 1e-12
        assert {tuple(x) for x in pg} == {tuple(x) for x in r.pairs} and len(r.pairs) > 0
    ctx.close()
    # graph replay == eager launches, and == the fused sweep's steps
    out = []
    for sweep, eager in ((1, False), (1, True), (0, False)):
        ctx = Q.Context(s, Q.make_params(sweep=sweep))
        ctx.profile(eager)
        ctx.step(0.05, 6)
        out.append(ctx.get_state())
        ctx.close()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    assert per_body_rel(out[0][0], out[2][0]) < 1e-12
