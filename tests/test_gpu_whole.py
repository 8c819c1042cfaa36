"""The whole-system Hermite rule (Sec. 2.3, after the steps; planet_mass > 0)
on the GPU, through the C ABI, against the FP64 oracle: lockstep steps of a
two-planet encounter, a whole system above the LDS stage, and a batch in
which only one system fires.  Tolerance 1e-12 relative per body per step."""
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


@pytest.mark.parametrize("n_small", [8, 100, 1100])
def test_whole_system_lockstep(Q, orc, n_small):
    s = inputs.two_planet_encounter(n_small, seed=3)
    say(f"whole system lockstep n={s.n}")
    ctx = Q.Context(s, Q.make_params(planet_mass=1e-4))
    p = orc.make_params(planet_mass=1e-4)
    q, v = s.q, s.v
    for k in range(3):
        ctx.set_state(s.m, s.h, q, v)
        ctx.step(0.05, 1)
        qg, vg = ctx.get_state()
        q, v, r = orc.step(p, 0.05, s.m, s.h, q, v)
        assert r.rc == 0 and r.stats["whole_system"] == 1
        st = ctx.stats()
        assert st["n_sets"] == 1 and st["max_set"] == s.n
        assert per_body_rel(qg, q) < 1e-12 and per_body_rel(vg, v) < 1e-12
    assert ctx.stats()["whole_system"] == 3
    _, sid = ctx.encounters()
    assert np.all(sid == sid[0])
    ctx.close()


def test_whole_system_in_a_batch(Q, orc):
    systems = [inputs.batch_system(0, 300), inputs.two_planet_encounter(20, seed=5),
               inputs.batch_system(2, 77)]
    say("whole system in a batch")
    ctx = Q.Context(systems, Q.make_params(planet_mass=1e-4))
    ctx.step(0.05, 2)
    qg, vg = ctx.get_state()
    off = ctx.offsets
    p = orc.make_params(planet_mass=1e-4)
    fired = 0
    for k, s in enumerate(systems):
        q, v = s.q, s.v
        for _ in range(2):
            q, v, r = orc.step(p, 0.05, s.m, s.h, q, v)
            fired += r.stats["whole_system"]
        sl = slice(off[k], off[k + 1])
        assert per_body_rel(qg[sl], q) < 1e-12 and per_body_rel(vg[sl], v) < 1e-12
    assert fired == 2 and ctx.stats()["whole_system"] == 2
    ctx.close()


def test_rule_off_leaves_the_hybrid_step(Q):
    s = inputs.two_planet_encounter(30, seed=9)
    out = []
    for pm in (0.0, 2e-3):     # off, and a threshold above both planets
        ctx = Q.Context(s, Q.make_params(planet_mass=pm))
        ctx.step(0.05, 3)
        out.append(ctx.get_state())
        assert ctx.stats()["whole_system"] == 0
        ctx.close()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
