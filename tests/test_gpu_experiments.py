"""The paper's parameter experiments (Sec. 3) on the GPU path, through the C
ABI: energy error over a fixed span vs the step size (slope 2, equal to the
oracle's figures), and the encounter sets as the encounter factor a_E grows
(a superset at the same state, equal to the oracle's lists)."""
import sys

import numpy as np
import pytest

from paper_1007_3458_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def X():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_1007_3458_amd import experiments, qsym
    qsym.lib()
    return experiments


def test_tau_scaling_matches_oracle(X, orc):
    s = inputs.small()
    taus = (0.4, 0.2, 0.1)
    say("tau scaling small, span 2")
    res = X.tau_scaling(taus=taus, span=2.0, system=s)
    assert 1.9 < res["slope_max"] < 2.1, res["slope_max"]
    for r in res["rows"]:
        assert r["status"] == 0 and r["encounters"] > 0
        p = orc.make_params()
        q, v = s.q, s.v
        E0 = orc.energy(s.G, s.m0, s.m, q, v)
        worst = 0.0
        for _ in range(r["steps"]):
            q, v, _ = orc.step(p, r["tau"], s.m, s.h, q, v)
            worst = max(worst, abs(orc.energy(s.G, s.m0, s.m, q, v) / E0 - 1.0))
        # the GPU samples the energy at 20 checkpoints, the oracle every step
        assert r["dE_max"] <= worst * (1 + 1e-3)
        assert abs(r["dE_final"] / (orc.energy(s.G, s.m0, s.m, q, v) / E0 - 1.0) - 1.0) < 1e-3


def test_tau_scaling_1024_bodies(X):
    say("tau scaling 1024 bodies, span 2")
    res = X.tau_scaling(taus=(0.4, 0.2, 0.1, 0.05), span=2.0)
    assert all(r["status"] == 0 for r in res["rows"])
    assert 1.8 < res["slope_max"] < 2.2, res["slope_max"]


def test_encounter_factor_superset_and_oracle_lists(X, orc):
    from paper_1007_3458_amd import qsym
    s = inputs.make_disk("crowd300", 3, 296, 1e-6, 4.5, 6.0, "uniform", "uniform", 0.05, 0.01)
    prev = None
    for aE in (0.5, 1.0, 2.0, 3.0, 4.0, 6.0):
        say(f"crowd300 first step, a_E {aE}")
        ctx = qsym.Context([s], qsym.make_params(aE=aE))
        ctx.step(0.05, 1)
        pairs, _ = ctx.encounters()
        ctx.close()
        _, _, r = orc.step(orc.make_params(aE=aE), 0.05, s.m, s.h, s.q, s.v)
        assert np.array_equal(pairs, r.pairs)
        cur = set(map(tuple, pairs.tolist()))
        if prev is not None:
            assert prev <= cur
        prev = cur
