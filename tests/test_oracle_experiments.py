"""The paper's parameter claims (Sec. 3) on the oracle, small synthetic
systems: the energy error over a fixed span falls as tau^2 (per step tau^3)
for this second-order scheme with encounters handled, and a larger
encounter factor a_E flags a superset of the pairs at the same state."""
import numpy as np

from paper_1007_3458_amd import inputs


def _span(orc, s, tau, span, **kw):
    p = orc.make_params(**kw)
    q, v = s.q, s.v
    E0 = orc.energy(s.G, s.m0, s.m, q, v)
    worst, enc = 0.0, 0
    for _ in range(int(round(span / tau))):
        q, v, r = orc.step(p, tau, s.m, s.h, q, v)
        assert r.rc == 0
        enc += len(r.pairs)
        worst = max(worst, abs(orc.energy(s.G, s.m0, s.m, q, v) / E0 - 1.0))
    return worst, enc


def test_energy_error_scales_as_tau_squared_over_a_span(orc):
    s = inputs.small()
    taus = np.array([0.4, 0.2, 0.1])
    rows = [_span(orc, s, t, 2.0) for t in taus]
    assert all(e > 0 for _, e in rows)          # encounters take part
    worst = np.array([w for w, _ in rows])
    slope = np.polyfit(np.log(taus), np.log(worst), 1)[0]
    assert 1.9 < slope < 2.1, slope
    # per-step average error: the tau^3 the paper quotes
    per_step = worst / (2.0 / taus)
    assert 2.9 < np.polyfit(np.log(taus), np.log(per_step), 1)[0] < 3.1


def test_larger_encounter_factor_flags_a_superset(orc):
    s = inputs.make_disk("crowd300", 3, 296, 1e-6, 4.5, 6.0, "uniform", "uniform", 0.05, 0.01)
    prev, counts = None, []
    for aE in (0.5, 1.0, 2.0, 3.0, 4.0, 6.0):
        _, _, r = orc.step(orc.make_params(aE=aE), 0.05, s.m, s.h, s.q, s.v)
        cur = set(map(tuple, r.pairs.tolist()))
        if prev is not None:
            assert prev <= cur
        prev = cur
        counts.append(len(cur))
    assert counts[-1] > counts[0]
