"""The bound the grid crude sweep (qsym_params.sweep = 1) rests on, checked on
the CPU with the oracle's pre-pass quantities: for every pair of "small"
bodies the exact crude limit (Sec. 2.4, first sweep) is at most
rho_i + rho_j with the separable per-body radius, and such a pair, if it
passes the exact test, lies within one grid cell (2 rho_lim) on every axis.
Mutual and summed Hill radii, a dense and a dispersed disk."""
import numpy as np
import pytest

from paper_1007_3458_amd import inputs


def _grid_constants(hill_mode, h, A, ve, aE, cs, tau):
    n = len(A)
    Alim = 2.0 * A.sum() / n if hill_mode == 0 else 0.0
    ch = h if hill_mode == 0 else h * A
    hA = ch.mean() * Alim if hill_mode == 0 else ch.mean()
    rlim = 1.5 * cs * (aE * hA + tau * ve.mean())
    rho = cs * (aE * (ch * Alim if hill_mode == 0 else ch) + tau * ve)
    small = rho <= rlim
    if hill_mode == 0:
        small &= A <= Alim
    return rho, rlim, small


@pytest.mark.parametrize("hill_mode", [0, 1])
@pytest.mark.parametrize("which", ["crowd", "disk"])
def test_separable_radius_bounds_the_exact_limit(orc, which, hill_mode):
    if which == "crowd":
        s = inputs.make_disk("crowd300", 3, 296, 1e-6, 4.5, 6.0, "uniform", "uniform", 0.05, 0.01)
    else:
        s = inputs.scaled_disk(2000, seed=31)
    aE, cs, tau = 3.0, 1.1, 0.05
    A, ve = orc.prepass(1.0, s.q, s.v)
    rho, rlim, small = _grid_constants(hill_mode, s.h, A, ve, aE, cs, tau)
    assert small.sum() > 0.9 * len(A)          # nearly every body takes the grid path
    idx = np.flatnonzero(small)
    hi, hj = s.h[idx][:, None], s.h[idx][None, :]
    Ai, Aj = A[idx][:, None], A[idx][None, :]
    if hill_mode == 0:
        Rup = aE * (hi + hj) * (Ai + Aj) / 2.0
    else:
        Rup = aE * (hi * Ai + hj * Aj)
    lim = cs * (Rup + tau * (ve[idx][:, None] + ve[idx][None, :]))
    bound = rho[idx][:, None] + rho[idx][None, :]
    assert np.all(lim <= bound * (1 + 1e-15))
    assert np.all(bound <= 2 * rlim * (1 + 1e-15))
    # the candidates among small bodies sit in adjacent cells of size 2 rho_lim
    cell = 2.0 * rlim * (1.0 + 1e-9)
    cand = orc.crude(orc.make_params(hill_mode=hill_mode), tau, s.q, s.h, A, ve)
    assert len(cand) > 0
    c = np.floor(s.q / cell)
    for i, j in cand:
        if small[i] and small[j]:
            assert np.all(np.abs(c[i] - c[j]) <= 1)
