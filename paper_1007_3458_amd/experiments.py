"""Parameter experiments of the paper on synthetic stand-ins, run on the GPU
path only (``python -m paper_1007_3458_amd.experiments --out FILE``).

* Step-size scaling (Sec. 3, test integrations): the same initial conditions
  integrated over one fixed span with several step sizes tau.  The scheme is
  second order, so the energy error per step goes as tau^3 and the error over
  the span as tau^2.  Reported: the final and the largest |dE/E0| over the
  span, their log-log slopes against tau, and the per-step average
  (final error / steps), the quantity the paper compares.
* Sensitivity (Sec. 3, sensitivity of parameters): a_E, the Hill factor of the
  encounter test, and a_H, the Hill factor of the transition radius r_crit.
  The paper finds the energy error insensitive to a_H and sensitive to a_E,
  with more encounters (and a slower step) for larger a_E.  Accuracy is
  measured on the giant planets with enhanced masses (the paper's primary
  test), cost on a planetesimal disk.

The paper's own initial conditions (1024 particles; the outer Solar System)
are not published, so the disks of ``inputs.make_disk`` stand in for them.
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import inputs, qsym


def tau_system(n_disk: int = 1020, seed: int = 8) -> inputs.System:
    """4 planets + 1020 planetesimals (1024 bodies, the paper's test size), the
    planetesimals in the benchmark disk's distributions."""
    return inputs.make_disk("tau1024", seed, n_disk, 1e-8, 15.0, 40.0, "rayleigh", "rayleigh",
                            0.05, 0.025)


def disk_system(n_disk: int = 4096, seed: int = 9) -> inputs.System:
    """4 planets + 4096 planetesimals crossing the outer planets' orbits."""
    return inputs.make_disk("disk4100", seed, n_disk, 1e-8, 15.0, 40.0, "rayleigh", "rayleigh",
                            0.05, 0.025)


def _slope(x, y):
    lx, ly = np.log(np.asarray(x, float)), np.log(np.asarray(y, float))
    return float(np.polyfit(lx, ly, 1)[0])


def run_span(systems, tau: float, nsteps: int, checkpoints: int = 20, **params):
    """Integrate the systems (one batched context) for ``nsteps`` steps of
    ``tau``; the energies are sampled at ``checkpoints`` evenly spaced steps.
    Returns per-system final and largest |dE/E0|, and the step statistics
    (time per step of the captured step, checkpoints excluded)."""
    systems = list(systems) if isinstance(systems, (list, tuple)) else [systems]
    ctx = qsym.Context(systems, qsym.make_params(**params))
    try:
        E0 = ctx.energy().copy()
        chunks = np.diff(np.round(np.linspace(0, nsteps, min(checkpoints, nsteps) + 1)).astype(int))
        worst = np.zeros(len(systems))
        dE = np.zeros(len(systems))
        wall, timed = 0.0, 0
        for c, k in enumerate(chunks):
            t0 = time.perf_counter()
            ctx.step(tau, int(k))
            ctx.sync()
            if c > 0:   # the first chunk includes capturing the step graph
                wall += time.perf_counter() - t0
                timed += int(k)
            dE = ctx.energy() / E0 - 1.0
            worst = np.maximum(worst, np.abs(dE))
        st = ctx.stats()
    finally:
        ctx.close()
    return dict(tau=tau, steps=int(nsteps), dE_final=dE.tolist(), dE_max=worst.tolist(),
                encounters=int(st["total_encounters"]), substeps=int(st["total_substeps"]),
                status=int(st["status"]), ms_per_step=1e3 * wall / timed if timed else None)


def tau_scaling(taus=(0.4, 0.2, 0.1, 0.05, 0.025), span: float = 4.0, system=None, **params):
    """Sec. 3, test integrations: one system over a fixed span, several tau."""
    system = system if system is not None else tau_system()
    rows = []
    for t in taus:
        n = int(round(span / t))
        if abs(n * t - span) > 1e-9 * span:
            raise ValueError("span must be a whole number of steps")
        r = run_span([system], t, n, **params)
        r.update(dE_final=r["dE_final"][0], dE_max=r["dE_max"][0])
        r["dE_per_step"] = r["dE_final"] / n
        rows.append(r)
    return dict(system=system.name, n=int(system.n), span=span, rows=rows,
                slope_final=_slope(taus, [abs(r["dE_final"]) for r in rows]),
                slope_max=_slope(taus, [r["dE_max"] for r in rows]),
                slope_per_step=_slope(taus, [abs(r["dE_per_step"]) for r in rows]))


def outer_period(G: float = 1.0, m0: float = 1.0) -> float:
    """Orbital period of the innermost giant planet (a = 5.2)."""
    return 2.0 * math.pi * math.sqrt(inputs.PLANET_A[0] ** 3 / (G * m0))


def sensitivity(aE_values=(0.5, 1.0, 1.5, 2.5, 4.0, 6.0), aH_values=(0.5, 1.0, 2.0, 4.0),
                periods: float = 20.0, seeds=tuple(range(8)), checkpoints: int = 400,
                disk_steps: int = 200, planet_mass: float = 0.0):
    """Sec. 3, sensitivity of parameters.

    Accuracy: the giant planets with 50 times their masses (the paper's
    enhanced outer Solar System, seeded elements), tau = 0.00255 P0, one
    batched context of ``len(seeds)`` realisations per value; the median and
    the largest over realisations of max |dE/E0| over ``periods`` P0.
    a_E is varied at a_H = 1, a_H at a_E = 2.5 (the paper's values).
    Cost: the 4100-body disk, tau = 0.05, ``disk_steps`` steps per a_E value:
    encounter pairs, Hermite substeps and the time per step."""
    systems = [inputs.enhanced_outer(s) for s in seeds]
    P0 = outer_period()
    tau = 0.00255 * P0
    nsteps = int(round(periods / 0.00255))

    def acc(**kw):
        r = run_span(systems, tau, nsteps, checkpoints, planet_mass=planet_mass, **kw)
        mx = np.asarray(r["dE_max"])
        r.update(dE_max_median=float(np.median(mx)), dE_max_worst=float(mx.max()))
        return r

    a_E = [dict(aE=a, **acc(aE=a, aH=1.0)) for a in aE_values]
    a_H = [dict(aH=a, **acc(aE=2.5, aH=a)) for a in aH_values]
    # the paper's values with the whole-system Hermite for planet-planet
    # encounters (every enhanced planet counts as a planet)
    whole = run_span(systems, tau, nsteps, checkpoints, aE=2.5, aH=1.0,
                     planet_mass=min(s.m.min() for s in systems))
    mx = np.asarray(whole["dE_max"])
    whole.update(aE=2.5, aH=1.0, dE_max_median=float(np.median(mx)), dE_max_worst=float(mx.max()))
    disk = disk_system()
    run_span([disk], 0.05, 2)   # warm-up, so the first timing is not an outlier
    cost = [dict(aE=a, **run_span([disk], 0.05, disk_steps, aE=a)) for a in aE_values]
    return dict(outer=dict(systems=[s.name for s in systems], tau=tau, P0=P0, steps=nsteps,
                           periods=periods, planet_mass=planet_mass, a_E=a_E, a_H=a_H,
                           whole_system=whole),
                disk=dict(system=disk.name, n=int(disk.n), tau=0.05, steps=disk_steps, a_E=cost))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default=None, help="write the results as JSON here")
    ap.add_argument("--quick", action="store_true", help="fewer values (a smoke run)")
    a = ap.parse_args()
    if a.quick:
        res = dict(tau_scaling=tau_scaling(taus=(0.2, 0.1, 0.05), span=2.0),
                   sensitivity=sensitivity(aE_values=(1.0, 2.5), aH_values=(1.0, 2.0), periods=2.0,
                                           seeds=(0, 1), disk_steps=40))
    else:
        res = dict(tau_scaling=tau_scaling(), sensitivity=sensitivity())
    res["command"] = "python -m paper_1007_3458_amd.experiments" + (" --quick" if a.quick else "") + \
        (f" --out {a.out}" if a.out else "")
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(json.dumps(res, indent=1) + "\n")
    ts = res["tau_scaling"]
    print(f"tau scaling ({ts['system']}, span {ts['span']}): slope of final |dE| {ts['slope_final']:.3f}, "
          f"of max |dE| {ts['slope_max']:.3f}, per step {ts['slope_per_step']:.3f}", flush=True)
    for r in ts["rows"]:
        print(f"  tau {r['tau']:<7} steps {r['steps']:<5} dE_final {r['dE_final']:+.3e} "
              f"dE_max {r['dE_max']:.3e} per step {r['dE_per_step']:+.3e} enc {r['encounters']}",
              flush=True)
    se = res["sensitivity"]["outer"]
    print(f"enhanced outer planets x{len(se['systems'])}, tau {se['tau']:.4f}, {se['steps']} steps", flush=True)
    for key in ("a_E", "a_H"):
        for r in se[key]:
            print(f"  {key} {r[key.replace('_', '')]:<5} max|dE| median {r['dE_max_median']:.3e} "
                  f"worst {r['dE_max_worst']:.3e} enc {r['encounters']:<7} substeps {r['substeps']:<8} "
                  f"status {r['status']}", flush=True)
    w = se["whole_system"]
    print(f"  whole-system rule on: max|dE| median {w['dE_max_median']:.3e} worst {w['dE_max_worst']:.3e} "
          f"substeps {w['substeps']}", flush=True)
    for r in res["sensitivity"]["disk"]["a_E"]:
        print(f"  disk a_E {r['aE']:<5} enc {r['encounters']:<7} substeps {r['substeps']:<8} "
              f"{r['ms_per_step'] or 0.0:.3f} ms/step", flush=True)


if __name__ == "__main__":
    main()
