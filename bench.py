#!/usr/bin/env python3
"""Benchmark of the hybrid symplectic step on one MI355X.

Default workload: the plain FP64 path on a 16388-body disk (4 planets +
16384 planetesimals of 1e-8, a ~ U[15, 40], Rayleigh e and i), tau = 0.05,
encounter radius 3 mutual Hill radii, encounters on.  One "step" is the
whole hybrid step: drift, kick with the fused crude sweep, Kepler, fine
sweep, sets, corrections + Hermite, second kick, drift.

Prints one JSON line.  `value` is pair-interactions per second (two all-pairs
kicks per step, N(N-1) ordered pairs each per system) over the timed steps,
inputs resident in HBM, as the library runs them: the captured step graph
replayed K times between two device synchronisations.  A separate profiled
pass of the same K steps (eager launches with HIP events around every kernel,
the energy evaluated between segments outside the timed time) gives the
per-kernel averages, the roofline's launch duration and the energy error;
its throughput is reported as `value_profiled`.

Other workloads: --workload disk128k (131076 bodies; with --precision 1 the
FP32 pair-term form, compared with the FP64 path on the same initial
conditions), --workload batch (512 independent systems of 64..4096 bodies),
--workload learned (the learned Kepler start: trained here on the GPU from
1e6 library solves, then the Kepler solve of 1,048,576 test bodies + a
65,540-body disk timed from each start, and whole steps of the disk with
the learned start against the first-order start).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector
FP32_PEAK_TFLOPS = 157.3     # MI355X FP32 vector
FLOP_PAIR = 20               # per ordered pair (sub 3, r^2 5, rsqrt 2, m/r^3 4, fma 6)
FLOP_CRUDE = 6               # per unordered pair (fused crude sweep)
FLOP_ENERGY_PAIR = 12        # per pair potential (sub 3, r^2 5, rsqrt 2, m/r 2)


def workload(name):
    from paper_1007_3458_amd import workloads
    try:
        return workloads.workload(name)
    except ValueError as e:
        raise SystemExit(str(e))


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("qsym_kernels.hpp", "qsym_common.hpp", "qsym.hip"):
        with open(os.path.join(ROOT, "paper_1007_3458_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(name, prec, kernel):
    """HBM bytes per launch of one kick kernel ("fused": with the crude sweep,
    "plain": without) from the committed rocprofv3 counter summary, when it
    was taken on the current kernel sources for that kernel; else None."""
    path = os.path.join(ROOT, "profiles", f"kick_{name}_p{prec}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("source_hash") != kernel_source_hash():
        return None
    return (t.get(kernel) or {}).get("bytes_per_launch")


def cpu_baseline(systems, tau, seconds, swapped=False):
    """The oracle (as it stands) on the host cores, a bounded sample of steps."""
    import oracle
    oracle.build()
    p = oracle.make_params()
    s = max(systems, key=lambda x: x.n)

    def one(q, v):
        if swapped:
            q, v, _, _ = oracle.step_swapped(p, tau, s.m, q, v)
            return q, v
        q, v, _ = oracle.step(p, tau, s.m, s.h, q, v)
        return q, v

    q, v = s.q, s.v
    t0 = time.perf_counter()
    q, v = one(q, v)
    first = time.perf_counter() - t0
    k = max(1, min(200, int(seconds / max(first, 1e-6))))
    t0 = time.perf_counter()
    for _ in range(k):
        q, v = one(q, v)
    dt = time.perf_counter() - t0
    n = s.n
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    cores = oracle.num_threads()
    kicks = 1.0 if swapped else 2.0
    kind = "swapped encounter-free" if swapped else "whole hybrid"
    out = {"value": kicks * n * (n - 1) * k / dt, "unit": "pair-interactions/s",
           "cores": cores, "kind": "oracle",
           "sample": f"{k} {kind} steps of the largest system ({n} bodies) after 1 untimed step",
           "steps_per_s": k / dt, "cpu": model}
    # one thread, one step, when that fits the same time budget
    if dt / k * cores <= seconds:
        oracle.set_threads(1)
        t0 = time.perf_counter()
        q, v = one(q, v)
        d1 = time.perf_counter() - t0
        oracle.set_threads(cores)
        out["single_thread"] = {"value": kicks * n * (n - 1) / d1, "steps": 1}
    return out


def make_context(systems, precision, tau, force_tune, kepler_mode=0, guess=None, sweep=0):
    from paper_1007_3458_amd import qsym
    ctx = qsym.Context(systems, precision=precision, kepler_mode=kepler_mode, guess=guess,
                       sweep=sweep)
    tune_us = None
    if force_tune or ctx.tuned is None:
        tune_us = ctx.autotune(tau)
    src = "autotuned now" if tune_us is not None else "tuned table"
    shape = {"plain": ctx.kick_shape(0), "crude": ctx.kick_shape(1), "source": src,
             "autotune_us": tune_us}
    return ctx, shape


def timed_run(ctx, tau, steps, warmup, graph_pass, checkpoints=10, swapped=False):
    """Warm-up, then `steps` profiled steps (HIP events per kernel) in
    `checkpoints` segments with the energy evaluated between them (outside
    the timed time); returns timings, energies and counters."""
    import torch
    from paper_1007_3458_amd import qsym
    stepper = ctx.step_swapped if swapped else ctx.step
    stepper(tau, warmup)
    ctx.sync()
    E0 = ctx.energy()
    ctx.profile(True)
    seg = max(1, steps // max(1, checkpoints))
    done, T, dEmax = 0, 0.0, np.zeros_like(E0)
    while done < steps:
        k = min(seg, steps - done)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stepper(tau, k)
        ctx.sync()
        torch.cuda.synchronize()
        T += time.perf_counter() - t0
        done += k
        E = ctx.energy()
        dEmax = np.maximum(dEmax, np.abs(E / E0 - 1.0))
    st = ctx.stats()
    ctx.profile(False)
    kern = {}
    for k, name in enumerate(qsym.PHASES):
        if st["phase_calls"][k] and name != "energy":
            kern[name] = st["phase_us"][k] / st["phase_calls"][k]
    ke = qsym.PHASES.index("energy")
    energy_us = st["phase_us"][ke] / st["phase_calls"][ke] if st["phase_calls"][ke] else None
    E1 = E
    graph_sps = None
    if graph_pass:
        torch.cuda.synchronize()
        g0 = time.perf_counter()
        stepper(tau, steps)
        ctx.sync()
        torch.cuda.synchronize()
        graph_sps = steps / (time.perf_counter() - g0)
    st2 = ctx.stats()
    return {"T": T, "kern": kern, "E0": E0, "E1": E1, "dEmax": dEmax, "graph_sps": graph_sps,
            "st": st, "st2": st2, "energy_us": energy_us}


def balance_report(ctx, tau, steps, swapped=False):
    """Load balance of the kick and Hermite launches over `steps` further
    steps profiled with workgroup records: per launch the busy time of each
    compute unit (the union of its workgroups' intervals), the busiest
    unit's against the mean over all the device's units."""
    stepper = ctx.step_swapped if swapped else ctx.step
    ctx.profile(True, records=True)
    stepper(tau, steps)
    ctx.sync()
    st = ctx.stats()
    ctx.profile(False)
    out = {}
    for name, ph in (("kick+crude", 1), ("hermite (k_hermite)", 5), ("kick2", 6)):
        n = st["busy_calls"][ph]
        if n and st["busy_mean_us"][ph] > 0:
            out[name] = {"max_over_mean": st["busy_max_us"][ph] / st["busy_mean_us"][ph],
                         "busy_max_us": st["busy_max_us"][ph] / n,
                         "busy_mean_us": st["busy_mean_us"][ph] / n,
                         "event_us": st["phase_us"][ph] / st["phase_calls"][ph], "launches": n}
    out["compute_units_seen"] = st["busy_units"]
    out["steps"] = steps
    return out


def oracle_energy_report(systems, tau, warmup, steps, dE):
    """The batch's per-system energy errors against the oracle's, integrated
    system by system under the same protocol (stored beside the tests)."""
    path = os.path.join(ROOT, "tests", "golden", "batch_energy_oracle.json")
    if not os.path.exists(path):
        return None
    g = json.load(open(path))
    if (g["n"] != [s_.n for s_ in systems] or g["tau"] != tau or g["warmup_steps"] != warmup
            or g["steps"] != steps or g["energy_every"] != max(1, steps // 10)):
        return None
    dE_o = np.array([float.fromhex(x) for x in g["dE_max"]])
    dE = np.asarray(dE, dtype=np.float64)
    return {"worst_system": int(np.argmax(dE)), "energy_error": float(dE.max()),
            "oracle_worst_system": int(np.argmax(dE_o)), "oracle_energy_error": float(dE_o.max()),
            "max_rel_diff": float(np.max(np.abs(dE - dE_o) / dE_o)),
            "source": "tests/golden/batch_energy_oracle.json (oracle, each system on its own, "
                      "same steps and energy checkpoints)"}


def kick_accels(ctx, m, h, q, v):
    """Accelerations at positions q through the library's kick (velocities
    zeroed so that v = a exactly), state (q, v) restored afterwards."""
    ctx.set_state(m, h, q, np.zeros_like(q))
    ctx.apply_kick(1.0)
    _, a = ctx.get_state()
    ctx.set_state(m, h, q, v)
    return a


def accel_err(a, ref):
    rel = np.linalg.norm(a - ref, axis=1) / np.maximum(np.linalg.norm(ref, axis=1), 1e-300)
    return float(rel.max()), float(np.sqrt(np.mean(rel ** 2)))


def _time_launches(fn, reps):
    """Average device time of `fn` (launches on torch's current stream)."""
    import torch
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        out = fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e3 / reps, out


def learned_report(reps=20):
    """Train the learned start on the GPU (1e6 library Laguerre solves), then
    time the Kepler solve of the 1,048,576 test bodies + 65,540-body disk
    from each start; returns (weights, report)."""
    import torch
    from paper_1007_3458_amd import inputs, learned_guess, qsym
    R = learned_guess.RECIPE
    q, v, dt = inputs.kepler_train(R["n"], R["seed"])
    w, curve, info = learned_guess.train(q, v, dt, batch=R["batch"], epochs=R["epochs"],
                                         lr=R["lr"], lr_final=R["lr_final"],
                                         init_seed=R["init_seed"])
    s = inputs.learned_workload()
    st = qsym.state_tensor(s.q, s.v)
    n = st.shape[1]
    dtt = torch.full((n,), 0.05, dtype=torch.float64, device=st.device)
    modes = {}
    roots = {}
    for mode, name in ((0, "laguerre_from_r0"), (1, "newton_first_order"), (2, "newton_learned")):
        us, (x, it) = _time_launches(
            lambda: qsym.kepler_solve(1.0, st, dtt, mode, w if mode == 2 else None), reps)
        itn = it.cpu().numpy()
        roots[mode] = x.cpu().numpy()
        nw = n // 64 * 64
        modes[name] = {"kernel_us": us, "solves_per_s": n / (us * 1e-6),
                       "iters_mean": float(itn.mean()), "iters_max": int(np.abs(itn).max()),
                       "wave_max_mean": float(np.abs(itn[:nw]).reshape(-1, 64).max(1).mean()),
                       "capped": int((itn < 0).sum())}
    us_g, _ = _time_launches(lambda: qsym.kepler_guess(1.0, st, dtt, w), reps)
    ref = roots[1]
    deltas = {name: float(np.max(np.abs(roots[m] - ref) / np.abs(ref)))
              for m, name in ((0, "laguerre_vs_newton"), (2, "learned_vs_newton"))}
    return w, {
        "kepler_bodies": n, "dt": 0.05,
        "kepler_test": "1048576 massless bodies a~U[0.5,50], e~U[0,0.9], i~U[0,0.1] (seed 6) "
                       "after 4 planets + 65536 planetesimals",
        "modes": modes, "guess_only_us": us_g, "root_rel_delta_max": deltas,
        "training": {"samples": info["n"], "labels": info["labels"], "epochs": R["epochs"],
                     "batch": R["batch"], "lr": [R["lr"], R["lr_final"]],
                     "train_s": info["train_s"], "loss_first_epoch": float(curve[0]),
                     "loss_last_epoch": float(curve[-1]),
                     "curve": [float(c) for c in curve]},
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="disk16k", choices=["disk16k", "disk128k", "small", "batch", "learned"])
    ap.add_argument("--precision", type=int, default=0, choices=[0, 1])
    ap.add_argument("--tau", type=float, default=0.05)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the kick shapes now instead of using the tuned table")
    ap.add_argument("--no-graph-pass", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="precision 1: skip the FP64 run on the same initial conditions")
    ap.add_argument("--no-forms", action="store_true",
                    help="precision 0: skip the FP32 form's run on the same initial conditions")
    ap.add_argument("--no-balance", action="store_true",
                    help="skip the load-balance pass (workgroup records) after the timed run")
    ap.add_argument("--swapped", action="store_true",
                    help="encounter-free steps with E_Kep and E_Int swapped (one kick per step)")
    ap.add_argument("--sweep", choices=["fused", "grid"], default="fused",
                    help="crude sweep fused into the first kick, or on the hashed grid ahead of it")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run 3 plain device-to-device copies of MIB MiB (the reference "
                         "kernel that scales the FETCH_SIZE / WRITE_SIZE counters to bytes)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        nb = args.calibrate_copy << 20
        a = torch.ones(nb, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nb, "copy_bytes_written": nb, "copies": 3}))
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library runs as one process on one MI355X; "
              "sharding a step over several GPUs is not implemented", file=sys.stderr)
        sys.exit(2)
    defaults = {"disk16k": (200, 20), "disk128k": (100, 5), "small": (1000, 50), "batch": (100, 10),
                "learned": (50, 5)}
    steps = args.steps if args.steps is not None else defaults[args.workload][0]
    warmup = args.warmup if args.warmup is not None else defaults[args.workload][1]

    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    systems, desc = workload(args.workload)
    if args.swapped:
        desc = desc.replace("encounters on", "encounter-free step with E_Kep and E_Int swapped")
    ntot = sum(s.n for s in systems)
    npairs = sum(float(s.n) * (s.n - 1) for s in systems)
    extra = {}
    kepler_mode, guess = 0, None
    if args.workload == "learned":
        guess, extra["learned_report"] = learned_report()
        kepler_mode = 2
    sweep = 1 if args.sweep == "grid" else 0
    ctx, shape = make_context(systems, args.precision, args.tau, args.autotune, kepler_mode, guess,
                              sweep)
    if args.workload == "learned" and not args.no_compare:
        # the same disk from the first-order Newton start
        ctx1, _ = make_context(systems, args.precision, args.tau, False, 1)
        r1 = timed_run(ctx1, args.tau, steps, warmup, not args.no_graph_pass)
        q1, _ = ctx1.get_state()
        sps1 = r1["graph_sps"] or steps / r1["T"]
        extra["learned_report"]["step_first_order"] = {
            "value": 2.0 * npairs * sps1, "apply+kepler_us": r1["kern"].get("apply+kepler"),
            "energy_error": float(np.max(r1["dEmax"])),
            "kepler_iters_total": r1["st"]["kepler_iters"]}
        ctx1.close()
    if args.precision == 1 and not args.no_compare:
        # accuracy of the FP32 pair terms against the FP64 kick (which is
        # itself checked against the oracle to 1e-13 by the test suite)
        ctx64, shape64 = make_context(systems, 0, args.tau, args.autotune)
        m = np.concatenate([s_.m for s_ in systems]); h = np.concatenate([s_.h for s_ in systems])
        q0 = np.concatenate([s_.q for s_ in systems]); v0 = np.concatenate([s_.v for s_ in systems])
        e_max, e_rms = accel_err(kick_accels(ctx, m, h, q0, v0), kick_accels(ctx64, m, h, q0, v0))
        r64 = timed_run(ctx64, args.tau, steps, warmup, not args.no_graph_pass)
        e64 = float(np.max(r64["dEmax"]))
        extra["precision_report"] = {
            "accel_rel_err_max": e_max, "accel_rel_err_rms": e_rms,
            "reference": "FP64 kick of the same library on the same state",
            "fp64_value": 2.0 * npairs * (r64["graph_sps"] or steps / r64["T"]),
            "fp64_kick_crude_us": r64["kern"].get("kick+crude"), "fp64_kick_us": r64["kern"].get("kick2"),
            "fp64_energy_error": e64, "fp64_kick_shape": shape64}
    r = timed_run(ctx, args.tau, steps, warmup, not args.no_graph_pass, swapped=args.swapped)
    if (args.precision == 0 and not args.swapped and not args.no_forms and sweep == 0
            and args.workload != "learned"):
        # the FP32 pair-term form on the same initial conditions, steps and
        # energy checkpoints: its speed and energy error against this run;
        # its accelerations at the initial state against a fresh FP64 context
        ctx32, shape32 = make_context(systems, 1, args.tau, args.autotune)
        r32 = timed_run(ctx32, args.tau, steps, warmup, not args.no_graph_pass)
        ctxa, _ = make_context(systems, 0, args.tau, False)
        m = np.concatenate([s_.m for s_ in systems]); h = np.concatenate([s_.h for s_ in systems])
        q0 = np.concatenate([s_.q for s_ in systems]); v0 = np.concatenate([s_.v for s_ in systems])
        e_max, e_rms = accel_err(kick_accels(ctx32, m, h, q0, v0), kick_accels(ctxa, m, h, q0, v0))
        ctx32.close()
        ctxa.close()
        extra["forms"] = {"fp32_pairs": {
            "value": 2.0 * npairs * (r32["graph_sps"] or steps / r32["T"]),
            "steps_per_s": r32["graph_sps"] or steps / r32["T"],
            "energy_error": float(np.max(r32["dEmax"])),
            "accel_rel_err_max": e_max, "accel_rel_err_rms": e_rms,
            "kick_crude_us": r32["kern"].get("kick+crude"), "kick_us": r32["kern"].get("kick2"),
            "kick_shape": shape32}}
    T = r["T"]
    kicks_per_step = 1.0 if args.swapped else 2.0
    value_profiled = kicks_per_step * npairs * steps / T
    gsps = r["graph_sps"]
    value = kicks_per_step * npairs * gsps if gsps else value_profiled
    sps = gsps if gsps else steps / T
    kern = r["kern"]
    energy_err = float(np.max(r["dEmax"]))
    if "precision_report" in extra:
        pr = extra["precision_report"]
        pr["energy_error"] = energy_err
        pr["energy_error_ratio_vs_fp64"] = energy_err / pr["fp64_energy_error"] if pr["fp64_energy_error"] else None
        pr["speedup_vs_fp64"] = value / pr["fp64_value"]
        # the same comparison on the state the FP32 run ended in
        qe, ve = ctx.get_state()
        e_max, e_rms = accel_err(kick_accels(ctx, m, h, qe, ve), kick_accels(ctx64, m, h, qe, ve))
        pr["accel_rel_err_max_end"], pr["accel_rel_err_rms_end"] = e_max, e_rms
        ctx64.close()
    if "forms" in extra:
        f32 = extra["forms"]["fp32_pairs"]
        f32["speedup_vs_fp64"] = f32["value"] / value
        f32["energy_error_ratio_vs_fp64"] = f32["energy_error"] / energy_err if energy_err else None
        f32["same"] = "initial conditions, tau, steps and energy checkpoints as the FP64 run"
    if "learned_report" in extra and "step_first_order" in extra["learned_report"]:
        lr_ = extra["learned_report"]
        q2, _ = ctx.get_state()
        lr_["step_learned"] = {"value": value, "apply+kepler_us": kern.get("apply+kepler"),
                               "energy_error": energy_err,
                               "kepler_iters_total": r["st"]["kepler_iters"]}
        lr_["step_position_rel_delta_max"] = float(np.max(
            np.linalg.norm(q2 - q1, axis=1) / np.linalg.norm(q1, axis=1)))

    # roofline of the dominant kernel: the kick with the fused crude sweep
    # (the plain kick for the swapped step).  Its flops are the algorithmic
    # count of all N(N-1) ordered interactions, also for the symmetric kick,
    # which evaluates each unordered pair once.
    # With the grid sweep both kicks are plain: the roofline is the plain kick.
    plain_roof = args.swapped or sweep == 1
    t_kick = kern.get("kick2") if plain_roof else kern.get("kick+crude")
    kick_name = "k_kick_sym" if shape["plain" if plain_roof else "crude"]["sym"] else "k_kick"
    flops = npairs * FLOP_PAIR + (0 if plain_roof else npairs / 2 * FLOP_CRUDE)
    peak = FP64_PEAK_TFLOPS if args.precision == 0 else FP32_PEAK_TFLOPS
    achieved = flops / (t_kick * 1e-6) / 1e12 if t_kick else None
    roof = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": (achieved / peak) if achieved else None,
            "traffic": measured_traffic(args.workload, args.precision,
                                        "plain" if plain_roof else "fused"),
            "kernel": kick_name + (" (E_Int)" if plain_roof else " (E_Int + fused crude sweep)"),
            "flop_per_launch": flops, "avg_launch_us": t_kick,
            "pairs_per_s_kernel": (npairs / (t_kick * 1e-6)) if t_kick else None}
    out = {
        "metric": "pair-interactions/s and steps/s vs plain FP64 path at matched energy error",
        "value": value,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": 1000.0 / sps,
        "steps_per_s": sps,
        "steps_per_s_graph": gsps,
        "value_profiled": value_profiled,
        "steps_per_s_profiled": steps / T,
        "timing": ("graph replay of the captured step" if gsps else "eager launches with HIP events")
        + "; per-kernel averages from the profiled pass",
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == 0 else "f32 m/r^3 on f64 separations, f64 elsewhere",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}", "n_bodies": ntot, "n_systems": len(systems),
                   "tau": args.tau, "precision": args.precision, "kepler_mode": kepler_mode,
                   "step": "swapped E_Kep/E_Int, no encounter search" if args.swapped else "hybrid",
                   "crude_sweep": None if args.swapped else args.sweep,
                   "kick_shape": shape},
        "energy_error": energy_err,
        "encounters_last_step": r["st"]["n_encounters"],
        "encounters_total": r["st2"]["total_encounters"],
        "hermite_substeps_total": r["st2"]["total_substeps"],
        "kepler_iters_total": r["st2"]["kepler_iters"],
        "kepler_iter_hist": r["st2"]["kepler_hist"],
        "kernel_avg_us": kern,
        "roofline": roof,
    }
    if r["energy_us"]:
        # the energy evaluation (between segments, outside the timed steps):
        # N(N-1)/2 pair potentials of 12 flop each per system
        ep = sum(float(s_.n) * (s_.n - 1) / 2 for s_ in systems)
        out["energy_eval"] = {"avg_us": r["energy_us"], "pair_potentials": ep,
                              "flop_per_pair": FLOP_ENERGY_PAIR,
                              "achieved_tflops": ep * FLOP_ENERGY_PAIR / (r["energy_us"] * 1e-6) / 1e12,
                              "frac_fp64_peak": ep * FLOP_ENERGY_PAIR / (r["energy_us"] * 1e-6) / 1e12
                              / FP64_PEAK_TFLOPS}
    if not args.no_balance:
        out["load_balance"] = balance_report(ctx, args.tau, 10 if args.workload != "disk128k" else 4,
                                             args.swapped)
    if args.workload == "batch" and not args.swapped:
        rep = oracle_energy_report(systems, args.tau, warmup, steps, r["dEmax"])
        if rep:
            out["energy_error_vs_oracle"] = rep
    out.update(extra)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(systems, args.tau, args.cpu_seconds, args.swapped)
    out["host"] = platform.node()
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
