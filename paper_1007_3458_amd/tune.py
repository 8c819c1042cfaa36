"""Kick launch-shape table: tune on the GPU and store per workload signature.

``python -m paper_1007_3458_amd.tune --workload disk16k`` runs the library's
autotuner (both kicks) on that workload and records the chosen shapes in
``tuned_shapes.json`` next to this file; contexts whose signature (system
sizes, precision, Hill mode) matches an entry start from those shapes.
"""
from __future__ import annotations

import argparse
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tuned_shapes.json")


def signature(sizes, precision, hill_mode) -> str:
    sizes = [int(n) for n in sizes]
    return f"n{sum(sizes)}_s{len(sizes)}_max{max(sizes) if sizes else 0}_p{precision}_h{hill_mode}"


def load() -> dict:
    if not os.path.exists(TABLE):
        return {}
    with open(TABLE) as fh:
        return json.load(fh)


def lookup(sizes, precision, hill_mode):
    return load().get(signature(sizes, precision, hill_mode))


def store(sizes, precision, hill_mode, entry, path=TABLE):
    table = load() if os.path.exists(path) else {}
    table[signature(sizes, precision, hill_mode)] = entry
    with open(path, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="disk16k")
    ap.add_argument("--precision", type=int, default=0)
    ap.add_argument("--tau", type=float, default=0.05)
    ap.add_argument("--copy-to", default=None)
    args = ap.parse_args()
    from paper_1007_3458_amd import qsym
    from paper_1007_3458_amd.workloads import workload
    systems, _ = workload(args.workload)
    ctx = qsym.Context(systems, precision=args.precision, shapes=None)
    us = ctx.autotune(args.tau)
    entry = {"plain": ctx.kick_shape(0), "crude": ctx.kick_shape(1), "us": list(us),
             "workload": args.workload}
    sizes = [s.n for s in systems]
    store(sizes, args.precision, ctx.params.hill_mode, entry)
    if args.copy_to:
        store(sizes, args.precision, ctx.params.hill_mode, entry, path=args.copy_to)
    print(json.dumps(entry), flush=True)


if __name__ == "__main__":
    main()
