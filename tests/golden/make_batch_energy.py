"""Write batch_energy_oracle.json: the oracle's relative energy error for
every system of the 512-system batch (tau = 0.05; 10 steps, then 100 steps
with the energy taken every 10 steps against the energy after the first 10).

This is the reference against which the library's energy error on the batch
is compared: each system is integrated by the oracle on its own (the systems
of a batch do not interact).  Only the oracle and the seeded input generators
are used.  Run from the repository root:  python tests/golden/make_batch_energy.py
"""
import json
import multiprocessing as mp
import os
import sys
import time

os.environ.setdefault("OMP_NUM_THREADS", "1")
ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

TAU, WARMUP, STEPS, EVERY = 0.05, 10, 100, 10
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch_energy_oracle.json")


def run(k):
    import numpy as np
    import oracle
    from paper_1007_3458_amd import inputs
    b = inputs.batch_system(k, int(inputs.batch_sizes()[k]))
    p = oracle.make_params(G=b.G, m0=b.m0)
    q, v = b.q, b.v
    enc = sub = 0
    for s in range(WARMUP + STEPS):
        if s == WARMUP:
            E0 = oracle.energy(b.G, b.m0, b.m, q, v)
            dE = 0.0
        q, v, r = oracle.step(p, TAU, b.m, b.h, q, v)
        assert r.rc == 0, (k, s, r.rc)
        enc += len(r.pairs)
        sub += int(r.stats["substeps"])
        if s + 1 > WARMUP and (s + 1 - WARMUP) % EVERY == 0:
            dE = max(dE, abs(oracle.energy(b.G, b.m0, b.m, q, v) / E0 - 1.0))
    return k, b.n, dE, enc, sub


def main():
    from paper_1007_3458_amd import inputs
    nsys = len(inputs.batch_sizes())
    t0 = time.time()
    with mp.Pool(min(8, os.cpu_count() or 1)) as pool:
        res = sorted(pool.imap_unordered(run, range(nsys), chunksize=1))
    out = {"what": "oracle energy error per system of the 512-system batch",
           "tau": TAU, "warmup_steps": WARMUP, "steps": STEPS, "energy_every": EVERY,
           "n": [r[1] for r in res], "dE_max": [float.hex(r[2]) for r in res],
           "encounter_pairs": [r[3] for r in res], "substeps": [r[4] for r in res]}
    with open(OUT, "w") as f:
        json.dump(out, f, indent=0)
    w = max(res, key=lambda r: r[2])
    print(f"{nsys} systems in {time.time() - t0:.0f} s; worst system {w[0]} (n={w[1]}) dE={w[2]:.3e}")


if __name__ == "__main__":
    main()
