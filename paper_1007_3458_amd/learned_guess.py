"""Learned starting value of the Kepler solve: GPU training and packaged weights.

The network, its features and its target are defined in ``include/qsym.h``
(kepler_mode 2).  Training runs entirely in the library's kernels: the
labels are the library's own converged Kepler roots (Laguerre, Appendix A)
unless the caller supplies roots, features and targets come from the
prepare kernel, the scalers from a reduction kernel, and the weights from
mini-batch Adam driven by the forward/backward kernels.

``python -m paper_1007_3458_amd.learned_guess`` trains on the standard
training solves (1e6 bound orbits, a ~ U[0.5, 50], e ~ U[0, 0.9], isotropic,
dt ~ log-U[0.005, 0.5], seed 5) and writes ``kepler_guess_weights.npy``.
"""
from __future__ import annotations

import argparse
import os
import time

import numpy as np

from . import inputs
from . import qsym

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "kepler_guess_weights.npy")

# training recipe of the packaged weights
RECIPE = dict(n=1_000_000, seed=5, init_seed=7, batch=8192, epochs=30, lr=3e-3, lr_final=3e-5)


def train(q, v, dt, x_root=None, mu=1.0, batch=8192, epochs=30, lr=3e-3, lr_final=3e-5,
          init_seed=7, device="cuda:0"):
    """Train the 4-32-32-1 start on bodies (q, v) with steps dt.

    Returns (weights float32 [1259], per-epoch mean loss, info dict)."""
    import torch

    t0 = time.perf_counter()
    state = qsym.state_tensor(q, v, device)
    n = state.shape[1]
    dt_t = torch.from_numpy(np.ascontiguousarray(np.broadcast_to(np.asarray(dt, np.float64),
                                                                 (n,)))).to(device)
    info = {"n": n, "labels": "given"}
    if x_root is None:
        x, it = qsym.kepler_solve(mu, state, dt_t, 0)
        if bool((it <= 0).any()):
            raise RuntimeError("Kepler solve reached its cap on a training sample")
        info["labels"] = "library Laguerre solve"
    else:
        x = torch.from_numpy(np.ascontiguousarray(x_root, dtype=np.float64)).to(device)
    tr = qsym.GuessTrainer(batch, device)
    try:
        feat = tr.prepare(mu, state, dt_t, x)
        w = torch.zeros(qsym.GUESS_WEIGHTS, dtype=torch.float32, device=device)
        w[:qsym.GUESS_PARAMS] = torch.from_numpy(inputs.guess_init(init_seed).astype(np.float32))
        tr.fit_scalers(feat, w)
        torch.cuda.synchronize(device)
        t1 = time.perf_counter()
        curve = tr.train(w, feat, batch, epochs, lr, lr_final)
        info["train_s"] = time.perf_counter() - t1
    finally:
        tr.close()
    info["total_s"] = time.perf_counter() - t0
    return w.cpu().numpy(), curve, info


def load(path: str = DEFAULT_WEIGHTS) -> np.ndarray:
    """Packaged (or saved) weights; plain .npy, never unpickled."""
    w = np.load(path, allow_pickle=False)
    if w.dtype != np.float32 or w.size != qsym.GUESS_WEIGHTS:
        raise ValueError(f"{path}: expected {qsym.GUESS_WEIGHTS} float32 values")
    return w


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--n", type=int, default=RECIPE["n"])
    ap.add_argument("--epochs", type=int, default=RECIPE["epochs"])
    args = ap.parse_args()
    q, v, dt = inputs.kepler_train(args.n, RECIPE["seed"])
    w, curve, info = train(q, v, dt, batch=RECIPE["batch"], epochs=args.epochs,
                           lr=RECIPE["lr"], lr_final=RECIPE["lr_final"],
                           init_seed=RECIPE["init_seed"])
    np.save(args.out, w)
    print({"out": args.out, "loss_first": float(curve[0]), "loss_last": float(curve[-1]), **info},
          flush=True)


if __name__ == "__main__":
    main()
