"""ctypes binding of ``libqsym.so`` (the C ABI of include/qsym.h).

Argument marshalling only: every step of the integrator runs in the HIP
kernels of the library.  PyTorch provides the device workspace and the
stream.  The library must have been built (``__graft_entry__.build()``);
importing this module on a machine without it raises immediately.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqsym.so")

QSYM_HOST, QSYM_DEVICE = 0, 1
ERRORS = {
    -1: "QSYM_EINVAL", -2: "QSYM_ENOMEM", -3: "QSYM_EHIP", -4: "QSYM_ENONFINITE",
    -5: "QSYM_EKEPLER", -6: "QSYM_EOVERFLOW", -7: "QSYM_ETRUNC", -8: "QSYM_EHERMITE",
}


class QsymError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("G", C.c_double), ("aE", C.c_double), ("aH", C.c_double), ("epsH", C.c_double),
                ("eta", C.c_double), ("eta_s", C.c_double), ("crude_safety", C.c_double),
                ("hill_mode", C.c_int32), ("kepler_mode", C.c_int32), ("precision", C.c_int32),
                ("max_substeps", C.c_int32), ("pair_capacity", C.c_int64),
                ("planet_mass", C.c_double), ("sweep", C.c_int32), ("pad2", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("n_candidates", C.c_int64), ("n_encounters", C.c_int64),
                ("n_sets", C.c_int64), ("max_set", C.c_int64), ("substeps", C.c_int64),
                ("total_encounters", C.c_int64), ("total_substeps", C.c_int64),
                ("kepler_iters", C.c_int64), ("kepler_max", C.c_int64),
                ("kepler_hist", C.c_int64 * 32), ("status", C.c_int64),
                ("phase_us", C.c_double * 12), ("phase_calls", C.c_int64 * 12),
                ("whole_system", C.c_int64), ("fallbacks", C.c_int64), ("overflows", C.c_int64),
                ("global_sets", C.c_int64), ("kepler_restarts", C.c_int64),
                ("busy_max_us", C.c_double * 12), ("busy_mean_us", C.c_double * 12),
                ("busy_calls", C.c_int64 * 12), ("busy_units", C.c_int64)]

    def as_dict(self):
        d = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            d[k] = list(v) if not isinstance(v, (int, float)) else v
        return d


PHASES = ["drift+prepass", "kick+crude", "apply+kepler", "fine", "sets", "hermite", "kick2",
          "apply2+momentum", "drift2", "energy", "momentum", "other"]

DEFAULTS = dict(G=1.0, aE=3.0, aH=1.0, epsH=1e-8, eta=0.02, eta_s=0.01, crude_safety=1.1,
                hill_mode=0, kepler_mode=0, precision=0, max_substeps=100000, pair_capacity=0,
                planet_mass=0.0, sweep=0)


def make_params(**kw) -> Params:
    d = dict(DEFAULTS)
    unknown = set(kw) - set(d)
    if unknown:
        raise TypeError(f"unknown parameters {sorted(unknown)}")
    d.update(kw)
    return Params(float(d["G"]), float(d["aE"]), float(d["aH"]), float(d["epsH"]), float(d["eta"]),
                  float(d["eta_s"]), float(d["crude_safety"]), int(d["hill_mode"]),
                  int(d["kepler_mode"]), int(d["precision"]), int(d["max_substeps"]),
                  int(d["pair_capacity"]), float(d["planet_mass"]), int(d["sweep"]), 0)


_lib = None
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_lp = C.POINTER(C.c_int64)

# name -> (restype, argtypes); kept in the order of include/qsym.h
SIGNATURES = {
    "qsym_workspace_bytes": (C.c_int, [C.POINTER(Params), C.c_int32, _lp, _lp]),
    "qsym_create": (C.c_int, [C.POINTER(Params), C.c_int32, _lp, _dp, C.c_void_p, C.c_int64,
                              C.c_void_p, C.POINTER(C.c_void_p)]),
    "qsym_destroy": (None, [C.c_void_p]),
    "qsym_set_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_int32]),
    "qsym_get_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    "qsym_step": (C.c_int, [C.c_void_p, C.c_double, C.c_int64]),
    "qsym_step_swapped": (C.c_int, [C.c_void_p, C.c_double, C.c_int64]),
    "qsym_sync": (C.c_int, [C.c_void_p]),
    "qsym_energy": (C.c_int, [C.c_void_p, _dp]),
    "qsym_encounters": (C.c_int, [C.c_void_p, _ip, C.c_int64, _lp, _ip]),
    "qsym_set_rcrit": (C.c_int, [C.c_void_p, _dp, C.c_int64, _lp]),
    "qsym_candidates": (C.c_int, [C.c_void_p, _ip, C.c_int64, _lp]),
    "qsym_stats": (C.c_int, [C.c_void_p, C.POINTER(Stats)]),
    "qsym_last_error": (C.c_char_p, [C.c_void_p]),
    "qsym_apply_drift": (C.c_int, [C.c_void_p, C.c_double]),
    "qsym_apply_kick": (C.c_int, [C.c_void_p, C.c_double, C.c_double]),
    "qsym_apply_kepler": (C.c_int, [C.c_void_p, C.c_double]),
    "qsym_fine_test": (C.c_int, [C.POINTER(Params), C.c_double, C.c_double, C.c_int64] +
                       [C.c_void_p] * 7 + [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.c_void_p, C.c_void_p]),
    "qsym_set_kick_shape": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int64,
                                      C.c_int32, C.c_int32]),
    "qsym_get_kick_shape": (C.c_int, [C.c_void_p, C.c_int32, _ip, _ip, _lp, _ip, _ip]),
    "qsym_autotune": (C.c_int, [C.c_void_p, C.c_double, _dp]),
    "qsym_profile": (C.c_int, [C.c_void_p, C.c_int32]),
    "qsym_set_guess": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32]),
    "qsym_kepler_solve": (C.c_int, [C.c_double, C.c_int64, C.c_void_p, C.c_void_p, C.c_int32,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "qsym_kepler_guess": (C.c_int, [C.c_double, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p]),
    "qsym_guess_trainer_create": (C.c_int, [C.c_int64, C.c_void_p, C.POINTER(C.c_void_p)]),
    "qsym_guess_trainer_destroy": (None, [C.c_void_p]),
    "qsym_guess_trainer_error": (C.c_char_p, [C.c_void_p]),
    "qsym_guess_reset": (C.c_int, [C.c_void_p]),
    "qsym_guess_prepare": (C.c_int, [C.c_void_p, C.c_double, C.c_int64, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_int64]),
    "qsym_guess_fit_scalers": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64,
                                         C.c_void_p]),
    "qsym_guess_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int64,
                                  C.c_void_p, _dp]),
    "qsym_guess_grad_static": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64,
                                         C.c_void_p, _dp, C.c_void_p]),
    "qsym_guess_adam": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_double,
                                  C.c_double, C.c_double]),
    "qsym_guess_train": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int64,
                                   C.c_int64, C.c_int32, C.c_double, C.c_double, _dp]),
}

GUESS_PARAMS = 1249
GUESS_WEIGHTS = 1259


def lib():
    """Load libqsym.so (raises if it has not been built).

    torch is imported first: torch carries its own HIP runtime with the same
    soname as the system one, and the process must use a single runtime (the
    one torch allocates device memory and streams with)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (loads torch's HIP runtime before ours binds to it)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _torch():
    import torch
    return torch


@dataclass
class Body:
    """Flattened input of one or several systems."""
    m: np.ndarray
    h: np.ndarray
    q: np.ndarray  # (n, 3)
    v: np.ndarray  # (n, 3)


def _soa(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1, 3).T)


class Context:
    """One library context over one or more independent systems.

    ``systems`` is a list of objects with attributes m, h, q, v, m0 (see
    paper_1007_3458_amd.inputs.System); bodies are concatenated in order.
    """

    def __init__(self, systems, params: Params | None = None, device="cuda:0", shapes="table",
                 guess="packaged", **kw):
        """shapes="table" starts from the tuned kick shapes recorded for this
        workload signature (paper_1007_3458_amd/tuned_shapes.json) when there
        is an entry; None keeps the library defaults.  guess="packaged" loads
        the packaged learned-start weights when kepler_mode is 2 (None
        leaves them unset; an array sets those)."""
        torch = _torch()
        if not isinstance(systems, (list, tuple)):
            systems = [systems]
        self.params = params if params is not None else make_params(**kw)
        self.device = torch.device(device)
        self.nsys = len(systems)
        sizes = [int(s.m.shape[0]) for s in systems]
        self.offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        self.n = int(self.offsets[-1])
        self.m0 = np.array([s.m0 for s in systems], dtype=np.float64)
        L = lib()
        nb = C.c_int64()
        self._check(L.qsym_workspace_bytes(C.byref(self.params), self.nsys,
                                           self.offsets.ctypes.data_as(_lp), C.byref(nb)), None)
        self.ws_bytes = int(nb.value)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        rc = L.qsym_create(C.byref(self.params), self.nsys, self.offsets.ctypes.data_as(_lp),
                           self.m0.ctypes.data_as(_dp), C.c_void_p(self._ws_ptr),
                           self.ws_bytes, C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc != 0:
            raise QsymError(rc, lib().qsym_last_error(None).decode())
        self.ctx = h
        m = np.concatenate([s.m for s in systems]).astype(np.float64)
        hh = np.concatenate([s.h for s in systems]).astype(np.float64)
        q = np.concatenate([np.asarray(s.q).reshape(-1, 3) for s in systems])
        v = np.concatenate([np.asarray(s.v).reshape(-1, 3) for s in systems])
        self.set_state(m, hh, q, v)
        self.tuned = None
        if shapes == "table":
            from . import tune
            e = tune.lookup(sizes, self.params.precision, self.params.hill_mode)
            if e:
                for w, key in ((0, "plain"), (1, "crude")):
                    sh = e[key]
                    self.set_kick_shape(sh["ipl"], sh["block"], sh["jchunk"], sh["remap"], which=w,
                                        sym=sh.get("sym", 0))
                self.tuned = e
        if self.params.kepler_mode == 2 and guess is not None:
            if isinstance(guess, str) and guess == "packaged":
                from . import learned_guess
                guess = learned_guess.load()
            self.set_guess(guess)

    # ---------------------------------------------------------- helpers
    def _check(self, rc, ctx):
        if rc != 0:
            raise QsymError(rc, lib().qsym_last_error(ctx).decode())

    def _c(self, rc):
        self._check(rc, self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            lib().qsym_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ state
    def set_state(self, m, h, q, v):
        self.m = np.ascontiguousarray(m, dtype=np.float64)
        self.h = np.ascontiguousarray(h, dtype=np.float64)
        qs, vs = _soa(q), _soa(v)
        self._c(lib().qsym_set_state(self.ctx, self.m.ctypes.data, self.h.ctypes.data,
                                     qs.ctypes.data, vs.ctypes.data, QSYM_HOST))

    def set_state_device(self, m, h, q, v):
        """Device tensors: m, h (n,), q, v (3, n) float64 on this device."""
        self._c(lib().qsym_set_state(self.ctx, m.data_ptr(), h.data_ptr(), q.data_ptr(),
                                     v.data_ptr(), QSYM_DEVICE))

    def get_state(self, check=True):
        """Positions and velocities (n, 3).  check=False returns them even when
        the device status reports an error (they are copied first)."""
        qs = np.empty((3, self.n)); vs = np.empty((3, self.n))
        rc = lib().qsym_get_state(self.ctx, qs.ctypes.data, vs.ctypes.data, QSYM_HOST)
        if check or rc in (-1, -3):
            self._c(rc)
        return qs.T.copy(), vs.T.copy()

    # ------------------------------------------------------------- steps
    def step(self, tau: float, nsteps: int = 1):
        self._c(lib().qsym_step(self.ctx, float(tau), int(nsteps)))

    def step_swapped(self, tau: float, nsteps: int = 1):
        """Encounter-free steps with E_Kep and E_Int swapped (one kick per step)."""
        self._c(lib().qsym_step_swapped(self.ctx, float(tau), int(nsteps)))

    def sync(self):
        self._c(lib().qsym_sync(self.ctx))

    def energy(self) -> np.ndarray:
        E = np.zeros(self.nsys)
        self._c(lib().qsym_energy(self.ctx, E.ctypes.data_as(_dp)))
        return E

    def encounters(self, cap: int | None = None):
        """Encounter pairs of the last step (sorted) and each body's set id."""
        if cap is None:
            cap = max(int(self.stats()["n_encounters"]), 1)
        pairs = np.zeros((cap, 2), np.int32)
        n = C.c_int64()
        sid = np.zeros(self.n, np.int32)
        self._c(lib().qsym_encounters(self.ctx, pairs.ctypes.data_as(_ip), cap, C.byref(n),
                                      sid.ctypes.data_as(_ip)))
        return pairs[: n.value].copy(), sid

    def set_rcrit(self) -> np.ndarray:
        """r_crit of each encounter set of the last step, sets numbered by
        their smallest member (as encounters() numbers them)."""
        n = C.c_int64()
        cap = max(int(self.stats()["n_sets"]), 1)
        out = np.zeros(cap)
        self._c(lib().qsym_set_rcrit(self.ctx, out.ctypes.data_as(_dp), cap, C.byref(n)))
        return out[: n.value].copy()

    def candidates(self, cap: int | None = None):
        cap = cap if cap is not None else 8 * self.n + 1024
        pairs = np.zeros((max(cap, 1), 2), np.int32)
        n = C.c_int64()
        self._c(lib().qsym_candidates(self.ctx, pairs.ctypes.data_as(_ip), cap, C.byref(n)))
        return pairs[: n.value].copy()

    def stats(self) -> dict:
        st = Stats()
        self._c(lib().qsym_stats(self.ctx, C.byref(st)))
        return st.as_dict()

    # ---------------------------------------------------- operator level
    def apply_drift(self, dt):
        self._c(lib().qsym_apply_drift(self.ctx, float(dt)))

    def apply_kick(self, dt, crude_tau=0.0):
        self._c(lib().qsym_apply_kick(self.ctx, float(dt), float(crude_tau)))

    def apply_kepler(self, dt):
        self._c(lib().qsym_apply_kepler(self.ctx, float(dt)))

    # -------------------------------------------------------- tuning
    def set_kick_shape(self, ipl, block, jchunk, remap=1, which=-1, sym=0):
        """which: 0 plain kick, 1 kick with the crude sweep, -1 both; sym > 0
        selects the symmetric kick with sym i-blocks per work item."""
        self._c(lib().qsym_set_kick_shape(self.ctx, which, ipl, block, jchunk, remap, sym))

    def kick_shape(self, which=1):
        a, b, r, y = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        j = C.c_int64()
        self._c(lib().qsym_get_kick_shape(self.ctx, which, C.byref(a), C.byref(b), C.byref(j),
                                          C.byref(r), C.byref(y)))
        return dict(ipl=a.value, block=b.value, jchunk=j.value, remap=r.value, sym=y.value)

    def autotune(self, tau):
        """Tune both kick shapes; returns (plain_us, crude_us)."""
        us = (C.c_double * 2)()
        self._c(lib().qsym_autotune(self.ctx, float(tau), us))
        return us[0], us[1]

    def profile(self, enable=True, records=False):
        """Per-kernel timings; records=True also collects the workgroup
        records behind the busy_* load-balance statistics."""
        self._c(lib().qsym_profile(self.ctx, (2 if records else 1) if enable else 0))

    def set_guess(self, weights):
        """Weights of the learned Kepler start (kepler_mode 2): a host array
        or a device tensor of GUESS_WEIGHTS float32 values."""
        torch = _torch()
        if isinstance(weights, torch.Tensor):
            if weights.dtype != torch.float32 or weights.numel() != GUESS_WEIGHTS or \
                    not weights.is_cuda or not weights.is_contiguous():
                raise ValueError("weights: contiguous float32 device tensor of 1259 values")
            torch.cuda.current_stream(weights.device).synchronize()
            self._c(lib().qsym_set_guess(self.ctx, C.c_void_p(weights.data_ptr()), QSYM_DEVICE))
        else:
            w = np.ascontiguousarray(weights, dtype=np.float32).ravel()
            if w.size != GUESS_WEIGHTS:
                raise ValueError("weights must hold 1259 values")
            self._c(lib().qsym_set_guess(self.ctx, C.c_void_p(w.ctypes.data), QSYM_HOST))


def fine_test(params: Params, m0, tau, m, h, A, q0, v0, q1, v1, pairs, device="cuda:0"):
    """Standalone fine sweep (Sec. 2.4) on the GPU; returns flags, lhs, rhs."""
    torch = _torch()
    dev = torch.device(device)

    def t(a, soa=False):
        a = _soa(a) if soa else np.ascontiguousarray(a, dtype=np.float64)
        return torch.from_numpy(a).to(dev)

    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    k = pairs.shape[0]
    n = int(np.asarray(m).shape[0])
    if k and (pairs.min() < 0 or pairs.max() >= n):
        raise ValueError("pair index outside [0, n)")
    for a in (h, A):
        if np.asarray(a).shape[0] != n:
            raise ValueError("per-body arrays must all have n entries")
    for a in (q0, v0, q1, v1):
        if np.asarray(a).reshape(-1, 3).shape[0] != n:
            raise ValueError("state arrays must be (n, 3)")
    tm, th, tA = t(m), t(h), t(A)
    tq0, tv0, tq1, tv1 = t(q0, True), t(v0, True), t(q1, True), t(v1, True)
    tp = torch.from_numpy(pairs).to(dev)
    flags = torch.zeros(max(k, 1), dtype=torch.int32, device=dev)
    lhs = torch.zeros(max(k, 1), dtype=torch.float64, device=dev)
    rhs = torch.zeros(max(k, 1), dtype=torch.float64, device=dev)
    st = torch.cuda.current_stream(dev)
    rc = lib().qsym_fine_test(C.byref(params), float(m0), float(tau), n, tm.data_ptr(), th.data_ptr(),
                              tA.data_ptr(), tq0.data_ptr(), tv0.data_ptr(), tq1.data_ptr(),
                              tv1.data_ptr(), k, tp.data_ptr(), flags.data_ptr(), lhs.data_ptr(),
                              rhs.data_ptr(), C.c_void_p(st.cuda_stream))
    if rc != 0:
        raise QsymError(rc, "qsym_fine_test failed")
    return (flags.cpu().numpy()[:k].astype(bool), lhs.cpu().numpy()[:k], rhs.cpu().numpy()[:k])


# ---------------------------------------------------------------------------
# stand-alone Kepler solves and the learned start
# ---------------------------------------------------------------------------
def state_tensor(q, v, device="cuda:0"):
    """(n, 3) positions and velocities -> device float64 SoA [6][n]."""
    torch = _torch()
    q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
    v = np.asarray(v, dtype=np.float64).reshape(-1, 3)
    if q.shape != v.shape:
        raise ValueError("q and v must have the same shape")
    return torch.from_numpy(np.ascontiguousarray(np.concatenate([q.T, v.T]))).to(device)


def _dev_f64(a, n, device):
    torch = _torch()
    if isinstance(a, torch.Tensor):
        if a.dtype != torch.float64 or a.numel() != n or not a.is_cuda or not a.is_contiguous():
            raise ValueError("expected a contiguous float64 device tensor of n values")
        return a
    a = np.ascontiguousarray(np.broadcast_to(np.asarray(a, np.float64), (n,)))
    return torch.from_numpy(a).to(device)


def _weights_dev(w, device):
    torch = _torch()
    if isinstance(w, torch.Tensor):
        if w.dtype != torch.float32 or w.numel() != GUESS_WEIGHTS or not w.is_cuda \
                or not w.is_contiguous():
            raise ValueError("weights: contiguous float32 device tensor of 1259 values")
        return w
    w = np.ascontiguousarray(w, dtype=np.float32).ravel()
    if w.size != GUESS_WEIGHTS:
        raise ValueError("weights must hold 1259 values")
    return torch.from_numpy(w).to(device)


def kepler_solve(mu, state, dt, mode=0, weights=None, device="cuda:0"):
    """Universal anomalies (Appendix A) of the bodies of a device SoA state
    [6][n] with per-body steps; returns device tensors (x, iters), iters < 0
    where every start reached the iteration cap."""
    torch = _torch()
    n = state.shape[1]
    if state.dtype != torch.float64 or state.shape[0] != 6 or not state.is_contiguous():
        raise ValueError("state: contiguous float64 device tensor [6][n]")
    dt_t = _dev_f64(dt, n, state.device)
    w = _weights_dev(weights, state.device) if weights is not None else None
    if mode == 2 and w is None:
        raise ValueError("mode 2 needs weights")
    x = torch.empty(max(n, 1), dtype=torch.float64, device=state.device)
    it = torch.empty(max(n, 1), dtype=torch.int32, device=state.device)
    st = torch.cuda.current_stream(state.device)
    rc = lib().qsym_kepler_solve(float(mu), n, C.c_void_p(state.data_ptr()),
                                 C.c_void_p(dt_t.data_ptr()), int(mode),
                                 C.c_void_p(w.data_ptr() if w is not None else 0),
                                 C.c_void_p(x.data_ptr()), C.c_void_p(it.data_ptr()),
                                 C.c_void_p(st.cuda_stream))
    if rc != 0:
        raise QsymError(rc, "qsym_kepler_solve failed")
    return x[:n], it[:n]


def kepler_guess(mu, state, dt, weights, device="cuda:0"):
    """The learned start alone (device tensor [n])."""
    torch = _torch()
    n = state.shape[1]
    dt_t = _dev_f64(dt, n, state.device)
    w = _weights_dev(weights, state.device)
    x = torch.empty(max(n, 1), dtype=torch.float64, device=state.device)
    st = torch.cuda.current_stream(state.device)
    rc = lib().qsym_kepler_guess(float(mu), n, C.c_void_p(state.data_ptr()),
                                 C.c_void_p(dt_t.data_ptr()), C.c_void_p(w.data_ptr()),
                                 C.c_void_p(x.data_ptr()), C.c_void_p(st.cuda_stream))
    if rc != 0:
        raise QsymError(rc, "qsym_kepler_guess failed")
    return x[:n]


GUESS_STATIC_MAX = 16384


def guess_grad_static(weights, feat, n=None, offset=0):
    """The learned start's loss gradient without a trainer and without any
    allocation by the library (its scratch is a static device array): returns
    (dL/dw device [1249], L) over samples [offset, offset + n) of feat."""
    torch = _torch()
    n = feat.shape[1] - offset if n is None else n
    g = torch.empty(GUESS_PARAMS, dtype=torch.float32, device=feat.device)
    loss = C.c_double()
    st = torch.cuda.current_stream(feat.device)
    rc = lib().qsym_guess_grad_static(C.c_void_p(weights.data_ptr()),
                                      C.c_void_p(feat.data_ptr() + 4 * offset), feat.shape[1], n,
                                      C.c_void_p(g.data_ptr()), C.byref(loss),
                                      C.c_void_p(st.cuda_stream))
    if rc != 0:
        raise QsymError(rc, lib().qsym_last_error(None).decode())
    return g, loss.value


class GuessTrainer:
    """Device-side training of the learned Kepler start (forward, backward
    and Adam kernels of the library) on torch's current stream."""

    def __init__(self, max_batch: int, device="cuda:0"):
        torch = _torch()
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        self.tr = C.c_void_p()
        rc = lib().qsym_guess_trainer_create(int(max_batch), C.c_void_p(self.stream.cuda_stream),
                                             C.byref(self.tr))
        if rc != 0:
            raise QsymError(rc, "qsym_guess_trainer_create failed")
        self.max_batch = int(max_batch)

    def _c(self, rc, what):
        if rc != 0:
            msg = lib().qsym_guess_trainer_error(self.tr)
            raise QsymError(rc, f"{what}: " + (msg.decode() if msg else ""))

    def close(self):
        if self.tr:
            lib().qsym_guess_trainer_destroy(self.tr)
            self.tr = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def prepare(self, mu, state, dt, x_root=None):
        """Features and targets [5][n] (device float32) of solved bodies."""
        torch = _torch()
        n = state.shape[1]
        dt_t = _dev_f64(dt, n, state.device)
        xr = _dev_f64(x_root, n, state.device) if x_root is not None else None
        feat = torch.empty((5, max(n, 1)), dtype=torch.float32, device=state.device)
        self._c(lib().qsym_guess_prepare(self.tr, float(mu), n, C.c_void_p(state.data_ptr()),
                                         C.c_void_p(dt_t.data_ptr()),
                                         C.c_void_p(xr.data_ptr() if xr is not None else 0),
                                         C.c_void_p(feat.data_ptr()), feat.shape[1]),
                "guess_prepare")
        return feat

    def fit_scalers(self, feat, weights, n=None):
        n = feat.shape[1] if n is None else n
        self._c(lib().qsym_guess_fit_scalers(self.tr, C.c_void_p(feat.data_ptr()), feat.shape[1],
                                             n, C.c_void_p(weights.data_ptr())), "fit_scalers")

    def grad(self, weights, feat, n=None, offset=0):
        """(dL/dw device [1249], L) over samples [offset, offset + n)."""
        torch = _torch()
        n = feat.shape[1] - offset if n is None else n
        g = torch.empty(GUESS_PARAMS, dtype=torch.float32, device=self.device)
        loss = C.c_double()
        self._c(lib().qsym_guess_grad(self.tr, C.c_void_p(weights.data_ptr()),
                                      C.c_void_p(feat.data_ptr() + 4 * offset), feat.shape[1], n,
                                      C.c_void_p(g.data_ptr()), C.byref(loss)), "guess_grad")
        return g, loss.value

    def adam(self, weights, grad, lr, b1=0.9, b2=0.999, eps=1e-8):
        self._c(lib().qsym_guess_adam(self.tr, C.c_void_p(weights.data_ptr()),
                                      C.c_void_p(grad.data_ptr()), lr, b1, b2, eps), "guess_adam")

    def reset(self):
        self._c(lib().qsym_guess_reset(self.tr), "guess_reset")

    def train(self, weights, feat, batch, epochs, lr, lr_final=0.0, n=None):
        """Mini-batch Adam over the samples; returns each epoch's mean loss."""
        n = feat.shape[1] if n is None else n
        curve = np.zeros(epochs)
        self._c(lib().qsym_guess_train(self.tr, C.c_void_p(weights.data_ptr()),
                                       C.c_void_p(feat.data_ptr()), feat.shape[1], n, int(batch),
                                       int(epochs), float(lr), float(lr_final),
                                       curve.ctypes.data_as(_dp)), "guess_train")
        return curve
