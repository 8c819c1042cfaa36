"""ctypes front-end of the FP64 CPU oracle (``qsym_oracle.c`` and
``kepler_guess_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg call it; the HIP product path never does.  Arrays are
numpy float64, positions/velocities shaped (n, 3).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "qsym_oracle.c"), os.path.join(HERE, "kepler_guess_oracle.c")]
LIB = os.path.join(HERE, "liboracle.so")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class Params(C.Structure):
    _fields_ = [("G", C.c_double), ("m0", C.c_double), ("aE", C.c_double), ("aH", C.c_double),
                ("epsH", C.c_double), ("eta", C.c_double), ("eta_s", C.c_double),
                ("crude_safety", C.c_double), ("hill_mode", C.c_int32),
                ("kepler_mode", C.c_int32), ("max_substeps", C.c_int32), ("pad", C.c_int32),
                ("planet_mass", C.c_double)]


class Stats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in (
        "n_candidates", "n_encounters", "n_sets", "max_set", "substeps", "kepler_iters",
        "kepler_max", "kepler_fail", "hermite_fail", "cand_overflow", "whole_system")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


DEFAULTS = dict(G=1.0, m0=1.0, aE=3.0, aH=1.0, epsH=1e-8, eta=0.02, eta_s=0.01,
                crude_safety=1.1, hill_mode=0, kepler_mode=0, max_substeps=100000,
                planet_mass=0.0)


def make_params(**kw) -> Params:
    d = dict(DEFAULTS)
    d.update(kw)
    return Params(d["G"], d["m0"], d["aE"], d["aH"], d["epsH"], d["eta"], d["eta_s"],
                  d["crude_safety"], int(d["hill_mode"]), int(d["kepler_mode"]),
                  int(d["max_substeps"]), 0, float(d["planet_mass"]))


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    stale = not os.path.exists(LIB) or any(
        os.path.getmtime(LIB) < os.path.getmtime(src) for src in SRCS)
    if force or stale:
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", "-fopenmp", "-o", tmp, *SRCS, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        i64, i32, d = C.c_int64, C.c_int32, C.c_double
        pp = C.POINTER(Params)
        sig = {
            "orc_stumpff": (None, [d, _dp, _dp]),
            "orc_kepler_body": (C.c_int, [d, _dp, _dp, d, i32, _dp, _dp, _ip]),
            "orc_kepler_root": (C.c_int, [d, _dp, _dp, d, i32, d, i32, _dp, _ip]),
            "orc_start_admissible": (C.c_int, [d, _dp, _dp, d, d]),
            "orc_kepler_all": (i64, [i64, d, _dp, _dp, d, i32, _dp, _dp, _ip]),
            "orc_drift": (None, [i64, d, _dp, _dp, _dp, d]),
            "orc_prepass": (None, [i64, d, _dp, _dp, _dp, _dp]),
            "orc_accel": (None, [i64, d, _dp, _dp, _dp]),
            "orc_kick": (None, [i64, d, _dp, _dp, _dp, d]),
            "orc_accel_rows": (None, [i64, d, _dp, _dp, i64, C.POINTER(C.c_int64), _dp]),
            "orc_crude": (i64, [i64, pp, d, _dp, _dp, _dp, _dp, _ip, i64]),
            "orc_fine_pair": (C.c_int, [pp, d, _dp, _dp, _dp, _dp, _dp, _dp, _dp, i64, i64,
                                        _dp, _dp, _dp]),
            "orc_fine": (i64, [i64, _ip, pp, d, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _ip, _dp, _dp]),
            "orc_fine_brute": (i64, [i64, i64, C.POINTER(C.c_int64), pp, d, _dp, _dp, _dp, _dp,
                                     _dp, _dp, _dp, _ip, i64]),
            "orc_sets": (i64, [i64, i64, _ip, _ip]),
            "orc_transition": (None, [d, d, _dp, _dp, _dp]),
            "orc_correct_set": (None, [i64, _ip, _dp, _dp, _dp, d, d, d]),
            "orc_hermite_force": (None, [i64, _dp, _dp, _dp, d, d, d, d, _dp, _dp]),
            "orc_hermite_set": (i64, [i64, _ip, _dp, _dp, _dp, pp, d, d]),
            "orc_hkep_set": (d, [i64, _ip, _dp, _dp, _dp, pp, d]),
            "orc_energy": (d, [i64, d, d, _dp, _dp, _dp]),
            "orc_angmom": (None, [i64, _dp, _dp, _dp, _dp]),
            "orc_step": (C.c_int, [i64, pp, d, _dp, _dp, _dp, _dp, i64, _ip, i64, _ip, _dp,
                                   C.POINTER(Stats)]),
            "orc_guess_features": (C.c_int, [d, _dp, _dp, d, _dp, _dp, _dp]),
            "orc_guess_net": (d, [_dp, _dp, _dp, _dp]),
            "orc_guess": (d, [_dp, d, _dp, _dp, d]),
            "orc_guess_target": (d, [d, _dp, _dp, d, d]),
            "orc_guess_dataset": (None, [i64, d, _dp, _dp, _dp, _dp, _dp, _dp]),
            "orc_guess_scalers": (None, [i64, _dp, _dp, _dp]),
            "orc_guess_loss_grad": (d, [_dp, i64, _dp, _dp, _dp]),
            "orc_adam": (None, [i64, _dp, _dp, _dp, _dp, i64, d, d, d, d]),
            "orc_kepler_roots": (i64, [i64, d, _dp, _dp, _dp, i32, _dp, _dp, _ip]),
            "orc_step_swapped": (i64, [i64, pp, d, _dp, _dp, _dp, C.POINTER(C.c_int64)]),
            "orc_num_threads": (C.c_int, []),
            "orc_set_threads": (None, [C.c_int]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a if shape is None else a.reshape(shape)


# ----------------------------------------------------------------- wrappers
def stumpff(y: float):
    c, s = C.c_double(), C.c_double()
    lib().orc_stumpff(float(y), C.byref(c), C.byref(s))
    return c.value, s.value


def kepler(mu, q, v, dt, mode=0):
    """Advance every body by dt on its two-body orbit; returns q1, v1, iters, fails."""
    q = _f64(q, (-1, 3)); v = _f64(v, (-1, 3))
    n = q.shape[0]
    q1 = np.empty_like(q); v1 = np.empty_like(v); it = np.zeros(n, np.int32)
    fails = lib().orc_kepler_all(n, mu, _d(q), _d(v), dt, mode, _d(q1), _d(v1), _i(it))
    return q1, v1, it, int(fails)


def start_admissible(mu, x0, v0, dt, xs):
    x0 = _f64(x0, (3,)); v0 = _f64(v0, (3,))
    return bool(lib().orc_start_admissible(mu, _d(x0), _d(v0), dt, xs))


def kepler_root(mu, x0, v0, dt, mode=0, x_start=None):
    x0 = _f64(x0, (3,)); v0 = _f64(v0, (3,))
    out = C.c_double(); it = C.c_int32()
    fail = lib().orc_kepler_root(mu, _d(x0), _d(v0), dt, mode, 0.0 if x_start is None else x_start,
                                 0 if x_start is None else 1, C.byref(out), C.byref(it))
    return out.value, it.value, fail


def drift(m0, m, q, v, dt):
    q = _f64(q, (-1, 3)).copy(); v = _f64(v, (-1, 3)); m = _f64(m)
    lib().orc_drift(q.shape[0], m0, _d(m), _d(v), _d(q), dt)
    return q


def prepass(mu, q, v):
    q = _f64(q, (-1, 3)); v = _f64(v, (-1, 3))
    n = q.shape[0]
    A = np.empty(n); ve = np.empty(n)
    lib().orc_prepass(n, mu, _d(q), _d(v), _d(A), _d(ve))
    return A, ve


def accel(G, m, q):
    q = _f64(q, (-1, 3)); m = _f64(m)
    a = np.empty_like(q)
    lib().orc_accel(q.shape[0], G, _d(m), _d(q), _d(a))
    return a


def accel_rows(G, m, q, rows):
    """Accelerations of the bodies listed in rows (over all j)."""
    q = _f64(q, (-1, 3)); m = _f64(m)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    a = np.empty((rows.shape[0], 3))
    lib().orc_accel_rows(q.shape[0], G, _d(m), _d(q), rows.shape[0],
                         rows.ctypes.data_as(C.POINTER(C.c_int64)), _d(a))
    return a


def kick(G, m, q, v, dt):
    q = _f64(q, (-1, 3)); v = _f64(v, (-1, 3)).copy(); m = _f64(m)
    lib().orc_kick(q.shape[0], G, _d(m), _d(q), _d(v), dt)
    return v


def crude(params: Params, tau, q, h, A, ve, cap=None):
    q = _f64(q, (-1, 3)); h = _f64(h); A = _f64(A); ve = _f64(ve)
    n = q.shape[0]
    cnt = lib().orc_crude(n, C.byref(params), tau, _d(q), _d(h), _d(A), _d(ve), None, 0)
    pairs = np.zeros((max(cnt, 1), 2), np.int32)
    lib().orc_crude(n, C.byref(params), tau, _d(q), _d(h), _d(A), _d(ve), _i(pairs), cnt)
    return pairs[:cnt]


def fine(params: Params, tau, pairs, m, h, A, q0, v0, q1, v1):
    """Fine-sweep flags of candidate pairs plus the two sides of the comparison."""
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    k = pairs.shape[0]
    flags = np.zeros(max(k, 1), np.int32); lhs = np.zeros(max(k, 1)); rhs = np.zeros(max(k, 1))
    args = [_f64(x) for x in (m, h, A)] + [_f64(x, (-1, 3)) for x in (q0, v0, q1, v1)]
    lib().orc_fine(k, _i(pairs), C.byref(params), tau, *[_d(x) for x in args], _i(flags),
                   _d(lhs), _d(rhs))
    return flags[:k].astype(bool), lhs[:k], rhs[:k]


def fine_brute(params: Params, tau, m, h, A, q0, v0, q1, v1, rows=None):
    """Fine-test flags of every pair that involves a body of rows (all
    bodies when None), without the crude sweep; returns the flagged pairs
    (min, max), unique, lexicographically sorted."""
    q0 = _f64(q0, (-1, 3)); n = q0.shape[0]
    rows = np.arange(n, dtype=np.int64) if rows is None else np.ascontiguousarray(rows, np.int64)
    args = [_f64(x) for x in (m, h, A)] + [q0] + [_f64(x, (-1, 3)) for x in (v0, q1, v1)]
    rp = rows.ctypes.data_as(C.POINTER(C.c_int64))
    cnt = lib().orc_fine_brute(n, rows.shape[0], rp, C.byref(params), tau,
                               *[_d(x) for x in args], None, 0)
    pairs = np.zeros((max(cnt, 1), 2), np.int32)
    lib().orc_fine_brute(n, rows.shape[0], rp, C.byref(params), tau, *[_d(x) for x in args],
                         _i(pairs), cnt)
    pairs = pairs[:cnt]
    if cnt == 0:
        return pairs
    return np.unique(pairs, axis=0)


def sets(n, pairs):
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    label = np.empty(max(n, 1), np.int32)
    ns = lib().orc_sets(n, pairs.shape[0], _i(pairs), _i(label))
    return label[:n], int(ns)


def transition(s, rcrit):
    K, Kp, Kpp = C.c_double(), C.c_double(), C.c_double()
    lib().orc_transition(s, rcrit, C.byref(K), C.byref(Kp), C.byref(Kpp))
    return K.value, Kp.value, Kpp.value


def correct_set(members, m, q, v, G, rcrit, dt):
    mem = np.ascontiguousarray(members, dtype=np.int32)
    v = _f64(v, (-1, 3)).copy()
    lib().orc_correct_set(mem.shape[0], _i(mem), _d(_f64(m)), _d(_f64(q, (-1, 3))), _d(v), G,
                          rcrit, dt)
    return v


def hermite_force(mm, x, u, G, mu, rcrit, eps):
    x = _f64(x, (-1, 3)); u = _f64(u, (-1, 3)); mm = _f64(mm)
    a = np.empty_like(x); j = np.empty_like(x)
    lib().orc_hermite_force(x.shape[0], _d(mm), _d(x), _d(u), G, mu, rcrit, eps, _d(a), _d(j))
    return a, j


def hermite_set(members, m, q, v, params: Params, rcrit, dt):
    mem = np.ascontiguousarray(members, dtype=np.int32)
    q = _f64(q, (-1, 3)).copy(); v = _f64(v, (-1, 3)).copy()
    ns = lib().orc_hermite_set(mem.shape[0], _i(mem), _d(_f64(m)), _d(q), _d(v),
                               C.byref(params), rcrit, dt)
    return q, v, int(ns)


def hkep_set(members, m, q, v, params: Params, rcrit):
    mem = np.ascontiguousarray(members, dtype=np.int32)
    return lib().orc_hkep_set(mem.shape[0], _i(mem), _d(_f64(m)), _d(_f64(q, (-1, 3))),
                              _d(_f64(v, (-1, 3))), C.byref(params), rcrit)


def energy(G, m0, m, q, v):
    q = _f64(q, (-1, 3)); v = _f64(v, (-1, 3))
    return lib().orc_energy(q.shape[0], G, m0, _d(_f64(m)), _d(q), _d(v))


def angmom(m, q, v):
    q = _f64(q, (-1, 3)); v = _f64(v, (-1, 3))
    L = np.zeros(3)
    lib().orc_angmom(q.shape[0], _d(_f64(m)), _d(q), _d(v), _d(L))
    return L


class StepResult:
    """rc, encounter pairs (i < j, lexicographic), component labels (the
    smallest member, -1 outside every set), r_crit of each set (sets in the
    order of their smallest member) and the step's statistics."""

    def __init__(self, rc, pairs, label, rcrit, stats):
        self.rc = rc
        self.pairs = pairs
        self.label = label
        self.rcrit = rcrit
        self.stats = stats


def step(params: Params, tau, m, h, q, v, cand_cap=None, enc_cap=None):
    """One hybrid step; returns (q, v, StepResult)."""
    q = _f64(q, (-1, 3)).copy(); v = _f64(v, (-1, 3)).copy()
    n = q.shape[0]
    cand_cap = 8 * n + 64 if cand_cap is None else cand_cap
    enc_cap = cand_cap if enc_cap is None else enc_cap
    pairs = np.zeros((max(enc_cap, 1), 2), np.int32)
    label = np.zeros(max(n, 1), np.int32)
    rcrit = np.zeros(max(n, 1))
    st = Stats()
    rc = lib().orc_step(n, C.byref(params), tau, _d(_f64(m)), _d(_f64(h)), _d(q), _d(v), cand_cap,
                        _i(pairs), enc_cap, _i(label), _d(rcrit), C.byref(st))
    ne = min(st.n_encounters, enc_cap)
    return q, v, StepResult(rc, pairs[:ne].copy(), label[:n].copy(),
                            rcrit[:st.n_sets].copy(), st.as_dict())


def step_swapped(params: Params, tau, m, q, v, nsteps=1):
    """nsteps encounter-free steps with E_Kep and E_Int swapped; returns
    (q, v, kepler_fails, kepler_iters)."""
    q = _f64(q, (-1, 3)).copy(); v = _f64(v, (-1, 3)).copy()
    m = _f64(m)
    fails, iters = 0, C.c_int64(0)
    for _ in range(nsteps):
        fails += lib().orc_step_swapped(q.shape[0], C.byref(params), tau, _d(m), _d(q), _d(v),
                                        C.byref(iters))
    return q, v, int(fails), int(iters.value)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(k: int) -> None:
    lib().orc_set_threads(int(k))


# ---------------------------------------------------------------------------
# learned starting value of the Kepler solve (kepler_guess_oracle.c)
# ---------------------------------------------------------------------------
GUESS_NPARAM = 1249
GUESS_NWEIGHTS = 1259   # parameters + 10 scalers


def guess_features(mu, x0, v0, dt):
    """(f[4], x_p, T) of one body, or None for dt == 0."""
    x0 = _f64(x0, (3,)); v0 = _f64(v0, (3,))
    f = np.zeros(4); xp = C.c_double(); T = C.c_double()
    if lib().orc_guess_features(mu, _d(x0), _d(v0), dt, _d(f), C.byref(xp), C.byref(T)):
        return None
    return f, xp.value, T.value


def guess_net(w, inp):
    """Network output and hidden activations on standardised inputs."""
    w = _f64(w); inp = _f64(inp, (4,))
    h1 = np.zeros(32); h2 = np.zeros(32)
    o = lib().orc_guess_net(_d(w), _d(inp), _d(h1), _d(h2))
    return o, h1, h2


def guess(w, mu, x0, v0, dt):
    w = _f64(w); x0 = _f64(x0, (3,)); v0 = _f64(v0, (3,))
    assert w.size == GUESS_NWEIGHTS
    return lib().orc_guess(_d(w), mu, _d(x0), _d(v0), dt)


def guess_target(mu, x0, v0, dt, x):
    x0 = _f64(x0, (3,)); v0 = _f64(v0, (3,))
    return lib().orc_guess_target(mu, _d(x0), _d(v0), dt, x)


def guess_dataset(mu, q, v, dt, x):
    """Raw features (n, 4) and targets (n,) of solved bodies."""
    q = _f64(q, (-1, 3)); v = _f64(v, (-1, 3)); n = q.shape[0]
    dt = _f64(np.broadcast_to(np.asarray(dt, np.float64), (n,))); x = _f64(x)
    f = np.zeros((n, 4)); y = np.zeros(n)
    lib().orc_guess_dataset(n, mu, _d(q), _d(v), _d(dt), _d(x), _d(f), _d(y))
    return f, y


def guess_scalers(f, y):
    f = _f64(f, (-1, 4)); y = _f64(y)
    sc = np.zeros(10)
    lib().orc_guess_scalers(f.shape[0], _d(f), _d(y), _d(sc))
    return sc


def guess_loss_grad(w, f, y, want_grad=True):
    w = _f64(w); f = _f64(f, (-1, 4)); y = _f64(y)
    assert w.size == GUESS_NWEIGHTS
    g = np.zeros(GUESS_NPARAM) if want_grad else None
    loss = lib().orc_guess_loss_grad(_d(w), f.shape[0], _d(f), _d(y),
                                     _d(g) if want_grad else None)
    return (loss, g) if want_grad else loss


def adam(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in place on float64 arrays w, m, v."""
    for a in (w, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _f64(g)
    lib().orc_adam(g.size, _d(w), _d(g), _d(m), _d(v), int(t), lr, b1, b2, eps)


def kepler_roots(mu, q, v, dt, mode=0, x_start=None):
    """Universal anomalies of n bodies (per-body dt); returns x, iters, fails."""
    q = _f64(q, (-1, 3)); v = _f64(v, (-1, 3)); n = q.shape[0]
    dt = _f64(np.broadcast_to(np.asarray(dt, np.float64), (n,)))
    xs = None if x_start is None else _f64(x_start)
    x = np.zeros(n); it = np.zeros(n, np.int32)
    fails = lib().orc_kepler_roots(n, mu, _d(q), _d(v), _d(dt), mode,
                                   None if xs is None else _d(xs), _d(x), _i(it))
    return x, it, int(fails)
