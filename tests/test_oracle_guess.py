"""Pins of the oracle of the learned Kepler starting value (features, network,
loss gradient, Adam) against finite differences, closed forms and the
symmetries of Kepler's equation in universal variables (Appendix A)."""
import numpy as np
import pytest

import oracle
from paper_1007_3458_amd import inputs

NP = oracle.GUESS_NPARAM


def _weights(seed, scale=0.5):
    rng = np.random.Generator(np.random.PCG64(seed))
    w = np.zeros(oracle.GUESS_NWEIGHTS)
    w[:NP] = rng.normal(size=NP) * scale
    w[NP:NP + 4] = rng.normal(size=4)
    w[NP + 4:NP + 8] = rng.uniform(0.5, 2.0, 4)
    w[NP + 8] = 0.1
    w[NP + 9] = 0.7
    return w


def _data(n, seed):
    q, u, dt = inputs.kepler_train(n, seed)
    x, it, fails = oracle.kepler_roots(1.0, q, u, dt, 0)
    assert fails == 0
    f, y = oracle.guess_dataset(1.0, q, u, dt, x)
    return q, u, dt, x, f, y


def test_gradient_matches_central_differences():
    """Backpropagated dL/dw equals the 4th-order central difference of the
    FP64 loss for every one of the 1249 parameters."""
    _, _, _, _, f, y = _data(48, 11)
    w = _weights(3)
    loss, g = oracle.guess_loss_grad(w, f, y)
    h = 1e-4
    fd = np.zeros(NP)
    for p in range(NP):
        vals = []
        for s in (-2, -1, 1, 2):
            ww = w.copy()
            ww[p] += s * h
            vals.append(oracle.guess_loss_grad(ww, f, y, want_grad=False))
        fd[p] = (vals[0] - 8 * vals[1] + 8 * vals[2] - vals[3]) / (12 * h)
    scale = np.abs(g).max()
    assert np.abs(fd - g).max() <= 1e-7 * scale
    # every block of the parameter vector is exercised
    for lo, hi in ((0, 128), (128, 160), (160, 1184), (1184, 1216), (1216, 1248), (1248, 1249)):
        assert np.abs(g[lo:hi]).max() > 1e-6 * scale


def test_network_wiring_closed_form():
    """With one path through the network, o = b3 + tanh(beta tanh(alpha i_j)):
    pins W1 row/column order, W2 orientation (row = second-layer unit) and
    the W3/b3 offsets."""
    inp = np.array([0.3, -0.7, 1.1, 0.25])
    for j in range(4):
        for k in (1, 17, 31):
            w = np.zeros(oracle.GUESS_NWEIGHTS)
            alpha, beta = 0.9, -1.3
            w[4 * (k - 1) + j] = alpha             # W1[k-1][j]
            w[160 + 32 * k + (k - 1)] = beta       # W2[k][k-1]
            w[1216 + k] = 2.0                      # W3[k]
            w[1248] = 0.125                        # b3
            o, h1, h2 = oracle.guess_net(w, inp)
            assert o == pytest.approx(0.125 + 2.0 * np.tanh(beta * np.tanh(alpha * inp[j])),
                                      rel=1e-15)
            assert h1[k - 1] == pytest.approx(np.tanh(alpha * inp[j]), rel=1e-15)
            assert np.count_nonzero(h1) == 1 and np.count_nonzero(h2) == 1
    # biases alone: o = b3 + sum_k W3_k tanh(b2_k + sum_c W2_kc tanh(b1_c))
    w = np.zeros(oracle.GUESS_NWEIGHTS)
    w[128:160] = np.linspace(-1, 1, 32)
    w[1184:1216] = np.linspace(0.5, -0.5, 32)
    w[160:1184] = np.eye(32).ravel() * 0.5
    w[1216:1248] = 1.0
    o, _, _ = oracle.guess_net(w, inp)
    assert o == pytest.approx(np.sum(np.tanh(np.linspace(0.5, -0.5, 32)
                                             + 0.5 * np.tanh(np.linspace(-1, 1, 32)))),
                              rel=1e-14)


def test_features_scale_invariance_and_time_reversal():
    """Lengths x lam and times x lam^1.5 (mu fixed) leave f1, f2, f3 and the
    target unchanged and shift f0 by ln lam; reversing v and dt together
    leaves every feature unchanged."""
    q, u, dt = inputs.kepler_train(20, 13)
    lam = 3.7
    for i in range(20):
        f, xp, T = oracle.guess_features(1.0, q[i], u[i], dt[i])
        fs, xps, Ts = oracle.guess_features(1.0, lam * q[i], u[i] / np.sqrt(lam),
                                            dt[i] * lam ** 1.5)
        assert fs[0] == pytest.approx(f[0] + np.log(lam), abs=1e-14)
        assert np.allclose(fs[1:], f[1:], rtol=1e-13, atol=1e-13)
        assert Ts == pytest.approx(T, rel=1e-13)
        assert xps == pytest.approx(xp * np.sqrt(lam), rel=1e-13)
        fr, xpr, Tr = oracle.guess_features(1.0, q[i], -u[i], -dt[i])
        assert np.array_equal(fr, f) and xpr == -xp and Tr == T
    assert oracle.guess_features(1.0, q[0], u[0], 0.0) is None


def test_kepler_root_is_odd_under_time_reversal():
    """x(x0, v0, -dt) = -x(x0, -v0, dt): the symmetry that lets the sign of
    the step ride on f1."""
    q, u, dt = inputs.kepler_train(200, 17)
    xf, _, ff = oracle.kepler_roots(1.0, q, -u, dt, 1)
    xb, _, fb = oracle.kepler_roots(1.0, q, u, -dt, 1)
    assert ff == 0 and fb == 0
    assert np.allclose(xb, -xf, rtol=1e-13, atol=0)


def test_guess_inverts_target():
    """A network whose output is the standardised target reproduces the root
    exactly (up to rounding), forward and backward in time."""
    q, u, dt = inputs.kepler_train(50, 19)
    for sgn in (1.0, -1.0):
        x, _, _ = oracle.kepler_roots(1.0, q, u, sgn * dt, 0)
        for i in range(50):
            y = oracle.guess_target(1.0, q[i], u[i], sgn * dt[i], x[i])
            w = np.zeros(oracle.GUESS_NWEIGHTS)
            w[NP + 4:NP + 8] = 1.0
            w[NP + 8], w[NP + 9] = 0.25, 2.0
            w[1248] = (y - 0.25) / 2.0            # o = b3
            g = oracle.guess(w, 1.0, q[i], u[i], sgn * dt[i])
            assert g == pytest.approx(x[i], rel=1e-12)


def test_adam_constant_gradient_closed_form():
    """Under a constant gradient the bias-corrected moments equal g and g^2,
    so every step moves w by exactly lr g / (|g| + eps)."""
    rng = np.random.Generator(np.random.PCG64(23))
    g = rng.normal(size=100) * np.logspace(-6, 2, 100)
    w0 = rng.normal(size=100)
    w, m, v = w0.copy(), np.zeros(100), np.zeros(100)
    T, lr, eps = 25, 3e-3, 1e-8
    for t in range(1, T + 1):
        oracle.adam(w, g, m, v, t, lr, 0.9, 0.999, eps)
    assert np.allclose(w, w0 - T * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-13)
    # moments are the exponential averages (1 - b^t) g and (1 - b^t) g^2
    assert np.allclose(m, (1 - 0.9 ** T) * g, rtol=1e-13)
    assert np.allclose(v, (1 - 0.999 ** T) * g * g, rtol=1e-12)
    # a zero gradient from zero moments leaves w unchanged
    w2, m2, v2 = w0.copy(), np.zeros(100), np.zeros(100)
    oracle.adam(w2, np.zeros(100), m2, v2, 1, lr)
    assert np.array_equal(w2, w0)


def test_scalers_arithmetic_sequence():
    n = 1001
    k = np.arange(n, dtype=np.float64)
    f = np.stack([k, 2 * k + 1, np.full(n, 3.0), -k], 1)
    sc = oracle.guess_scalers(f, 0.5 * k)
    sd = np.sqrt((n * n - 1) / 12.0)
    assert np.allclose(sc[:4], [(n - 1) / 2, n, 3.0, -(n - 1) / 2], rtol=1e-15)
    assert np.allclose(sc[4:8], [sd, 2 * sd, 1.0, sd], rtol=1e-13)
    assert np.allclose(sc[8:], [(n - 1) / 4, sd / 2], rtol=1e-13)


def test_guess_iterations_from_exact_start():
    """Newton started at the converged root stops after one step; started at
    a learned guess it converges to the same root as from the first-order
    guess (converged results unchanged)."""
    q, u, dt = inputs.kepler_train(300, 29)
    x, _, _ = oracle.kepler_roots(1.0, q, u, dt, 1)
    x2, it2, f2 = oracle.kepler_roots(1.0, q, u, dt, 2, x)
    assert f2 == 0 and np.all(it2 == 1)
    assert np.allclose(x2, x, rtol=1e-14, atol=0)
    w = _weights(31, scale=0.05)
    w[NP + 8], w[NP + 9] = 0.0, 0.01
    xs = np.array([oracle.guess(w, 1.0, q[i], u[i], dt[i]) for i in range(300)])
    x3, _, f3 = oracle.kepler_roots(1.0, q, u, dt, 2, xs)
    assert f3 == 0
    assert np.allclose(x3, x, rtol=1e-13, atol=0)


def test_training_lowers_loss():
    """Full-batch Adam on 2048 oracle solves lowers the loss of the
    Glorot-initialised network a hundredfold within 150 steps."""
    _, _, _, _, f, y = _data(2048, 37)
    w = np.zeros(oracle.GUESS_NWEIGHTS)
    w[:NP] = inputs.guess_init()
    w[NP:] = oracle.guess_scalers(f, y)
    m, v = np.zeros(NP), np.zeros(NP)
    wp = w[:NP].copy()
    l0 = oracle.guess_loss_grad(w, f, y, want_grad=False)
    for t in range(1, 151):
        w[:NP] = wp
        _, g = oracle.guess_loss_grad(w, f, y)
        oracle.adam(wp, g, m, v, t, 1e-2)
    w[:NP] = wp
    l1 = oracle.guess_loss_grad(w, f, y, want_grad=False)
    assert l1 < 0.01 * l0


def _orbits(n, seed):
    """Bound orbits (e in [0.05, 0.95]) and unbound ones (1.05 to 2 times the
    escape speed) with positive and negative steps up to half a period."""
    rng = np.random.Generator(np.random.PCG64(seed))
    q, u, dt = inputs.kepler_train(n, seed, e_hi=0.95)
    out = []
    for i in range(n):
        out.append((q[i], u[i], dt[i] * (1 if i % 2 else -1)))
        r = rng.normal(size=3)
        r *= rng.uniform(0.5, 20) / np.linalg.norm(r)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        vesc = np.sqrt(2.0 / np.linalg.norm(r))
        out.append((r, d * vesc * rng.uniform(1.05, 2.0), rng.uniform(0.01, 2.0)))
    return out


def test_root_ratio_lies_in_admissible_range():
    """x / (sqrt(mu) dt / r0) = r0 <1/r> lies in [r0/r_max, r0/q]: every
    converged root is an admissible start; scaled, negated or non-finite
    values are not."""
    for q0, u0, h in _orbits(200, 71):
        f, xp, T = oracle.guess_features(1.0, q0, u0, h)
        if abs(f[2] - 2.0) < 1e-3:    # nearly at rest: h -> 0, the range is unbounded
            continue
        x, it, fail = oracle.kepler_root(1.0, q0, u0, h, 0)
        assert fail == 0
        if abs(x / xp - 1.0) > 1e-9:
            assert oracle.start_admissible(1.0, q0, u0, h, x)
        assert not oracle.start_admissible(1.0, q0, u0, h, 1e6 * x)
        assert not oracle.start_admissible(1.0, q0, u0, h, -x)
        assert not oracle.start_admissible(1.0, q0, u0, h, float("nan"))


def test_universal_anomaly_is_time_integral_of_inverse_radius():
    """dx/dt = sqrt(mu)/r (the relation behind the admissible range):
    Simpson's rule over exact Kepler positions reproduces the root."""
    for q0, u0, h in _orbits(4, 73)[:6]:
        ts = np.linspace(0.0, h, 2001)
        inv_r = []
        for t in ts:
            q1, _, _, fails = oracle.kepler(1.0, q0[None], u0[None], t)
            assert fails == 0
            inv_r.append(1.0 / np.linalg.norm(q1[0]))
        inv_r = np.array(inv_r)
        dtq = ts[1] - ts[0]
        simpson = dtq / 3 * (inv_r[0] + inv_r[-1] + 4 * inv_r[1:-1:2].sum() + 2 * inv_r[2:-1:2].sum())
        x, _, _ = oracle.kepler_root(1.0, q0, u0, h, 0)
        assert simpson == pytest.approx(x, rel=1e-8)


def test_inadmissible_start_falls_back_to_first_order_guess():
    """A wild start (here 1e30 times the root) gives the same root as the
    first-order guess, in the same number of iterations."""
    q, u, dt = inputs.kepler_train(200, 79)
    x1, it1, _ = oracle.kepler_roots(1.0, q, u, dt, 1)
    x2, it2, f2 = oracle.kepler_roots(1.0, q, u, dt, 2, 1e30 * x1)
    assert f2 == 0
    assert np.array_equal(x1, x2) and np.array_equal(it1, it2)
