"""Learned Kepler start on the GPU (through the C ABI) against the FP64 oracle:
stand-alone roots, the start itself, the loss gradient, Adam, training on
oracle solves, what the trained start gains, and that converged results do
not depend on it.

Tolerances: roots 1e-14 relative (both sides iterate to |dx| <= 1e-14 |x|);
the FP32 start 1e-4 relative per unit of scaled step T; FP32 gradients
1e-3 relative to the largest component (FP64 backprop on the CPU); Adam
1e-6 relative (FP32 state)."""
import sys

import numpy as np
import pytest

from paper_1007_3458_amd import inputs

pytestmark = pytest.mark.gpu

NP, NW = 1249, 1259


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def Q():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_1007_3458_amd import qsym
    qsym.lib()
    return qsym


def _rand_weights(seed, scale=0.3):
    rng = np.random.Generator(np.random.PCG64(seed))
    w = np.zeros(NW)
    w[:NP] = rng.normal(size=NP) * scale
    w[NP:NP + 4] = [2.0, 0.0, 0.9, -3.0]
    w[NP + 4:NP + 8] = [1.2, 0.5, 0.5, 1.5]
    w[NP + 8], w[NP + 9] = 0.0, 0.2
    return w.astype(np.float32).astype(np.float64)


def _train_set(n, seed, negative=False):
    q, u, dt = inputs.kepler_train(n, seed)
    if negative:
        dt = dt.copy()
        dt[1::2] *= -1.0
    return q, u, dt


def test_kepler_solve_roots_match_oracle(Q, orc):
    import torch
    for mode in (0, 1):
        q, u, dt = _train_set(20011, 41, negative=True)
        say(f"kepler_solve mode {mode} n={len(dt)}")
        x_o, it_o, f_o = orc.kepler_roots(1.0, q, u, dt, mode)
        st = Q.state_tensor(q, u)
        x_g, it_g = Q.kepler_solve(1.0, st, dt, mode)
        torch.cuda.synchronize()
        x_g = x_g.cpu().numpy()
        it_g = it_g.cpu().numpy()
        assert f_o == 0 and np.all(it_g > 0)
        assert np.max(np.abs(x_g - x_o) / np.abs(x_o)) <= 1e-14
        # the same iteration in the same order: counts agree but for rare
        # rounding ties at the stopping test
        assert np.mean(it_g != it_o) < 1e-3 and np.max(np.abs(it_g - it_o)) <= 1


def test_kepler_solve_edges(Q, orc):
    import torch
    q, u, dt = _train_set(257, 43)
    dt[5] = 0.0
    st = Q.state_tensor(q, u)
    x, it = Q.kepler_solve(1.0, st, dt, 1)
    torch.cuda.synchronize()
    assert x[5].item() == 0.0 and it[5].item() == 0
    x_o, _, _ = orc.kepler_roots(1.0, q, u, dt, 1)
    assert np.allclose(x.cpu().numpy(), x_o, rtol=1e-14, atol=0)
    x0, it0 = Q.kepler_solve(1.0, Q.state_tensor(np.zeros((0, 3)), np.zeros((0, 3))),
                             np.zeros(0), 1)
    assert x0.numel() == 0
    with pytest.raises(ValueError):
        Q.kepler_solve(1.0, st, dt, 2)   # mode 2 without weights


def test_guess_matches_oracle(Q, orc):
    import torch
    w = _rand_weights(45)
    q, u, dt = _train_set(5003, 47, negative=True)
    say("kepler_guess n=5003")
    g = Q.kepler_guess(1.0, Q.state_tensor(q, u), dt, w).cpu().numpy()
    torch.cuda.synchronize()
    g_o = np.array([orc.guess(w, 1.0, q[i], u[i], dt[i]) for i in range(len(dt))])
    T = np.sqrt(1.0) * np.abs(dt) / np.linalg.norm(q, axis=1) ** 1.5
    err = np.abs(g - g_o) / np.abs(g_o)
    assert np.all(np.isfinite(g))
    assert np.max(err / np.maximum(T, 1.0)) <= 1e-4


def _both_datasets(Q, orc, n, seed):
    """Each side solves and featurises the same bodies on its own."""
    q, u, dt = _train_set(n, seed, negative=True)
    x_o, _, f = orc.kepler_roots(1.0, q, u, dt, 0)
    assert f == 0
    F_o, y_o = orc.guess_dataset(1.0, q, u, dt, x_o)
    st = Q.state_tensor(q, u)
    x_g, it = Q.kepler_solve(1.0, st, dt, 0)
    tr = Q.GuessTrainer(max(n, 64))
    feat = tr.prepare(1.0, st, dt, x_g)
    return tr, feat, F_o, y_o


def test_prepare_and_scalers_match_oracle(Q, orc):
    import torch
    n = 30001
    say(f"guess_prepare/fit_scalers n={n}")
    tr, feat, F_o, y_o = _both_datasets(Q, orc, n, 49)
    fg = feat.cpu().numpy()
    assert np.allclose(fg[:4].T, F_o, rtol=2e-6, atol=2e-6)
    assert np.allclose(fg[4], y_o, rtol=1e-5, atol=1e-6 * np.abs(y_o).max())
    w = torch.zeros(NW, dtype=torch.float32, device="cuda")
    tr.fit_scalers(feat, w)
    sc = w.cpu().numpy()[NP:]
    sc_o = orc.guess_scalers(F_o, y_o)
    assert np.allclose(sc, sc_o, rtol=1e-5, atol=1e-6)
    # a zero step is rejected
    q, u, dt = _train_set(100, 51)
    dt[7] = 0.0
    with pytest.raises(Q.QsymError):
        tr.prepare(1.0, Q.state_tensor(q, u), dt)
    tr.close()


@pytest.mark.parametrize("n", [64, 4096 + 17])
def test_gradient_matches_oracle_backprop(Q, orc, n):
    import torch
    say(f"guess_grad n={n}")
    tr, feat, F_o, y_o = _both_datasets(Q, orc, n, 53 + n)
    w = _rand_weights(55)
    wt = torch.from_numpy(w.astype(np.float32)).cuda()
    g, loss = tr.grad(wt, feat)
    g = g.cpu().numpy()
    loss_o, g_o = orc.guess_loss_grad(w, F_o, y_o)
    scale = np.abs(g_o).max()
    assert np.abs(g - g_o).max() <= 1e-3 * scale
    for lo, hi in ((0, 128), (128, 160), (160, 1184), (1184, 1216), (1216, 1248), (1248, 1249)):
        blk = np.abs(g_o[lo:hi]).max()
        assert np.abs(g[lo:hi] - g_o[lo:hi]).max() <= 1e-3 * max(blk, 1e-3 * scale)
    assert loss == pytest.approx(loss_o, rel=1e-4)
    tr.close()


def test_adam_matches_oracle(Q, orc):
    import torch
    rng = np.random.Generator(np.random.PCG64(57))
    w = rng.normal(size=NW).astype(np.float32).astype(np.float64)
    tr = Q.GuessTrainer(64)
    wt = torch.from_numpy(w.astype(np.float32)).cuda()
    wo, m, v = w[:NP].copy(), np.zeros(NP), np.zeros(NP)
    for t in range(1, 4):
        g = (rng.normal(size=NP) * np.logspace(-5, 1, NP)).astype(np.float32).astype(np.float64)
        tr.adam(wt, torch.from_numpy(g.astype(np.float32)).cuda(), 1e-2, 0.9, 0.999, 1e-8)
        orc.adam(wo, g, m, v, t, 1e-2, 0.9, 0.999, 1e-8)
    wg = wt.cpu().numpy()
    assert np.allclose(wg[:NP], wo, rtol=1e-6, atol=1e-7)
    assert np.array_equal(wg[NP:], w[NP:].astype(np.float32))   # scalers untouched
    tr.close()


@pytest.fixture(scope="module")
def trained(Q, orc):
    """Weights trained on the GPU on 2^18 solves generated by the oracle."""
    import torch
    n = 1 << 18
    q, u, dt = inputs.kepler_train(n, 5)
    x, _, f = orc.kepler_roots(1.0, q, u, dt, 0)
    assert f == 0
    say(f"training on {n} oracle solves")
    tr = Q.GuessTrainer(8192)
    st = Q.state_tensor(q, u)
    feat = tr.prepare(1.0, st, dt, x)
    w = torch.zeros(NW, dtype=torch.float32, device="cuda")
    w[:NP] = torch.from_numpy(inputs.guess_init(7).astype(np.float32))
    tr.fit_scalers(feat, w)
    curve = tr.train(w, feat, 8192, 30, 3e-3, 3e-5)
    tr.close()
    say("curve", curve[:3], curve[-3:])
    return w.cpu().numpy(), curve


def test_training_curve(trained):
    w, curve = trained
    assert np.all(np.isfinite(curve)) and np.all(np.isfinite(w))
    assert curve[-1] < 0.02 * curve[0]
    assert curve[-1] <= curve[len(curve) // 2]


def test_trained_start_gains_and_leaves_roots_unchanged(Q, orc, trained):
    """On the learned-guess test bodies (a ~ U[0.5, 50], e ~ U[0, 0.9],
    dt = 0.05): fewer Newton iterations than from the first-order guess and
    than the Laguerre start, also per 64-lane wave, with the same roots."""
    import torch
    w, _ = trained
    s = inputs.kepler_test(1 << 16)
    st = Q.state_tensor(s.q, s.v)
    res = {}
    for mode in (0, 1, 2):
        x, it = Q.kepler_solve(1.0, st, 0.05, mode, w if mode == 2 else None)
        torch.cuda.synchronize()
        res[mode] = (x.cpu().numpy(), it.cpu().numpy())
    for mode in (0, 1, 2):
        it = res[mode][1]
        say(f"mode {mode}: mean {it.mean():.3f} max {it.max()} "
            f"wave-max {it.reshape(-1, 64).max(1).mean():.3f}")
        assert np.all(it > 0)
    mean = {m: res[m][1].mean() for m in res}
    wave = {m: res[m][1].reshape(-1, 64).max(1).mean() for m in res}
    assert mean[2] < 0.9 * mean[1] < mean[0]
    assert wave[2] < wave[1] < wave[0]
    x1, x2 = res[1][0], res[2][0]
    assert np.max(np.abs(x2 - x1) / np.abs(x1)) <= 1e-14
    # the oracle started from its own evaluation of the same network
    # converges in the same number of iterations almost everywhere
    sub = slice(0, 4096)
    g_o = np.array([orc.guess(w.astype(np.float64), 1.0, s.q[i], s.v[i], 0.05)
                    for i in range(4096)])
    x_o, it_o, f_o = orc.kepler_roots(1.0, s.q[sub], s.v[sub], 0.05, 2, g_o)
    assert f_o == 0
    assert np.mean(it_o != res[2][1][sub]) < 0.01
    assert np.max(np.abs(x_o - x2[sub]) / np.abs(x_o)) <= 1e-14


def test_step_with_learned_start_matches_first_order_start(Q, trained):
    """Whole steps with kepler_mode 2 and 1 give the same trajectory."""
    w, _ = trained
    s = inputs.small()
    out = {}
    for mode in (1, 2):
        ctx = Q.Context([s], Q.make_params(kepler_mode=mode), guess=w if mode == 2 else None)
        say(f"20 steps kepler_mode {mode}")
        ctx.step(0.05, 20)
        out[mode] = ctx.get_state()
        ctx.close()
    q1, q2 = out[1][0], out[2][0]
    assert np.max(np.linalg.norm(q2 - q1, axis=1) / np.linalg.norm(q1, axis=1)) <= 1e-12


def test_mode2_needs_weights_and_survives_garbage(Q):
    import torch
    s = inputs.small()
    ctx = Q.Context([s], Q.make_params(kepler_mode=2), guess=None)
    with pytest.raises(Q.QsymError):
        ctx.step(0.05, 1)
    ctx.set_guess(np.full(NW, np.nan, np.float32))   # unusable start: first-order guess
    ctx.step(0.05, 1)
    ctx.close()
    q, u, dt = _train_set(4099, 59, negative=True)
    st = Q.state_tensor(q, u)
    x1, it1 = Q.kepler_solve(1.0, st, dt, 1)
    rng = np.random.Generator(np.random.PCG64(61))
    huge = rng.normal(size=NW) * 1e3
    huge[NP + 4:NP + 8] = 1.0
    huge[NP + 9] = 1.0
    nan = np.full(NW, np.nan)
    for name, w in (("huge", huge), ("nan", nan)):
        say(f"garbage weights: {name}")
        x2, it2 = Q.kepler_solve(1.0, st, dt, 2, w)
        torch.cuda.synchronize()
        a, b = x1.cpu().numpy(), x2.cpu().numpy()
        assert np.all(it2.cpu().numpy() > 0)
        assert np.max(np.abs(a - b) / np.abs(a)) <= 1e-14
        if name == "nan":   # not-finite start -> first-order guess: identical
            assert np.array_equal(a, b) and torch.equal(it1, it2)


def test_packaged_weights_gain(Q):
    """The packaged weights (trained on 1e6 library solves) gain over the
    first-order start on the test orbits."""
    import torch
    from paper_1007_3458_amd import learned_guess
    w = learned_guess.load()
    s = inputs.kepler_test(1 << 15, seed=83)
    st = Q.state_tensor(s.q, s.v)
    _, it1 = Q.kepler_solve(1.0, st, 0.05, 1)
    _, it2 = Q.kepler_solve(1.0, st, 0.05, 2, w)
    torch.cuda.synchronize()
    a, b = it1.cpu().numpy(), it2.cpu().numpy()
    say(f"packaged weights: mean {a.mean():.3f} -> {b.mean():.3f}")
    assert np.all(b > 0) and b.mean() < 0.9 * a.mean()
