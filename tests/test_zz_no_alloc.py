"""The allocation-free loss gradient of the learned Kepler start
(qsym_guess_grad_static, scratch in a static device array) against the
trainer's qsym_guess_grad through the C ABI: two calls in a row, the second
with fewer samples (the static scratch keeps the first call's partial sums),
each equal to the trainer's result on the same samples -- the same kernels
over the same partial layout, so the same bits -- and within the FP32
gradient bar of the FP64 oracle backprop.  Sizes beyond the static scratch
are refused with a message."""
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


def _weights(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    w = np.zeros(NW)
    w[:NP] = rng.normal(size=NP) * 0.3
    w[NP:NP + 4] = [2.0, 0.0, 0.9, -3.0]
    w[NP + 4:NP + 8] = [1.2, 0.5, 0.5, 1.5]
    w[NP + 8], w[NP + 9] = 0.0, 0.2
    return w.astype(np.float32).astype(np.float64)


def test_static_gradient_equals_trainer_gradient(Q, orc):
    import torch
    n1, n2 = 12000 + 37, 1000 + 5
    q, u, dt = inputs.kepler_train(n1, 77)
    x, _, fails = orc.kepler_roots(1.0, q, u, dt, 1)
    assert fails == 0
    st = Q.state_tensor(q, u)
    tr = Q.GuessTrainer(Q.GUESS_STATIC_MAX)
    feat = tr.prepare(1.0, st, dt, x)
    w = _weights(78)
    wt = torch.from_numpy(w.astype(np.float32)).cuda()
    F_o, y_o = orc.guess_dataset(1.0, q, u, dt, x)
    for n, off in ((n1, 0), (n2, 500)):
        say(f"static gradient n={n} offset={off}")
        g_s, l_s = Q.guess_grad_static(wt, feat, n=n, offset=off)
        g_t, l_t = tr.grad(wt, feat, n=n, offset=off)
        g_s, g_t = g_s.cpu().numpy(), g_t.cpu().numpy()
        assert np.array_equal(g_s, g_t)
        assert l_s == l_t
        loss_o, g_o = orc.guess_loss_grad(w, F_o[off:off + n], y_o[off:off + n])
        assert np.abs(g_s - g_o).max() <= 1e-3 * np.abs(g_o).max()
        assert l_s == pytest.approx(loss_o, rel=1e-4)
    tr.close()


def test_static_gradient_refuses_sizes_beyond_its_scratch(Q):
    import torch
    feat = torch.zeros((5, Q.GUESS_STATIC_MAX + 1), dtype=torch.float32, device="cuda:0")
    wt = torch.zeros(NW, dtype=torch.float32, device="cuda:0")
    with pytest.raises(Q.QsymError) as e:
        Q.guess_grad_static(wt, feat)
    assert e.value.code == -1 and "16384" in str(e.value)
