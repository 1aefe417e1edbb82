"""Pins of the FP64 warm-start network reference (oracle/cnn.py)."""
import numpy as np
import pytest

from oracle import cnn


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.uniform(-30, 30, 10000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0, 65504.0]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(cnn.bf16(x), ref)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_conv_brute_force(d):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 5, 6, 3))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    z = cnn.conv(x, W, b, d)
    ref = np.zeros_like(z)
    for bb in range(2):
        for y in range(5):
            for xx in range(6):
                for n in range(4):
                    s = b[n]
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            yy, x2 = y + d * dy, xx + d * dx
                            if 0 <= yy < 5 and 0 <= x2 < 6:
                                s += W[n, dy + 1, dx + 1] @ x[bb, yy, x2]
                    ref[bb, y, xx, n] = s
    assert np.max(np.abs(z - ref)) < 1e-12


@pytest.mark.parametrize("d", [1, 2, 4])
def test_conv_transpose_is_adjoint(d):
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 9, 7, 3))
    g = rng.standard_normal((2, 9, 7, 4))
    W = rng.standard_normal((4, 3, 3, 3))
    lhs = np.sum(cnn.conv(x, W, np.zeros(4), d) * g)
    rhs = np.sum(x * cnn.conv_transpose(g, W, d))
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)
    dW, db = cnn.conv_wgrad(g, x, d)
    # d/dW <conv(x, W), g> = conv_wgrad(g, x)
    eps = 1e-6
    for idx in [(0, 0, 0, 0), (3, 2, 1, 2), (1, 1, 1, 1)]:
        Wp = W.copy(); Wp[idx] += eps
        num = (np.sum(cnn.conv(x, Wp, np.zeros(4), d) * g) - lhs) / eps
        assert abs(num - dW[idx]) < 1e-5 * max(1, abs(dW[idx]))
    assert np.allclose(db, g.reshape(-1, 4).sum(0))


def test_gradients_by_finite_differences():
    """Backward of the full network (FP64, no rounding) vs central differences."""
    rng = np.random.default_rng(3)
    x0 = rng.standard_normal((2, 12, 11, 4))
    target = rng.standard_normal((2, 12, 11))
    mask = np.zeros((12, 11), bool)
    mask[1:-1, 1:-1] = True
    W, b = cnn.init_params(4, seed=5)
    b = [rng.standard_normal(v.shape) * 0.1 for v in b]
    loss, dW, db, _ = cnn.loss_and_grads(x0, target, mask, W, b, rounding=False)
    h = 1e-6
    for l in range(4):
        for _ in range(4):
            idx = tuple(rng.integers(0, s) for s in W[l].shape)
            Wp = [w.copy() for w in W]; Wm = [w.copy() for w in W]
            Wp[l][idx] += h; Wm[l][idx] -= h
            lp = cnn.loss_and_grads(x0, target, mask, Wp, b, rounding=False)[0]
            lm = cnn.loss_and_grads(x0, target, mask, Wm, b, rounding=False)[0]
            num = (lp - lm) / (2 * h)
            assert abs(num - dW[l][idx]) <= 1e-7 * max(1.0, abs(num)) + 1e-9, (l, idx, num, dW[l][idx])
        k = int(rng.integers(0, b[l].shape[0]))
        bp = [v.copy() for v in b]; bm = [v.copy() for v in b]
        bp[l][k] += h; bm[l][k] -= h
        num = (cnn.loss_and_grads(x0, target, mask, W, bp, rounding=False)[0]
               - cnn.loss_and_grads(x0, target, mask, W, bm, rounding=False)[0]) / (2 * h)
        assert abs(num - db[l][k]) <= 1e-7 * max(1.0, abs(num)) + 1e-9


def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(4)
    p = [rng.standard_normal((3, 4)), rng.standard_normal(5)]
    tp = [torch.tensor(v, dtype=torch.float64, requires_grad=True) for v in p]
    opt = torch.optim.Adam(tp, lr=1e-2)
    state = ([np.zeros_like(v) for v in p], [np.zeros_like(v) for v in p], 0)
    for _ in range(5):
        g = [rng.standard_normal(v.shape) for v in p]
        for t, gg in zip(tp, g):
            t.grad = torch.tensor(gg)
        opt.step()
        p, state = cnn.adam(p, g, state, lr=1e-2)
    for a, t in zip(p, tp):
        assert np.max(np.abs(a - t.detach().numpy())) < 1e-12
