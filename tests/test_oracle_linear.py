"""Pins for the oracle's linear-layer forward/backward (the differentiation row of the
K-factor pipeline): central finite differences in fp64 (eps = 1e-6) on a width-64 two-layer
MLP with tanh and loss 0.5 ||y - t||^2 / B, and the bias-as-ones-column identity used by the
fused backward ([dW | db] = g^T [x | 1])."""
import numpy as np

import oracle as O


def _mlp(params, x, t):
    (W1, b1), (W2, b2) = params
    s1 = O.linear_forward(x, W1, b1)
    h = np.tanh(s1)
    y = O.linear_forward(h, W2, b2)
    loss = 0.5 * np.sum((y - t) ** 2) / x.shape[0]
    return loss, (s1, h, y)


def _grads(params, x, t):
    (W1, b1), (W2, b2) = params
    loss, (s1, h, y) = _mlp(params, x, t)
    g2 = (y - t) / x.shape[0]
    dh, dW2, db2 = O.linear_backward(h, W2, g2)
    g1 = dh * (1.0 - h ** 2)
    dx, dW1, db1 = O.linear_backward(x, W1, g1)
    return [(dW1, db1), (dW2, db2)], dx


def test_linear_backward_matches_central_differences():
    rng = np.random.default_rng(0)
    B, w = 8, 64
    x = rng.standard_normal((B, w))
    t = rng.standard_normal((B, w))
    params = [(rng.standard_normal((w, w)) / 8, rng.standard_normal(w) / 8) for _ in range(2)]
    grads, dx = _grads(params, x, t)
    eps = 1e-6
    for li in range(2):
        for which in range(2):
            P = params[li][which]
            G = grads[li][which]
            for idx in [tuple(rng.integers(0, s) for s in P.shape) for _ in range(12)]:
                old = P[idx]
                P[idx] = old + eps
                lp, _ = _mlp(params, x, t)
                P[idx] = old - eps
                lm, _ = _mlp(params, x, t)
                P[idx] = old
                fd = (lp - lm) / (2 * eps)
                assert abs(fd - G[idx]) <= 1e-7 + 1e-6 * abs(G[idx]), (li, which, idx, fd, G[idx])
    # input gradient as well
    for idx in [tuple(rng.integers(0, s) for s in x.shape) for _ in range(12)]:
        old = x[idx]
        x[idx] = old + eps
        lp, _ = _mlp(params, x, t)
        x[idx] = old - eps
        lm, _ = _mlp(params, x, t)
        x[idx] = old
        assert abs((lp - lm) / (2 * eps) - dx[idx]) <= 1e-7 + 1e-6 * abs(dx[idx])


def test_bias_gradient_is_the_ones_column():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((5, 3))
    W = rng.standard_normal((4, 3))
    g = rng.standard_normal((5, 4))
    _, dW, db = O.linear_backward(x, W, g)
    xh = np.concatenate([x, np.ones((5, 1))], axis=1)
    np.testing.assert_allclose(g.T @ xh, np.concatenate([dW, db[:, None]], axis=1), rtol=0, atol=1e-14)
