"""GPU parity of the K-FAC linear layer (kfac_linear_forward / kfac_linear_backward and the
autograd Function) against the FP64 oracle, on bf16 inputs (exactly representable in fp64).

Tolerances: fp32 outputs ([dW | db], the backward factor) <= 1e-5 relative Frobenius (bf16
products are exact in fp32, only the accumulation rounds); bf16 outputs (y, dx) within the
bf16 rounding of the exact value (relative Frobenius <= 4e-3)."""
import numpy as np
import pytest
import torch

import oracle as O

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def K():
    import paper_2206_15397_amd as k
    return k


def to_np(t):
    return t.detach().double().cpu().numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def bf16(a, scale=1.0):
    return (torch.from_numpy(np.asarray(a, dtype=np.float32) * scale)).to(torch.bfloat16).to(DEV)


SHAPES = [(512, 1024, 768), (300, 200, 130), (1, 7, 9), (129, 64, 64), (70, 257, 100), (0, 33, 17)]


@pytest.mark.parametrize("n,d_in,d_out", SHAPES)
def test_linear_forward(n, d_in, d_out):
    rng = np.random.default_rng(n + d_in)
    x = bf16(rng.standard_normal((n, d_in)))
    W = bf16(rng.standard_normal((d_out, d_in)) / np.sqrt(d_in))
    b = torch.from_numpy(rng.standard_normal(d_out).astype(np.float32)).to(DEV)
    y = K().ops.linear_forward(x, W, b)
    torch.cuda.synchronize()
    if n == 0:
        assert y.shape == (0, d_out)
        return
    yo = O.linear_forward(to_np(x), to_np(W), to_np(b))
    assert rel(to_np(y), yo) <= 4e-3
    # each element is the bf16 rounding of an fp32-accumulated value
    assert np.all(np.abs(to_np(y) - yo) <= 2 ** -8 * np.abs(yo) + 1e-5 * np.abs(yo).max())


@pytest.mark.parametrize("n,d_in,d_out", SHAPES)
@pytest.mark.parametrize("bias", [True, False])
def test_linear_backward_and_fused_gamma(n, d_in, d_out, bias):
    rng = np.random.default_rng(7 * n + d_out)
    x = bf16(rng.standard_normal((n, d_in)))
    W = bf16(rng.standard_normal((d_out, d_in)) / np.sqrt(d_in))
    g = bf16(rng.standard_normal((n, d_out)))
    G0 = np.eye(d_out, dtype=np.float32) + 0.01
    Gam = torch.from_numpy(G0).to(DEV)
    Gb = K().bf16_shadow(Gam)
    rho, scale = 0.95, 1.0 / max(n, 1)
    dx, dWb = K().ops.linear_backward(g, x, W, with_bias=bias, Gamma=Gam, Gamma_bf16=Gb, rho=rho, scale=scale)
    torch.cuda.synchronize()
    xo, Wo, go = to_np(x), to_np(W), to_np(g)
    dxo, dWo, dbo = O.linear_backward(xo, Wo, go)
    Go = O.ea_update(G0.astype(np.float64), go, rho, scale)
    if n > 0:
        assert rel(to_np(dx), dxo) <= 4e-3
        assert rel(to_np(dWb[:, :d_in]), dWo) <= 1e-5
        if bias:
            assert rel(to_np(dWb[:, d_in]), dbo) <= 1e-5
    else:
        assert np.all(to_np(dWb) == 0)
    assert rel(to_np(Gam), Go) <= 1e-5
    Gg = Gam.cpu().numpy()
    assert np.array_equal(Gg, Gg.T)
    assert torch.equal(Gb, Gam.to(torch.bfloat16))


def test_linear_backward_without_dx_and_gamma():
    rng = np.random.default_rng(3)
    x = bf16(rng.standard_normal((200, 300)))
    W = bf16(rng.standard_normal((150, 300)) / 17)
    g = bf16(rng.standard_normal((200, 150)))
    dx, dWb = K().ops.linear_backward(g, x, W, with_bias=True, want_dx=False)
    torch.cuda.synchronize()
    assert dx is None
    _, dWo, dbo = O.linear_backward(to_np(x), to_np(W), to_np(g))
    assert rel(to_np(dWb), np.concatenate([dWo, dbo[:, None]], axis=1)) <= 1e-5


class _MLP:
    """Width-w MLP with tanh between KFAC linear layers (bf16 weights, fp32 biases)."""

    def __init__(self, w, depth, seed):
        from paper_2206_15397_amd.autograd import KFACLinearState
        rng = np.random.default_rng(seed)
        self.W = [bf16(rng.standard_normal((w, w)) / np.sqrt(w)).requires_grad_(True) for _ in range(depth)]
        self.b = [torch.from_numpy(0.1 * rng.standard_normal(w).astype(np.float32)).to(DEV).requires_grad_(True)
                  for _ in range(depth)]
        self.st = [KFACLinearState(w, w, bias=True, rho=0.95, device=DEV) for _ in range(depth)]

    def __call__(self, x):
        from paper_2206_15397_amd.autograd import kfac_linear
        h = x
        for i, (W, b, s) in enumerate(zip(self.W, self.b, self.st)):
            h = kfac_linear(h, W, b, s)
            if i + 1 < len(self.W):
                h = torch.tanh(h)
        return h


def test_autograd_mlp_gradients_match_fp64_reference():
    """4-layer MLP: the Function's gradients against an fp64 reference run on the activations
    the GPU produced (so only each layer's own arithmetic is compared)."""
    w, B = 256, 64
    net = _MLP(w, 4, 11)
    rng = np.random.default_rng(12)
    x = bf16(rng.standard_normal((B, w)))
    t = torch.from_numpy(rng.standard_normal((B, w)).astype(np.float32)).to(DEV)
    acts = []
    h = x
    from paper_2206_15397_amd.autograd import kfac_linear
    for i in range(4):
        acts.append(h)
        h = kfac_linear(h, net.W[i], net.b[i], net.st[i])
        h.retain_grad()
        acts.append(h)
        if i < 3:
            h = torch.tanh(h)
    loss = 0.5 * ((h.float() - t) ** 2).sum() / B
    loss.backward()
    torch.cuda.synchronize()
    for i in range(4):
        a_in, s_out = acts[2 * i], acts[2 * i + 1]
        g = to_np(s_out.grad.to(torch.bfloat16))      # the bf16 gradient the layer received
        dxo, dWo, dbo = O.linear_backward(to_np(a_in), to_np(net.W[i]), g)
        assert rel(to_np(net.st[i].J[:, :w]), dWo) <= 1e-5, i
        assert rel(to_np(net.b[i].grad), dbo) <= 1e-5, i
        assert rel(to_np(net.W[i].grad), dWo) <= 4e-3, i
        # backward factor: one EA step from I with per-sample gradients B * g
        Go = O.ea_update(np.eye(w), g, 0.95, float(B))
        assert rel(to_np(net.st[i].G), Go) <= 1e-5, i
        # forward factor: one EA step from I with [a | 1]
        Ao = O.ea_update(np.eye(w + 1), to_np(a_in), 0.95, 1.0 / B, append_ones=True)
        assert rel(to_np(net.st[i].A), Ao) <= 1e-5, i


def test_kfac_step_after_autograd_matches_oracle():
    """A few forward/backward steps of a 4-layer MLP, then each layer's factors go through
    SREVD and the damped inverse: eigenvalues against the oracle at r = 32 (p = 8, q = 1), and
    at full rank (r = d, the exact regime) the preconditioned [dW | db] against the exact
    (G + lambda I)^{-1} J (A + lambda I)^{-1}."""
    w, B = 128, 96
    net = _MLP(w, 4, 21)
    rng = np.random.default_rng(22)
    for step in range(3):
        x = bf16(rng.standard_normal((B, w)))
        t = torch.from_numpy(rng.standard_normal((B, w)).astype(np.float32)).to(DEV)
        for p in net.W + net.b:
            p.grad = None
        loss = 0.5 * ((net(x).float() - t) ** 2).sum() / B
        loss.backward()
    torch.cuda.synchronize()
    lam, r, p, q = 0.1, 32, 8, 1
    for i, st in enumerate(net.st):
        _, Da, s1 = K().rand_eig(st.A, r, p, q, seed=5, stream_id=2 * i)
        _, Dg, s2 = K().rand_eig(st.G, r, p, q, seed=5, stream_id=2 * i + 1)
        torch.cuda.synchronize()
        assert int(s1.item()) == 0 and int(s2.item()) == 0
        _, Doa = O.srevd(to_np(st.A), r, p, q, 5, 2 * i)
        _, Dog = O.srevd(to_np(st.G), r, p, q, 5, 2 * i + 1)
        assert np.max(np.abs(to_np(Da) - Doa) / Doa) <= 1e-4
        assert np.max(np.abs(to_np(Dg) - Dog) / Dog) <= 1e-4
        J = st.J.contiguous()
        Ua, Da, _ = K().rand_eig(st.A, w + 1, 8, q, seed=5)
        Ug, Dg, _ = K().rand_eig(st.G, w, 8, q, seed=5)
        S = K().precondition(J, Ua, Da, Ug, Dg, lam)
        torch.cuda.synchronize()
        Sx = O.exact_precondition(to_np(J), to_np(st.A), to_np(st.G), lam)
        assert rel(to_np(S), Sx) <= 1e-4, i
