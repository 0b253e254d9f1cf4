"""K-FAC convolution layer (KFC factors over im2col patches; Sec. 2.1 and the VGG16_bn layers
of Sec. 5): the input factor's EA with the patches gathered from the NHWC input by the EA
kernel, and the weight gradient [dW | db] = g^T [P | 1] as an implicit GEMM with the output
factor's EA fused.  References: the oracle's EA (Alg. 1 EA lines) and fp64 products on
patches built on the host with torch.nn.functional.unfold, reordered to the (dy, dx, c)
column order.  Tolerances: EA and fp32-accumulated bf16 products <= 1e-5 relative."""
import numpy as np
import pytest
import torch
import torch.nn.functional as Fn

import oracle as O

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def K():
    import paper_2206_15397_amd as k
    return k


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def patches(x_nhwc, kh, kw, pad, stride):
    """im2col of an NHWC tensor on the host in fp64: rows (b, oh, ow), columns (dy, dx, c)."""
    x = torch.from_numpy(x_nhwc).permute(0, 3, 1, 2)                   # NCHW fp64
    B, C = x.shape[0], x.shape[1]
    u = Fn.unfold(x, (kh, kw), padding=pad, stride=stride)              # B x (C kh kw) x L, cols (c, dy, dx)
    L = u.shape[2]
    u = u.reshape(B, C, kh * kw, L).permute(0, 3, 2, 1).reshape(B * L, kh * kw * C)
    return u.numpy()


CASES = [  # (B, H, W, C_in, C_out, kh, kw, pad, stride)
    (4, 8, 8, 16, 24, 3, 3, 1, 1),       # 16-byte channel runs
    (3, 7, 9, 3, 8, 3, 3, 1, 1),         # C = 3 (the first VGG layer): element loads
    (2, 9, 9, 8, 16, 3, 3, 0, 2),        # stride 2, no padding
    (2, 6, 5, 32, 40, 1, 1, 0, 1),       # 1 x 1
    (32, 16, 16, 16, 24, 3, 3, 1, 1),    # n = 8192 positions: the weight gradient runs in K slices
]


@pytest.mark.parametrize("case", CASES)
def test_conv_factor_ea_and_weight_gradient(case):
    B, H, W, C, Co, kh, kw, pad, st = case
    rng = np.random.default_rng(sum(case))
    x = torch.from_numpy(rng.standard_normal((B, H, W, C)).astype(np.float32)).to(torch.bfloat16).to(DEV)
    Ho, Wo = (H + 2 * pad - kh) // st + 1, (W + 2 * pad - kw) // st + 1
    g = torch.from_numpy(rng.standard_normal((B, Ho, Wo, Co)).astype(np.float32)).to(torch.bfloat16).to(DEV)
    P = patches(x.double().cpu().numpy(), kh, kw, pad, st)
    n = P.shape[0]
    assert n == B * Ho * Wo
    d = kh * kw * C + 1
    F0 = np.eye(d) + 0.01 * (lambda m: m + m.T)(rng.standard_normal((d, d)))
    F = torch.from_numpy(F0.astype(np.float32)).to(DEV)
    Fb = K().bf16_shadow(F)
    K().conv_ea_update(F, x, kh, kw, pad, st, 0.9, 1.0 / n, append_ones=True, F_bf16=Fb)
    G0 = np.eye(Co)
    G = torch.eye(Co, device=DEV)
    dWb = K().conv_backward_weight(g, x, kh, kw, pad, st, with_bias=True, Gamma=G, rho=0.9, scale=0.5)
    torch.cuda.synchronize()
    Fo = O.ea_update(F0.astype(np.float32).astype(np.float64), P, 0.9, 1.0 / n, append_ones=True)
    assert rel(F.double().cpu().numpy(), Fo) <= 1e-5
    assert torch.equal(Fb, F.to(torch.bfloat16))
    g2 = g.double().cpu().numpy().reshape(n, Co)
    want = g2.T @ np.concatenate([P, np.ones((n, 1))], 1)
    assert rel(dWb.double().cpu().numpy(), want) <= 1e-5
    Go = O.ea_update(G0, g2, 0.9, 0.5)
    assert rel(G.double().cpu().numpy(), Go) <= 1e-5


# (case, bias, misalign): the two im2col loader forms without the ones column (the 16-byte
# form's groups past the patch are then all zero), and the element form on a channel count
# that is a multiple of 8 (an input 2 bytes off 16-byte alignment)
EXTRA = [((4, 8, 8, 16, 24, 3, 3, 1, 1), False, False),
         ((3, 7, 9, 3, 8, 3, 3, 1, 1), False, False),
         ((4, 8, 8, 16, 24, 3, 3, 1, 1), True, True),
         ((2, 9, 9, 8, 16, 3, 3, 0, 2), False, True)]


@pytest.mark.parametrize("implicit", [False, True])
@pytest.mark.parametrize("case,bias,misalign", EXTRA)
def test_conv_factor_loader_forms(case, bias, misalign, implicit):
    """implicit: an empty workspace, so that neither call stages the patches and both gather
    them inside the EA and weight-gradient kernels (the staged path is the default for these
    small patch matrices)."""
    B, H, W, C, Co, kh, kw, pad, st = case
    rng = np.random.default_rng(sum(case) + 7 * bias + 3 * misalign)
    xs = torch.from_numpy(rng.standard_normal((B, H, W, C)).astype(np.float32)).to(torch.bfloat16)
    if misalign:
        buf = torch.empty(B * H * W * C + 8, dtype=torch.bfloat16, device=DEV)
        x = buf[1:1 + B * H * W * C].view(B, H, W, C)
        x.copy_(xs.to(DEV))
        assert x.data_ptr() % 16 != 0 and x.is_contiguous()
    else:
        x = xs.to(DEV)
    Ho, Wo = (H + 2 * pad - kh) // st + 1, (W + 2 * pad - kw) // st + 1
    g = torch.from_numpy(rng.standard_normal((B, Ho, Wo, Co)).astype(np.float32)).to(torch.bfloat16).to(DEV)
    P = patches(x.double().cpu().numpy(), kh, kw, pad, st)
    n = P.shape[0]
    d = kh * kw * C + (1 if bias else 0)
    F0 = np.eye(d) + 0.01 * (lambda m: m + m.T)(rng.standard_normal((d, d)))
    F = torch.from_numpy(F0.astype(np.float32)).to(DEV)
    Fb = K().bf16_shadow(F)
    ws = torch.empty(0, dtype=torch.uint8, device=DEV) if implicit else None
    K().conv_ea_update(F, x, kh, kw, pad, st, 0.9, 1.0 / n, append_ones=bias, F_bf16=Fb, workspace=ws)
    dWb = K().conv_backward_weight(g, x, kh, kw, pad, st, with_bias=bias, workspace=ws)
    torch.cuda.synchronize()
    Fo = O.ea_update(F0.astype(np.float32).astype(np.float64), P, 0.9, 1.0 / n, append_ones=bias)
    assert rel(F.double().cpu().numpy(), Fo) <= 1e-5
    assert torch.equal(Fb, F.to(torch.bfloat16))
    g2 = g.double().cpu().numpy().reshape(n, Co)
    Pb = np.concatenate([P, np.ones((n, 1))], 1) if bias else P
    assert rel(dWb.double().cpu().numpy(), g2.T @ Pb) <= 1e-5


def test_conv_layer_autograd_matches_reference():
    """The autograd Function: output, input gradient (framework convolutions on the same bf16
    operands), dW / db against fp32 autograd of the same convolution, J = [dW | db] in the
    factor's column order, and both factors updated."""
    from paper_2206_15397_amd.autograd import KFACConv2dState, kfac_conv2d
    torch.manual_seed(0)
    B, C, Co, H = 8, 16, 32, 12
    x = torch.randn((B, C, H, H)).to(torch.bfloat16)
    W = (torch.randn((Co, C, 3, 3)) / 12).to(torch.bfloat16)
    b = torch.randn(Co) * 0.1
    st = KFACConv2dState(C, Co, 3, 3, 1, 1, bias=True, rho=0.9, device=DEV)
    xd, Wd, bd = x.to(DEV).requires_grad_(True), W.to(DEV).requires_grad_(True), b.to(DEV).requires_grad_(True)
    y = kfac_conv2d(xd, Wd, bd, st)
    t = torch.randn(y.shape).to(DEV)
    ((y.float() - t) ** 2).sum().mul(0.5 / B).backward()
    torch.cuda.synchronize()
    # fp32 reference on the host, from the same bf16 values
    xr, Wr, br = x.float().requires_grad_(True), W.float().requires_grad_(True), b.clone().requires_grad_(True)
    yr = Fn.conv2d(xr, Wr, br, padding=1)
    gy = (y.detach().float().cpu() - t.cpu()) / B                        # the gradient the layer received
    yr.backward(gy)
    assert rel(y.detach().float().cpu().numpy(), yr.detach().numpy()) <= 1e-2        # bf16 output
    assert rel(xd.grad.float().cpu().numpy(), xr.grad.numpy()) <= 1e-2
    gyb = gy.to(torch.bfloat16).double()                                 # dW uses the bf16 gradient
    Pn = patches(x.double().permute(0, 2, 3, 1).numpy(), 3, 3, 1, 1)
    g2 = gyb.permute(0, 2, 3, 1).reshape(-1, Co).numpy()
    J = g2.T @ np.concatenate([Pn, np.ones((Pn.shape[0], 1))], 1)
    assert rel(st.J.double().cpu().numpy(), J) <= 1e-5
    dW = J[:, :9 * C].reshape(Co, 3, 3, C).transpose(0, 3, 1, 2)
    assert rel(Wd.grad.double().cpu().numpy(), dW) <= 1e-2                # returned in the weight's bf16
    assert rel(bd.grad.double().cpu().numpy(), J[:, 9 * C]) <= 1e-5
    n = Pn.shape[0]
    A0 = np.eye(9 * C + 1)
    assert rel(st.A.double().cpu().numpy(), O.ea_update(A0, Pn, 0.9, 1.0 / n, append_ones=True)) <= 1e-5
    Gw = O.ea_update(np.eye(Co), g2, 0.9, float(B * B) / n)
    assert rel(st.G.double().cpu().numpy(), Gw) <= 1e-5


def test_conv_factor_vgg_layer_sampled():
    """Full size: VGG16_bn conv6 (256 -> 256 at 8 x 8, batch 128; d_A = 2305, n = 8192 rows):
    sampled entries of the input factor against fp64 sums over the im2col rows computed on
    the GPU from the same bf16 input."""
    B, H, C = 128, 8, 256
    g = torch.Generator(device=DEV).manual_seed(9)
    x = torch.randn((B, H, H, C), generator=g, device=DEV).to(torch.bfloat16)
    d = 9 * C + 1
    F = K().fill_identity(torch.empty((d, d), device=DEV))
    n = B * H * H
    K().conv_ea_update(F, x, 3, 3, 1, 1, 0.95, 1.0 / n, append_ones=True)
    torch.cuda.synchronize()
    xp = Fn.pad(x.double().permute(0, 3, 1, 2), (1, 1, 1, 1))               # B x C x 10 x 10, fp64
    rng = np.random.default_rng(3)
    cols = rng.choice(d, 48, replace=False)

    def col(j):          # column j of [P | 1] over all n rows, fp64 on the GPU
        if j == 9 * C:
            return torch.ones(n, dtype=torch.float64, device=DEV)
        tap, c = divmod(j, C)
        dy, dx = divmod(tap, 3)
        return xp[:, c, dy:dy + H, dx:dx + H].reshape(-1)

    Fs = F.double()
    worst = 0.0
    for a, bcol in zip(cols[:24], cols[24:]):
        for i, j in ((a, bcol), (a, a)):
            want = 0.95 * (i == j) + 0.05 * float((col(i) * col(j)).sum()) / n
            got = float(Fs[i, j])
            worst = max(worst, abs(got - want) / (abs(want) + 1e-3))
    assert worst <= 1e-4, worst
    # the weight gradient of the same layer at full size (K slices) with the fused output-factor
    # EA: sampled entries of dW and Gamma against fp64 sums over the n positions
    Co = 256
    gy = (1e-2 * torch.randn((B, H, H, Co), generator=g, device=DEV)).to(torch.bfloat16)
    G = K().fill_identity(torch.empty((Co, Co), device=DEV))
    dWb = K().conv_backward_weight(gy, x, 3, 3, 1, 1, with_bias=True, Gamma=G, rho=0.95, scale=2.0)
    torch.cuda.synchronize()
    g2 = gy.double().reshape(n, Co)
    outs = rng.choice(Co, 24, replace=False)
    worst_w = worst_g = 0.0
    for o, j, o2 in zip(outs, cols[:24], outs[::-1]):
        want = float((g2[:, o] * col(j)).sum())
        worst_w = max(worst_w, abs(float(dWb[o, j]) - want) / (abs(want) + 1e-3))
        wg = 0.95 * (o == o2) + 0.05 * 2.0 * float((g2[:, o] * g2[:, o2]).sum())
        worst_g = max(worst_g, abs(float(G[o, o2]) - wg) / (abs(wg) + 1e-3))
    assert worst_w <= 1e-4, worst_w
    assert worst_g <= 1e-4, worst_g
    assert torch.equal(G, G.T)
