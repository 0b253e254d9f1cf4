"""K-FAC linear and convolution layers behind torch.autograd.Function (the differentiation
pattern of the K-factor pipeline).  The linear layer is described here; the convolution
(KFC factors over im2col patches) at KFACConv2dFn.

Forward  : y = x W^T + b on bf16 MFMA; the layer input x is captured and, when enabled, the
           forward factor is updated in the same step, A <- rho A + (1 - rho) s [x|1]^T [x|1]
           (Alg. 1's EA of the activations).
Backward : one library call gives dx = g W (bf16), [dW | db] = g^T [x | 1] (fp32) and the
           fused backward-factor EA G <- rho G + (1 - rho) s_g g^T g (Alg. 1's EA of the
           back-propagated gradients).  The fp32 [dW | db] is kept in the state as the
           gradient matrix J of the layer for the damped inverse (Sec. 4.1).

Every numeric step runs in libkfac's kernels; torch supplies memory, streams and the tape.
"""
from __future__ import annotations

import torch

from . import ops


class KFACLinearState:
    """Per-layer factors and the last gradient matrix of a K-FAC linear layer.

    d_in, d_out: layer sizes; bias: whether the layer has a bias (the forward factor then
    has size d_in + 1, the bias column of J is the last one).
    rho: EA decay.  g_scale: the EA scale of g^T g for the backward factor.  The default, n
    (the batch size), fits the gradients g of a batch-mean loss: the per-sample gradients are
    n g, and their average outer product is (1/n) sum (n g_i)(n g_i)^T = n g^T g."""

    def __init__(self, d_in: int, d_out: int, bias: bool = True, rho: float = 0.95, device="cuda",
                 ea_forward: bool = True, ea_backward: bool = True, g_scale: float = None):
        self.d_in, self.d_out, self.bias, self.rho = d_in, d_out, bias, rho
        self.ea_forward, self.ea_backward, self.g_scale = ea_forward, ea_backward, g_scale
        d_a = d_in + (1 if bias else 0)
        self.A = ops.fill_identity(torch.empty((d_a, d_a), dtype=torch.float32, device=device))
        self.G = ops.fill_identity(torch.empty((d_out, d_out), dtype=torch.float32, device=device))
        self.A_bf16 = ops.bf16_shadow(self.A)
        self.G_bf16 = ops.bf16_shadow(self.G)
        self.J = None           # fp32 [dW | db] of the last backward (d_out x d_a)

    @property
    def d_a(self):
        return self.d_in + (1 if self.bias else 0)


class KFACLinearFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, W, b, state: KFACLinearState):
        lead = x.shape[:-1]
        x2 = x.reshape(-1, x.shape[-1])
        if x2.dtype != torch.bfloat16 or x2.stride(-1) != 1:
            x2 = x2.to(torch.bfloat16).contiguous()
        y = ops.linear_forward(x2, W, b)
        if state.ea_forward:
            ops.ea_update(state.A, x2, state.rho, 1.0 / max(x2.shape[0], 1), append_ones=state.bias,
                          F_bf16=state.A_bf16)
        ctx.save_for_backward(x2, W)
        ctx.state = state
        ctx.has_bias = b is not None
        ctx.lead = lead
        ctx.x_dtype = x.dtype
        return y.reshape(*lead, W.shape[0])

    @staticmethod
    def backward(ctx, gy):
        x2, W = ctx.saved_tensors
        st = ctx.state
        g = gy.reshape(-1, gy.shape[-1])
        if g.dtype != torch.bfloat16 or g.stride(-1) != 1:
            g = g.to(torch.bfloat16).contiguous()
        n = g.shape[0]
        g_scale = float(max(n, 1)) if st.g_scale is None else float(st.g_scale)
        dx, dWb = ops.linear_backward(
            g, x2, W, with_bias=ctx.has_bias, want_dx=ctx.needs_input_grad[0],
            Gamma=st.G if st.ea_backward else None, Gamma_bf16=st.G_bf16 if st.ea_backward else None,
            rho=st.rho, scale=g_scale)
        st.J = dWb
        d_in = x2.shape[1]
        dW = dWb[:, :d_in].to(W.dtype) if ctx.needs_input_grad[1] else None
        db = dWb[:, d_in].contiguous() if (ctx.has_bias and ctx.needs_input_grad[2]) else None
        gx = dx.reshape(*ctx.lead, d_in).to(ctx.x_dtype) if dx is not None else None
        return gx, dW, db, None


def kfac_linear(x, W, b, state: KFACLinearState):
    return KFACLinearFn.apply(x, W, b, state)


class KFACConv2dState:
    """Per-layer factors and the last gradient matrix of a K-FAC convolution (KFC factors).

    The forward factor is the EA of the im2col patches of the input (one row per output
    position, columns (dy, dx, c) plus the bias column): d_a = kh kw c_in + bias.  The
    backward factor is the EA of the output gradients over positions: d_g = c_out.
    g_scale: EA scale of g^T g; the default B^2 / n (B the batch, n = B out_h out_w positions)
    fits the gradients of a batch-mean loss (per-example gradients B g, averaged over the n
    position rows)."""

    def __init__(self, c_in: int, c_out: int, kh: int = 3, kw: int = 3, pad: int = 1, stride: int = 1,
                 bias: bool = True, rho: float = 0.95, device="cuda", ea_forward: bool = True,
                 ea_backward: bool = True, g_scale: float = None):
        self.c_in, self.c_out, self.kh, self.kw, self.pad, self.stride = c_in, c_out, kh, kw, pad, stride
        self.bias, self.rho = bias, rho
        self.ea_forward, self.ea_backward, self.g_scale = ea_forward, ea_backward, g_scale
        d_a = kh * kw * c_in + (1 if bias else 0)
        self.A = ops.fill_identity(torch.empty((d_a, d_a), dtype=torch.float32, device=device))
        self.G = ops.fill_identity(torch.empty((c_out, c_out), dtype=torch.float32, device=device))
        self.A_bf16 = ops.bf16_shadow(self.A)
        self.G_bf16 = ops.bf16_shadow(self.G)
        self.J = None           # fp32 [dW | db] of the last backward (c_out x d_a), columns (dy, dx, c)

    @property
    def d_a(self):
        return self.kh * self.kw * self.c_in + (1 if self.bias else 0)


class KFACConv2dFn(torch.autograd.Function):
    """Convolution y = conv(x, W) + b whose K-FAC work runs in libkfac: the forward factor's
    EA over the im2col patches of x (gathered from the NHWC input by the EA kernel), and in
    the backward the weight gradient [dW | db] = g^T [P | 1] as an implicit GEMM with the
    backward factor's EA fused into the same launch.  The output and the input gradient are
    ordinary convolutions of the framework (MIOpen through torch): K-FAC leaves them as they
    are.  x: N x C x H x W (any memory format), W: C_out x C_in x kh x kw."""

    @staticmethod
    def forward(ctx, x, W, b, state: KFACConv2dState):
        import torch.nn.functional as F
        xb = x.to(torch.bfloat16)
        Wb = W.to(torch.bfloat16)
        y = F.conv2d(xb, Wb, None, stride=state.stride, padding=state.pad)
        if b is not None:
            y = y + b.to(y.dtype)[None, :, None, None]
        x_nhwc = xb.permute(0, 2, 3, 1).contiguous()
        if state.ea_forward:
            ops.conv_ea_update(state.A, x_nhwc, state.kh, state.kw, state.pad, state.stride, state.rho,
                               append_ones=state.bias, F_bf16=state.A_bf16)
        ctx.save_for_backward(x_nhwc, Wb)
        ctx.state = state
        ctx.has_bias = b is not None
        ctx.x_shape, ctx.x_dtype, ctx.w_dtype = x.shape, x.dtype, W.dtype
        return y

    @staticmethod
    def backward(ctx, gy):
        x_nhwc, Wb = ctx.saved_tensors
        st = ctx.state
        g_nhwc = gy.to(torch.bfloat16).permute(0, 2, 3, 1).contiguous()
        n = g_nhwc.shape[0] * g_nhwc.shape[1] * g_nhwc.shape[2]
        B = g_nhwc.shape[0]
        g_scale = float(B * B) / max(n, 1) if st.g_scale is None else float(st.g_scale)
        dWb = ops.conv_backward_weight(
            g_nhwc, x_nhwc, st.kh, st.kw, st.pad, st.stride, with_bias=ctx.has_bias,
            Gamma=st.G if st.ea_backward else None, Gamma_bf16=st.G_bf16 if st.ea_backward else None,
            rho=st.rho, scale=g_scale)
        st.J = dWb
        c_out, c_in = Wb.shape[0], Wb.shape[1]
        k = st.kh * st.kw * c_in
        dW = None
        if ctx.needs_input_grad[1]:
            dW = dWb[:, :k].reshape(c_out, st.kh, st.kw, c_in).permute(0, 3, 1, 2).to(ctx.w_dtype)
        db = dWb[:, k].contiguous() if (ctx.has_bias and ctx.needs_input_grad[2]) else None
        gx = None
        if ctx.needs_input_grad[0]:
            gx = torch.nn.grad.conv2d_input(ctx.x_shape, Wb, gy.to(torch.bfloat16), stride=st.stride,
                                            padding=st.pad).to(ctx.x_dtype)
        return gx, dW, db, None


def kfac_conv2d(x, W, b, state: KFACConv2dState):
    return KFACConv2dFn.apply(x, W, b, state)
