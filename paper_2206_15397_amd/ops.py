"""Python wrappers of the libkfac C ABI.  Argument marshalling only: tensors provide
device memory (and workspaces), torch's current stream provides the HIP stream."""
from __future__ import annotations

import torch

from . import _lib
from ._lib import check, lib


def _stream():
    return ctypes_void(torch.cuda.current_stream().cuda_stream)


def ctypes_void(x):
    import ctypes
    return ctypes.c_void_p(int(x))


def _ptr(t):
    import ctypes
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _require_cuda(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise ValueError("libkfac operates on device tensors")


def _workspace(nbytes: int, device):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def fill_identity(F: torch.Tensor) -> torch.Tensor:
    _require_cuda(F)
    assert F.dtype == torch.float32 and F.dim() == 2 and F.shape[0] == F.shape[1] and F.stride(1) == 1
    check("kfac_fill_identity", lib().kfac_fill_identity(_ptr(F), F.shape[0], F.stride(0), _stream()))
    return F


def ea_update(F: torch.Tensor, X: torch.Tensor, rho: float, scale: float = None,
              append_ones: bool = False, F_bf16: torch.Tensor = None, workspace=None) -> torch.Tensor:
    """In place: F <- rho F + (1 - rho) scale [X|1]^T [X|1]; optionally refreshes F_bf16."""
    _require_cuda(F, X, F_bf16)
    d = F.shape[0]
    n, d_in = X.shape
    assert F.dtype == torch.float32 and F.stride(1) == 1 and (n == 0 or X.stride(1) == 1)
    xtype = {torch.float32: _lib.KFAC_FP32, torch.bfloat16: _lib.KFAC_BF16}[X.dtype]
    if scale is None:
        scale = 1.0 / max(n, 1)
    L = lib()
    if workspace is None:
        ws_bytes = L.kfac_ea_update_workspace(d, n)
        workspace = _workspace(ws_bytes, F.device) if ws_bytes else None
    ws_bytes = 0 if workspace is None else workspace.numel()
    fb_ld = 0 if F_bf16 is None else F_bf16.stride(0)
    check("kfac_ea_update", L.kfac_ea_update(
        _ptr(F), d, F.stride(0), _ptr(X), xtype, n, d_in, X.stride(0) if n else d_in,
        1 if append_ones else 0, float(rho), float(scale), _ptr(F_bf16), fb_ld,
        _ptr(workspace), ws_bytes, _stream()))
    return F


def gaussian_omega(d: int, l: int, seed: int, stream_id: int = 0, inversion_index: int = 0,
                   device="cuda", want_words: bool = False):
    Om = torch.empty((d, l), dtype=torch.float32, device=device)
    words = torch.empty((d, (l + 3) // 4, 4), dtype=torch.int32, device=device) if want_words else None
    check("kfac_gaussian_omega", lib().kfac_gaussian_omega(
        _ptr(Om), d, l, l, int(seed), int(stream_id), int(inversion_index), _ptr(words), _stream()))
    return (Om, words) if want_words else Om


def _prec(sketch) -> int:
    """Sketch / power-iteration product precision: "fp32", "bf16" (bf16 copy of F) or
    "split" (fp32 operands as bf16 hi/lo pairs on bf16 MFMA)."""
    try:
        return {"fp32": _lib.KFAC_SKETCH_FP32, "bf16": _lib.KFAC_SKETCH_BF16, "split": _lib.KFAC_SKETCH_SPLIT}[sketch]
    except KeyError:
        raise ValueError(f"sketch must be 'fp32', 'bf16' or 'split', not {sketch!r}") from None


def _variant(v) -> int:
    if v in ("srevd", _lib.KFAC_SREVD):
        return _lib.KFAC_SREVD
    if v in ("rsvd", _lib.KFAC_RSVD):
        return _lib.KFAC_RSVD
    raise ValueError(f"variant must be 'srevd' or 'rsvd', not {v!r}")


def rand_eig_workspace_bytes(d, r, p, q, sketch="fp32", variant="srevd") -> int:
    prec = _prec(sketch)
    return int(lib().kfac_rand_eig_workspace(d, r, p, q, _variant(variant), prec))


def rand_eig(F: torch.Tensor, r: int, p: int, q: int, seed: int, stream_id: int = 0,
             inversion_index: int = 0, sketch: str = "fp32", F_bf16: torch.Tensor = None,
             U: torch.Tensor = None, D: torch.Tensor = None, workspace=None, status=None,
             variant: str = "srevd"):
    """Randomized low-rank eigendecomposition of the symmetric PSD factor F (variant
    "srevd": Alg. 3; "rsvd": Alg. 2 returning its V factor): returns (U d x r, D r
    descending, status int32)."""
    _require_cuda(F, F_bf16)
    d = F.shape[0]
    prec = _prec(sketch)
    if prec == _lib.KFAC_SKETCH_BF16 and F_bf16 is None:
        F_bf16 = bf16_shadow(F)
    if U is None:
        U = torch.empty((d, r), dtype=torch.float32, device=F.device)
    if D is None:
        D = torch.empty((r,), dtype=torch.float32, device=F.device)
    if status is None:
        status = torch.zeros((1,), dtype=torch.int32, device=F.device)
    L = lib()
    v = _variant(variant)
    if workspace is None:
        workspace = _workspace(L.kfac_rand_eig_workspace(d, r, p, q, v, prec), F.device)
    check("kfac_rand_eig", L.kfac_rand_eig(
        _ptr(F), d, F.stride(0), _ptr(F_bf16), 0 if F_bf16 is None else F_bf16.stride(0),
        int(r), int(p), int(q), int(seed), int(stream_id), int(inversion_index), v, prec,
        _ptr(U), U.stride(0), _ptr(D), _ptr(workspace), workspace.numel(), _ptr(status), _stream()))
    return U, D, status


def rand_eig_noalloc(F: torch.Tensor, r: int, p: int, q: int, seed: int, stream_id: int = 0,
                     inversion_index: int = 0, sketch: str = "fp32", F_bf16: torch.Tensor = None,
                     U: torch.Tensor = None, D: torch.Tensor = None, status=None):
    """rand_eig through kfac_rand_eig_noalloc: no workspace, the library's static scratch.
    U, D and status must be given by callers that allocate nothing during the call."""
    _require_cuda(F, F_bf16, U, D, status)
    d = F.shape[0]
    prec = _prec(sketch)
    if U is None:
        U = torch.empty((d, r), dtype=torch.float32, device=F.device)
    if D is None:
        D = torch.empty((r,), dtype=torch.float32, device=F.device)
    if status is None:
        status = torch.zeros((1,), dtype=torch.int32, device=F.device)
    check("kfac_rand_eig_noalloc", lib().kfac_rand_eig_noalloc(
        _ptr(F), d, F.stride(0), _ptr(F_bf16), 0 if F_bf16 is None else F_bf16.stride(0),
        int(r), int(p), int(q), int(seed), int(stream_id), int(inversion_index), _lib.KFAC_SREVD, prec,
        _ptr(U), U.stride(0), _ptr(D), _ptr(status), _stream()))
    return U, D, status


def precondition_workspace_bytes(d_g, d_a, r_a, r_g) -> int:
    return int(lib().kfac_precondition_workspace(d_g, d_a, r_a, r_g))


def precondition(J: torch.Tensor, Ua: torch.Tensor, Da: torch.Tensor, Ug: torch.Tensor,
                 Dg: torch.Tensor, lam: float, S: torch.Tensor = None, workspace=None) -> torch.Tensor:
    """S = (U_g D_g U_g^T + lam I)^{-1} J (U_a D_a U_a^T + lam I)^{-1} via the low-rank identity."""
    _require_cuda(J, Ua, Da, Ug, Dg)
    d_g, d_a = J.shape
    r_a, r_g = Ua.shape[1], Ug.shape[1]
    if S is None:
        S = torch.empty((d_g, d_a), dtype=torch.float32, device=J.device)
    L = lib()
    if workspace is None:
        workspace = _workspace(L.kfac_precondition_workspace(d_g, d_a, r_a, r_g), J.device)
    check("kfac_precondition", L.kfac_precondition(
        _ptr(J), d_g, d_a, J.stride(0), _ptr(Ua), Ua.stride(0), _ptr(Da), r_a, _ptr(Ug), Ug.stride(0),
        _ptr(Dg), r_g, float(lam), _ptr(S), S.stride(0), _ptr(workspace), workspace.numel(), _stream()))
    return S


def linear_forward(x: torch.Tensor, W: torch.Tensor, bias: torch.Tensor = None, y: torch.Tensor = None):
    """y = x W^T + b on bf16 MFMA (x: n x d_in bf16, W: d_out x d_in bf16, bias fp32)."""
    _require_cuda(x, W, bias)
    n, d_in = x.shape
    d_out = W.shape[0]
    assert x.dtype == torch.bfloat16 and W.dtype == torch.bfloat16 and W.shape[1] == d_in
    assert (n == 0 or x.stride(1) == 1) and W.stride(1) == 1
    assert bias is None or (bias.dtype == torch.float32 and bias.is_contiguous() and bias.numel() == d_out)
    if y is None:
        y = torch.empty((n, d_out), dtype=torch.bfloat16, device=x.device)
    check("kfac_linear_forward", lib().kfac_linear_forward(
        _ptr(x), n, d_in, x.stride(0) if n else d_in, _ptr(W), d_out, W.stride(0), _ptr(bias), _ptr(y),
        y.stride(0), _stream()))
    return y


def linear_backward(g: torch.Tensor, x: torch.Tensor, W: torch.Tensor, with_bias: bool = True,
                    want_dx: bool = True, Gamma: torch.Tensor = None, Gamma_bf16: torch.Tensor = None,
                    rho: float = 0.95, scale: float = None):
    """dx = g W (bf16), [dW | db] = g^T [x | 1] (fp32, d_out x (d_in + with_bias)), and, when
    Gamma is given, Gamma <- rho Gamma + (1 - rho) scale g^T g in place (fused)."""
    _require_cuda(g, x, W, Gamma, Gamma_bf16)
    n, d_out = g.shape
    d_in = x.shape[1]
    assert g.dtype == torch.bfloat16 and x.dtype == torch.bfloat16 and W.dtype == torch.bfloat16
    assert (n == 0 or (g.stride(1) == 1 and x.stride(1) == 1)) and W.stride(1) == 1 and x.shape[0] == n
    dx = torch.empty((n, d_in), dtype=torch.bfloat16, device=g.device) if want_dx else None
    dWb = torch.empty((d_out, d_in + (1 if with_bias else 0)), dtype=torch.float32, device=g.device)
    if scale is None:
        scale = 1.0 / max(n, 1)
    if Gamma is not None:
        assert Gamma.dtype == torch.float32 and Gamma.stride(1) == 1 and Gamma.shape == (d_out, d_out)
    check("kfac_linear_backward", lib().kfac_linear_backward(
        _ptr(g), n, d_out, g.stride(0) if n else d_out, _ptr(x), d_in, x.stride(0) if n else d_in, _ptr(W),
        W.stride(0), _ptr(dx), d_in if dx is None else dx.stride(0), _ptr(dWb), dWb.stride(0),
        1 if with_bias else 0, _ptr(Gamma), d_out if Gamma is None else Gamma.stride(0), _ptr(Gamma_bf16),
        d_out if Gamma_bf16 is None else Gamma_bf16.stride(0), float(rho), float(scale), _stream()))
    return dx, dWb


def _conv_geom(x: torch.Tensor, kh: int, kw: int, pad: int, stride: int):
    """kfac_conv_geom of an NHWC bf16 input (batch, height, width, channels), contiguous."""
    assert x.dim() == 4 and x.dtype == torch.bfloat16 and x.is_contiguous(), "x: contiguous NHWC bf16"
    B, H, W, C = x.shape
    return _lib.ConvGeom(B, H, W, C, int(kh), int(kw), int(pad), int(stride))


def conv_out_size(h: int, k: int, pad: int, stride: int) -> int:
    return (h + 2 * pad - k) // stride + 1


def conv_ea_update(F: torch.Tensor, x: torch.Tensor, kh: int, kw: int, pad: int, stride: int, rho: float,
                   scale: float = None, append_ones: bool = False, F_bf16: torch.Tensor = None,
                   workspace=None) -> torch.Tensor:
    """In place: F <- rho F + (1 - rho) scale [P|1]^T [P|1], P the im2col patches of the NHWC
    input x (rows: output positions; columns: (dy, dx, c)); optionally refreshes F_bf16."""
    import ctypes
    _require_cuda(F, x, F_bf16)
    g = _conv_geom(x, kh, kw, pad, stride)
    n = x.shape[0] * conv_out_size(x.shape[1], kh, pad, stride) * conv_out_size(x.shape[2], kw, pad, stride)
    if scale is None:
        scale = 1.0 / max(n, 1)
    L = lib()
    d = F.shape[0]
    if workspace is None:
        ws_bytes = L.kfac_conv_ea_update_workspace(d, ctypes.byref(g))
        workspace = _workspace(ws_bytes, F.device) if ws_bytes else None
    ws_bytes = 0 if workspace is None else workspace.numel()
    check("kfac_conv_ea_update", L.kfac_conv_ea_update(
        _ptr(F), d, F.stride(0), _ptr(x), ctypes.byref(g), 1 if append_ones else 0, float(rho), float(scale),
        _ptr(F_bf16), 0 if F_bf16 is None else F_bf16.stride(0), _ptr(workspace), ws_bytes, _stream()))
    return F


def conv_backward_weight(g: torch.Tensor, x: torch.Tensor, kh: int, kw: int, pad: int, stride: int,
                         with_bias: bool = True, Gamma: torch.Tensor = None, Gamma_bf16: torch.Tensor = None,
                         rho: float = 0.95, scale: float = None, workspace=None, dWb: torch.Tensor = None):
    """[dW | db] = g^T [P | 1] (fp32, c_out x (kh kw C + with_bias), columns (dy, dx, c) then the
    bias) from the NHWC output gradient g (batch, out_h, out_w, c_out; bf16) and the NHWC
    input x; with Gamma, also Gamma <- rho Gamma + (1 - rho) scale g^T g in place (fused).
    workspace: K-slice partials (default: the size the library asks for)."""
    import ctypes
    _require_cuda(g, x, Gamma, Gamma_bf16)
    geo = _conv_geom(x, kh, kw, pad, stride)
    assert g.dim() == 4 and g.dtype == torch.bfloat16 and g.is_contiguous()
    c_out = g.shape[3]
    ncol = kh * kw * x.shape[3] + (1 if with_bias else 0)
    if dWb is None:
        dWb = torch.empty((c_out, ncol), dtype=torch.float32, device=g.device)
    assert dWb.dtype == torch.float32 and dWb.shape == (c_out, ncol) and dWb.stride(1) == 1
    if scale is None:
        scale = 1.0 / max(g.shape[0] * g.shape[1] * g.shape[2], 1)
    L = lib()
    if workspace is None:
        ws_bytes = L.kfac_conv_backward_weight_workspace(c_out, ctypes.byref(geo), 1 if with_bias else 0)
        workspace = _workspace(ws_bytes, g.device) if ws_bytes else None
    ws_bytes = 0 if workspace is None else workspace.numel()
    check("kfac_conv_backward_weight", L.kfac_conv_backward_weight(
        _ptr(g), c_out, _ptr(x), ctypes.byref(geo), _ptr(dWb), dWb.stride(0), 1 if with_bias else 0, _ptr(Gamma),
        c_out if Gamma is None else Gamma.stride(0), _ptr(Gamma_bf16),
        c_out if Gamma_bf16 is None else Gamma_bf16.stride(0), float(rho), float(scale), _ptr(workspace), ws_bytes,
        _stream()))
    return dWb


def bf16_shadow(F: torch.Tensor) -> torch.Tensor:
    """bf16 copy of F whose row pitch is a multiple of 64 elements (128 bytes), so the
    bf16 sketch kernels read it with aligned 16-byte loads."""
    d = F.shape[0]
    ld = (F.shape[1] + 63) // 64 * 64
    buf = torch.empty((d, ld), dtype=torch.bfloat16, device=F.device)
    out = buf[:, :F.shape[1]]
    out.copy_(F)
    return out


class Plan:
    """Grouped K-factor step over many factors and layers (kfac_plan_* in the C ABI).

    factors: list of dicts with keys F (d x d fp32), r, p, q, stream_id, and optionally
             F_bf16, X (n x d_in, fp32 or bf16), append_ones, scale, U, D, variant ("srevd" or
             "rsvd").
    layers:  list of dicts with keys fa, fg (factor indices), J (d_g x d_a); S optional.
    The plan owns its workspace and status tensors; launch() only enqueues kernels and may
    be captured in a CUDA/HIP graph after upload()."""

    def __init__(self, factors, layers=(), sketch="bf16", device=None):
        import ctypes
        L = lib()
        self._L = L
        self.factors = [dict(f) for f in factors]
        self.layers = [dict(l) for l in layers]
        dev = device or self.factors[0]["F"].device
        prec = _prec(sketch)
        fds = (_lib.FactorDesc * len(self.factors))()
        for i, f in enumerate(self.factors):
            F = f["F"]
            d = F.shape[0]
            r = int(f["r"])
            _require_cuda(F)
            if prec == _lib.KFAC_SKETCH_BF16 and f.get("F_bf16") is None:
                f["F_bf16"] = bf16_shadow(F)
            f.setdefault("U", torch.empty((d, r), dtype=torch.float32, device=dev))
            f.setdefault("D", torch.empty((r,), dtype=torch.float32, device=dev))
            x = f.get("X")
            fd = fds[i]
            fd.F, fd.d, fd.ldf = F.data_ptr(), d, F.stride(0)
            fb = f.get("F_bf16")
            fd.F_bf16, fd.ldfb = (fb.data_ptr(), fb.stride(0)) if fb is not None else (None, 0)
            fd.r, fd.p, fd.q, fd.stream_id = r, int(f["p"]), int(f["q"]), int(f.get("stream_id", i))
            if x is not None:
                fd.X = x.data_ptr()
                fd.xtype = _lib.KFAC_BF16 if x.dtype == torch.bfloat16 else _lib.KFAC_FP32
                fd.n, fd.d_in, fd.ldx = x.shape[0], x.shape[1], x.stride(0)
                fd.append_ones = 1 if f.get("append_ones") else 0
                fd.scale = float(f.get("scale", 1.0 / x.shape[0]))
            fd.U, fd.ldu, fd.D = f["U"].data_ptr(), f["U"].stride(0), f["D"].data_ptr()
            fd.variant = _variant(f.get("variant", "srevd"))
        lds = (_lib.LayerDesc * max(1, len(self.layers)))()
        for k, l in enumerate(self.layers):
            J = l["J"]
            l.setdefault("S", torch.empty_like(J))
            ld = lds[k]
            ld.fa, ld.fg = int(l["fa"]), int(l["fg"])
            ld.J, ld.ldj, ld.S, ld.lds = J.data_ptr(), J.stride(0), l["S"].data_ptr(), l["S"].stride(0)
        self._fds, self._lds = fds, lds
        h = ctypes.c_void_p()
        check("kfac_plan_create", L.kfac_plan_create(ctypes.byref(fds), len(self.factors),
                                                     ctypes.byref(lds) if self.layers else None,
                                                     len(self.layers), prec, ctypes.byref(h)))
        self._h = h
        self.workspace = torch.empty(int(L.kfac_plan_workspace(h)), dtype=torch.uint8, device=dev)
        self.status = torch.zeros((1,), dtype=torch.int32, device=dev)

    def set_scalars(self, rho=0.95, lam=0.1, seed=0, inversion_index=0, do_ea=True, do_eig=True,
                    do_precondition=True):
        check("kfac_plan_set_scalars", self._L.kfac_plan_set_scalars(
            self._h, float(rho), float(lam), int(seed), int(inversion_index), int(do_ea), int(do_eig),
            int(do_precondition)))
        return self

    def upload(self):
        check("kfac_plan_upload", self._L.kfac_plan_upload(self._h, _ptr(self.workspace), self.workspace.numel(),
                                                           _ptr(self.status), _stream()))
        return self

    @property
    def launch_count(self):
        return int(self._L.kfac_plan_launch_count(self._h))

    def launch(self):
        check("kfac_plan_launch", self._L.kfac_plan_launch(self._h, _stream()))

    def launch_range(self, first, count):
        check("kfac_plan_launch_range", self._L.kfac_plan_launch_range(self._h, int(first), int(count), _stream()))

    def autotune(self, cache_path=None, reps=3):
        """Pick the fastest tile configuration of every grouped fp32 GEMM launch (timed on the
        device; results cached in `cache_path`).  Re-uploads the tables."""
        cp = None if cache_path is None else str(cache_path).encode()
        check("kfac_plan_autotune", self._L.kfac_plan_autotune(self._h, _ptr(self.workspace), self.workspace.numel(),
                                                               _ptr(self.status), cp, int(reps), _stream()))
        return self

    def force_config(self, gemm_f32=-1, sketch_bf16=-1):
        """Fix the kernel configuration of every fp32 GEMM / bf16 sketch launch (-1: default);
        re-uploads the tables."""
        check("kfac_plan_force_config", self._L.kfac_plan_force_config(self._h, int(gemm_f32), int(sketch_bf16)))
        return self.upload()

    def set_branches(self, nbranch):
        """Run the plan's layer groups on `nbranch` concurrent streams (1..4); re-uploads."""
        check("kfac_plan_set_branches", self._L.kfac_plan_set_branches(self._h, int(nbranch)))
        return self.upload()

    def launch_branches(self):
        return [int(self._L.kfac_plan_launch_branch(self._h, i)) for i in range(self.launch_count)]

    def launch_configs(self):
        return [int(self._L.kfac_plan_launch_config(self._h, i)) for i in range(self.launch_count)]

    def launch_work(self, index):
        """(flops, bytes) of launch `index`: algorithmic work over all its tasks."""
        import ctypes
        f, b = ctypes.c_double(), ctypes.c_double()
        check("kfac_plan_launch_work", self._L.kfac_plan_launch_work(self._h, int(index), ctypes.byref(f),
                                                                     ctypes.byref(b)))
        return f.value, b.value

    def launch_names(self):
        return [self._L.kfac_plan_launch_name(self._h, i).decode() for i in range(self.launch_count)]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._L.kfac_plan_destroy(h)
            self._h = None
