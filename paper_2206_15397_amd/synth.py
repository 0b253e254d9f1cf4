"""Seeded synthetic inputs shaped like the paper's workloads.

This module builds *inputs* only (activation batches, back-propagated gradients,
directly-constructed PSD factors, gradient matrices and layer shape tables).  It holds
none of the K-factor method's arithmetic: EA updates, sketches, eigensolves and the
damped inverse are computed elsewhere (GPU library, or the CPU oracle in tests).

Recipes (the paper measures CIFAR-10 / VGG16_bn, which is not available here, so these
stand in for it; spectra follow the decay the paper reports for K-factors, Sec. 3):
  * rotation R: Haar-random orthogonal matrix (QR of a Gaussian, signs fixed by diag(R));
  * power-law spectrum sigma_i = i^-1.5, or exponential sigma_i = exp(-i/40);
  * activation batch a = Z diag(sqrt(sigma)) R^T with Z ~ N(0,1)^{n x m}, fresh Z per
    EA step, so E[a^T a]/n = R diag(sigma) R^T;
  * direct factor F = U diag(sigma) U^T;
  * layer gradient J = g^T [a | 1] / n (the weight-gradient of a linear map).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# Seeds of the input streams (kept apart from the Omega seed of the method).
SEED_ROT_A = 101
SEED_ROT_G = 102
SEED_ACT_A = 201
SEED_ACT_G = 202
SEED_J = 203


def power_spectrum(m: int, alpha: float = 1.5) -> np.ndarray:
    return np.arange(1, m + 1, dtype=np.float64) ** (-alpha)


def exp_spectrum(m: int, scale: float = 40.0) -> np.ndarray:
    return np.exp(-np.arange(1, m + 1, dtype=np.float64) / scale)


def haar_orthogonal(m: int, seed: int, k: Optional[int] = None) -> np.ndarray:
    """m x k matrix with orthonormal columns, Haar-distributed (Mezzadri's sign fix)."""
    k = m if k is None else k
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((m, k))
    Q, R = np.linalg.qr(Z)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s[None, :]


def psd_factor(d: int, spectrum: np.ndarray, seed: int) -> np.ndarray:
    """F = U diag(spectrum) U^T in float64 (len(spectrum) <= d: thin U)."""
    k = len(spectrum)
    U = haar_orthogonal(d, seed, k)
    return (U * spectrum[None, :]) @ U.T


def activation_batch(n: int, rot: np.ndarray, spectrum: np.ndarray, seed: int,
                     step: int = 0) -> np.ndarray:
    """n x m batch a = Z diag(sqrt(sigma)) R^T (row = one sample)."""
    rng = np.random.default_rng([seed, step])
    Z = rng.standard_normal((n, rot.shape[1]))
    return (Z * np.sqrt(spectrum)[None, :]) @ rot.T


def gaussian(shape, seed: int, step: int = 0) -> np.ndarray:
    return np.random.default_rng([seed, step]).standard_normal(shape)


# ----------------------------------------------------------------------------------------
# Torch (device) versions of the same recipes, for workloads too large for the host.
# ----------------------------------------------------------------------------------------
def torch_haar_orthogonal(m: int, seed: int, device, k: Optional[int] = None):
    import torch
    k = m if k is None else k
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) * 1000003 + m)
    Z = torch.randn((m, k), generator=g, device=device, dtype=torch.float32)
    Q, R = torch.linalg.qr(Z)
    s = torch.sign(torch.diagonal(R))
    s[s == 0] = 1.0
    return Q * s[None, :]


def torch_activation_batch(n: int, rot, spectrum_t, seed: int, step: int, device, out_dtype=None):
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) * 7919 + int(step) * 104729 + rot.shape[0])
    Z = torch.randn((n, rot.shape[1]), generator=g, device=device, dtype=torch.float32)
    a = (Z * torch.sqrt(spectrum_t)[None, :]) @ rot.T
    return a if out_dtype is None else a.to(out_dtype)


# ----------------------------------------------------------------------------------------
# Layer tables.
# ----------------------------------------------------------------------------------------
@dataclass
class LayerShape:
    name: str
    m_a: int            # input features (9*C_in for a 3x3 conv, fan-in for FC)
    d_g: int            # output features (C_out)
    n: int              # sample rows per EA step (B*H*W for conv, B for FC)
    bias: bool = True

    @property
    def d_a(self) -> int:
        return self.m_a + (1 if self.bias else 0)


# (C_in, C_out, input height = width) of VGG16_bn's 3x3 convolutions (padding 1, stride 1)
# on 32x32 inputs
VGG16_BN_CONVS = [(3, 64, 32), (64, 64, 32), (64, 128, 16), (128, 128, 16), (128, 256, 8),
                  (256, 256, 8), (256, 256, 8), (256, 512, 4), (512, 512, 4), (512, 512, 4),
                  (512, 512, 2), (512, 512, 2), (512, 512, 2)]


def vgg16_bn_cifar_layers(batch: int = 128) -> List[LayerShape]:
    """VGG16_bn on 32x32 inputs with the paper's extra 512->512 FC layer (Sec. 5):
    13 3x3 convolutions (channels 64,64,128,128,256x3,512x6, spatial size halving after
    each block) and FC 512->512->512->10.  A-factor dim = 9*C_in + 1, G-factor dim = C_out."""
    out = []
    for i, (ci, co, hw) in enumerate(VGG16_BN_CONVS):
        out.append(LayerShape(f"conv{i + 1}", 9 * ci, co, batch * hw * hw, True))
    for i, (fi, fo) in enumerate([(512, 512), (512, 512), (512, 10)]):
        out.append(LayerShape(f"fc{i + 1}", fi, fo, batch, True))
    return out


def c5_factor_sizes(count: int = 64, lo: int = 64, hi: int = 8192) -> List[int]:
    """Deterministic log-uniform quantile grid of factor sizes in [lo, hi]."""
    e = np.log2(hi / lo)
    return [int(round(lo * 2.0 ** (e * i / (count - 1)))) for i in range(count)]


@dataclass
class Workload:
    """A synthetic K-factor workload description (sizes and hyper-parameters)."""
    name: str
    layers: List[LayerShape] = field(default_factory=list)
    rho: float = 0.95
    lam: float = 0.1
    r_cap: int = 256
    p: int = 16
    q: int = 1
    seed: int = 0
    ea_steps_before: int = 10


def single_fc_workload() -> Workload:
    """One FC layer 256->128 with bias, batch 128: A 257x257, G 128x128, r=32, p=10,
    q=1, lambda=0.1, 10 EA steps from identity with rho=0.95."""
    return Workload("fc256x128", [LayerShape("fc", 256, 128, 128, True)],
                    rho=0.95, lam=0.1, r_cap=32, p=10, q=1, seed=0, ea_steps_before=10)


def vgg16_bn_workload() -> Workload:
    return Workload("vgg16_bn_cifar_b128", vgg16_bn_cifar_layers(128), rho=0.95, lam=0.1,
                    r_cap=256, p=16, q=1, seed=0, ea_steps_before=10)
