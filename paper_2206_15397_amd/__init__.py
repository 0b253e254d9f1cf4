"""MI355X-native Randomized K-FAC K-factor pipeline (EA update, randomized symmetric
eigendecomposition, damped low-rank inverse application) behind a C ABI (libkfac.so).

This module only marshals arguments: tensors supply device memory, the current torch
stream supplies the HIP stream, and every step runs in the library's HIP kernels.  The
library is loaded lazily; a missing or unloadable library raises, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

from ._lib import (KFAC_BF16, KFAC_FP32, KFAC_SKETCH_BF16, KFAC_SKETCH_FP32, KFAC_SREVD,
                   KFAC_RSVD, STATUS_BITS, KfacError, lib, library_path)
from .ops import (Plan, bf16_shadow, conv_backward_weight, conv_ea_update, ea_update, fill_identity,
                  gaussian_omega, precondition, rand_eig, rand_eig_noalloc, rand_eig_workspace_bytes,
                  precondition_workspace_bytes)

__all__ = [
    "ea_update", "fill_identity", "gaussian_omega", "rand_eig", "rand_eig_noalloc", "precondition", "lib",
    "library_path", "KfacError", "rand_eig_workspace_bytes", "precondition_workspace_bytes",
    "STATUS_BITS", "Plan", "bf16_shadow", "conv_ea_update", "conv_backward_weight",
]
