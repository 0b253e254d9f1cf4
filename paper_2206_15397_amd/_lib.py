"""ctypes declarations of libkfac.so (see include/kfac.h)."""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(HERE, "libkfac.so")

KFAC_OK, KFAC_EINVAL, KFAC_EWORKSPACE, KFAC_EHIP, KFAC_EUNSUPPORTED, KFAC_ESCRATCH = 0, 1, 2, 3, 4, 5
NOALLOC_SCRATCH_BYTES = 128 << 20
KFAC_FP32, KFAC_BF16 = 0, 1
KFAC_SREVD, KFAC_RSVD = 0, 1
KFAC_SKETCH_FP32, KFAC_SKETCH_BF16, KFAC_SKETCH_SPLIT = 0, 1, 2
STATUS_BITS = {1: "CHOL_SHIFTED", 2: "CHOL_FAILED", 4: "NONFINITE", 8: "EIG_NOCONV"}

# Every function exported by include/kfac.h, with (restype, argtypes).
_p, _i64, _u64, _u32, _i, _f, _sz = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64,
                                     ctypes.c_uint32, ctypes.c_int, ctypes.c_float, ctypes.c_size_t)
SIGNATURES = {
    "kfac_status_string": (ctypes.c_char_p, [_i]),
    "kfac_build_info": (ctypes.c_char_p, []),
    "kfac_fill_identity": (_i, [_p, _i64, _i64, _p]),
    "kfac_ea_update_workspace": (_sz, [_i64, _i64]),
    "kfac_ea_update": (_i, [_p, _i64, _i64, _p, _i, _i64, _i64, _i64, _i, _f, _f, _p, _i64, _p, _sz, _p]),
    "kfac_gaussian_omega": (_i, [_p, _i64, _i64, _i64, _u64, _u64, _u32, _p, _p]),
    "kfac_rand_eig_workspace": (_sz, [_i64, _i64, _i64, _i, _i, _i]),
    "kfac_rand_eig": (_i, [_p, _i64, _i64, _p, _i64, _i64, _i64, _i, _u64, _u64, _u32, _i, _i,
                           _p, _i64, _p, _p, _sz, _p, _p]),
    "kfac_rand_eig_noalloc": (_i, [_p, _i64, _i64, _p, _i64, _i64, _i64, _i, _u64, _u64, _u32, _i, _i,
                                   _p, _i64, _p, _p, _p]),
    "kfac_precondition_workspace": (_sz, [_i64, _i64, _i64, _i64]),
    "kfac_precondition": (_i, [_p, _i64, _i64, _i64, _p, _i64, _p, _i64, _p, _i64, _p, _i64, _f,
                               _p, _i64, _p, _sz, _p]),
    "kfac_linear_forward": (_i, [_p, _i64, _i64, _i64, _p, _i64, _i64, _p, _p, _i64, _p]),
    "kfac_linear_backward": (_i, [_p, _i64, _i64, _i64, _p, _i64, _i64, _p, _i64, _p, _i64, _p, _i64, _i,
                                  _p, _i64, _p, _i64, _f, _f, _p]),
    "kfac_conv_ea_update_workspace": (_sz, [_i64, _p]),
    "kfac_conv_ea_update": (_i, [_p, _i64, _i64, _p, _p, _i, _f, _f, _p, _i64, _p, _sz, _p]),
    "kfac_conv_backward_weight_workspace": (_sz, [_i64, _p, _i]),
    "kfac_conv_backward_weight": (_i, [_p, _i64, _p, _p, _p, _i64, _i, _p, _i64, _p, _i64, _f, _f, _p, _sz, _p]),
    "kfac_plan_create": (_i, [_p, _i, _p, _i, _i, _p]),
    "kfac_plan_workspace": (_sz, [_p]),
    "kfac_plan_set_scalars": (_i, [_p, _f, _f, _u64, _u32, _i, _i, _i]),
    "kfac_plan_upload": (_i, [_p, _p, _sz, _p, _p]),
    "kfac_plan_launch_count": (_i, [_p]),
    "kfac_plan_launch": (_i, [_p, _p]),
    "kfac_plan_launch_range": (_i, [_p, _i, _i, _p]),
    "kfac_plan_launch_name": (ctypes.c_char_p, [_p, _i]),
    "kfac_plan_launch_work": (_i, [_p, _i, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "kfac_plan_autotune": (_i, [_p, _p, _sz, _p, ctypes.c_char_p, _i, _p]),
    "kfac_plan_force_config": (_i, [_p, _i, _i]),
    "kfac_plan_launch_config": (_i, [_p, _i]),
    "kfac_plan_set_branches": (_i, [_p, _i]),
    "kfac_plan_launch_branch": (_i, [_p, _i]),
    "kfac_plan_destroy": (None, [_p]),
}


class FactorDesc(ctypes.Structure):
    """Mirror of kfac_factor_desc (include/kfac.h)."""
    _fields_ = [("F", _p), ("d", _i64), ("ldf", _i64), ("F_bf16", _p), ("ldfb", _i64),
                ("r", _i64), ("p", _i64), ("q", _i), ("stream_id", _u64),
                ("X", _p), ("xtype", _i), ("n", _i64), ("d_in", _i64), ("ldx", _i64),
                ("append_ones", _i), ("scale", _f), ("U", _p), ("ldu", _i64), ("D", _p), ("variant", _i)]


class ConvGeom(ctypes.Structure):
    """Mirror of kfac_conv_geom (include/kfac.h)."""
    _fields_ = [("batch", _i64), ("height", _i64), ("width", _i64), ("channels", _i64),
                ("kh", _i64), ("kw", _i64), ("pad", _i64), ("stride", _i64)]


class LayerDesc(ctypes.Structure):
    """Mirror of kfac_layer_desc (include/kfac.h)."""
    _fields_ = [("fa", _i), ("fg", _i), ("J", _p), ("ldj", _i64), ("S", _p), ("lds", _i64)]


_lock = threading.Lock()
_handle = None


class KfacError(RuntimeError):
    def __init__(self, fn: str, code: int):
        self.code = code
        super().__init__(f"{fn} failed: {status_string(code)} ({code})")


def library_path() -> str:
    return _SO


def lib():
    """The loaded libkfac.so.  Raises if it has not been built: there is no fallback."""
    global _handle
    with _lock:
        if _handle is None:
            if not os.path.exists(_SO):
                raise RuntimeError(
                    f"libkfac.so not found at {_SO}; build it with "
                    "`python -c 'import __graft_entry__ as g; g.build()'` (hipcc, gfx950)")
            h = ctypes.CDLL(_SO)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(h, name)
                fn.restype = res
                fn.argtypes = args
            _handle = h
    return _handle


def status_string(code: int) -> str:
    return lib().kfac_status_string(int(code)).decode()


def check(fn: str, code: int):
    if code != KFAC_OK:
        raise KfacError(fn, code)
