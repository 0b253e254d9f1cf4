"""The allocation-free entry point kfac_rand_eig_noalloc (static device scratch, no
workspace argument) against kfac_rand_eig with a caller workspace, through the C ABI: two
calls in a row per sketch precision, the second on a smaller factor, so the second call
runs on the scratch contents the first one left.  Both entry points run the same kernels
in the same order, so the outputs must be bit-identical."""
import numpy as np
import pytest
import torch

from paper_2206_15397_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def K():
    import paper_2206_15397_amd as k
    return k


def factor(d, seed):
    sig = np.exp(-np.arange(d) / 30.0) + 0.05
    return torch.from_numpy(synth.psd_factor(d, sig, seed).astype(np.float32)).to(DEV)


@pytest.mark.parametrize("sketch", ["fp32", "bf16"])
def test_noalloc_matches_workspace_entry_point_twice(sketch):
    cases = [(2305, 256, 16, 1, 7), (300, 40, 10, 2, 8)]       # second call: smaller factor
    for d, r, p, q, sid in cases:
        F = factor(d, 900 + d)
        Fb = K().bf16_shadow(F) if sketch == "bf16" else None
        U0, D0, s0 = K().rand_eig(F, r, p, q, seed=5, stream_id=sid, sketch=sketch, F_bf16=Fb)
        U1 = torch.full((d, r), float("nan"), device=DEV)
        D1 = torch.full((r,), float("nan"), device=DEV)
        s1 = torch.zeros((1,), dtype=torch.int32, device=DEV)
        K().rand_eig_noalloc(F, r, p, q, seed=5, stream_id=sid, sketch=sketch, F_bf16=Fb, U=U1, D=D1, status=s1)
        torch.cuda.synchronize()
        assert int(s0.item()) == 0 and int(s1.item()) == 0, (d, sketch)
        assert torch.equal(D0, D1), (d, sketch)
        assert torch.equal(U0, U1), (d, sketch)


def test_noalloc_rejects_problems_beyond_its_scratch():
    from paper_2206_15397_amd import _lib
    L = K().lib()
    need = L.kfac_rand_eig_workspace(16384, 256, 16, 2, _lib.KFAC_SREVD, _lib.KFAC_SKETCH_BF16)
    assert need > _lib.NOALLOC_SCRATCH_BYTES
    F = torch.zeros((8, 8), device=DEV)
    U = torch.zeros((8, 4), device=DEV)
    st = torch.zeros((1,), dtype=torch.int32, device=DEV)
    code = L.kfac_rand_eig_noalloc(F.data_ptr(), 16384, 16384, F.data_ptr(), 16384, 256, 16, 2, 0, 0, 0,
                                   _lib.KFAC_SREVD, _lib.KFAC_SKETCH_BF16, U.data_ptr(), 256, U.data_ptr(),
                                   st.data_ptr(), None)
    assert code == _lib.KFAC_ESCRATCH
    assert b"scratch" in L.kfac_status_string(code)
