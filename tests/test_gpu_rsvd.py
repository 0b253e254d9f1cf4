"""GPU parity of the RSVD variant (Alg. 2 returning the V factor that Sec. 2.2.2 prescribes
for symmetric PSD factors; used by RS-KFAC, Alg. 4) against the oracle's rsvd with the same
Omega: singular values (e_lambda) <= 1e-4 on the fp32 and split-bf16 sketch paths and
<= 5e-3 on the bf16 one; orthonormal V; the damped inverse built from (V, Sigma) against the oracle's (e_S) where
the top-r space is separated from the rest; Sigma sits between the SREVD Ritz values and the
eigenvalues of F (both on the GPU); and, in a grouped plan mixing both variants, every factor
and layer equals the per-factor entry points' result."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2206_15397_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def K():
    import paper_2206_15397_amd as k
    return k


def to_np(t):
    return t.detach().double().cpu().numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def e_lambda(D, Do):
    return np.max(np.abs(D - Do) / np.abs(Do))


def gapped(d, r, seed):
    sig = np.exp(-2.0 * np.arange(d) / max(r, 1)) + 0.01
    sig[r:] *= 0.25
    return synth.psd_factor(d, sig, seed).astype(np.float32)


@pytest.mark.parametrize("sketch", ["fp32", "bf16", "split"])
@pytest.mark.parametrize("d,r,p,q", [(257, 32, 10, 1), (500, 64, 16, 2), (1100, 100, 16, 0), (2305, 256, 16, 1),
                                     (300, 280, 30, 1)])
def test_rsvd_matches_oracle(sketch, d, r, p, q):
    F = gapped(d, r, 50 + d)
    Ft = torch.from_numpy(F).to(DEV)
    Fb = K().bf16_shadow(Ft) if sketch == "bf16" else None
    V, S, st = K().rand_eig(Ft, r, p, q, seed=4, stream_id=6, sketch=sketch, F_bf16=Fb, variant="rsvd")
    U, D, st2 = K().rand_eig(Ft, r, p, q, seed=4, stream_id=6, sketch=sketch, F_bf16=Fb)
    torch.cuda.synchronize()
    assert int(st.item()) == 0 and int(st2.item()) == 0
    F64 = F.astype(np.float64)
    Vo, So = O.rsvd(F64, r, p, q, 4, 6)
    tol = 5e-3 if sketch == "bf16" else 1e-4
    Vg, Sg = to_np(V), to_np(S)
    assert e_lambda(Sg, So) <= tol, e_lambda(Sg, So)
    assert bool(np.all(np.diff(Sg) <= 0))
    assert np.abs(Vg.T @ Vg - np.eye(r)).max() <= 1e-4
    idx = np.argmax(np.abs(Vg), axis=0)
    assert np.all(Vg[idx, np.arange(r)] > 0)
    # SREVD Ritz value <= RSVD singular value <= eigenvalue of F (same Q)
    lam = np.sort(np.linalg.eigvalsh(F64))[::-1][:r]
    Dg = to_np(D)
    assert np.all(Dg <= Sg * (1 + 1e-5) + 1e-7) and np.all(Sg <= lam * (1 + 1e-5) + 1e-7)
    # damped inverse from (V, Sigma) on a random gradient, both sides
    J = np.random.default_rng(d).standard_normal((64, d)).astype(np.float32)
    Ug_small = synth.haar_orthogonal(64, 3)[:, :16]
    Dsm = np.linspace(1.0, 0.2, 16)
    Sg_ = K().precondition(torch.from_numpy(J).to(DEV), V, S, torch.from_numpy(Ug_small.astype(np.float32)).to(DEV),
                           torch.from_numpy(Dsm.astype(np.float32)).to(DEV), 0.1)
    So_ = O.precondition(J.astype(np.float64), Vo, So, Ug_small, Dsm, 0.1)
    assert rel(to_np(Sg_), So_) <= tol


def test_rsvd_projection_error_not_worse_than_srevd():
    # Sec. 2.2.2: V Sigma V^T is the preferable rank-r approximation; on average over draws
    # its error ||F - V Sigma V^T||_F does not exceed SREVD's ||F - U D U^T||_F
    d, r, p, q = 600, 40, 8, 0
    F = synth.psd_factor(d, synth.power_spectrum(d), 77).astype(np.float32)
    Ft = torch.from_numpy(F).to(DEV)
    F64 = F.astype(np.float64)
    er, es = [], []
    for seed in range(8):
        V, S, _ = K().rand_eig(Ft, r, p, q, seed=seed, variant="rsvd")
        U, D, _ = K().rand_eig(Ft, r, p, q, seed=seed)
        torch.cuda.synchronize()
        V, S, U, D = to_np(V), to_np(S), to_np(U), to_np(D)
        er.append(np.linalg.norm(F64 - (V * S) @ V.T))
        es.append(np.linalg.norm(F64 - (U * D) @ U.T))
    assert np.mean(er) <= np.mean(es) * (1 + 1e-6), (np.mean(er), np.mean(es))


@pytest.mark.parametrize("sketch", ["fp32", "bf16", "split"])
def test_plan_mixed_variants_match_single_factor_calls(sketch):
    specs = [(257, 32, 10, 1, "rsvd"), (128, 32, 10, 1, "srevd"), (513, 64, 16, 2, "rsvd"), (40, 30, 16, 1, "rsvd")]
    facs = []
    for i, (d, r, p, q, v) in enumerate(specs):
        F = torch.from_numpy(gapped(d, r, 70 + i)).to(DEV)
        facs.append(dict(F=F, F_bf16=K().bf16_shadow(F), r=r, p=p, q=q, stream_id=i, variant=v))
    rng = np.random.default_rng(3)
    lays = [dict(fa=0, fg=1, J=torch.from_numpy(rng.standard_normal((128, 257)).astype(np.float32)).to(DEV)),
            dict(fa=2, fg=3, J=torch.from_numpy(rng.standard_normal((40, 513)).astype(np.float32)).to(DEV))]
    plan = K().Plan(facs, lays, sketch=sketch)
    plan.set_scalars(0.95, 0.1, 9, 0, do_ea=False).upload()
    plan.launch()
    torch.cuda.synchronize()
    assert int(plan.status.item()) == 0
    outs = []
    for i, f in enumerate(facs):
        U, D, st = K().rand_eig(f["F"], f["r"], f["p"], f["q"], seed=9, stream_id=i, sketch=sketch,
                                F_bf16=f["F_bf16"], variant=f["variant"])
        torch.cuda.synchronize()
        assert int(st.item()) == 0
        outs.append((U, D))
        assert e_lambda(to_np(plan.factors[i]["D"]), to_np(D)) <= 1e-5, i
        assert rel(to_np(plan.factors[i]["U"]), to_np(U)) <= 1e-4, i
    for l in plan.layers:
        S = K().precondition(l["J"], outs[l["fa"]][0], outs[l["fa"]][1], outs[l["fg"]][0], outs[l["fg"]][1], 0.1)
        torch.cuda.synchronize()
        assert rel(to_np(l["S"]), to_np(S)) <= 1e-4
