"""GPU checks at the full sizes of the measured workloads, on outputs the oracle (or an fp64
reference formula on the GPU's own inputs) can compute one by one, and on properties that
hold at any size.

* 4-layer MLP, width 4096, batch 512, bf16 (the differentiation workload): sampled columns of
  [dW | db], sampled entries of both EA factors, then one K-factor step at
  r = 256, p = 16, q = 1 with the bf16 sketch: orthonormal U, Ritz values equal to the
  Rayleigh quotients of their vectors, and sampled rows of S against the damped-inverse
  formula (Sec. 4.1) evaluated in fp64 on the GPU's U, D and J.
* One d = 16384 factor built by 50 EA steps of 512 bf16 rows (the wide-factor workload), in
  the grouped plan as bench.py times it: orthonormal U, descending D equal to the Rayleigh
  quotients of U's columns, D interlacing the eigenvalues from a library eigensolver
  (torch.linalg.eigvalsh, fp32) and the leading 16 within the bf16-sketch gate 5e-3.

Tolerances: fp32-accumulated bf16 products <= 1e-5 relative; bf16 outputs within bf16
rounding (4e-3); Ritz values vs Rayleigh quotients <= 1e-4 relative; U^T U - I <= 1e-4."""
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


def test_mlp_width4096_batch512_sampled():
    from paper_2206_15397_amd.autograd import KFACLinearState, kfac_linear
    w, B, depth, rho, lam = 4096, 512, 4, 0.95, 0.1
    g = torch.Generator(device="cpu").manual_seed(41)
    Ws = [(torch.randn((w, w), generator=g) / np.sqrt(w)).to(torch.bfloat16).to(DEV).requires_grad_(True)
          for _ in range(depth)]
    bs = [(0.1 * torch.randn(w, generator=g)).to(DEV).requires_grad_(True) for _ in range(depth)]
    st = [KFACLinearState(w, w, bias=True, rho=rho, device=DEV) for _ in range(depth)]
    x = torch.randn((B, w), generator=g).to(torch.bfloat16).to(DEV)
    t = torch.randn((B, w), generator=g).to(DEV)
    acts, h = [], x
    for i in range(depth):
        acts.append(h)
        h = kfac_linear(h, Ws[i], bs[i], st[i])
        h.retain_grad()
        acts.append(h)
        if i + 1 < depth:
            h = torch.tanh(h)
    loss = 0.5 * ((h.float() - t) ** 2).sum() / B
    loss.backward()
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    cols = rng.choice(w, 16, replace=False)
    rows = rng.choice(B, 4, replace=False)
    for i in range(depth):
        a_in = to_np(acts[2 * i])
        gi = to_np(acts[2 * i + 1].grad.to(torch.bfloat16))   # the bf16 gradient the layer received
        # [dW | db] columns: g^T a  (and g^T 1 for the bias)
        J = st[i].J
        assert rel(to_np(J[:, cols]), gi.T @ a_in[:, cols]) <= 1e-5, i
        assert rel(to_np(J[:, w]), gi.sum(0)) <= 1e-5, i
        # factors: sampled entries
        Gs = to_np(st[i].G)
        Ah = np.concatenate([a_in, np.ones((B, 1))], 1)
        ii, jj = rng.integers(0, w, 32), rng.integers(0, w, 32)
        Go = rho * (ii == jj) + (1 - rho) * B * np.einsum("bi,bi->i", gi[:, ii], gi[:, jj])
        Ao = rho * (ii == jj) + (1 - rho) * np.einsum("bi,bi->i", Ah[:, ii], Ah[:, jj]) / B
        assert np.max(np.abs(Gs[ii, jj] - Go) / (np.abs(Go) + 1e-3 * np.abs(np.diag(Gs)).max())) <= 1e-4, i
        As = to_np(st[i].A)
        assert np.max(np.abs(As[ii, jj] - Ao) / (np.abs(Ao) + 1e-3 * np.abs(np.diag(As)).max())) <= 1e-4, i
    # one K-factor step on the last layer's factors: r = 256, p = 16, q = 1, bf16 sketch
    s = st[depth - 1]
    Ua, Da, s1 = K().rand_eig(s.A, 256, 16, 1, seed=0, stream_id=0, sketch="bf16", F_bf16=s.A.to(torch.bfloat16))
    Ug, Dg, s2 = K().rand_eig(s.G, 256, 16, 1, seed=0, stream_id=1, sketch="bf16", F_bf16=s.G.to(torch.bfloat16))
    J = s.J.contiguous()
    S = K().precondition(J, Ua, Da, Ug, Dg, lam)
    torch.cuda.synchronize()
    assert int(s1.item()) == 0 and int(s2.item()) == 0
    for U, D, F in ((Ua, Da, s.A), (Ug, Dg, s.G)):
        U64, F64 = U.double(), F.double()
        assert (U64.T @ U64 - torch.eye(256, device=DEV, dtype=torch.float64)).abs().max().item() <= 1e-4
        rq = ((F64 @ U64) * U64).sum(0)
        assert ((rq - D.double()).abs() / D.double()).max().item() <= 1e-4
        assert bool((D[:-1] >= D[1:]).all())
    # S rows against the damped-inverse formula in fp64 on the GPU's own U, D, J
    Ua64, Ug64, J64 = Ua.double(), Ug.double(), J.double()
    fa = 1.0 / (Da.double() + lam) - 1.0 / lam
    fg = 1.0 / (Dg.double() + lam) - 1.0 / lam
    M = (J64 @ Ua64) * fa @ Ua64.T + J64 / lam
    r_idx = torch.tensor(rows.tolist() + [0, w - 1], device=DEV)
    Sr = (Ug64[r_idx] * fg) @ (Ug64.T @ M) + M[r_idx] / lam
    assert rel(to_np(S[r_idx]), to_np(Sr)) <= 1e-5


def test_wide_factor_d16384_plan_properties():
    from paper_2206_15397_amd import synth
    d, n, steps, r, p, q = 16384, 512, 50, 256, 16, 2
    k = 2048
    U = synth.torch_haar_orthogonal(d, 301, DEV, k)
    spec = torch.exp(-torch.arange(k, device=DEV, dtype=torch.float32) / 40.0)
    F = K().fill_identity(torch.empty((d, d), device=DEV))
    Fb = K().bf16_shadow(F)
    for st in range(steps):
        a = synth.torch_activation_batch(n, U, spec, 302, st, DEV, out_dtype=torch.bfloat16)
        K().ea_update(F, a, 0.95, 1.0 / n, F_bf16=Fb)
    del U
    plan = K().Plan([dict(F=F, F_bf16=Fb, r=r, p=p, q=q, stream_id=0)], [], sketch="bf16")
    plan.set_scalars(0.95, 0.1, 0, 0, do_ea=False, do_eig=True, do_precondition=False).upload()
    plan.launch()
    torch.cuda.synchronize()
    assert int(plan.status.item()) == 0
    Uo, Do = plan.factors[0]["U"], plan.factors[0]["D"]
    assert bool((Do[:-1] >= Do[1:]).all())
    U64 = Uo.double()
    assert (U64.T @ U64 - torch.eye(r, device=DEV, dtype=torch.float64)).abs().max().item() <= 1e-4
    FU = torch.empty((d, r), device=DEV, dtype=torch.float64)
    for c0 in range(0, d, 4096):                      # F U in fp64, 4096 rows at a time
        FU[c0:c0 + 4096] = F[c0:c0 + 4096].double() @ U64
    rq = (FU * U64).sum(0)
    assert ((rq - Do.double()).abs() / Do.double()).max().item() <= 1e-4
    # against the eigenvalues of a library eigensolver on the same factor (fp32): Ritz values
    # interlace (D_i <= lambda_i for any subspace), and the leading ones, well separated from
    # the rest of the spectrum, are resolved within the bf16-sketch gate (further down the
    # decay the randomized approximation itself, not the arithmetic, sets the error)
    ev = torch.linalg.eigvalsh(F).double().flip(0)[:r]
    assert bool((Do.double() <= ev * (1 + 1e-5) + 1e-7).all())
    assert ((Do.double()[:16] - ev[:16]).abs() / ev[:16]).max().item() <= 5e-3
