"""Non-finite factors: a NaN or Inf entry in a K-factor must surface as the status bit
KFAC_DS_NONFINITE (set where a Gram or the projected matrix C of Alg. 3 is formed), the
launches must still complete (every loop of the small eigensolver has a fixed trip count and
the descending selection orders NaN last, so every index it hands on is a valid row), and in
a grouped plan the other factors and layers must come out bitwise as they do without the
bad factor (the factors of a step are independent through Alg. 3 and the Sec. 4.1 inverse)."""
import numpy as np
import pytest
import torch

from paper_2206_15397_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
NONFINITE = 0x4


def K():
    import paper_2206_15397_amd as k
    return k


def gapped(d, r, seed):
    sig = np.exp(-2.0 * np.arange(d) / max(r, 1))
    sig[r:] *= 0.25
    return synth.psd_factor(d, sig, seed).astype(np.float32)


def poison(F, bad, i, j):
    F = F.copy()
    F[i, j] = bad
    F[j, i] = bad
    return F


@pytest.mark.parametrize("sketch", ["fp32", "bf16", "split"])
@pytest.mark.parametrize("bad", [np.nan, np.inf])
@pytest.mark.parametrize("d,r,p,q", [(300, 32, 8, 1), (600, 300, 16, 0)])
def test_rand_eig_nonfinite_factor_sets_status(sketch, bad, d, r, p, q):
    if sketch != "fp32" and r + p > 288:
        pytest.skip("the bf16 sketch paths take l <= 288")
    print(f"nonfinite rand_eig sketch={sketch} bad={bad} d={d} r={r} p={p} q={q}", flush=True)
    F0 = gapped(d, r, 7)
    ws = torch.empty(K().rand_eig_workspace_bytes(d, r, p, q, sketch), dtype=torch.uint8, device=DEV)
    Fb = torch.from_numpy(poison(F0, bad, 3, d // 2)).to(DEV)
    _, _, st = K().rand_eig(Fb, r, p, q, seed=5, sketch=sketch, workspace=ws)
    torch.cuda.synchronize()
    assert int(st.item()) & NONFINITE, int(st.item())
    # the same workspace then serves a clean factor exactly as a fresh one does
    Fc = torch.from_numpy(F0).to(DEV)
    U1, D1, st1 = K().rand_eig(Fc, r, p, q, seed=5, sketch=sketch, workspace=ws)
    U2, D2, st2 = K().rand_eig(Fc, r, p, q, seed=5, sketch=sketch)
    torch.cuda.synchronize()
    assert int(st1.item()) == 0 and int(st2.item()) == 0
    assert torch.equal(D1, D2) and torch.equal(U1, U2)


@pytest.mark.parametrize("sketch", ["fp32", "bf16"])
def test_plan_nonfinite_factor_is_contained(sketch):
    shapes = [(257, 32, 8, 1), (130, 24, 8, 1), (300, 40, 8, 2)]
    F0 = [gapped(d, r, 50 + i) for i, (d, r, p, q) in enumerate(shapes)]
    rng = np.random.default_rng(3)
    layers = [(0, 2), (1, 0)]
    Js = [rng.standard_normal((shapes[g][0], shapes[a][0])).astype(np.float32) for a, g in layers]

    def run(Fs):
        fd = [dict(F=torch.from_numpy(F).to(DEV), r=r, p=p, q=q, stream_id=i)
              for i, (F, (d, r, p, q)) in enumerate(zip(Fs, shapes))]
        ld = [dict(fa=a, fg=g, J=torch.from_numpy(J).to(DEV)) for (a, g), J in zip(layers, Js)]
        plan = K().Plan(fd, ld, sketch=sketch)
        plan.set_scalars(0.95, 0.1, 9, 0, do_ea=False).upload()
        plan.launch()
        torch.cuda.synchronize()
        return plan

    print(f"nonfinite plan sketch={sketch}", flush=True)
    clean = run(F0)
    assert int(clean.status.item()) == 0
    bad = run([F0[0], poison(F0[1], np.nan, 5, 77), F0[2]])
    assert int(bad.status.item()) & NONFINITE
    for i in (0, 2):
        assert torch.equal(bad.factors[i]["D"], clean.factors[i]["D"]), i
        assert torch.equal(bad.factors[i]["U"], clean.factors[i]["U"]), i
    assert torch.equal(bad.layers[0]["S"], clean.layers[0]["S"])
    assert not torch.isfinite(bad.layers[1]["S"]).all()
