"""GPU parity of the grouped plan (kfac_plan_* in the C ABI): one K-factor step over many
factors and layers in grouped launches, checked against the FP64 oracle (EA, SREVD and
damped inverse of Alg. 1/3/5 and the Sec. 4.1 identity) and against the per-factor entry
points, plus hipGraph replays checked bitwise against an eager launch.

Tolerances as in the per-entry-point tests: EA <= 1e-5 relative Frobenius; e_lambda and e_S
<= 1e-4 on the fp32 and split-bf16 sketch paths, <= 5e-3 on the bf16 sketch path."""
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


def gapped_factor(d, r, seed):
    """F = R diag(sigma) R^T with sigma_i = exp(-2i/r) and a 4x drop after index r: the
    top-r eigenspace is well separated, so S is well conditioned (inside a near-degenerate
    cluster the truncated preconditioner depends on which basis of the cluster is kept, and
    then no two correct implementations need agree)."""
    sig = np.exp(-2.0 * np.arange(d) / max(r, 1))
    sig[r:] *= 0.25
    return synth.psd_factor(d, sig, seed).astype(np.float32)


# (m, bias, r, p, q, ea_batch or 0, ea dtype); l = min(r+p, d); row 2 is the exact regime,
# row 3 has no EA input this step, row 4 has two power iterations and a ragged d = 513
FACTORS = [
    (256, True, 32, 10, 1, 128, "fp32"),
    (128, False, 32, 10, 1, 128, "fp32"),
    (64, True, 60, 10, 1, 100, "bf16"),
    (300, False, 20, 5, 0, 0, None),
    (512, True, 64, 16, 2, 1000, "bf16"),
    (1, False, 1, 0, 0, 7, "fp32"),
]
LAYERS = [(0, 1), (3, 2), (4, 1), (5, 5), (2, 4)]


def make_problem(seed=0):
    facs, inputs = [], []
    for i, (m, bias, r, p, q, n, dt) in enumerate(FACTORS):
        F0 = gapped_factor(m + (1 if bias else 0), r, 1000 + 17 * i)
        X = None
        if n:
            R = synth.haar_orthogonal(m, 2000 + i)
            X = synth.activation_batch(n, R, 0.2 * synth.power_spectrum(m), 3000 + i, seed).astype(np.float32)
        facs.append(dict(F0=F0, X=X, r=r, p=p, q=q, bias=bias, dt=dt, n=n))
    rng = np.random.default_rng(seed + 5)
    Js = [rng.standard_normal((facs[g]["F0"].shape[0], facs[a]["F0"].shape[0])).astype(np.float32)
          for a, g in LAYERS]
    return facs, Js


def device_inputs(facs, Js):
    fd, ld = [], []
    for i, f in enumerate(facs):
        F = torch.from_numpy(f["F0"]).to(DEV)
        desc = dict(F=F, r=f["r"], p=f["p"], q=f["q"], stream_id=i)
        if f["X"] is not None:
            X = torch.from_numpy(f["X"]).to(DEV)
            if f["dt"] == "bf16":
                X = X.to(torch.bfloat16)
            desc.update(X=X, append_ones=f["bias"], scale=1.0 / f["n"])
        fd.append(desc)
    for (a, g), J in zip(LAYERS, Js):
        ld.append(dict(fa=a, fg=g, J=torch.from_numpy(J).to(DEV)))
    return fd, ld


RHO, LAM, SEED, INV = 0.95, 0.1, 11, 2


@pytest.mark.parametrize("sketch", ["fp32", "bf16", "split"])
def test_plan_matches_oracle(sketch):
    facs, Js = make_problem()
    fd, ld = device_inputs(facs, Js)
    plan = K().Plan(fd, ld, sketch=sketch)
    plan.set_scalars(RHO, LAM, SEED, INV).upload()
    assert plan.launch_count > 10
    plan.launch()
    torch.cuda.synchronize()
    assert int(plan.status.item()) == 0
    tol = 5e-3 if sketch == "bf16" else 1e-4
    U_or, D_or = [], []
    for i, f in enumerate(facs):
        Fg = plan.factors[i]["F"]
        if f["X"] is not None:
            Xo = to_np(plan.factors[i]["X"])
            Fo = O.ea_update(f["F0"].astype(np.float64), Xo, RHO, 1.0 / f["n"], append_ones=f["bias"])
            assert rel(to_np(Fg), Fo) <= 1e-5, i
            if sketch == "bf16":
                assert torch.equal(plan.factors[i]["F_bf16"], Fg.to(torch.bfloat16)), i
        else:
            assert np.array_equal(to_np(Fg), f["F0"].astype(np.float64))
        # the oracle continues from the exact factor the GPU holds
        Uo, Do = O.srevd(to_np(Fg), f["r"], f["p"], f["q"], SEED, i, INV)
        U_or.append(Uo)
        D_or.append(Do)
        Dg, Ug = to_np(plan.factors[i]["D"]), to_np(plan.factors[i]["U"])
        assert e_lambda(Dg, Do) <= tol, (i, e_lambda(Dg, Do))
        assert np.abs(Ug.T @ Ug - np.eye(f["r"])).max() < 1e-4, i
    for k, ((a, g), J) in enumerate(zip(LAYERS, Js)):
        So = O.precondition(J.astype(np.float64), U_or[a], D_or[a], U_or[g], D_or[g], LAM)
        assert rel(to_np(plan.layers[k]["S"]), So) <= tol, (k, rel(to_np(plan.layers[k]["S"]), So))


def test_plan_matches_per_factor_entry_points():
    """The grouped launches run the same kernel bodies as the per-factor calls."""
    facs, Js = make_problem(seed=3)
    fd, ld = device_inputs(facs, Js)
    plan = K().Plan(fd, ld, sketch="fp32")
    plan.set_scalars(RHO, LAM, SEED, INV).upload()
    plan.launch()
    torch.cuda.synchronize()
    for i, f in enumerate(facs):
        F = torch.from_numpy(f["F0"]).to(DEV)
        if f["X"] is not None:
            K().ea_update(F, fd[i]["X"], RHO, 1.0 / f["n"], append_ones=f["bias"])
        U, D, st = K().rand_eig(F, f["r"], f["p"], f["q"], seed=SEED, stream_id=i, inversion_index=INV)
        torch.cuda.synchronize()
        assert int(st.item()) == 0
        assert rel(to_np(plan.factors[i]["F"]), to_np(F)) <= 1e-6
        assert e_lambda(to_np(plan.factors[i]["D"]), to_np(D)) <= 1e-5
        Ug, Ue = to_np(plan.factors[i]["U"]), to_np(U)
        k = min(4, f["r"])
        assert np.linalg.norm(Ug[:, :k] @ Ug[:, :k].T - Ue[:, :k] @ Ue[:, :k].T) < 1e-3
    for k, (a, g) in enumerate(LAYERS):
        S = K().precondition(ld[k]["J"], plan.factors[a]["U"], plan.factors[a]["D"], plan.factors[g]["U"],
                             plan.factors[g]["D"], LAM)
        torch.cuda.synchronize()
        assert rel(to_np(plan.layers[k]["S"]), to_np(S)) <= 1e-5


@pytest.mark.parametrize("sketch", ["fp32", "bf16", "split"])
def test_plan_graph_replays_match_eager(sketch):
    facs, Js = make_problem(seed=1)
    fd, ld = device_inputs(facs, Js)
    plan = K().Plan(fd, ld, sketch=sketch)
    plan.set_scalars(RHO, LAM, SEED, INV).upload()
    F0 = [f["F"].clone() for f in plan.factors]
    Fb0 = [f["F_bf16"].clone() if f.get("F_bf16") is not None else None for f in plan.factors]

    def restore():
        for f, a, b in zip(plan.factors, F0, Fb0):
            f["F"].copy_(a)
            if b is not None:
                f["F_bf16"].copy_(b)
        plan.status.zero_()

    def snapshot():
        out = [f[k].clone() for f in plan.factors for k in ("F", "U", "D")]
        return out + [l["S"].clone() for l in plan.layers]

    restore()
    plan.launch()
    torch.cuda.synchronize()
    ref = snapshot()
    assert int(plan.status.item()) == 0
    restore()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.launch()
    torch.cuda.synchronize()
    for rep in range(3):
        restore()
        # unrelated eager work between replays
        junk = torch.randn(1000, 1000, device=DEV) @ torch.randn(1000, 1000, device=DEV)
        g.replay()
        torch.cuda.synchronize()
        got = snapshot()
        for x, y in zip(got, ref):
            assert torch.equal(x, y), rep
        assert int(plan.status.item()) == 0
        del junk


def test_plan_phase_switches():
    """do_ea / do_eig / do_precondition select phases; with EA off the factors are untouched."""
    facs, Js = make_problem(seed=2)
    fd, ld = device_inputs(facs, Js)
    plan = K().Plan(fd, ld, sketch="fp32")
    plan.set_scalars(RHO, LAM, SEED, INV, do_ea=False).upload()
    plan.launch()
    torch.cuda.synchronize()
    for i, f in enumerate(facs):
        assert np.array_equal(to_np(plan.factors[i]["F"]), f["F0"].astype(np.float64))
        Uo, Do = O.srevd(f["F0"].astype(np.float64), f["r"], f["p"], f["q"], SEED, i, INV)
        assert e_lambda(to_np(plan.factors[i]["D"]), Do) <= 1e-4
    n_all = plan.launch_count
    plan.set_scalars(RHO, LAM, SEED, INV, do_ea=False, do_eig=False).upload()
    assert 0 < plan.launch_count < n_all
    S_before = [l["S"].clone() for l in plan.layers]
    plan.launch()
    torch.cuda.synchronize()
    for l, s in zip(plan.layers, S_before):
        assert torch.equal(l["S"], s)   # same U, D and J: same result


def test_plan_rejects_bad_descriptors():
    F = torch.eye(300, device=DEV)
    with pytest.raises(K().KfacError):
        K().Plan([dict(F=F, r=280, p=20, q=1)], sketch="fp32")   # l = 300 > 288 in a plan
    with pytest.raises(K().KfacError):
        K().Plan([dict(F=F, r=0, p=20, q=1)], sketch="fp32")


def test_plan_autotune_keeps_results_bitwise(tmp_path):
    """Every fp32 GEMM tile configuration accumulates each output over k in the same order,
    so the autotuned plan reproduces the default plan bit for bit; the cache is written and
    reused."""
    facs, Js = make_problem(seed=4)
    fd, ld = device_inputs(facs, Js)
    plan = K().Plan(fd, ld, sketch="bf16")
    plan.set_scalars(RHO, LAM, SEED, INV).upload()
    F0 = [f["F"].clone() for f in plan.factors]
    Fb0 = [f["F_bf16"].clone() for f in plan.factors]

    def run():
        for f, a, b in zip(plan.factors, F0, Fb0):
            f["F"].copy_(a)
            f["F_bf16"].copy_(b)
        plan.status.zero_()
        plan.launch()
        torch.cuda.synchronize()
        return [f[k].clone() for f in plan.factors for k in ("F", "U", "D")] + [l["S"].clone() for l in plan.layers]

    ref = run()
    cache = tmp_path / "tune.txt"
    plan.autotune(cache_path=cache, reps=2)
    assert cache.exists() and len(cache.read_text().splitlines()) > 0
    got = run()
    for x, y in zip(got, ref):
        assert torch.equal(x, y)
    plan.autotune(cache_path=cache, reps=2)     # served from the cache
    assert len(cache.read_text().splitlines()) == len(set(cache.read_text().splitlines()))
    got = run()
    for x, y in zip(got, ref):
        assert torch.equal(x, y)


@pytest.mark.parametrize("f32_cfg", [0, 1, 2, 3, 4])
def test_plan_every_gemm_config_matches(f32_cfg):
    """Each fp32 GEMM tile configuration reproduces the default bit for bit (same k order) on
    the fp32-sketch plan, whose Rayleigh-Ritz product can take every configuration; the two
    bf16 sketch kernels (96 x 128 tiles; whole-width tiles with split-K) both meet the bf16
    gates against the oracle under each fp32 configuration."""
    facs, Js = make_problem(seed=6)

    def run(sketch, f32, bf):
        fd, ld = device_inputs(facs, Js)
        plan = K().Plan(fd, ld, sketch=sketch)
        plan.set_scalars(RHO, LAM, SEED, INV).upload()
        plan.force_config(gemm_f32=f32, sketch_bf16=bf)
        plan.launch()
        torch.cuda.synchronize()
        assert int(plan.status.item()) == 0
        return plan

    ref, got = run("fp32", 0, -1), run("fp32", f32_cfg, -1)
    assert any(n == "gemm_f32" and c == f32_cfg for n, c in zip(got.launch_names(), got.launch_configs()))
    for a, b in zip(ref.factors, got.factors):
        assert torch.equal(a["U"], b["U"]) and torch.equal(a["D"], b["D"])
    for a, b in zip(ref.layers, got.layers):
        assert torch.equal(a["S"], b["S"])
    for bf_cfg in (0, 1):
        plan = run("bf16", f32_cfg, bf_cfg)
        names = plan.launch_names()
        assert any(n == ("gemm_bf16_skinny" if bf_cfg else "gemm_bf16") for n in names)
        assert "gemm_bf16x3" in names
        for i, f in enumerate(facs):
            Uo, Do = O.srevd(to_np(plan.factors[i]["F"]), f["r"], f["p"], f["q"], SEED, i, INV)
            assert e_lambda(to_np(plan.factors[i]["D"]), Do) <= 5e-3


@pytest.mark.parametrize("sketch", ["fp32", "split", "bf16"])
@pytest.mark.parametrize("nb", [2, 3, 4])
def test_plan_branches_match_one_branch(sketch, nb):
    """The same plan run as nb concurrent branches (fork / join around plan-owned streams),
    eagerly and as a captured graph, gives the one-branch results: bitwise where every launch
    keeps its kernel (fp32 and split sketches), within the bf16 gate where a branch's own
    sketch-kernel default may differ."""
    facs, Js = make_problem(seed=5)
    outs = []
    for nbr in (1, nb, nb):
        fd, ld = device_inputs(facs, Js)
        plan = K().Plan(fd, ld, sketch=sketch)
        plan.set_scalars(RHO, LAM, SEED, INV).upload()
        if nbr > 1:
            plan.set_branches(nbr)
            br = plan.launch_branches()
            assert set(br) <= set(range(nbr + 1)) and len(set(br)) > 1
        if len(outs) < 2:
            plan.launch()
        else:                                    # third run: a graph capture of the branches
            Fs = [f["F"].clone() for f in plan.factors]
            g = torch.cuda.CUDAGraph()
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s):
                with torch.cuda.graph(g):
                    plan.launch()
            torch.cuda.current_stream().wait_stream(s)
            torch.cuda.synchronize()
            for f, F0 in zip(plan.factors, Fs):
                f["F"].copy_(F0)                 # capture ran nothing: restore anyway
            g.replay()
        torch.cuda.synchronize()
        assert int(plan.status.item()) == 0
        outs.append(([to_np(f["F"]) for f in plan.factors], [to_np(f["D"]) for f in plan.factors],
                     [to_np(f["U"]) for f in plan.factors], [to_np(l["S"]) for l in plan.layers]))
    for o in outs[1:]:
        for a, b in zip(outs[0][0], o[0]):
            assert np.array_equal(a, b)
        for k in (1, 2, 3):
            for a, b in zip(outs[0][k], o[k]):
                if sketch == "bf16":
                    assert rel(a, b) <= 5e-3
                else:
                    assert np.array_equal(a, b)
