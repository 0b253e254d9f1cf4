"""Oracle parity on the workloads bench.py measures, built by bench.py's own builders and
run in the launch configuration it times: the autotuned bf16 grouped plan of the VGG16_bn
factor set (whose EA launch runs the grouped split-K tiles and the finalize), the plain
per-layer fp32 path of the same set, the d = 16384 wide factor, and the 64-factor batch.

For every factor the oracle continues from the exact factor the GPU holds (its pre-step
factor and the step's activations for the EA; its post-EA factor for the randomized
eigendecomposition, with the same Omega) and every layer's damped inverse is compared with
the oracle's (Alg. 3 SREVD, Alg. 5 and the Sec. 4.1 identity):

* EA (Alg. 1 EA lines): relative Frobenius error <= 1e-5; the bf16 shadow is RNE(F) bitwise.
* e_lambda = max_i |D_i - D_i^or| / D_i^or over the top r: <= 1e-4 (fp32 and split-bf16
  sketches), <= 5e-3 (bf16 sketch).
* the damped inverse applied to the GPU's own (U, D): <= 1e-5 against the fp64 formula.
* e_S = ||S - S^or||_F / ||S^or||_F: <= 1e-4 (fp32 / split sketch), <= 5e-3 (bf16 sketch)
  where both factors' top-r Ritz values are separated from the next one (relative gap at
  the cut >= 1e-2).  Where the cut falls inside a cluster (the VGG16_bn factors: ten EA
  steps from I leave every eigenvalue past the leading few within ~1e-4 of rho^10 = 0.599),
  which directions of the cluster are kept depends on perturbations far below fp32
  rounding, and S with it (Sec. 4.1: kept directions are damped by 1/(D + lambda), dropped
  ones by 1/lambda); there e_S is measured, recorded and held to a bound that documents
  its size (5e-3 fp32 sketch, 2e-2 split-bf16 and bf16 sketches), not to the gate.

Every measured error is appended as a JSON line to the file named by the environment
variable KFAC_PARITY_LOG (when set)."""
import json
import os

import numpy as np
import pytest
import torch

import bench
import oracle as O

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def to_np(t):
    return t.detach().double().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def e_lambda(D, Do):
    return float(np.max(np.abs(D - Do) / np.abs(Do)))


def record(**kw):
    path = os.environ.get("KFAC_PARITY_LOG")
    if path:
        with open(path, "a") as fh:
            fh.write(json.dumps(kw) + "\n")
    print(json.dumps(kw), flush=True)


def check_factor(tag, F_post, F_pre, X, append_ones, n, rho, U, D, r, p, q, seed, stream_id, tol, F_bf16=None):
    """EA and eigen parity of one factor; returns the oracle's (U, D)."""
    F64 = to_np(F_post)
    out = {"case": tag, "d": F64.shape[0]}
    if X is not None:
        Fo = O.ea_update(to_np(F_pre), to_np(X), rho, 1.0 / n, append_ones=append_ones)
        out["e_ea"] = rel(F64, Fo)
        assert out["e_ea"] <= 1e-5, out
    if F_bf16 is not None:
        assert torch.equal(F_bf16, F_post.to(torch.bfloat16)), tag
    Uo, Do, aux = O.srevd(F64, r, p, q, seed, stream_id, return_all=True)
    lam = aux["lam"]
    gap = float((lam[r - 1] - lam[r]) / lam[r - 1]) if r < len(lam) else float("inf")
    Dg = to_np(D)
    out["e_lambda"] = e_lambda(Dg, Do)
    out["cut_gap"] = gap
    record(**out)
    assert bool(np.all(np.diff(Dg) <= 0)), tag
    assert out["e_lambda"] <= tol, out
    Ug = to_np(U)
    assert np.abs(Ug.T @ Ug - np.eye(r)).max() <= 1e-4, tag
    return Uo, Do, gap


# e_S bound where the cut falls inside a cluster: fp32 products (~1e-7 relative) leave
# ~1e-3, split-bf16 products (~1e-5 relative, the dropped lo x lo term and the 8-bit lo
# parts) and bf16 products ~1e-2
FLAT_TOL = {"fp32": 5e-3, "split": 2e-2, "bf16": 2e-2}
# the damped inverse on the GPU's own (U, D): fp32 MFMA products
STAGE_TOL = {"fp32": 1e-5, "split": 1e-5, "bf16": 1e-5}


def check_layer(tag, J, S, Ua, Da, Ug, Dg, oa, og, lam, tol, flat, stage_tol=1e-5):
    J64, S64 = to_np(J), to_np(S)
    Ua64, Da64, Ug64, Dg64 = to_np(Ua), to_np(Da), to_np(Ug), to_np(Dg)
    stage = rel(S64, O.precondition(J64, Ua64, Da64, Ug64, Dg64, lam))
    So = O.precondition(J64, oa[0], oa[1], og[0], og[1], lam)
    sep = min(oa[2], og[2]) >= 1e-2
    out = {"case": tag, "e_S_stage": stage, "e_S": rel(S64, So), "separated_cut": bool(sep),
           "dD_damped": float(max(np.max(np.abs(Da64 - oa[1]) / (oa[1] + lam)),
                                  np.max(np.abs(Dg64 - og[1]) / (og[1] + lam))))}
    record(**out)
    assert stage <= stage_tol, out
    assert out["e_S"] <= (tol if sep else flat), out


# ---- VGG16_bn factor set: the autotuned grouped plans (split-bf16 and bf16 sketches) ------
@pytest.fixture(scope="module", params=["split", "bf16"])
def vgg_plan(request):
    dev = torch.device(DEV)
    wl, layers = bench.build_workload(dev, act_dtype_bf16=True)
    bench.make_buffers(wl, layers, dev, "bf16")
    plan = bench.make_plan(wl, layers, sketch=request.param, autotune=True)
    bench.restore(layers)
    plan.status.zero_()
    plan.launch()
    torch.cuda.synchronize()
    assert int(plan.status.item()) == 0
    yield request.param, wl, layers, plan
    del plan


@pytest.mark.parametrize("li", range(16))
def test_vgg16_bn_plan_layer_matches_oracle(vgg_plan, li):
    sketch, wl, layers, plan = vgg_plan
    L = layers[li]
    tol = 5e-3 if sketch == "bf16" else 1e-4
    sh = sketch == "bf16"
    oa = check_factor(f"vgg_plan_{sketch}/{L.shape.name}/A", L.A, L.A0, L.a, L.shape.bias, L.n, wl.rho, L.Ua, L.Da,
                      L.ra, wl.p, wl.q, wl.seed, 2 * li, tol, F_bf16=L.Ab if sh else None)
    og = check_factor(f"vgg_plan_{sketch}/{L.shape.name}/G", L.G, L.G0, L.g, False, L.n, wl.rho, L.Ug, L.Dg, L.rg,
                      wl.p, wl.q, wl.seed, 2 * li + 1, tol, F_bf16=L.Gb if sh else None)
    check_layer(f"vgg_plan_{sketch}/{L.shape.name}", L.J, L.S, L.Ua, L.Da, L.Ug, L.Dg, oa, og, wl.lam, tol,
                FLAT_TOL[sketch], stage_tol=STAGE_TOL[sketch])


# ---- VGG16_bn factor set: the plain per-layer fp32 path (the bench's comparator) -----------
@pytest.fixture(scope="module")
def vgg_plain():
    dev = torch.device(DEV)
    wl, layers = bench.build_workload(dev, act_dtype_bf16=True)
    for L in layers:
        L.a, L.g = L.a.float(), L.g.float()
    bench.make_buffers(wl, layers, dev, "fp32")
    bench.restore(layers)
    for li, L in enumerate(layers):
        bench.layer_step(wl, li, L, "fp32", False)
    torch.cuda.synchronize()
    for L in layers:
        assert int(L.st.abs().sum().item()) == 0
    return wl, layers


@pytest.mark.parametrize("li", range(16))
def test_vgg16_bn_plain_fp32_layer_matches_oracle(vgg_plain, li):
    wl, layers = vgg_plain
    L = layers[li]
    tol = 1e-4
    oa = check_factor(f"vgg_plain/{L.shape.name}/A", L.A, L.A0, L.a, L.shape.bias, L.n, wl.rho, L.Ua, L.Da, L.ra,
                      wl.p, wl.q, wl.seed, 2 * li, tol)
    og = check_factor(f"vgg_plain/{L.shape.name}/G", L.G, L.G0, L.g, False, L.n, wl.rho, L.Ug, L.Dg, L.rg, wl.p,
                      wl.q, wl.seed, 2 * li + 1, tol)
    check_layer(f"vgg_plain/{L.shape.name}", L.J, L.S, L.Ua, L.Da, L.Ug, L.Dg, oa, og, wl.lam, tol,
                FLAT_TOL["fp32"])


# ---- wide factor d = 16384 (r = 256, p = 16, q = 2), the plan as bench.py times it ---------
def test_wide_factor_d16384_matches_oracle():
    import paper_2206_15397_amd as K
    d = 16384
    F, Fb, F_prev, a = bench.build_wide(d, torch.device(DEV), keep_last_input=True)
    plan = K.Plan([dict(F=F, F_bf16=Fb, r=bench.WIDE_R, p=bench.WIDE_P, q=bench.WIDE_Q, stream_id=0)], [],
                  sketch="bf16")
    plan.set_scalars(0.95, 0.1, 0, 0, do_ea=False, do_eig=True, do_precondition=False).upload()
    plan.launch()
    torch.cuda.synchronize()
    assert int(plan.status.item()) == 0
    check_factor("wide_d16384", F, F_prev, a, False, bench.WIDE_N, 0.95, plan.factors[0]["U"],
                 plan.factors[0]["D"], bench.WIDE_R, bench.WIDE_P, bench.WIDE_Q, 0, 0, 5e-3, F_bf16=Fb)


# ---- 64 factors of log-uniform sizes, the batched plan as bench.py times it (split-bf16
# sketch: the bf16 copy of these factors perturbs them by ~2^-9 ||F||, a sizeable fraction
# of lambda_r for their e^(-j/40) spectra, so only the fp32-class sketch meets the gates) ---
@pytest.fixture(scope="module")
def batched64():
    import paper_2206_15397_amd as K
    facs, lays = bench.build_batched64(torch.device(DEV))
    plan = K.Plan(facs, lays, sketch=bench.BATCHED64_SKETCH)
    plan.set_scalars(0.95, 0.1, 0, 0, do_ea=False).upload()
    plan.autotune(cache_path=None, reps=1)
    plan.launch()
    torch.cuda.synchronize()
    assert int(plan.status.item()) == 0
    yield plan
    del plan


@pytest.mark.parametrize("grp", range(8))
def test_batched64_layers_match_oracle(batched64, grp):
    plan = batched64
    for j in range(4 * grp, 4 * grp + 4):
        lay = plan.layers[j]
        ors = {}
        for side in ("fg", "fa"):
            i = lay[side]
            f = plan.factors[i]
            ors[side] = check_factor(f"batched64/f{i}", f["F"], None, None, False, 0, 0.95, f["U"], f["D"], f["r"],
                                     f["p"], f["q"], 0, i, 1e-4)
        fa, fg = plan.factors[lay["fa"]], plan.factors[lay["fg"]]
        check_layer(f"batched64/l{j}", lay["J"], lay["S"], fa["U"], fa["D"], fg["U"], fg["D"], ors["fa"], ors["fg"],
                    0.1, 1e-4, FLAT_TOL[bench.BATCHED64_SKETCH], stage_tol=STAGE_TOL[bench.BATCHED64_SKETCH])
