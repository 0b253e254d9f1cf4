#!/usr/bin/env python3
"""K-factor step benchmark on one MI355X.

Workload: the VGG16_bn-shaped factor set on CIFAR-sized inputs (batch 128, 3x32x32):
13 3x3 convolutions (A-factor dims 9*C_in+1 = 28..4609, G-factor dims C_out = 64..512)
and the FC head 512->512->512->10, i.e. 16 layers / 32 K-factors.  Synthetic activations
follow a 1/i^1.5 covariance under a seeded rotation; factors are built by 10 EA steps
from I (rho 0.95) during untimed setup.  One timed step = EA step 11 for all 32 factors,
the randomized eigendecomposition (SREVD, r=min(256,d), p=16, q=1) of all 32 factors and
the damped inverse (lambda 0.1) for all 16 layer gradients -- with inputs resident in HBM.

Oracle leg (skipped with --no-check): after the timings the FP64 CPU oracle runs the full
step from the GPU's own pre-step factors and the step's activations (EA, SREVD with the same
Omega, damped inverse); its wall time is the `cpu_baseline` and its outputs give the
`parity` object (EA error, e_lambda, e_S per path against the 5e-3 / 1e-4 gates).

Paths measured on the same GPU:
  plan    : the grouped plan (kfac_plan_*): every phase of all 32 factors / 16 layers in one
            launch, bf16 activations and the split-bf16 sketch (fp32 factors as bf16 hi/lo
            pairs on bf16 MFMA), captured once in a hipGraph and replayed -- this is the
            reported `value` (32 factors / median step time);
  plan bf16: the same plan with the sketch on the bf16 shadow of the factors;
  plain   : per-layer entry-point calls on one stream, fp32 activations and fp32 sketch;
  streams : (optional, --streams N) per-factor calls spread over N streams in a hipGraph.
After the timed replays the plan's launches are replayed eagerly with a HIP event between
consecutive launches (queue pre-filled behind a spin kernel), which gives each grouped
launch's duration; the `roofline` object reports the kernel with the largest share of the
step against the published MI355X peak for its arithmetic type.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--streams", type=int, default=0,
                    help="also time per-factor calls spread over this many streams (0: skip)")
    ap.add_argument("--branches", type=int, default=4,
                    help="concurrent branches (streams) of the grouped plan, 1..4")
    ap.add_argument("--no-check", action="store_true",
                    help="skip the oracle leg (CPU baseline timing and parity of the timed outputs)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default GEMM tile configurations")
    ap.add_argument("--config", choices=["vgg", "wide", "batched64", "copy", "vgg_ea", "conv", "driver"],
                    default="vgg",
                    help="vgg: VGG16_bn factor set (default); wide: one d x d factor (--d); "
                         "batched64: 64 factors of log-uniform sizes 64..8192; copy: a plain 1 GiB "
                         "device copy that calibrates the HBM byte counters of rocprofv3; vgg_ea: the "
                         "VGG16_bn EA phase alone (counter harness); conv: the K-FAC work of the VGG16_bn "
                         "convolutions (implicit im2col); driver: the K-FAC driver over one inversion "
                         "period of the paper's schedule")
    ap.add_argument("--sketch", default="split", choices=["bf16", "split", "fp32"],
                    help="--config driver: sketch precision of the driver's plans")
    ap.add_argument("--d", type=int, default=16384, help="factor size of --config wide")
    ap.add_argument("--full-eig", action="store_true", help="--config wide: also time torch.linalg.eigh")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class Layer:
    pass


def build_workload(dev, act_dtype_bf16: bool):
    import torch
    import paper_2206_15397_amd as K
    from paper_2206_15397_amd import synth
    wl = synth.vgg16_bn_workload()
    layers = []
    for li, s in enumerate(wl.layers):
        L = Layer()
        L.shape = s
        L.d_a, L.d_g, L.n = s.d_a, s.d_g, s.n
        Ra = synth.torch_haar_orthogonal(s.m_a, synth.SEED_ROT_A + li, dev)
        Rg = synth.torch_haar_orthogonal(s.d_g, synth.SEED_ROT_G + li, dev)
        sa = torch.tensor(synth.power_spectrum(s.m_a), dtype=torch.float32, device=dev)
        sg = torch.tensor(synth.power_spectrum(s.d_g), dtype=torch.float32, device=dev)
        L.A = K.fill_identity(torch.empty((s.d_a, s.d_a), device=dev))
        L.G = K.fill_identity(torch.empty((s.d_g, s.d_g), device=dev))
        for k in range(wl.ea_steps_before):
            a = synth.torch_activation_batch(s.n, Ra, sa, synth.SEED_ACT_A + li, k, dev)
            g = synth.torch_activation_batch(s.n, Rg, sg, synth.SEED_ACT_G + li, k, dev)
            if act_dtype_bf16:
                a, g = a.to(torch.bfloat16), g.to(torch.bfloat16)
            K.ea_update(L.A, a, wl.rho, 1.0 / s.n, append_ones=s.bias)
            K.ea_update(L.G, g, wl.rho, 1.0 / s.n)
            del a, g
        # the timed step's batch, resident in HBM
        a = synth.torch_activation_batch(s.n, Ra, sa, synth.SEED_ACT_A + li, wl.ea_steps_before, dev)
        g = synth.torch_activation_batch(s.n, Rg, sg, synth.SEED_ACT_G + li, wl.ea_steps_before, dev)
        ah = torch.cat([a, torch.ones((s.n, 1), device=dev)], dim=1)
        L.J = (g.T @ ah / s.n).contiguous()
        del ah
        if act_dtype_bf16:
            a, g = a.to(torch.bfloat16), g.to(torch.bfloat16)
        L.a, L.g = a.contiguous(), g.contiguous()
        L.A0, L.G0 = L.A.clone(), L.G.clone()      # restored before every timed step
        L.Ab = K.bf16_shadow(L.A)
        L.Gb = K.bf16_shadow(L.G)
        L.ra, L.rg = min(wl.r_cap, s.d_a), min(wl.r_cap, s.d_g)
        layers.append(L)
        torch.cuda.synchronize()
    return wl, layers


def make_buffers(wl, layers, dev, sketch):
    import torch
    import paper_2206_15397_amd as K
    for li, L in enumerate(layers):
        L.Ua = torch.empty((L.d_a, L.ra), device=dev)
        L.Da = torch.empty((L.ra,), device=dev)
        L.Ug = torch.empty((L.d_g, L.rg), device=dev)
        L.Dg = torch.empty((L.rg,), device=dev)
        L.S = torch.empty((L.d_g, L.d_a), device=dev)
        L.st = torch.zeros((2,), dtype=torch.int32, device=dev)
        L.ws_a = torch.empty(K.rand_eig_workspace_bytes(L.d_a, L.ra, wl.p, wl.q, sketch), dtype=torch.uint8, device=dev)
        L.ws_g = torch.empty(K.rand_eig_workspace_bytes(L.d_g, L.rg, wl.p, wl.q, sketch), dtype=torch.uint8, device=dev)
        L.ws_p = torch.empty(K.precondition_workspace_bytes(L.d_g, L.d_a, L.ra, L.rg), dtype=torch.uint8, device=dev)
        L.ws_ea_a = torch.empty(max(1, K.lib().kfac_ea_update_workspace(L.d_a, L.n)), dtype=torch.uint8, device=dev)
        L.ws_ea_g = torch.empty(max(1, K.lib().kfac_ea_update_workspace(L.d_g, L.n)), dtype=torch.uint8, device=dev)


def layer_step(wl, li, L, sketch, bf16_shadow):
    """One layer's share of the K-factor step on the current stream."""
    import paper_2206_15397_amd as K
    K.ea_update(L.A, L.a, wl.rho, 1.0 / L.n, append_ones=L.shape.bias, F_bf16=L.Ab if bf16_shadow else None,
                workspace=L.ws_ea_a)
    K.ea_update(L.G, L.g, wl.rho, 1.0 / L.n, F_bf16=L.Gb if bf16_shadow else None, workspace=L.ws_ea_g)
    K.rand_eig(L.A, L.ra, wl.p, wl.q, wl.seed, 2 * li, 0, sketch=sketch, F_bf16=L.Ab if sketch == "bf16" else None,
               U=L.Ua, D=L.Da, workspace=L.ws_a, status=L.st[0:1])
    K.rand_eig(L.G, L.rg, wl.p, wl.q, wl.seed, 2 * li + 1, 0, sketch=sketch, F_bf16=L.Gb if sketch == "bf16" else None,
               U=L.Ug, D=L.Dg, workspace=L.ws_g, status=L.st[1:2])
    K.precondition(L.J, L.Ua, L.Da, L.Ug, L.Dg, wl.lam, S=L.S, workspace=L.ws_p)


def restore(layers):
    for L in layers:
        L.A.copy_(L.A0)
        L.G.copy_(L.G0)


def cost(L):
    return L.d_a ** 2 * (L.ra + 16) + L.d_g ** 2 * (L.rg + 16) + L.n * (L.d_a ** 2 + L.d_g ** 2) / 64


def run_plain(wl, layers, steps, warmup):
    import torch
    for _ in range(warmup):
        restore(layers)
        for li, L in enumerate(layers):
            layer_step(wl, li, L, "fp32", False)
    torch.cuda.synchronize()
    times = []
    for _ in range(steps):
        restore(layers)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for li, L in enumerate(layers):
            layer_step(wl, li, L, "fp32", False)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    return times


def capture_batched(wl, layers, nstreams):
    """Capture one K-factor step: layers assigned to streams by longest-processing-time."""
    import torch
    streams = [torch.cuda.Stream() for _ in range(nstreams)]
    load = [0.0] * nstreams
    assign = [[] for _ in range(nstreams)]
    for li in sorted(range(len(layers)), key=lambda i: -cost(layers[i])):
        k = min(range(nstreams), key=lambda s: load[s])
        assign[k].append(li)
        load[k] += cost(layers[li])

    def body():
        main = torch.cuda.current_stream()      # the capturing stream inside torch.cuda.graph
        fork = torch.cuda.Event()
        fork.record(main)
        joins = []
        for s, lis in zip(streams, assign):
            s.wait_event(fork)
            with torch.cuda.stream(s):
                for li in lis:
                    layer_step(wl, li, layers[li], "bf16", True)
            ev = torch.cuda.Event()
            ev.record(s)
            joins.append(ev)
        for ev in joins:
            main.wait_event(ev)

    # warm the allocator / first-launch paths outside the capture
    body()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        body()
    torch.cuda.synchronize()
    return g


def run_batched(wl, layers, steps, warmup, nstreams):
    import torch
    restore(layers)
    g = capture_batched(wl, layers, nstreams)
    for _ in range(warmup):
        restore(layers)
        g.replay()
    torch.cuda.synchronize()
    times = []
    for _ in range(steps):
        restore(layers)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    return g, times


def make_plan(wl, layers, sketch="bf16", autotune=True, branches=1, variant="srevd"):
    """All 32 factors and 16 layers of the step in one grouped plan (bf16 activations; sketch
    "split": split-bf16 products of the fp32 factors, "bf16": products of the bf16 shadow,
    which the EA phase refreshes): factor 2i is layer i's A factor, 2i+1 its G factor."""
    import paper_2206_15397_amd as K
    fd, ld = [], []
    sh = sketch == "bf16"
    for li, L in enumerate(layers):
        fd.append(dict(F=L.A, F_bf16=L.Ab if sh else None, X=L.a, append_ones=L.shape.bias, scale=1.0 / L.n, r=L.ra,
                       p=wl.p, q=wl.q, stream_id=2 * li, U=L.Ua, D=L.Da, variant=variant))
        fd.append(dict(F=L.G, F_bf16=L.Gb if sh else None, X=L.g, append_ones=False, scale=1.0 / L.n, r=L.rg,
                       p=wl.p, q=wl.q, stream_id=2 * li + 1, U=L.Ug, D=L.Dg, variant=variant))
        ld.append(dict(fa=2 * li, fg=2 * li + 1, J=L.J, S=L.S))
    plan = K.Plan(fd, ld, sketch=sketch)
    plan.set_scalars(wl.rho, wl.lam, wl.seed, 0).upload()
    if branches > 1:
        plan.set_branches(branches)
    if autotune:
        import tempfile
        restore(layers)
        plan.autotune(cache_path=os.path.join(tempfile.gettempdir(), "kfac_autotune_cache.txt"), reps=3)
        restore(layers)
    return plan


def run_plan(wl, layers, steps, warmup, autotune=True, sketch="bf16", branches=1, variant="srevd"):
    import torch
    plan = make_plan(wl, layers, sketch=sketch, autotune=autotune, branches=branches, variant=variant)
    restore(layers)
    plan.launch()                       # first-launch paths outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.launch()
    torch.cuda.synchronize()
    for _ in range(warmup):
        restore(layers)
        g.replay()
    torch.cuda.synchronize()
    times = []
    for _ in range(steps):
        restore(layers)
        plan.status.zero_()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    return plan, g, times


def phase_times(plan, layers, reps, restore_fn=None):
    """Average duration of every grouped launch of the plan: HIP events on the launch
    stream between consecutive launches, with the queue pre-filled behind a spin kernel so
    that host enqueue gaps do not show up as kernel time."""
    import torch
    names = plan.launch_names()
    n = len(names)
    acc = [0.0] * n
    for _ in range(reps):
        if restore_fn is not None:
            restore_fn()
        else:
            restore(layers)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(n + 1)]
        torch.cuda._sleep(20_000_000)
        ev[0].record()
        for i in range(n):
            plan.launch_range(i, 1)
            ev[i + 1].record()
        torch.cuda.synchronize()
        for i in range(n):
            acc[i] += ev[i].elapsed_time(ev[i + 1])
    return names, [a / reps for a in acc]


# Published MI355X peaks: HBM3E bandwidth and dense matrix / vector throughput.
PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"bf16": 2500.0, "fp32": 157.3, "fp64": 78.6}
# split-bf16 products of fp32 operands issue three bf16 MFMAs per product: their peak in
# useful flops is a third of the bf16 one
PEAK_TFLOPS["bf16x3"] = PEAK_TFLOPS["bf16"] / 3
# arithmetic type and unit kind of each grouped launch: "mfma" for matrix-core kernels,
# "alu" for the fp64 vector kernels (single-workgroup factorisations and eigensolver)
KIND = {
    "ea_tiles_bf16": ("bf16", "mfma"), "gemm_bf16": ("bf16", "mfma"), "gemm_bf16_skinny": ("bf16", "mfma"),
    "gemm_bf16x3": ("bf16x3", "mfma"),
    "ea_tiles": ("fp32", "mfma"), "gemm_f32": ("fp32", "mfma"),
    "gram_partial": ("fp64", "mfma"), "trmm": ("fp64", "mfma"),
    "cholinv": ("fp64", "alu"), "trtri_cols": ("fp64", "mfma"),
    "tridiag": ("fp64", "alu"), "backtransform": ("fp64", "alu"),
}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` on `workload` from the rocprofv3 FETCH_SIZE /
    WRITE_SIZE passes recorded in profiles/hbm_traffic.json (scaled by the counters' reading
    for a plain copy of known size), or None when there is no record or the library was
    built from other sources than the ones measured."""
    try:
        import paper_2206_15397_amd as K
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
        src = K.lib().kfac_build_info().decode().rsplit(" src ", 1)[-1]
        if rec.get("src_hash") != src:
            return None
        return rec["workloads"][workload][kernel]["traffic_bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        return None


# Kernel families of the step: the launch sequence is walked in
# order, since a gemm_f32 / slice_reduce launch belongs to the phase it sits in.
A8 = {"tridiag", "tri_prep", "tri_bisect", "tri_select", "tri_vec", "tri_cluster_lead", "tri_cluster",
      "backtransform"}


def families(names):
    """Family of every launch: ea, omega, sketch (sketch and power-iteration products),
    cholqr (Gram, Cholesky, triangular inverse and product), rr (Rayleigh-Ritz product),
    eig (the small eigensolver), ritz (U = QP and column signs), precondition."""
    fam = []
    for nm in names:
        if nm.startswith("ea_"):
            fam.append("ea")
        elif nm == "omega":
            fam.append("omega")
        elif nm in ("gemm_bf16", "gemm_bf16_skinny"):
            fam.append("sketch")
        elif nm == "gemm_bf16x3":
            fam.append(None)            # split-bf16 products: sketch / power or Rayleigh-Ritz
        elif nm in ("gram_partial", "gram_reduce", "cholinv", "trtri_cols", "trmm"):
            fam.append("cholqr")
        elif nm in A8:
            fam.append("eig")
        elif nm.startswith("sign_"):
            fam.append("ritz")
        else:
            fam.append(None)            # fp32 GEMMs and K-slice reductions: by position
    eig = [i for i, f in enumerate(fam) if f == "eig"]
    first_eig, last_eig = (eig[0], eig[-1]) if eig else (len(names), -1)
    # the Rayleigh-Ritz product is the last product before the eigensolver
    prods = [i for i in range(first_eig) if names[i] in ("gemm_f32", "gemm_bf16x3", "gemm_bf16", "gemm_bf16_skinny")]
    rr_at = prods[-1] if prods else None
    seen_ritz = False
    for i, nm in enumerate(names):
        if fam[i] is not None:
            continue
        if nm in ("slice_reduce", "gemm_f32_reduce"):
            fam[i] = fam[i - 1] if i > 0 else "other"
        elif i < first_eig:
            fam[i] = "rr" if i == rr_at else "sketch"
        elif i > last_eig and eig and not seen_ritz:
            fam[i] = "ritz"
            seen_ritz = True
        else:
            fam[i] = "precondition"
    return fam


# arithmetic type each family's roofline is taken against (the EA is priced on HBM bytes)
FAMILY_BOUND = {"sketch": ("bf16", "mfma"), "rr": ("bf16x3", "mfma"), "cholqr": ("fp64", "mfma"),
                "ritz": ("fp32", "mfma"), "precondition": ("fp32", "mfma"), "ea": (None, "hbm"),
                "omega": (None, "hbm")}


def roofline(plan, names, times_ms, workload=None, precondition_dtype="fp32"):
    """Roofline of the step, per kernel family and for the dominant kernel.

    by_family: time per step of each family and its achieved fraction of the roofline that
    bounds it (EA and Omega: HBM on their algorithmic bytes; products: MFMA peak of their
    arithmetic type); the small eigensolver is reported in absolute microseconds only.
    The returned top-level object is the dominant kernel outside the small eigensolver:
    algorithmic work of its launches (kfac_plan_launch_work) over their measured time."""
    fam = families(names)
    bound = dict(FAMILY_BOUND)
    for f in ("sketch", "rr"):            # priced on the arithmetic of the family's product kernel
        ks = [nm for nm, fa in zip(names, fam) if fa == f and nm in KIND]
        if ks:
            bound[f] = (KIND[ks[0]][0], "mfma")
    bound["precondition"] = (precondition_dtype, "mfma")
    byf = {}
    for i, (nm, t) in enumerate(zip(names, times_ms)):
        f, b = plan.launch_work(i)
        a = byf.setdefault(fam[i], [0.0, 0.0, 0.0])
        a[0] += t
        a[1] += f
        a[2] += b
    by_family = {}
    for k, (t_ms, fl, nb) in byf.items():
        e = {"us_per_step": round(1e3 * t_ms, 1)}
        if k in bound and t_ms > 0:
            dt, kind = bound[k]
            if kind == "hbm":
                ach = nb / (t_ms * 1e-3) / 1e9
                e.update({"bound": "hbm", "achieved_GBs": round(ach, 1), "frac": round(ach / PEAK_HBM_GBS, 4)})
            else:
                ach = fl / (t_ms * 1e-3) / 1e12
                e.update({"bound": "mfma", "dtype": dt, "achieved_TFLOPs": round(ach, 2),
                          "frac": round(ach / PEAK_TFLOPS[dt], 4)})
        by_family[k] = e
    tot = {}
    for i, (nm, t) in enumerate(zip(names, times_ms)):
        if nm in A8:
            continue
        f, b = plan.launch_work(i)
        a = tot.setdefault(nm, [0.0, 0.0, 0.0, 0])
        a[0] += t
        a[1] += f
        a[2] += b
        a[3] += 1
    nm = max(tot, key=lambda k: tot[k][0])
    t_ms, flops, nbytes, count = tot[nm]
    dt, unit_kind = KIND.get(nm, ("fp32", "hbm"))
    if nm.startswith("gemm_f32") and fam[names.index(nm)] == "precondition":
        dt = precondition_dtype
    peak_f = PEAK_TFLOPS[dt] * 1e12
    if unit_kind == "hbm" or nm.startswith("ea_") or nbytes / (PEAK_HBM_GBS * 1e9) >= flops / peak_f:
        ach = nbytes / (t_ms * 1e-3) / 1e9
        out = {"bound": "hbm", "achieved": round(ach, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
               "frac": round(ach / PEAK_HBM_GBS, 5)}
    else:
        ach = flops / (t_ms * 1e-3) / 1e12
        out = {"bound": unit_kind, "achieved": round(ach, 4), "peak": PEAK_TFLOPS[dt], "unit": "TFLOP/s",
               "frac": round(ach / PEAK_TFLOPS[dt], 6)}
    traffic = measured_traffic(workload, nm) if workload else None
    out.update({"traffic": traffic, "kernel": nm, "dtype": dt,
                "launches_per_step": count,
                "avg_launch_us": round(1e3 * t_ms / count, 2),
                "flops_per_launch": flops / count, "bytes_per_launch": nbytes / count,
                "traffic_over_algorithmic": None if traffic is None else round(traffic / (nbytes / count), 3),
                "share_of_step": round(t_ms / sum(times_ms), 4),
                "small_eigensolver_us_per_step": round(1e3 * sum(t for n_, t in zip(names, times_ms) if n_ in A8), 1),
                "by_family": by_family})
    return out


def median(xs):
    s = sorted(xs)
    return s[len(s) // 2]


def snapshot(layers, status=None):
    """Host copies of one step of every layer: the pre-step factors and the step's inputs
    (exactly the values the GPU consumed) and every output of the step.  status: the device
    status word of the path (default: the per-layer words of the entry-point calls)."""
    out = []
    for L in layers:
        out.append({k: getattr(L, k).detach().cpu() for k in
                    ("A0", "G0", "a", "g", "J", "A", "G", "Ua", "Da", "Ug", "Dg", "S")})
        out[-1].update(name=L.shape.name, bias=L.shape.bias, n=L.n, ra=L.ra, rg=L.rg,
                       status=int(L.st.abs().sum().item()) if status is None else 0)
    if status is not None and out:
        out[0]["status"] = int(status)
    return out


GATES = {"plan_bf16": 5e-3, "plan_split": 5e-3, "plain_fp32": 1e-4}


def cpu_baseline(wl, snaps):
    """The FP64 oracle on the full step of the same workload, timed on the host cores: for
    every layer the EA of both factors from the GPU's own pre-step factors and the step's
    activations, the randomized eigendecomposition (SREVD, same Omega) of the GPU's post-EA
    factors, and the damped inverse.  snaps: {path: snapshot}, the first being the reported
    path, whose oracle step is the one timed.  The oracle's outputs also give the parity of
    every path (the eigendecompositions are repeated, untimed, from each other path's own
    post-EA factors): EA error, e_lambda (top-r relative eigenvalue error), e_S (relative
    Frobenius error of the preconditioned gradient), the damped inverse applied to the
    GPU's own (U, D) (stage error), the damping-aware eigenvalue error |dD| / (D + lambda)
    and the relative gap of the oracle's Ritz values at the rank cut."""
    import numpy as np
    import oracle as O

    def f64(t):
        return t.double().numpy()

    def rel(a, b):
        return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))

    def eig(F, r, sid):
        U, D, aux = O.srevd(F, r, wl.p, wl.q, wl.seed, sid, return_all=True)
        lam = aux["lam"]
        return U, D, float((lam[r - 1] - lam[r]) / lam[r - 1]) if r < len(lam) else float("inf")

    def layer_errors(s, A, G, oa, og, So):
        Da, Dg = f64(s["Da"]), f64(s["Dg"])
        S = f64(s["S"])
        st = O.precondition(f64(s["J"]), f64(s["Ua"]), Da, f64(s["Ug"]), Dg, wl.lam)
        return {"e_ea": max(rel(f64(s["A"]), A), rel(f64(s["G"]), G)),
                "e_lambda": float(max(np.max(np.abs(Da - oa[1]) / oa[1]), np.max(np.abs(Dg - og[1]) / og[1]))),
                "e_S": rel(S, So), "e_S_stage": rel(S, st),
                "dD_damped": float(max(np.max(np.abs(Da - oa[1]) / (oa[1] + wl.lam)),
                                       np.max(np.abs(Dg - og[1]) / (og[1] + wl.lam)))),
                "cut_gap": min(oa[2], og[2])}

    names = list(snaps)
    first = snaps[names[0]]
    t = {"ea": 0.0, "eig": 0.0, "precondition": 0.0}
    per = {k: [] for k in names}
    t_all = time.perf_counter()
    for li, s in enumerate(first):
        n = s["n"]
        t0 = time.perf_counter()
        A = O.ea_update(f64(s["A0"]), f64(s["a"]), wl.rho, 1.0 / n, append_ones=s["bias"])
        G = O.ea_update(f64(s["G0"]), f64(s["g"]), wl.rho, 1.0 / n)
        t["ea"] += time.perf_counter() - t0
        for k, name in enumerate(names):
            q = snaps[name][li]
            t1 = time.perf_counter()
            oa = eig(f64(q["A"]), q["ra"], 2 * li)
            og = eig(f64(q["G"]), q["rg"], 2 * li + 1)
            t2 = time.perf_counter()
            So = O.precondition(f64(q["J"]), oa[0], oa[1], og[0], og[1], wl.lam)
            t3 = time.perf_counter()
            per[name].append(layer_errors(q, A, G, oa, og, So))
            if k == 0:
                t["eig"] += t2 - t1
                t["precondition"] += t3 - t2
                # conditioning of S: the oracle's own S moves by this much when its input
                # factors are perturbed entrywise at fp32 rounding (relative 2^-24, symmetric)
                rng = np.random.default_rng(1000 + li)

                def pert(F):
                    E = rng.uniform(-1.0, 1.0, F.shape)
                    return F * (1.0 + 2.0 ** -24 * (E + E.T) / 2)
                pa = eig(pert(f64(q["A"])), q["ra"], 2 * li)
                pg = eig(pert(f64(q["G"])), q["rg"], 2 * li + 1)
                per[name][-1]["e_S_floor_fp32_input"] = rel(
                    O.precondition(f64(q["J"]), pa[0], pa[1], pg[0], pg[1], wl.lam), So)
        log(f"  oracle {s['name']}: " + "; ".join(
            f"{nm} e_lambda {per[nm][-1]['e_lambda']:.1e} e_S {per[nm][-1]['e_S']:.1e}" for nm in names))
    t_step = t["ea"] + t["eig"] + t["precondition"]
    nfac = 2 * len(first)
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    except Exception:       # pragma: no cover
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    base = {"value": round(nfac / t_step, 4), "unit": "K-factor eig-inversions/s", "cores": threads,
            "kind": "oracle",
            "sample": f"the full step (all {len(first)} layers / {nfac} factors): FP64 oracle EA "
                      f"{t['ea']:.1f}s + SREVD {t['eig']:.1f}s + damped inverse {t['precondition']:.1f}s = "
                      f"{t_step:.1f}s; its products and QR run in the host BLAS/LAPACK ({threads} threads), "
                      f"its Jacobi sweeps on one core; host nproc={os.cpu_count()}"}
    parity = {}
    for name in names:
        rows = per[name]
        gate = GATES.get(name, 5e-3)
        mx = {k: max(r[k] for r in rows) for k in rows[0] if k not in ("cut_gap", "e_S_floor_fp32_input")}
        sep = [r["cut_gap"] >= 1e-2 for r in rows]
        parity[name] = {"gate": gate, **{k + "_max": float(f"{v:.4g}") for k, v in mx.items()},
                        "e_S_per_layer": [float(f"{r['e_S']:.3g}") for r in rows],
                        "separated_cut_per_layer": sep,
                        **({"e_S_floor_fp32_input_per_layer": [float(f"{r['e_S_floor_fp32_input']:.3g}") for r in rows]}
                           if "e_S_floor_fp32_input" in rows[0] else {}),
                        "e_S_max_separated_cuts": max([r["e_S"] for r, ok in zip(rows, sep) if ok] or [0.0]),
                        "status": sum(sn["status"] for sn in snaps[name]),
                        "pass_e_lambda": bool(mx["e_lambda"] <= gate), "pass_e_S": bool(mx["e_S"] <= gate),
                        "pass_e_S_separated_cuts": bool(max([r["e_S"] for r, ok in zip(rows, sep) if ok] or [0.0])
                                                        <= gate),
                        "pass_ea": bool(mx["e_ea"] <= 1e-5)}
    log(f"  oracle step {time.perf_counter() - t_all:.1f}s")
    return base, parity


def mfma_fraction(plan, names, times_ms):
    """Sum of GEMM flops over sum of (time x peak of the GEMM's arithmetic type), over the
    sketch / power (bf16), Rayleigh-Ritz (fp32 or split-bf16) and Ritz-vector (fp32) GEMM
    launches; a K-slice reduction counts with the GEMM it completes."""
    gemm = {"gemm_bf16": "bf16", "gemm_bf16_skinny": "bf16", "gemm_bf16x3": "bf16x3", "gemm_f32": "fp32"}
    fl, tp, last = 0.0, 0.0, None
    for i, (nm, t) in enumerate(zip(names, times_ms)):
        if nm in gemm:
            last = gemm[nm]
        elif nm not in ("slice_reduce", "gemm_f32_reduce") or last is None:
            last = None
            continue
        f, _ = plan.launch_work(i)
        fl += f
        tp += t * 1e-3 * PEAK_TFLOPS[last] * 1e12
    return fl / tp if tp > 0 else None


def graph_times(plan, steps, warmup, restore_fn):
    import torch
    restore_fn()
    plan.launch()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.launch()
    torch.cuda.synchronize()
    for _ in range(warmup):
        restore_fn()
        g.replay()
    torch.cuda.synchronize()
    times = []
    for _ in range(steps):
        restore_fn()
        plan.status.zero_()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    return g, times


WIDE_N, WIDE_EA_STEPS, WIDE_R, WIDE_P, WIDE_Q = 512, 50, 256, 16, 2


def build_wide(d, dev, keep_last_input=False):
    """The wide-factor workload: d x d factor built from I by 50 EA steps (rho 0.95) of 512
    bf16 activation rows whose covariance has the spectrum e^(-i/40) on a thin Haar basis of
    min(d, 2048) columns; the bf16 shadow is refreshed by the last step.  Returns (F, F_bf16)
    or, with keep_last_input, (F, F_bf16, F before the last step, the last step's rows)."""
    import torch
    import paper_2206_15397_amd as K
    from paper_2206_15397_amd import synth
    n, ea_steps = WIDE_N, WIDE_EA_STEPS
    k = min(d, 2048)
    U = synth.torch_haar_orthogonal(d, 301, dev, k)
    spec = torch.exp(-torch.arange(k, device=dev, dtype=torch.float32) / 40.0)
    F = K.fill_identity(torch.empty((d, d), device=dev))
    Fb = K.bf16_shadow(F)
    prev = a = None
    for st in range(ea_steps):
        a = synth.torch_activation_batch(n, U, spec, 302, st, dev, out_dtype=torch.bfloat16)
        if keep_last_input and st == ea_steps - 1:
            prev = F.clone()
        K.ea_update(F, a, 0.95, 1.0 / n, F_bf16=Fb)
    torch.cuda.synchronize()
    del U
    return (F, Fb, prev, a) if keep_last_input else (F, Fb)


def main_wide(args, dev):
    """One wide factor (build_wide); randomized eig with r = 256, p = 16, q = 2 through a
    one-factor plan (eig phases only)."""
    import tempfile
    import torch
    import paper_2206_15397_amd as K
    d = args.d
    log(f"building d={d} factor ({WIDE_EA_STEPS} EA steps of {WIDE_N} rows) ...")
    t0 = time.time()
    F, Fb = build_wide(d, dev)
    log(f"  setup {time.time() - t0:.1f}s")
    r, p, q = WIDE_R, WIDE_P, WIDE_Q
    plan = K.Plan([dict(F=F, F_bf16=Fb, r=r, p=p, q=q, stream_id=0)], [], sketch="bf16")
    plan.set_scalars(0.95, 0.1, 0, 0, do_ea=False, do_eig=True, do_precondition=False).upload()
    if not args.no_autotune:
        plan.autotune(cache_path=os.path.join(tempfile.gettempdir(), "kfac_autotune_cache.txt"), reps=3)
    nothing = lambda: None
    g, times = graph_times(plan, args.steps, args.warmup, nothing)
    ms = median(times)
    names, pt = phase_times(plan, None, max(3, args.steps // 2), restore_fn=nothing)
    tot = sum(pt)
    for i, (nm, t) in enumerate(zip(names, pt)):
        log(f"  [{i:2d}] {nm:18s} {t * 1e3:9.1f} us  {100 * t / tot:5.1f}%")
    frac = mfma_fraction(plan, names, pt)
    log(f"rand-eig d={d}: median {ms:.3f} ms, GEMM MFMA fraction {frac:.3f}, status={int(plan.status.item())}")
    full_ms = None
    if args.full_eig:
        Fc = F.clone()
        torch.linalg.eigh(Fc)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        torch.linalg.eigh(Fc)
        e1.record()
        torch.cuda.synchronize()
        full_ms = e0.elapsed_time(e1)
        log(f"full eig (torch.linalg.eigh, fp32, comparison only): {full_ms:.1f} ms")
    res = {"metric": "K-factor eig-inversions/s (wide factor)", "value": round(1e3 / ms, 3),
           "unit": "K-factor eig-inversions/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "bf16+fp32+fp64", "data": "synthetic",
           "config": {"workload": f"wide_factor_d{d}_ea50_b512", "d": d, "r": r, "p": p, "q": q},
           "gemm_mfma_fraction": None if frac is None else round(frac, 4),
           "roofline": roofline(plan, names, pt, f"wide_factor_d{d}_ea50_b512"), "full_eig_ms": full_ms}
    print(json.dumps(res), flush=True)


def event_times(calls, reps):
    """Average duration of each callable (one library call each) on the current stream: HIP
    events between consecutive calls, the queue pre-filled behind a spin kernel so that host
    enqueue gaps do not show up as kernel time."""
    import torch
    acc = [0.0] * len(calls)
    for _ in range(reps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(calls) + 1)]
        torch.cuda._sleep(20_000_000)
        ev[0].record()
        for i, c in enumerate(calls):
            c()
            ev[i + 1].record()
        torch.cuda.synchronize()
        for i in range(len(calls)):
            acc[i] += ev[i].elapsed_time(ev[i + 1])
    return [a / reps for a in acc]


def graph_of(fn, steps, warmup):
    """Capture fn once in a graph and time `steps` replays (ms each)."""
    import torch
    fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    times = []
    for _ in range(steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    return g, times


CONV_BATCH = 128


def main_conv(args, dev):
    """The K-FAC work of VGG16_bn's 13 convolutions in one step (batch 128, 32x32 inputs, KFC
    factors): per layer the input factor's EA over the im2col patches of the NHWC input and
    the weight gradient [dW | db] = g^T [P | 1] with the output factor's EA fused, through the
    implicit-im2col kernels (kfac_conv_ea_update, kfac_conv_backward_weight).  Beside it the
    same work with the patches materialised (torch unfold into an n x 9C matrix) and the dense
    kernels (kfac_ea_update, kfac_linear_backward without dx).  Inputs: post-ReLU-like
    activations |N(0, 1)| and N(0, 1e-3) output gradients, bf16, seeded."""
    import torch
    import torch.nn.functional as Fn
    import paper_2206_15397_amd as K
    from paper_2206_15397_amd import synth
    gen = torch.Generator(device=dev)
    gen.manual_seed(4242)
    rho, B = 0.95, CONV_BATCH
    layers = []
    for ci, co, hw in synth.VGG16_BN_CONVS:
        L = Layer()
        L.ci, L.co, L.hw = ci, co, hw
        L.d_a, L.n = 9 * ci + 1, B * hw * hw
        L.x = torch.randn((B, hw, hw, ci), generator=gen, device=dev).abs_().to(torch.bfloat16)
        L.g = (1e-3 * torch.randn((B, hw, hw, co), generator=gen, device=dev)).to(torch.bfloat16)
        L.A = K.fill_identity(torch.empty((L.d_a, L.d_a), device=dev))
        L.G = K.fill_identity(torch.empty((co, co), device=dev))
        L.Ab, L.Gb = K.bf16_shadow(L.A), K.bf16_shadow(L.G)
        geo = K.ops._conv_geom(L.x, 3, 3, 1, 1)
        import ctypes
        wsb = K.lib().kfac_conv_ea_update_workspace(L.d_a, ctypes.byref(geo))
        L.ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev) if wsb else None
        wsd = K.lib().kfac_ea_update_workspace(L.d_a, L.n)
        L.wsd = torch.empty(max(wsd, 1), dtype=torch.uint8, device=dev) if wsd else None
        wsw = K.lib().kfac_conv_backward_weight_workspace(co, ctypes.byref(geo), 1)
        L.wsw = torch.empty(max(wsw, 1), dtype=torch.uint8, device=dev) if wsw else None
        L.dW = torch.empty((co, L.d_a), device=dev)
        L.Wd = torch.zeros((co, 9 * ci), dtype=torch.bfloat16, device=dev)
        L.gs = float(B * B) / L.n
        layers.append(L)

    def ea_call(L):
        return lambda: K.conv_ea_update(L.A, L.x, 3, 3, 1, 1, rho, append_ones=True, F_bf16=L.Ab, workspace=L.ws)

    def dw_call(L):
        return lambda: K.conv_backward_weight(L.g, L.x, 3, 3, 1, 1, with_bias=True, Gamma=L.G, Gamma_bf16=L.Gb,
                                              rho=rho, scale=L.gs, workspace=L.wsw, dWb=L.dW)

    def implicit_step():
        for L in layers:
            ea_call(L)()
            dw_call(L)()

    def patches(L):
        xn = L.x.permute(0, 3, 1, 2)
        u = Fn.unfold(xn, (3, 3), padding=1)                            # B x (C 9) x L, (c, dy, dx)
        return u.view(B, L.ci, 9, -1).permute(0, 3, 2, 1).reshape(L.n, 9 * L.ci).contiguous()

    def explicit_step():
        for L in layers:
            P = patches(L)
            K.ea_update(L.A, P, rho, 1.0 / L.n, append_ones=True, F_bf16=L.Ab, workspace=L.wsd)
            K.ops.linear_backward(L.g.view(L.n, L.co), P, L.Wd, with_bias=True, want_dx=False, Gamma=L.G,
                                  Gamma_bf16=L.Gb, rho=rho, scale=L.gs)

    g1, t_imp = graph_of(implicit_step, args.steps, args.warmup)
    ms_imp = median(t_imp)
    del g1
    log(f"implicit im2col (13 convolutions): median {ms_imp:.3f} ms per step")
    g2, t_exp = graph_of(explicit_step, max(3, args.steps // 2), 1)
    ms_exp = median(t_exp)
    del g2
    log(f"materialised patches + dense kernels: median {ms_exp:.3f} ms per step")
    calls, kinds = [], []
    for L in layers:
        calls += [ea_call(L), dw_call(L)]
        kinds += [("conv_ea", L), ("conv_dw", L)]
    ts = event_times(calls, max(3, args.steps // 2))
    fam = {"conv_ea": [0.0, 0.0, 0.0, 0], "conv_dw": [0.0, 0.0, 0.0, 0]}
    for (kind, L), t in zip(kinds, ts):
        d, n = L.d_a, L.n
        if kind == "conv_ea":
            fl = float(n) * d * (d + 1)                                  # upper triangle of [P|1]^T [P|1]
            by = 2.0 * B * L.hw * L.hw * L.ci + 10.0 * d * d           # NHWC input, factor r/w + bf16 shadow
        else:
            fl = 2.0 * n * L.co * d + float(n) * L.co * (L.co + 1)     # g^T [P|1] and the fused g^T g
            by = 2.0 * B * L.hw * L.hw * (L.ci + L.co) + 4.0 * L.co * d + 10.0 * L.co * L.co
        a = fam[kind]
        a[0] += t
        a[1] += fl
        a[2] += by
        a[3] += 1
        log(f"  {kind} C_in={L.ci:3d} C_out={L.co:3d} {L.hw:2d}x{L.hw:<2d} d_A={d:4d}: {t * 1e3:8.1f} us")
    by_kind = {}
    for kind, (t, fl, by, cnt) in fam.items():
        by_kind[kind] = {"us_per_step": round(1e3 * t, 1), "launches": cnt,
                         "achieved_TFLOPs": round(fl / (t * 1e-3) / 1e12, 2),
                         "mfma_frac_bf16": round(fl / (t * 1e-3) / 1e12 / PEAK_TFLOPS["bf16"], 4),
                         "achieved_GBs": round(by / (t * 1e-3) / 1e9, 1),
                         "hbm_frac": round(by / (t * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
    dom = max(fam, key=lambda k: fam[k][0])
    t, fl, by, cnt = fam[dom]
    ach = fl / (t * 1e-3) / 1e12
    roof = {"bound": "mfma", "achieved": round(ach, 3), "peak": PEAK_TFLOPS["bf16"], "unit": "TFLOP/s",
            "frac": round(ach / PEAK_TFLOPS["bf16"], 5), "traffic": None, "kernel": dom,
            "avg_launch_us": round(1e3 * t / cnt, 2), "flops_per_launch": fl / cnt, "bytes_per_launch": by / cnt,
            "by_kind": by_kind}
    res = {"metric": "K-FAC convolution work per step (VGG16_bn, 13 convolutions)", "value": round(ms_imp, 4),
           "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_imp, 4),
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "bf16+fp32",
           "data": "synthetic",
           "config": {"workload": "vgg16_bn_cifar_b128_convolutions", "batch": B, "layers": 13, "kernel": "3x3/p1/s1"},
           "materialised_patches_ms_per_step": round(ms_exp, 4),
           "speedup_vs_materialised": round(ms_exp / ms_imp, 3), "roofline": roof}
    print(json.dumps(res), flush=True)


def main_driver(args, dev):
    """The K-FAC driver over one inversion period of the paper's Sec. 5 schedule on the
    VGG16_bn layer set (batch 256, the paper's): EA every T_KU = 10 iterations, inversion every
    T_KI = 50 (epoch 0: r = 220, r_l = 10, n_pwr-it = 4), the damped inverse every iteration,
    each iteration one replay of a captured graph.  Reports the K-factor work per training
    iteration amortised over the period, and the three kinds of iteration separately.
    Inputs (the K-factor step benchmark's recipe) are written into the driver's buffers once."""
    import torch
    import paper_2206_15397_amd as K
    from paper_2206_15397_amd import synth
    from paper_2206_15397_amd.driver import KFACDriver, LayerSpec
    from paper_2206_15397_amd.schedule import PaperSchedule
    sched = PaperSchedule()
    shapes = synth.vgg16_bn_cifar_layers(sched.batch)
    drv = KFACDriver([LayerSpec(s.m_a, s.d_g, s.n, s.bias) for s in shapes], schedule=sched, sketch=args.sketch,
                     device=dev)
    # the same input recipe as the K-factor step benchmark: layer inputs and gradients with
    # power-law covariance spectra on Haar bases, J = g^T [a | 1] / n
    for l, s in enumerate(shapes):
        a, g, J = drv.inputs(l)
        Ra = synth.torch_haar_orthogonal(s.m_a, synth.SEED_ROT_A + l, dev)
        Rg = synth.torch_haar_orthogonal(s.d_g, synth.SEED_ROT_G + l, dev)
        sa = torch.tensor(synth.power_spectrum(s.m_a), dtype=torch.float32, device=dev)
        sg = torch.tensor(synth.power_spectrum(s.d_g), dtype=torch.float32, device=dev)
        af = synth.torch_activation_batch(s.n, Ra, sa, synth.SEED_ACT_A + l, 0, dev)
        gf = synth.torch_activation_batch(s.n, Rg, sg, synth.SEED_ACT_G + l, 0, dev)
        J.copy_(gf.T @ torch.cat([af, torch.ones((s.n, 1), device=dev)], dim=1) / s.n)
        a.copy_(af)
        g.copy_(gf)
        del Ra, Rg, af, gf
    torch.cuda.synchronize()
    period = sched.T_KI(0)
    # the first period builds the plans and graphs; the second is timed
    for it in range(period):
        drv.step(it, 0)
    torch.cuda.synchronize()
    kinds = {}
    tot = []
    for rep in range(max(1, args.steps // 10)):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(period + 1)]
        e[0].record()
        for it in range(period):
            drv.step(period * (rep + 1) + it, 0)
            e[it + 1].record()
        torch.cuda.synchronize()
        for it in range(period):
            k = period * (rep + 1) + it
            key = "EA+inversion+precondition" if k % period == 0 else \
                ("EA+precondition" if k % sched.T_KU == 0 else "precondition")
            kinds.setdefault(key, []).append(e[it].elapsed_time(e[it + 1]))
        tot.append(e[0].elapsed_time(e[period]))
    per_it = median(tot) / period
    log(f"driver: {period} iterations in {median(tot):.3f} ms, {per_it:.4f} ms per iteration (amortised)")
    for k, v in kinds.items():
        log(f"  {k}: median {median(v):.3f} ms over {len(v)}")
    # the parts of an inversion iteration: the host's re-upload of the plans' tables (new
    # lambda and inversion index) and the replay of the inversion graph alone
    t0 = time.perf_counter()
    drv._upload_all(drv.inversions)
    up_ms = 1e3 * (time.perf_counter() - t0)
    ginv, tinv = None, []
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        drv._graphs["EIP"].replay()
        e1.record()
        torch.cuda.synchronize()
        tinv.append(e0.elapsed_time(e1))
    log(f"  inversion iteration: table upload {up_ms:.2f} ms (host), graph replay {median(tinv):.3f} ms")
    names, pt = phase_times(drv._plans["EIP"], None, 2, restore_fn=lambda: None)
    agg = {}
    for nm, t in zip(names, pt):
        agg[nm] = agg.get(nm, 0.0) + t
    for nm, t in sorted(agg.items(), key=lambda kv: -kv[1])[:12]:
        log(f"    {nm:18s} {t * 1e3:9.1f} us")
    res = {"metric": "K-factor work per training iteration (amortised over T_KI)", "value": round(per_it, 4),
           "unit": "ms/iteration", "n_gpus": 1, "steps": period * max(1, args.steps // 10), "warmup": period,
           "ms_per_step": round(per_it, 4), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "bf16+fp32+fp64", "data": "synthetic",
           "config": {"workload": "vgg16_bn_cifar_b256_paper_schedule_epoch0", "layers": len(shapes),
                      "T_KU": sched.T_KU, "T_KI": period, "r": sched.rank(0), "r_l": sched.oversampling(0),
                      "q": sched.q, "rho": sched.rho, "lambda": sched.lam(0), "sketch": args.sketch},
           "iteration_ms": {k: round(median(v), 4) for k, v in kinds.items()},
           "inversion_graph_ms": round(median(tinv), 4), "inversion_upload_host_ms": round(up_ms, 3)}
    print(json.dumps(res), flush=True)


BATCHED64_SKETCH = "split"


def build_batched64(dev):
    """64 factors of log-uniform sizes 64..8192 with e^(-j/40) spectra (built in fp64 on a thin
    Haar basis, rounded to fp32 + bf16 shadow); r = min(256, d/2), p = 16, q = 1; 32 layers
    pair (F_2j, F_2j+1) with J ~ N(0, 1).  Returns (factor descriptors, layer descriptors)."""
    import torch
    import paper_2206_15397_amd as K
    from paper_2206_15397_amd import synth
    sizes = synth.c5_factor_sizes(64, 64, 8192)
    facs = []
    for i, d in enumerate(sizes):
        k = min(d, 2048)
        Ud = synth.torch_haar_orthogonal(d, 400 + i, dev, k).double()
        sig = torch.exp(-torch.arange(k, device=dev, dtype=torch.float64) / 40.0)
        F = ((Ud * sig[None, :]) @ Ud.T).float().contiguous()
        del Ud
        facs.append(dict(F=F, F_bf16=K.bf16_shadow(F), r=min(256, d // 2), p=16, q=1, stream_id=i))
    gen = torch.Generator(device=dev)
    gen.manual_seed(203)
    lays = []
    for j in range(32):
        dg, da = sizes[2 * j], sizes[2 * j + 1]
        lays.append(dict(fg=2 * j, fa=2 * j + 1, J=torch.randn((dg, da), generator=gen, device=dev)))
    torch.cuda.synchronize()
    return facs, lays


def main_batched64(args, dev):
    """The 64-factor workload (build_batched64), lambda 0.1.  No EA in the step (factors are
    given)."""
    import tempfile
    import torch
    import paper_2206_15397_amd as K
    log("building 64 factors ...")
    t0 = time.time()
    facs, lays = build_batched64(dev)
    log(f"  setup {time.time() - t0:.1f}s")
    nothing = lambda: None
    alt_ms = {}
    for sk in ("bf16", BATCHED64_SKETCH):          # the reported sketch last (its plan is kept)
        plan = K.Plan(facs, lays, sketch=sk)
        plan.set_scalars(0.95, 0.1, 0, 0, do_ea=False).upload()
        if not args.no_autotune:
            plan.autotune(cache_path=os.path.join(tempfile.gettempdir(), "kfac_autotune_cache.txt"), reps=3)
        g, times = graph_times(plan, args.steps, args.warmup, nothing)
        alt_ms[sk] = median(times)
        log(f"batched64 {sk} sketch: median {alt_ms[sk]:.3f} ms, status={int(plan.status.item())}")
        del g
    ms = alt_ms[BATCHED64_SKETCH]
    names, pt = phase_times(plan, None, max(3, args.steps // 2), restore_fn=nothing)
    plain_ms = None
    if not args.no_plain:
        Fs = [f["F"] for f in facs]
        outs = []
        for f in facs:
            d, r = f["F"].shape[0], f["r"]
            outs.append(dict(U=torch.empty((d, r), device=dev), D=torch.empty((r,), device=dev),
                             ws=torch.empty(K.rand_eig_workspace_bytes(d, r, 16, 1, "fp32"), dtype=torch.uint8,
                                            device=dev), st=torch.zeros((1,), dtype=torch.int32, device=dev)))

        def plain_step():
            for i, f in enumerate(facs):
                o = outs[i]
                K.rand_eig(f["F"], f["r"], 16, 1, 0, i, 0, sketch="fp32", U=o["U"], D=o["D"], workspace=o["ws"],
                           status=o["st"])
            for l in lays:
                K.precondition(l["J"], outs[l["fa"]]["U"], outs[l["fa"]]["D"], outs[l["fg"]]["U"],
                               outs[l["fg"]]["D"], 0.1)
        plain_step()
        torch.cuda.synchronize()
        tpl = []
        for _ in range(max(2, args.steps // 4)):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            plain_step()
            e1.record()
            torch.cuda.synchronize()
            tpl.append(e0.elapsed_time(e1))
        plain_ms = median(tpl)
        log(f"plain per-factor fp32: median {plain_ms:.3f} ms")
    res = {"metric": "K-factor eig-inversions/s (64 factors, batched)", "value": round(64 / (ms / 1e3), 2),
           "unit": "K-factor eig-inversions/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "bf16+fp32+fp64", "data": "synthetic",
           "config": {"workload": "batched64_loguniform_64_8192", "factors": 64, "layers": 32,
                      "r": "min(256,d/2)", "p": 16, "q": 1, "lambda": 0.1, "sketch": BATCHED64_SKETCH},
           "bf16_sketch_ms_per_step": round(alt_ms["bf16"], 4),
           "plain_fp32_ms_per_step": plain_ms,
           "speedup_vs_plain_fp32": None if plain_ms is None else round(plain_ms / ms, 3),
           "roofline": roofline(plan, names, pt, "batched64_loguniform_64_8192")}
    print(json.dumps(res), flush=True)


def main_vgg_ea(args):
    """Counter harness for the EA phase: the VGG16_bn factor set's EA inputs (bf16 activation
    rows of the real shapes, drawn on the host with numpy: no device linear-algebra library
    runs during setup) in a plan with only its EA phase, launched --steps times.  Traffic
    counters do not depend on the values, so these stand in for the benchmark's inputs."""
    import numpy as np
    import torch
    import paper_2206_15397_amd as K
    from paper_2206_15397_amd import synth
    dev = torch.device("cuda:0")
    wl = synth.vgg16_bn_workload()
    rng = np.random.default_rng(7)
    fd, keep = [], []
    for li, s_ in enumerate(wl.layers):
        for d, din, bias in ((s_.d_a, s_.m_a, s_.bias), (s_.d_g, s_.d_g, False)):
            F = K.fill_identity(torch.empty((d, d), device=dev))
            X = torch.from_numpy(rng.standard_normal((s_.n, din), dtype=np.float32)).to(dev).to(torch.bfloat16)
            keep += [F, X]
            fd.append(dict(F=F, F_bf16=K.bf16_shadow(F), X=X, append_ones=bias, scale=1.0 / s_.n,
                           r=min(wl.r_cap, d), p=wl.p, q=wl.q, stream_id=len(fd)))
    plan = K.Plan(fd, [], sketch="bf16")
    plan.set_scalars(wl.rho, wl.lam, wl.seed, 0, do_ea=True, do_eig=False, do_precondition=False).upload()
    names = plan.launch_names()
    for _ in range(max(1, args.steps)):
        plan.launch()
    torch.cuda.synchronize()
    print(json.dumps({"harness": "vgg16_bn EA phase", "launches": names, "steps": max(1, args.steps),
                      "work": [plan.launch_work(i) for i in range(len(names))],
                      "src": K.lib().kfac_build_info().decode().rsplit(" src ", 1)[-1]}), flush=True)


def main_copy(args):
    """Counter calibration: a plain elementwise copy (1 GiB read, 1 GiB written per launch)."""
    import torch
    dev = torch.device("cuda:0")
    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, device=dev)
    dst = torch.empty_like(src)
    for _ in range(max(1, args.steps)):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "elementwise copy", "bytes_read_per_launch": nbytes,
                      "bytes_written_per_launch": nbytes, "launches": max(1, args.steps)}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the library runs on one GPU "
              "per process and has no multi-GPU sharding.", file=sys.stderr)
        sys.exit(2)
    if args.config == "copy":
        return main_copy(args)
    if args.config == "vgg_ea":
        return main_vgg_ea(args)
    if args.config != "vgg":
        import torch
        import paper_2206_15397_amd as K
        K.lib()
        dev = torch.device("cuda:0")
        if args.config == "conv":
            return main_conv(args, dev)
        if args.config == "driver":
            return main_driver(args, dev)
        return main_wide(args, dev) if args.config == "wide" else main_batched64(args, dev)
    import torch
    import paper_2206_15397_amd as K
    dev = torch.device("cuda:0")
    K.lib()
    log("building workload (bf16 activations) ...")
    t0 = time.time()
    wl, layers = build_workload(dev, act_dtype_bf16=True)
    make_buffers(wl, layers, dev, "bf16")
    log(f"  setup {time.time() - t0:.1f}s")
    snaps = {}
    # the reported path: the grouped plan with the bf16-shadow sketch
    plan, gp, tp_ = run_plan(wl, layers, args.steps, args.warmup, autotune=not args.no_autotune, sketch="bf16",
                             branches=args.branches)
    ms_b = median(tp_)
    log(f"plan bf16 sketch ({plan.launch_count} grouped launches, {args.branches} branches): median {ms_b:.3f} ms  "
        f"(min {min(tp_):.3f}, max {max(tp_):.3f}) status={int(plan.status.item())}")
    launches = plan.launch_count
    del gp
    # The roofline is timed on the one-branch schedule of the same plan: there every launch
    # runs one phase of all factors alone on the GPU, so its duration is the kernel's own
    # (concurrent branches share the compute units, and an eager pass over their launches
    # would add up latency-bound launches that the graph overlaps).
    ms_1 = ms_b
    if args.branches > 1:
        plan.set_branches(1)
        if not args.no_autotune:
            import tempfile
            restore(layers)
            plan.autotune(cache_path=os.path.join(tempfile.gettempdir(), "kfac_autotune_cache.txt"), reps=3)
        g1, t1 = graph_times(plan, max(3, args.steps // 2), 1, lambda: restore(layers))
        ms_1 = median(t1)
        del g1
        log(f"  same plan on one branch ({plan.launch_count} launches): median {ms_1:.3f} ms")
    names, pt = phase_times(plan, layers, max(3, args.steps // 2))
    tot = sum(pt)
    cfgs = plan.launch_configs()
    for i, (nm, t) in enumerate(zip(names, pt)):
        log(f"  [{i:2d}] {nm:18s} {t * 1e3:9.1f} us  {100 * t / tot:5.1f}%  cfg {cfgs[i]}")
    roof = roofline(plan, names, pt, "vgg16_bn_cifar_b128_factor_set")
    roof["schedule"] = "one branch (per-launch durations of the same plan's kernels)"
    log(f"roofline: {roof}")
    # the step's outputs (the eager replay above ran one whole step from the restored factors)
    if not args.no_check:
        snaps["plan_bf16"] = snapshot(layers, int(plan.status.item()))
    del plan
    # the same plan with the split-bf16 sketch (fp32-class products)
    plan_b, gb, tb_ = run_plan(wl, layers, max(3, args.steps // 2), 1, autotune=not args.no_autotune, sketch="split",
                               branches=args.branches)
    ms_sp = median(tb_)
    log(f"plan split-bf16 sketch: median {ms_sp:.3f} ms status={int(plan_b.status.item())}")
    del gb
    if not args.no_check:
        restore(layers)
        plan_b.launch()
        torch.cuda.synchronize()
        snaps["plan_split"] = snapshot(layers, int(plan_b.status.item()))
    del plan_b
    # the RSVD variant (Alg. 2) of the same step: timed only (its parity is a GPU test)
    plan_r, gr, tr_ = run_plan(wl, layers, max(3, args.steps // 2), 1, autotune=not args.no_autotune, sketch="bf16",
                               branches=args.branches, variant="rsvd")
    ms_rs = median(tr_)
    log(f"plan bf16 sketch, RSVD variant: median {ms_rs:.3f} ms status={int(plan_r.status.item())}")
    del gr, plan_r
    plain_ms = None
    if args.streams > 0:
        g, tb = run_batched(wl, layers, args.steps, args.warmup, args.streams)
        ms_s = median(tb)
        status_b = [int(x) for L in layers for x in L.st.cpu().tolist()]
        log(f"per-factor bf16 over {args.streams} streams: median {ms_s:.3f} ms status={set(status_b)}")
        del g
    if not args.no_plain:
        for L in layers:
            for n in ("a", "g"):
                setattr(L, n, getattr(L, n).float())
        make_buffers(wl, layers, dev, "fp32")
        tp = run_plain(wl, layers, max(3, args.steps // 4), 1)
        plain_ms = median(tp)
        log(f"plain fp32: median {plain_ms:.3f} ms")
        if not args.no_check:
            snaps["plain_fp32"] = snapshot(layers)
    nfac = 2 * len(layers)
    res = {
        "metric": "K-factor eig-inversions/s + K-FAC step ms vs plain FP32 at <=1e-4/<=5e-3 err",
        "value": round(nfac / (ms_b / 1e3), 2),
        "unit": "K-factor eig-inversions/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_b, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16+fp32+fp64",
        "data": "synthetic",
        "config": {"workload": "vgg16_bn_cifar_b128_factor_set", "factors": nfac, "layers": len(layers),
                   "r": "min(256,d)", "p": wl.p, "q": wl.q, "rho": wl.rho, "lambda": wl.lam,
                   "path": "grouped plan (%d launches, %d branches), bf16 sketch, hipGraph" % (launches, args.branches)},
        "plain_fp32_ms_per_step": None if plain_ms is None else round(plain_ms, 4),
        "speedup_vs_plain_fp32": None if plain_ms is None else round(plain_ms / ms_b, 3),
        "one_branch_ms_per_step": round(ms_1, 4),
        "split_sketch_plan_ms_per_step": round(ms_sp, 4),
        "rsvd_variant_plan_ms_per_step": round(ms_rs, 4),
        "roofline": roof,
    }
    if not args.no_check:
        log("oracle: full step, timed (cpu_baseline) and compared with the GPU outputs (parity) ...")
        base, parity = cpu_baseline(wl, snaps)
        res["cpu_baseline"] = base
        res["parity"] = parity
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
