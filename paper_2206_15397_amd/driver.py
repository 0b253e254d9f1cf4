"""K-FAC driver: the K-factor side of RS-KFAC / SRE-KFAC (Alg. 4 / Alg. 5) over training
iterations, with the periods and schedules of the paper's experiments (Sec. 5), on grouped
plans replayed as captured hipGraphs.

At iteration k of epoch n (schedule: schedule.PaperSchedule or any object with the same
methods):
  * k % T_KU == 0      EA update of every factor from this iteration's layer inputs a and
                       back-propagated gradients g (Alg. 1 EA lines);
  * k % T_KI(n) == 0   randomized decomposition of every factor (SREVD, Alg. 3, or RSVD,
                       Alg. 2) at rank r(n) (or the adaptive rank), oversampling r_l(n), q
                       power iterations, with a fresh Omega (the inversion index counts the
                       inversions);
  * every iteration    damped inverse of every layer's gradient J with the current (U, D)
                       and lambda(n) (Sec. 4.1 identity), into S.
Every combination that occurs (EA + inversion + precondition, EA + precondition, inversion +
precondition, precondition) is one grouped plan captured once in a hipGraph and replayed.
lambda and the inversion index live in the plans' device tables, re-uploaded between
replays; a change of rank or oversampling rebuilds the plans (and their graphs) right before
the inversion that first uses it, so between two inversions every step applies the ranks of
the last one.  Host work per iteration: choosing and replaying one graph.

The caller writes each iteration's inputs into the driver's buffers (`inputs(l)`): the
layer input a (n x d_in, bf16), the gradient g (n x d_out, bf16) and J = Mat(grad W)
(d_out x (d_in + bias), fp32); S (same shape as J) holds the preconditioned gradient after
`step`.  Factors start from the identity (Alg. 1)."""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional, Sequence

import torch

from .ops import Plan, bf16_shadow, fill_identity
from .schedule import AdaptiveRank, PaperSchedule


@dataclass
class LayerSpec:
    d_in: int            # input features of the layer (without the bias column)
    d_out: int           # output features
    n: int               # sample rows per iteration (batch, or batch x positions for a conv)
    bias: bool = True

    @property
    def d_a(self) -> int:
        return self.d_in + (1 if self.bias else 0)


class KFACDriver:
    def __init__(self, layers: Sequence[LayerSpec], schedule=None, sketch: str = "split",
                 variant: str = "srevd", seed: int = 0, rank_cap: int = 256,
                 adaptive: Optional[AdaptiveRank] = None, device="cuda"):
        self.specs = [s if isinstance(s, LayerSpec) else LayerSpec(*s) for s in layers]
        self.sched = schedule or PaperSchedule()
        self.sketch, self.variant, self.seed = sketch, variant, int(seed)
        self.adaptive = adaptive
        self.dev = torch.device(device)
        self.inversions = 0
        self._lam = None
        self._gen = None              # (per-factor ranks, p, q) of the current plans
        self._plans = {}
        self._graphs = {}
        self._ranks = None            # per-factor ranks of the last inversion
        self._want = None             # per-factor ranks requested for the next inversion
        dev = self.dev
        self.F, self.Fb, self.U, self.D, self.X = [], [], [], [], []
        self.J, self.S = [], []
        for s in self.specs:
            for d, din in ((s.d_a, s.d_in), (s.d_out, s.d_out)):
                F = fill_identity(torch.empty((d, d), device=dev))
                self.F.append(F)
                self.Fb.append(bf16_shadow(F) if sketch == "bf16" else None)
                ra = min(d, rank_cap)
                self.U.append(torch.zeros((d, ra), device=dev))
                self.D.append(torch.zeros((ra,), device=dev))
                self.X.append(torch.zeros((s.n, din), dtype=torch.bfloat16, device=dev))
            self.J.append(torch.zeros((s.d_out, s.d_a), device=dev))
            self.S.append(torch.zeros((s.d_out, s.d_a), device=dev))

    # ---- inputs / outputs --------------------------------------------------------------------
    def inputs(self, l: int):
        """(a, g, J) buffers of layer l for the caller to fill before `step`."""
        return self.X[2 * l], self.X[2 * l + 1], self.J[l]

    def factors(self, l: int):
        return self.F[2 * l], self.F[2 * l + 1]

    def decomposition(self, l: int):
        """Current ((U_A, D_A), (U_G, D_G)) of layer l, at the ranks of the last inversion."""
        ra, rg = self._ranks[2 * l], self._ranks[2 * l + 1]
        return ((self.U[2 * l][:, :ra], self.D[2 * l][:ra]), (self.U[2 * l + 1][:, :rg], self.D[2 * l + 1][:rg]))

    def ranks(self) -> List[int]:
        return list(self._ranks) if self._ranks else []

    # ---- plans and graphs --------------------------------------------------------------------
    def _desired_ranks(self, epoch: int) -> List[int]:
        cap = self.sched.rank(epoch)
        base = [min(cap, F.shape[0], self.U[i].shape[1]) for i, F in enumerate(self.F)]
        if self.adaptive is None or self._want is None:
            return base
        return [min(w, b) for w, b in zip(self._want, base)]

    def _build(self, ranks: List[int], p: int, q: int):
        for g in self._graphs.values():
            del g
        self._graphs, self._plans = {}, {}
        fds, lds = [], []
        for i, F in enumerate(self.F):
            s = self.specs[i // 2]
            a_side = i % 2 == 0
            fds.append(dict(F=F, F_bf16=self.Fb[i], X=self.X[i], append_ones=s.bias if a_side else False,
                            scale=1.0 / s.n, r=ranks[i], p=p, q=q, stream_id=i, U=self.U[i], D=self.D[i],
                            variant=self.variant))
        for l in range(len(self.specs)):
            lds.append(dict(fa=2 * l, fg=2 * l + 1, J=self.J[l], S=self.S[l]))
        for key, (ea, eig) in {"EIP": (1, 1), "EP": (1, 0), "IP": (0, 1), "P": (0, 0)}.items():
            pl = Plan(fds, lds, sketch=self.sketch, device=self.dev)
            pl.set_scalars(self.sched.rho, self._lam, self.seed, self.inversions, do_ea=ea, do_eig=eig,
                           do_precondition=True).upload()
            self._plans[key] = pl
        # one eager launch of the precondition-only plan (it writes S only) before capturing,
        # so that no first-launch work happens inside a capture
        self._plans["P"].launch()
        torch.cuda.synchronize(self.dev)
        for key, pl in self._plans.items():
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                pl.launch()
            self._graphs[key] = g
        torch.cuda.synchronize(self.dev)
        self._gen = (tuple(ranks), p, q)

    def _upload_all(self, inv_index: int):
        for key, pl in self._plans.items():
            ea, eig = key in ("EIP", "EP"), key in ("EIP", "IP")
            pl.set_scalars(self.sched.rho, self._lam, self.seed, inv_index, do_ea=ea, do_eig=eig,
                           do_precondition=True).upload()

    # ---- one iteration -----------------------------------------------------------------------
    def step(self, it: int, epoch: int):
        """K-factor work of iteration `it` (of epoch `epoch`) on the current stream; returns the
        list of preconditioned gradients S (one per layer)."""
        ea = it % self.sched.T_KU == 0
        inv = it % self.sched.T_KI(epoch) == 0 or self._ranks is None
        lam = float(self.sched.lam(epoch))
        if inv:
            ranks = self._desired_ranks(epoch)
            p, q = int(self.sched.oversampling(epoch)), int(self.sched.q)
            if self._gen != (tuple(ranks), p, q):
                self._lam = lam
                self._build(ranks, p, q)
            self._lam = lam
            self._upload_all(self.inversions)
        elif lam != self._lam:
            self._lam = lam
            self._upload_all(max(self.inversions - 1, 0))
        key = ("EI" if ea else "I") + "P" if inv else ("EP" if ea else "P")
        self._graphs[key].replay()
        if inv:
            self.inversions += 1
            self._ranks = list(self._gen[0])
            if self.adaptive is not None:
                self._adapt(epoch)
        return self.S

    def _adapt(self, epoch: int):
        Ds = [D[:r].cpu() for D, r in zip(self.D, self._ranks)]
        want = []
        for i, D in enumerate(Ds):
            s = self.specs[i // 2]
            want.append(self.adaptive.next_rank(D.tolist(), self._ranks[i], self.U[i].shape[1], self.F[i].shape[0],
                                                s.n, self.sched.rho))
        self._want = want
