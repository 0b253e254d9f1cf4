"""Hyper-parameter schedules and rank rules of Randomized K-FAC (host-side arithmetic only).

* PaperSchedule: the schedules of the paper's VGG16_bn experiments (Sec. 5, implementation
  details) as functions of the current epoch n_ce: factor-update period T_KU = 10,
  inversion period T_KI(n) = 50 - 20 [n >= 20], damping lambda(n) = 0.1 - 0.05 [n >= 25]
  - 0.04 [n >= 35], step size alpha(n) = 0.3 - 0.1 [n >= 2] - 0.1 [n >= 3] - 0.07 [n >= 13]
  - 0.02 [n >= 18] - 0.007 [n >= 27] - 0.002 [n >= 40], target rank r(n) = 220 + 10
  [n >= 15], oversampling r_l(n) = 10 + [n >= 22] + [n >= 30], n_pwr-it = 4, rho = 0.95.
  Epochs are counted from 0.
* prop31_r_eps / prop31_max_modes: Proposition 3.1 (Sec. 3): an EA K-factor built from
  d_M x n_M batch matrices has at most min(r_eps n_M, d_M) eigenvalues above eps lambda_max,
  r_eps = ceil(log(alpha eps) / log(rho)).
* AdaptiveRank: per-factor target rank from the spectrum of the previous inversion (the
  per-layer adaptive rank the paper leaves to future work, Sec. 6): keep the Ritz values
  above eps lambda_max (eps = 1/33, the level below which the paper treats eigenvalues as
  zero at lambda ~ lambda_max / 10, Sec. 3), capped by the schedule's rank and by
  Proposition 3.1's bound.
"""
from __future__ import annotations

import math
from dataclasses import dataclass


def _ind(c: bool) -> int:
    return 1 if c else 0


@dataclass(frozen=True)
class PaperSchedule:
    """Sec. 5 schedules; `n` is the current epoch (0-based)."""
    rho: float = 0.95
    T_KU: int = 10
    q: int = 4
    batch: int = 256

    def T_KI(self, n: int) -> int:
        return 50 - 20 * _ind(n >= 20)

    def lam(self, n: int) -> float:
        return 0.1 - 0.05 * _ind(n >= 25) - 0.04 * _ind(n >= 35)

    def lr(self, n: int) -> float:
        return (0.3 - 0.1 * _ind(n >= 2) - 0.1 * _ind(n >= 3) - 0.07 * _ind(n >= 13) - 0.02 * _ind(n >= 18)
                - 0.007 * _ind(n >= 27) - 0.002 * _ind(n >= 40))

    def rank(self, n: int) -> int:
        return 220 + 10 * _ind(n >= 15)

    def oversampling(self, n: int) -> int:
        return 10 + _ind(n >= 22) + _ind(n >= 30)


def prop31_r_eps(rho: float, alpha: float, eps: float) -> int:
    """r_eps = ceil(log(alpha eps) / log(rho)) (Proposition 3.1)."""
    if not (0 < rho < 1 and 0 < alpha < 1 and 0 < eps < 1):
        raise ValueError("rho, alpha and eps must lie in (0, 1)")
    return int(math.ceil(math.log(alpha * eps) / math.log(rho)))


def prop31_max_modes(rho: float, alpha: float, eps: float, n_M: int, d_M: int) -> int:
    """At most min(r_eps n_M, d_M) eigenvalues of the EA factor exceed eps lambda_max."""
    return min(prop31_r_eps(rho, alpha, eps) * n_M, d_M)


@dataclass
class AdaptiveRank:
    """Target rank of one factor for its next inversion, from the Ritz values D (descending)
    its last inversion returned with rank r_prev:

        k   = #{i : D_i >= eps D_0}                     (modes above the cut)
        r   = 2 r_prev           if k == r_prev          (the spectrum may continue past r)
              k + margin         otherwise
        r  <- min(r, r_cap, Prop. 3.1 bound min(r_eps n_M, d), d), rounded up to `granule`
              (then clipped to the caps again), and at least r_min.

    alpha is Proposition 3.1's lambda_max / sigma_max^2 lower bound."""
    eps: float = 1.0 / 33.0
    alpha: float = 0.1
    margin: int = 8
    granule: int = 16
    r_min: int = 16

    def next_rank(self, D, r_prev: int, r_cap: int, d: int, n_M: int, rho: float) -> int:
        D = [float(x) for x in D]
        if not D or D[0] <= 0.0:
            return max(1, min(self.r_min, r_cap, d))
        k = sum(1 for x in D if x >= self.eps * D[0])
        r = 2 * r_prev if k >= r_prev else k + self.margin
        cap = min(r_cap, prop31_max_modes(rho, self.alpha, self.eps, n_M, d), d)
        r = min(r, cap)
        r = min(-(-r // self.granule) * self.granule, cap)
        return max(min(self.r_min, cap), r)
