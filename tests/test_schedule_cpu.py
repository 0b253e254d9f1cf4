"""Host logic of the K-FAC driver: the Sec. 5 schedules at their switching epochs, the
Proposition 3.1 bound against the paper's worked numbers (tests/golden/), and the adaptive
rank rule on synthetic spectra."""
import json
import os

import pytest

from paper_2206_15397_amd.schedule import AdaptiveRank, PaperSchedule, prop31_max_modes, prop31_r_eps

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_paper_schedule_switches():
    # Sec. 5: T_KU = 10, rho = 0.95, n_pwr-it = 4; T_KI 50 -> 30 at epoch 20; lambda 0.1 ->
    # 0.05 at 25 -> 0.01 at 35; r 220 -> 230 at 15; r_l 10 -> 11 at 22 -> 12 at 30; the step
    # size 0.3 decreasing at epochs 2, 3, 13, 18, 27, 40
    s = PaperSchedule()
    assert (s.T_KU, s.rho, s.q, s.batch) == (10, 0.95, 4, 256)
    assert [s.T_KI(n) for n in (0, 19, 20, 49)] == [50, 50, 30, 30]
    assert [round(s.lam(n), 12) for n in (0, 24, 25, 34, 35, 49)] == [0.1, 0.1, 0.05, 0.05, 0.01, 0.01]
    assert [s.rank(n) for n in (0, 14, 15, 49)] == [220, 220, 230, 230]
    assert [s.oversampling(n) for n in (0, 21, 22, 29, 30, 49)] == [10, 10, 11, 11, 12, 12]
    want = {0: 0.3, 1: 0.3, 2: 0.2, 3: 0.1, 12: 0.1, 13: 0.03, 17: 0.03, 18: 0.01, 26: 0.01, 27: 0.003,
            39: 0.003, 40: 0.001, 49: 0.001}
    for n, v in want.items():
        assert abs(s.lr(n) - v) < 1e-12, (n, s.lr(n), v)


def test_prop31_matches_worked_numbers():
    with open(os.path.join(GOLDEN, "prop31_worked_numbers.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        assert prop31_max_modes(c["rho"], c["alpha"], c["eps"], c["n_M"], 10 ** 9) == c["modes"]
        assert prop31_max_modes(c["rho"], c["alpha"], c["eps"], c["n_M"], 1000) == 1000
        assert prop31_r_eps(c["rho"], c["alpha"], c["eps"]) * c["n_M"] == c["modes"]
    with pytest.raises(ValueError):
        prop31_r_eps(1.0, 0.1, 0.03)


def test_adaptive_rank_rule():
    ar = AdaptiveRank(eps=1 / 33, alpha=0.1, margin=8, granule=16, r_min=16)
    # 40 modes above D_0/33 out of 128 kept: 40 + 8 -> 48
    D = [1.0 / (1 + i) ** 1.0 for i in range(128)]
    k = sum(1 for x in D if x >= D[0] / 33)
    assert k == 33
    assert ar.next_rank(D, 128, 256, 4096, 256, 0.95) == 48       # 33 + 8 = 41 -> 48
    # every kept value above the cut: the spectrum may continue, double (capped)
    flat = [1.0] * 64
    assert ar.next_rank(flat, 64, 256, 4096, 256, 0.95) == 128
    assert ar.next_rank([1.0] * 200, 200, 256, 4096, 256, 0.95) == 256
    assert ar.next_rank(flat, 64, 100, 4096, 256, 0.95) == 100     # schedule cap, not rounded past it
    # Proposition 3.1's bound with rho = 0.5, n_M = 1 (r_eps = 9 modes) caps the rank
    assert prop31_max_modes(0.5, 0.1, 1 / 33, 1, 4096) == 9
    assert ar.next_rank(flat, 64, 256, 4096, 1, 0.5) == 9
    # never below r_min (nor the factor size)
    assert ar.next_rank([1.0] + [1e-6] * 63, 64, 256, 4096, 256, 0.95) == 16
    assert ar.next_rank([1.0] * 4, 4, 256, 12, 256, 0.95) == 12    # 8 -> granule 16 -> d = 12
    assert ar.next_rank([], 4, 256, 12, 256, 0.95) == 12
