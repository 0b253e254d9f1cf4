"""Pins for the oracle's EA K-factor update (Alg. 1 EA lines, Sec. 3 matrix form) and
Proposition 3.1 (Sec. 3), checked against closed forms, brute force and the paper's own
worked numbers."""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2206_15397_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def brute_force_ea(F, X, rho, s, ones):
    """Scalar triple loop of F_ij <- rho F_ij + (1-rho) s sum_k xh_ki xh_kj."""
    n, m = len(X), len(X[0])
    d = m + (1 if ones else 0)
    xh = [list(row) + ([1.0] if ones else []) for row in X]
    out = [[0.0] * d for _ in range(d)]
    for i in range(d):
        for j in range(d):
            acc = 0.0
            for k in range(n):
                acc += xh[k][i] * xh[k][j]
            out[i][j] = rho * F[i][j] + (1.0 - rho) * s * acc
    return np.array(out)


@pytest.mark.parametrize("ones", [False, True])
def test_ea_brute_force_tiny(ones):
    X = [[0.5, -1.25], [2.0, 0.75], [-0.5, 3.0]]        # 3 samples x 2 features
    d = 2 + (1 if ones else 0)
    F0 = np.eye(d) * 0.3 + 0.1
    got = O.ea_update(F0, np.array(X), 0.9, 1.0 / 3.0, append_ones=ones)
    want = brute_force_ea(F0.tolist(), X, 0.9, 1.0 / 3.0, ones)
    np.testing.assert_allclose(got, want, rtol=1e-14, atol=1e-15)


def test_ea_geometric_closed_form():
    # k+1 steps with the same batch from F = I give rho^{k+1} I + (1 - rho^{k+1}) s Xh^T Xh.
    rng = np.random.default_rng(3)
    X = rng.standard_normal((7, 5))
    rho, s, steps = 0.95, 1.0 / 7, 12
    F = np.eye(6)
    for _ in range(steps):
        F = O.ea_update(F, X, rho, s, append_ones=True)
    Xh = np.concatenate([X, np.ones((7, 1))], axis=1)
    want = rho ** steps * np.eye(6) + (1 - rho ** steps) * s * (Xh.T @ Xh)
    assert np.linalg.norm(F - want) / np.linalg.norm(want) < 1e-14


def test_ea_symmetry_psd_and_rank_one():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((9, 11))
    F = O.ea_update(np.eye(11), X, 0.95, 1 / 9)
    assert np.array_equal(F, F.T)                              # exact symmetry
    lam, _ = O.jacobi_eig(F)
    assert lam[-1] >= -1e-14 * lam[0]                          # PSD
    # rank-one sample x = e_3 touches only entry (3, 3) by (1-rho)*s.
    e = np.zeros((1, 11)); e[0, 3] = 1.0
    G = O.ea_update(F, e, 0.8, 0.5)
    D = G - 0.8 * F
    expect = np.zeros((11, 11)); expect[3, 3] = 0.2 * 0.5
    np.testing.assert_allclose(D, expect, atol=1e-15)


def test_prop31_worked_numbers():
    with open(os.path.join(GOLDEN, "prop31_worked_numbers.json")) as f:
        g = json.load(f)
    for c in g["cases"]:
        r_eps = O.prop31_r_eps(c["rho"], c["alpha"], c["eps"])
        assert r_eps * c["n_M"] == c["modes"]
        assert O.prop31_max_modes(c["rho"], c["alpha"], c["eps"], c["n_M"], 10 ** 6) == c["modes"]
        assert O.prop31_max_modes(c["rho"], c["alpha"], c["eps"], c["n_M"], 100) == 100


@pytest.mark.parametrize("rho,n_M,d_M", [(0.5, 2, 40), (0.7, 3, 60), (0.5, 1, 30)])
def test_prop31_bound_holds_on_zero_init_ea(rho, n_M, d_M):
    # Matrix form of the EA (zero initialisation), random batches M_i (d_M x n_M).  With
    # sigma_M = max_i ||M_i||_2 and alpha = lambda_M / sigma_M^2, at most
    # min(r_eps n_M, d_M) eigenvalues exceed eps * lambda_M.
    rng = np.random.default_rng(11)
    Ms = [rng.standard_normal((d_M, n_M)) * (1.0 + 0.5 * rng.random()) for _ in range(80)]
    F = np.zeros((d_M, d_M))
    for M in Ms:
        F = O.ea_update(F, M.T, rho, 1.0)
    lam, _ = O.jacobi_eig(F)
    sigma_M = max(np.linalg.norm(M, 2) for M in Ms)
    alpha = lam[0] / sigma_M ** 2
    assert 0 < alpha < 1
    for eps in [0.3, 0.1, 0.03, 0.01]:
        count = int(np.sum(lam >= eps * lam[0]))
        assert count <= O.prop31_max_modes(rho, alpha, eps, n_M, d_M)


def test_activation_recipe_covariance():
    # The synthetic activation recipe has covariance R diag(sigma) R^T.
    m = 6
    R = synth.haar_orthogonal(m, 5)
    sig = synth.power_spectrum(m)
    a = synth.activation_batch(200000, R, sig, 7)
    cov = a.T @ a / a.shape[0]
    want = (R * sig) @ R.T
    assert np.abs(cov - want).max() < 0.02
