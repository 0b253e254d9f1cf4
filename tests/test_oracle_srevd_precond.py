"""Pins for the oracle's randomized eigendecomposition (Alg. 3 SREVD, Alg. 2 RSVD with
the Sec. 2.2 power iterations) and the damped low-rank inverse (Sec. 4.1 identity,
Alg. 4/5), against exact recovery, Rayleigh-Ritz theory, the Halko-Martinsson-Tropp
average error bounds, Cholesky solves and a Kronecker-product brute force."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2206_15397_amd import synth


def factor(d, spec, seed):
    return synth.psd_factor(d, spec, seed)


def test_exact_recovery_low_rank():
    # rank(F) = k <= l: the sketch captures range(F) exactly and SREVD returns the exact
    # top eigenpairs (HMT, exact-rank case).
    d, k = 64, 10
    spec = np.concatenate([np.geomspace(2.0, 0.1, k), np.zeros(d - k)])
    F = factor(d, spec, 1)
    U, D = O.srevd(F, r=8, p=4, q=1, seed=3)
    np.testing.assert_allclose(D, spec[:8], atol=1e-12 * spec[0])
    U0 = synth.haar_orthogonal(d, 1, d)[:, :8]
    np.testing.assert_allclose(np.abs(U.T @ U0), np.eye(8), atol=1e-10)
    V, Dv = O.rsvd(F, r=8, p=4, q=1, seed=3)
    np.testing.assert_allclose(Dv, spec[:8], atol=1e-12 * spec[0])


def test_full_width_sketch_equals_full_eig():
    # l = min(r + p, d) = d: the randomized method reduces to the full eigendecomposition.
    d = 24
    F = factor(d, synth.power_spectrum(d), 2)
    U, D = O.srevd(F, r=20, p=8, q=0, seed=1)
    lam = np.sort(np.linalg.eigvalsh(F))[::-1]
    np.testing.assert_allclose(D, lam[:20], atol=1e-13)
    w, V = np.linalg.eigh(F)
    w, V = w[::-1], V[:, ::-1]
    np.testing.assert_allclose((U * D) @ U.T, (V[:, :20] * w[:20]) @ V[:, :20].T, atol=1e-12)


@pytest.mark.parametrize("q", [0, 1, 2])
def test_ritz_interlacing_residual_orthonormality(q):
    d = 120
    F = factor(d, synth.exp_spectrum(d, 10.0) + 0.01, 5)
    U, D, aux = O.srevd(F, r=12, p=6, q=q, seed=9, return_all=True)
    Q = aux["Q"]
    lam = np.sort(np.linalg.eigvalsh(F))[::-1]
    assert np.abs(Q.T @ Q - np.eye(18)).max() < 1e-13
    assert np.all(np.diff(D) <= 0)
    assert np.all(D <= lam[:12] + 1e-13)                    # Cauchy interlacing
    for i in range(12):
        res = F @ U[:, i] - D[i] * U[:, i]
        proj = F @ U[:, i] - Q @ (Q.T @ (F @ U[:, i]))
        assert abs(np.linalg.norm(res) - np.linalg.norm(proj)) < 1e-12
    # every column of U has its largest-magnitude entry positive (the sign convention)
    cols = np.arange(U.shape[1])
    assert np.all(U[np.argmax(np.abs(U), axis=0), cols] > 0)
    # RSVD singular values sit between SREVD Ritz values and the true eigenvalues.
    V, S = O.rsvd(F, r=12, p=6, q=q, seed=9)
    assert np.all(D <= S + 1e-12) and np.all(S <= lam[:12] + 1e-12)


def _sin_largest_angle(Q1, Q2):
    """sin of the largest principal angle between span(Q1) and span(Q2) (orthonormal)."""
    return np.linalg.norm(Q2 - Q1 @ (Q1.T @ Q2), 2)


@pytest.mark.parametrize("q", [0, 1, 2])
def test_range_finder_spans_power_of_factor_times_omega(q):
    # q power iterations (Sec. 2.2): span(Q) = span(F^{q+1} Omega).  F is well conditioned
    # (spectrum in [1, 3]) so F^{q+1} Omega has full rank in fp64; the spans of different
    # powers are far apart, so one multiply too many or too few fails the check.
    d, l = 40, 10
    F = factor(d, np.linspace(3.0, 1.0, d), 31)
    omega = O.gaussian_test_matrix(d, l, seed=5, stream_id=1)
    Q = O.range_finder(F, omega, q)
    assert Q.shape == (d, l) and np.abs(Q.T @ Q - np.eye(l)).max() < 1e-13
    for m in range(4):
        ref, _ = np.linalg.qr(np.linalg.matrix_power(F, m) @ omega)
        s = _sin_largest_angle(Q, ref)
        if m == q + 1:
            assert s <= 1e-10, (q, m, s)
        else:
            assert s > 1e-3, (q, m, s)


def test_power_iterations_reduce_projection_error_on_gapped_spectrum():
    # On a spectrum with a gap after k modes, each power iteration raises the decay of the
    # tail relative to the head, so the range error ||(I - QQ^T) F|| falls strictly.
    d, k, l = 120, 10, 12
    sig = np.concatenate([np.linspace(1.0, 0.5, k), np.linspace(0.1, 0.01, d - k)])
    F = factor(d, sig, 41)
    omega = O.gaussian_test_matrix(d, l, seed=3)
    err = []
    for q in range(3):
        Q = O.range_finder(F, omega, q)
        err.append(np.linalg.norm(F - Q @ (Q.T @ F), 2))
    assert err[1] < 0.5 * err[0] and err[2] < err[1], err
    assert err[2] >= sig[l] * (1 - 1e-12)       # never below the rank-l truncation floor


def test_kfactor_step_draws_omega_from_stream_2l_and_2l_plus_1():
    # One K-factor step over two layers equals the per-layer steps it is made of, with the
    # Omega stream of layer l's A factor 2l and of its G factor 2l+1 (and not swapped).
    rng = np.random.default_rng(17)
    rho, lam, r_cap, p, q, seed = 0.9, 0.1, 6, 3, 1, 11
    layers = []
    for li, (m, dg, n) in enumerate([(12, 9, 20), (10, 14, 25)]):
        layers.append({"A": np.eye(m + 1), "G": np.eye(dg), "a": rng.standard_normal((n, m)),
                       "g": rng.standard_normal((n, dg)), "bias": True,
                       "J": rng.standard_normal((dg, m + 1))})
    out = O.kfactor_step(layers, rho, lam, r_cap, p, q, seed)
    for li, (L, o) in enumerate(zip(layers, out)):
        n = L["a"].shape[0]
        A = O.ea_update(L["A"], L["a"], rho, 1.0 / n, append_ones=True)
        G = O.ea_update(L["G"], L["g"], rho, 1.0 / n)
        np.testing.assert_array_equal(o["A"], A)
        np.testing.assert_array_equal(o["G"], G)
        Ua, Da = O.srevd(A, r_cap, p, q, seed, 2 * li)
        Ug, Dg = O.srevd(G, r_cap, p, q, seed, 2 * li + 1)
        np.testing.assert_array_equal(o["U_a"], Ua)
        np.testing.assert_array_equal(o["D_a"], Da)
        np.testing.assert_array_equal(o["U_g"], Ug)
        np.testing.assert_array_equal(o["D_g"], Dg)
        np.testing.assert_array_equal(o["S"], O.precondition(L["J"], Ua, Da, Ug, Dg, lam))
        # the other stream gives a different draw, hence different Ritz values
        _, Da_other = O.srevd(A, r_cap, p, q, seed, 2 * li + 1)
        assert np.abs(Da_other - Da).max() > 1e-8


def _hmt_spectral_bound(sig, k, p, m):
    # E ||(I - QQ^T) F^m||_2 <= (1 + sqrt(k/(p-1))) s_{k+1}^m
    #                          + e sqrt(k+p)/p (sum_{j>k} s_j^{2m})^{1/2};
    # and ||(I-QQ^T)F||^m <= ||(I-QQ^T)F^m|| for PSD F, then Jensen.
    t = (1 + math.sqrt(k / (p - 1))) * sig[k] ** m + \
        math.e * math.sqrt(k + p) / p * math.sqrt(np.sum(sig[k:] ** (2 * m)))
    return t ** (1.0 / m)


@pytest.mark.parametrize("q", [0, 1])
def test_hmt_average_bounds(q):
    d, k, p = 80, 10, 5
    sig = synth.exp_spectrum(d, 6.0)
    F = factor(d, sig, 21)
    errs2, errsF = [], []
    for seed in range(60):
        omega = O.gaussian_test_matrix(d, k + p, seed)
        Q = O.range_finder(F, omega, q)
        E = F - Q @ (Q.T @ F)
        errs2.append(np.linalg.norm(E, 2))
        errsF.append(np.linalg.norm(E, "fro"))
    assert np.mean(errs2) <= 1.05 * _hmt_spectral_bound(sig, k, p, q + 1)
    if q == 0:
        # E ||(I - QQ^T) F||_F <= (1 + k/(p-1))^{1/2} (sum_{j>k} s_j^2)^{1/2}
        assert np.mean(errsF) <= 1.05 * math.sqrt(1 + k / (p - 1)) * math.sqrt(np.sum(sig[k:] ** 2))
    # the bound is not vacuous: truncation error is a floor
    assert min(errs2) >= sig[k + p] * (1 - 1e-12)   # rank-(k+p) truncation is a floor (Eckart-Young)


def test_rsvd_projection_error_not_worse_than_srevd():
    # RSVD keeps V~ (Sec. 2.2.2), whose projection error is smaller than SREVD's (Sec. 2.3).
    d, r, p = 100, 10, 3
    F = factor(d, synth.power_spectrum(d, 1.0), 4)
    lam, V0 = np.linalg.eigh(F)
    best = (V0[:, ::-1][:, :r] * lam[::-1][:r]) @ V0[:, ::-1][:, :r].T
    e_s, e_r = [], []
    for seed in range(30):
        U, D = O.srevd(F, r, p, 0, seed)
        V, S = O.rsvd(F, r, p, 0, seed)
        e_s.append(np.linalg.norm((U * D) @ U.T - best))
        e_r.append(np.linalg.norm((V * S) @ V.T - best))
    assert np.mean(e_r) < np.mean(e_s)


# ---------------------------------------------------------------------------------------
# Damped inverse application
# ---------------------------------------------------------------------------------------
def test_full_rank_identity_solves_damped_system():
    d, lam = 30, 0.1
    F = factor(d, synth.power_spectrum(d), 8)
    w_, V = np.linalg.eigh(F)
    rng = np.random.default_rng(0)
    v = rng.standard_normal((d, 3))
    f = O.damping_weights(w_, lam)
    w = V @ ((V.T @ v) * f[:, None]) + v / lam
    np.testing.assert_allclose((F + lam * np.eye(d)) @ w, v, atol=1e-12)


def test_precondition_full_rank_equals_cholesky_solve():
    dg, da, lam = 12, 17, 0.05
    A = factor(da, synth.power_spectrum(da), 1)
    G = factor(dg, synth.exp_spectrum(dg, 3.0), 2)
    J = np.random.default_rng(3).standard_normal((dg, da))
    Ua, Da = O.srevd(A, da, 0, 0, 0)
    Ug, Dg = O.srevd(G, dg, 0, 0, 0)
    S = O.precondition(J, Ua, Da, Ug, Dg, lam)
    S_star = O.exact_precondition(J, A, G, lam)
    assert np.linalg.norm(S - S_star) / np.linalg.norm(S_star) < 1e-12


def test_precondition_kronecker_brute_force():
    # (A (x) G)^{-1} vec(J) = vec(G^{-1} J A^{-1}) with column-major vec (Sec. 2.1), both
    # factors damped by lam; the Kronecker matrix is built explicitly with np.kron.
    dg, da, lam = 4, 6, 0.2
    A = factor(da, synth.power_spectrum(da), 11) + 0.0
    G = factor(dg, synth.power_spectrum(dg), 12)
    J = np.random.default_rng(5).standard_normal((dg, da))
    K = np.kron(A + lam * np.eye(da), G + lam * np.eye(dg))
    vecS = np.linalg.solve(K, J.reshape(-1, order="F"))
    S_kron = vecS.reshape((dg, da), order="F")
    Ua, Da = O.srevd(A, da, 0, 0, 0)
    Ug, Dg = O.srevd(G, dg, 0, 0, 0)
    S = O.precondition(J, Ua, Da, Ug, Dg, lam)
    np.testing.assert_allclose(S, S_kron, atol=1e-12 * np.abs(S_kron).max())
    np.testing.assert_allclose(O.exact_precondition(J, A, G, lam), S_kron, atol=1e-12 * np.abs(S_kron).max())


def test_precondition_diagonal_factors_closed_form():
    dg, da, lam = 5, 7, 0.3
    a = np.linspace(2.0, 0.1, da)
    g = np.linspace(1.5, 0.2, dg)
    J = np.random.default_rng(6).standard_normal((dg, da))
    Ua, Da = O.srevd(np.diag(a), da, 0, 0, 0)
    Ug, Dg = O.srevd(np.diag(g), dg, 0, 0, 0)
    S = O.precondition(J, Ua, Da, Ug, Dg, lam)
    want = J / ((g[:, None] + lam) * (a[None, :] + lam))
    np.testing.assert_allclose(S, want, rtol=1e-12)


def test_truncated_precondition_exact_on_exact_low_rank_factors():
    # If each factor has exactly r non-zero eigenvalues, the rank-r identity is exact.
    dg, da, r, lam = 20, 30, 5, 0.1
    sa = np.concatenate([np.geomspace(3, 0.5, r), np.zeros(da - r)])
    sg = np.concatenate([np.geomspace(2, 0.3, r), np.zeros(dg - r)])
    A, G = factor(da, sa, 1), factor(dg, sg, 2)
    J = np.random.default_rng(7).standard_normal((dg, da))
    Ua, Da = O.srevd(A, r, 4, 1, 1)
    Ug, Dg = O.srevd(G, r, 4, 1, 2)
    S = O.precondition(J, Ua, Da, Ug, Dg, lam)
    S_star = O.exact_precondition(J, A, G, lam)
    assert np.linalg.norm(S - S_star) / np.linalg.norm(S_star) < 1e-11
    # dropping the +J/lam term (a plausible slip) would break this
    bad = ((J @ Ua) * O.damping_weights(Da, lam)) @ Ua.T
    assert np.linalg.norm(bad - S_star) / np.linalg.norm(S_star) > 0.1


def test_jacobi_on_rayleigh_ritz_matrix_matches_lapack():
    d = 200
    F = factor(d, synth.power_spectrum(d), 13) * 0.4 + 0.6 * np.eye(d)
    U, D, aux = O.srevd(F, 32, 10, 1, 0, return_all=True)
    ref = np.sort(np.linalg.eigvalsh(aux["C"]))[::-1]
    np.testing.assert_allclose(aux["lam"], ref, atol=1e-13)


def test_sketch_operand_enters_only_the_range_finder():
    # F_sketch replaces F in the sketch and power-iteration products only: with F_sketch = F
    # the result is unchanged, and with a rank-k F_sketch whose range holds F's top-k
    # eigenvectors the range finder returns exactly that span while the Rayleigh-Ritz step
    # still projects F itself (Ritz values = F's top-k eigenvalues).
    d, k = 60, 8
    sig = np.concatenate([np.geomspace(4.0, 1.0, k), np.geomspace(0.5, 0.05, d - k)])
    F = factor(d, sig, 61)
    U1, D1 = O.srevd(F, 6, 4, 1, 3, 2)
    U2, D2 = O.srevd(F, 6, 4, 1, 3, 2, F_sketch=F.copy())
    np.testing.assert_array_equal(D1, D2)
    np.testing.assert_array_equal(U1, U2)
    Uf = synth.haar_orthogonal(d, 61, d)[:, :k]
    Fs = (Uf * np.linspace(2.0, 1.0, k)[None, :]) @ Uf.T
    U3, D3, aux = O.srevd(F, k - 2, 2, 1, 3, 2, F_sketch=Fs, return_all=True)
    np.testing.assert_allclose(D3, sig[:k - 2], rtol=1e-12)
    assert _sin_largest_angle(aux["Q"], Uf) < 1e-10
