"""Pins for the oracle's dense building blocks: thin Householder QR (the paper's thin
"QR_decomp"), the cyclic Jacobi eigensolver (Alg. 1 "eig", Alg. 3 "Eigen_decomp") and the
one-sided Jacobi SVD (Alg. 2), against closed forms and LAPACK."""
import math

import numpy as np
import pytest

import oracle as O


@pytest.mark.parametrize("m,k", [(40, 7), (9, 9), (300, 42)])
def test_householder_qr_definition_and_lapack(m, k):
    rng = np.random.default_rng(m * 100 + k)
    Y = rng.standard_normal((m, k))
    Q, R = O.householder_qr(Y)
    assert np.abs(Q @ R - Y).max() < 1e-13 * np.abs(Y).max() * k
    assert np.abs(Q.T @ Q - np.eye(k)).max() < 1e-14 * k
    assert np.all(np.tril(R, -1) == 0) and np.all(np.diag(R) > 0)
    Ql, Rl = np.linalg.qr(Y)
    s = np.sign(np.diag(Rl))
    np.testing.assert_allclose(Q, Ql * s, atol=1e-12)


@pytest.mark.parametrize("m,k", [(40, 7), (9, 9), (300, 42)])
def test_thin_qr_equals_householder_qr(m, k):
    # the range finder's library-backed thin QR is the same factorisation as the reflector
    # loop above (positive diagonal of R makes the thin QR of a full-rank Y unique)
    rng = np.random.default_rng(m * 7 + k)
    Y = rng.standard_normal((m, k))
    Q, R = O.thin_qr(Y)
    Qh, Rh = O.householder_qr(Y)
    np.testing.assert_allclose(Q, Qh, atol=1e-12)
    np.testing.assert_allclose(R, Rh, atol=1e-12 * np.abs(Rh).max())


def test_jacobi_tridiagonal_toeplitz_closed_form():
    # tridiag(b, a, b) of size n has eigenvalues a + 2 b cos(k pi / (n + 1)), k = 1..n,
    # with eigenvectors sin(i k pi / (n+1)).
    n, a, b = 37, 2.5, -0.75
    T = np.diag(np.full(n, a)) + np.diag(np.full(n - 1, b), 1) + np.diag(np.full(n - 1, b), -1)
    lam, V = O.jacobi_eig(T)
    want = np.sort(a + 2 * b * np.cos(np.arange(1, n + 1) * np.pi / (n + 1)))[::-1]
    np.testing.assert_allclose(lam, want, atol=1e-13)
    # eigenvector of the largest eigenvalue (b < 0 -> k = n)
    k = n
    v = np.sin(np.arange(1, n + 1) * k * np.pi / (n + 1))
    v /= np.linalg.norm(v)
    assert abs(abs(v @ V[:, 0]) - 1) < 1e-12


@pytest.mark.parametrize("n", [2, 8, 64, 150])
def test_jacobi_vs_lapack_and_orthogonality(n):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n)); A = A + A.T
    lam, V = O.jacobi_eig(A)
    ref = np.sort(np.linalg.eigvalsh(A))[::-1]
    scale = np.abs(ref).max()
    np.testing.assert_allclose(lam, ref, atol=1e-12 * scale)
    assert np.abs(V.T @ V - np.eye(n)).max() < 1e-13 * max(1, n / 10)
    assert np.abs(V @ np.diag(lam) @ V.T - A).max() < 1e-12 * scale


def test_jacobi_repeated_eigenvalues():
    rng = np.random.default_rng(2)
    U = np.linalg.qr(rng.standard_normal((20, 20)))[0]
    sig = np.array([3.0] * 5 + [1.0] * 10 + [0.0] * 5)
    A = (U * sig) @ U.T
    lam, V = O.jacobi_eig(A)
    np.testing.assert_allclose(lam, sig, atol=1e-13)
    # projector onto the eigenvalue-3 cluster is basis independent
    P = V[:, :5] @ V[:, :5].T
    np.testing.assert_allclose(P, U[:, :5] @ U[:, :5].T, atol=1e-12)


@pytest.mark.parametrize("m,n", [(50, 6), (300, 30), (12, 12)])
def test_jacobi_svd_closed_form(m, n):
    rng = np.random.default_rng(m + n)
    Ul = np.linalg.qr(rng.standard_normal((m, n)))[0]
    Vr = np.linalg.qr(rng.standard_normal((n, n)))[0]
    s = np.geomspace(5.0, 1e-3, n)
    W = (Ul * s) @ Vr.T
    U, sv, V = O.jacobi_svd(W)
    np.testing.assert_allclose(sv, s, rtol=1e-12)
    assert np.abs(U @ np.diag(sv) @ V.T - W).max() < 1e-13 * 5
    assert np.abs(V.T @ V - np.eye(n)).max() < 1e-13
    np.testing.assert_allclose(sv, np.linalg.svd(W, compute_uv=False), rtol=1e-12)


def test_sign_normalize_convention():
    U = np.array([[0.1, -0.5, 0.3], [-0.9, 0.5, -0.3], [0.2, 0.0, 0.1]])
    N = O.sign_normalize(U)
    np.testing.assert_array_equal(N[:, 0], -U[:, 0])   # largest |.| is -0.9
    np.testing.assert_array_equal(N[:, 1], -U[:, 1])   # tie -0.5 vs 0.5: lowest row
    np.testing.assert_array_equal(N[:, 2], U[:, 2])
