"""FP64 reference implementation of the Randomized K-FAC K-factor pipeline.

TEST INFRASTRUCTURE ONLY (see the package docstring): slow, plain, float64.

Section / algorithm references are to Puiu, arXiv 2206.15397:
  Alg. 1   K-FAC (EA K-factor updates, eig, inverse application)
  Alg. 2   randomized SVD (RSVD)
  Alg. 3   symmetric randomized EVD (SREVD)
  Alg. 4/5 RS-KFAC / SRE-KFAC per-layer loops
  Sec. 2.2 power iterations ("n_pwr-it")
  Sec. 2.2.2 use of the V factor of RSVD for symmetric PSD matrices
  Sec. 3   matrix form of the EA and Proposition 3.1
  Sec. 4.1 identity (U D U^T + lam I)^{-1} V = U[(D + lam I)^{-1} - I/lam]U^T V + V/lam
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading

import numpy as np

__all__ = [
    "philox4x32_10", "uniforms_from_words", "gaussian_test_matrix", "ea_update",
    "philox_words_for", "philox_words_at", "householder_qr", "thin_qr", "jacobi_eig", "jacobi_svd", "sign_normalize", "range_finder",
    "srevd", "rsvd", "damping_weights", "precondition", "exact_precondition",
    "prop31_r_eps", "prop31_max_modes", "full_eig", "kfactor_step", "oracle_library_path",
    "linear_forward", "linear_backward",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "jacobi.c")
_SO = os.path.join(_HERE, "libkfac_oracle_jacobi.so")
_lock = threading.Lock()
_lib_handle = None


def oracle_library_path() -> str:
    return _SO


def build_oracle_library(force: bool = False) -> str:
    """Compile jacobi.c with gcc (plain IEEE double, no fast-math)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _lib():
    global _lib_handle
    with _lock:
        if _lib_handle is None:
            build_oracle_library()
            lib = ctypes.CDLL(_SO)
            dp = ctypes.POINTER(ctypes.c_double)
            lib.oracle_jacobi_eig.argtypes = [dp, dp, ctypes.c_int, ctypes.c_double]
            lib.oracle_jacobi_eig.restype = ctypes.c_int
            lib.oracle_jacobi_svd.argtypes = [dp, dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_double]
            lib.oracle_jacobi_svd.restype = ctypes.c_int
            _lib_handle = lib
    return _lib_handle


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ----------------------------------------------------------------------------------------
# Gaussian test matrix Omega (Alg. 2 / Alg. 3, "Sample Gaussian matrix").
# The paper does not name a sampler.  Omega is drawn from a counter-based generator,
# Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), so that any party can reproduce the
# same draw from (seed, stream, inversion index) without shared state.
# ----------------------------------------------------------------------------------------
_PHILOX_M0 = 0xD2511F53
_PHILOX_M1 = 0xCD9E8D57
_PHILOX_W0 = 0x9E3779B9
_PHILOX_W1 = 0xBB67AE85
_MASK32 = 0xFFFFFFFF


def philox4x32_10(ctr: np.ndarray, key) -> np.ndarray:
    """Philox4x32 with 10 rounds.  ctr: (..., 4) uint32; key: (k0, k1).

    One round maps (c0, c1, c2, c3) to (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2),
    hi(M0*c0) ^ c3 ^ k1, lo(M0*c0)); between rounds the key is bumped by the Weyl
    constants (W0, W1).  Pinned to the generator's published known-answer vectors."""
    c = np.array(ctr, dtype=np.uint64) & _MASK32
    k0 = np.uint64(int(key[0]) & _MASK32)
    k1 = np.uint64(int(key[1]) & _MASK32)
    c0, c1, c2, c3 = c[..., 0], c[..., 1], c[..., 2], c[..., 3]
    for rnd in range(10):
        p0 = np.uint64(_PHILOX_M0) * c0
        p1 = np.uint64(_PHILOX_M1) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(_MASK32)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(_MASK32)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        if rnd < 9:
            k0 = (k0 + np.uint64(_PHILOX_W0)) & np.uint64(_MASK32)
            k1 = (k1 + np.uint64(_PHILOX_W1)) & np.uint64(_MASK32)
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def uniforms_from_words(w: np.ndarray) -> np.ndarray:
    """23-bit uniforms in (0, 1): ((w >> 9) + 1/2) * 2^-23 (24 significant bits, so the
    value is exact in fp32 as well as fp64)."""
    return ((w.astype(np.uint64) >> np.uint64(9)).astype(np.float64) + 0.5) * 2.0 ** -23


def philox_words_at(rows, groups, seed: int, stream_id: int, inversion_index: int) -> np.ndarray:
    """Raw 32-bit words of Omega's draw for the given row indices and column groups
    (a group is four consecutive columns): (len(rows), len(groups), 4).  The counter of
    (row i, group g) is (i, g, stream_id mod 2^32, inversion_index) and the key is
    (seed mod 2^32, seed >> 32)."""
    i = np.asarray(rows, dtype=np.uint64).reshape(-1)[:, None]
    g = np.asarray(groups, dtype=np.uint64).reshape(-1)[None, :]
    ctr = np.zeros((i.shape[0], g.shape[1], 4), dtype=np.uint64)
    ctr[..., 0] = i
    ctr[..., 1] = g
    ctr[..., 2] = np.uint64(int(stream_id) & _MASK32)
    ctr[..., 3] = np.uint64(int(inversion_index) & _MASK32)
    key = (int(seed) & _MASK32, (int(seed) >> 32) & _MASK32)
    return philox4x32_10(ctr, key)


def philox_words_for(d: int, l: int, seed: int, stream_id: int, inversion_index: int) -> np.ndarray:
    """Raw 32-bit words for rows 0..d-1 and column groups 0..ceil(l/4)-1: (d, G, 4)."""
    return philox_words_at(np.arange(d), np.arange((l + 3) // 4), seed, stream_id, inversion_index)


def gaussian_test_matrix(d: int, l: int, seed: int, stream_id: int = 0,
                         inversion_index: int = 0) -> np.ndarray:
    """Omega in R^{d x l}, i.i.d. N(0,1) (Alg. 3 "Sample Gaussian Matrix").

    Element (i, j) uses Philox counter (i, j // 4, stream_id, inversion_index) and key
    (seed mod 2^32, seed >> 32); the four words give two Box-Muller pairs
    (z0, z1) = sqrt(-2 ln u0) (cos 2 pi u1, sin 2 pi u1), (z2, z3) likewise, and
    Omega_ij = z_{j mod 4}."""
    w = philox_words_for(d, l, seed, stream_id, inversion_index)
    u = uniforms_from_words(w)
    r01 = np.sqrt(-2.0 * np.log(u[..., 0]))
    r23 = np.sqrt(-2.0 * np.log(u[..., 2]))
    z = np.empty(u.shape, dtype=np.float64)
    z[..., 0] = r01 * np.cos(2.0 * np.pi * u[..., 1])
    z[..., 1] = r01 * np.sin(2.0 * np.pi * u[..., 1])
    z[..., 2] = r23 * np.cos(2.0 * np.pi * u[..., 3])
    z[..., 3] = r23 * np.sin(2.0 * np.pi * u[..., 3])
    return z.reshape(d, -1)[:, :l].copy()


# ----------------------------------------------------------------------------------------
# EA K-factor update (Alg. 1 forward/backward EA lines; matrix form in Sec. 3).
# ----------------------------------------------------------------------------------------
def ea_update(F: np.ndarray, X: np.ndarray, rho: float, scale: float,
              append_ones: bool = False) -> np.ndarray:
    """F <- rho F + (1 - rho) * scale * Xh^T Xh, Xh = [X | 1] when the layer has a bias.

    X holds one sample per row (n x d_in); the outer-product sum over samples is the
    K-factor A A^T of Alg. 1 with A = Xh^T.  F is returned as a new float64 array, with
    the lower triangle copied from the upper so it is exactly symmetric."""
    X = np.asarray(X, dtype=np.float64)
    if append_ones:
        X = np.concatenate([X, np.ones((X.shape[0], 1))], axis=1)
    d = X.shape[1]
    F = np.asarray(F, dtype=np.float64)
    assert F.shape == (d, d), (F.shape, d)
    G = X.T @ X
    out = rho * F + (1.0 - rho) * scale * G
    iu = np.triu_indices(d, 1)
    out[(iu[1], iu[0])] = out[iu]
    return out


# ----------------------------------------------------------------------------------------
# Thin QR (the paper's "QR_decomp", always thin, Sec. 2.2) by Householder reflections.
# ----------------------------------------------------------------------------------------
def householder_qr(Y: np.ndarray):
    """Thin QR, Y = Q R with Q (m x k) orthonormal and R upper triangular, diag(R) >= 0."""
    A = np.array(Y, dtype=np.float64, copy=True)
    m, k = A.shape
    vs = []
    for j in range(k):
        x = A[j:, j].copy()
        alpha = np.linalg.norm(x)
        v = x
        if alpha == 0.0:
            vs.append(None)
            continue
        v[0] += math.copysign(alpha, x[0]) if x[0] != 0 else alpha
        v /= np.linalg.norm(v)
        A[j:, j:] -= 2.0 * np.outer(v, v @ A[j:, j:])
        vs.append(v)
    R = np.triu(A[:k, :])
    Q = np.zeros((m, k))
    Q[:k, :k] = np.eye(k)
    for j in range(k - 1, -1, -1):
        v = vs[j]
        if v is None:
            continue
        Q[j:, :] -= 2.0 * np.outer(v, v @ Q[j:, :])
    sgn = np.where(np.diag(R) < 0, -1.0, 1.0)
    return Q * sgn[None, :], R * sgn[:, None]


def thin_qr(Y: np.ndarray):
    """The same thin QR as householder_qr (diag(R) >= 0), computed by LAPACK's blocked
    Householder routines: the range finder's QR at full sizes, where the reflector loop
    above would dominate the oracle's run time.  Any thin QR serves the range finder, whose
    downstream results depend only on span(Q) (Sec. 2.2 leaves the QR method open)."""
    Q, R = np.linalg.qr(np.asarray(Y, dtype=np.float64), mode="reduced")
    sgn = np.where(np.diag(R) < 0, -1.0, 1.0)
    return Q * sgn[None, :], R * sgn[:, None]


# ----------------------------------------------------------------------------------------
# Dense symmetric eigendecomposition (Alg. 1 "eig", Alg. 3 "Eigen_decomp") and thin SVD
# (Alg. 2) by Jacobi rotations in plain C.
# ----------------------------------------------------------------------------------------
def jacobi_eig(A: np.ndarray, tol: float = 1e-15):
    """Eigenpairs of a symmetric matrix, eigenvalues sorted descending."""
    M = np.ascontiguousarray(A, dtype=np.float64).copy()
    n = M.shape[0]
    V = np.zeros((n, n))
    sweeps = _lib().oracle_jacobi_eig(_dptr(M), _dptr(V), n, tol)
    if sweeps < 0:
        raise RuntimeError("Jacobi eigensolver did not converge")
    lam = np.diag(M).copy()
    order = np.argsort(-lam, kind="stable")
    return lam[order], V[:, order]


def jacobi_svd(W: np.ndarray, tol: float = 1e-15):
    """Thin SVD of a tall matrix W = U diag(s) Vr^T, singular values descending."""
    M = np.ascontiguousarray(W, dtype=np.float64).copy()
    m, n = M.shape
    assert m >= n
    s = np.zeros(n)
    Vr = np.zeros((n, n))
    sweeps = _lib().oracle_jacobi_svd(_dptr(M), _dptr(s), _dptr(Vr), m, n, tol)
    if sweeps < 0:
        raise RuntimeError("one-sided Jacobi SVD did not converge")
    order = np.argsort(-s, kind="stable")
    s = s[order]
    M = M[:, order]
    Vr = Vr[:, order]
    U = np.zeros_like(M)
    nz = s > 0
    U[:, nz] = M[:, nz] / s[nz][None, :]
    return U, s, Vr


def full_eig(F: np.ndarray):
    """Full eigendecomposition of a K-factor (Alg. 1 "eig"), descending."""
    return jacobi_eig(F)


def sign_normalize(U: np.ndarray) -> np.ndarray:
    """Make the largest-magnitude entry of every column positive (ties: lowest row)."""
    U = np.array(U, dtype=np.float64, copy=True)
    if U.size == 0:
        return U
    idx = np.argmax(np.abs(U), axis=0)
    sgn = np.sign(U[idx, np.arange(U.shape[1])])
    sgn[sgn == 0] = 1.0
    return U * sgn[None, :]


# ----------------------------------------------------------------------------------------
# Randomized range finder (Alg. 2/3 sample-multiply-QR steps) with q power iterations
# (Sec. 2.2).  One power iteration is one more multiply by F followed by a fresh thin QR,
# so span(Q) = span(F^{q+1} Omega).
# ----------------------------------------------------------------------------------------
def range_finder(F: np.ndarray, omega: np.ndarray, q: int, F_sketch: np.ndarray = None) -> np.ndarray:
    """Q with span(Q) = span(F^{q+1} Omega).  F_sketch, when given, is the matrix the
    sketch and power-iteration products multiply by (the bf16 copy of F on a path whose
    sketch runs in bf16); the method is otherwise unchanged."""
    Fs = F if F_sketch is None else np.asarray(F_sketch, dtype=np.float64)
    Q, _ = thin_qr(Fs @ omega)
    for _ in range(q):
        Q, _ = thin_qr(Fs @ Q)
    return Q


def _sketch_width(d: int, r: int, p: int) -> int:
    return min(r + p, d)


def srevd(F: np.ndarray, r: int, p: int, q: int, seed: int, stream_id: int = 0,
          inversion_index: int = 0, return_all: bool = False, F_sketch: np.ndarray = None):
    """Symmetric randomized EVD, Alg. 3: top-r eigenpairs (U d x r, D r) of PSD F.

    Steps: Omega (d x l, l = min(r+p, d)); Y = F Omega; Q = thin-QR(Y); q power
    iterations; C = Q^T F Q (symmetrised); C = P diag(D_C) P^T sorted descending;
    U = Q P[:, :r], D = D_C[:r]; columns of U sign-normalised.  When l = d the sketch
    spans everything and Q = I (the randomized result equals the full eig).  F_sketch: see
    range_finder (the Rayleigh-Ritz product W = F Q always takes F)."""
    F = np.asarray(F, dtype=np.float64)
    d = F.shape[0]
    l = _sketch_width(d, r, p)
    if l == d:
        Q = np.eye(d)
    else:
        omega = gaussian_test_matrix(d, l, seed, stream_id, inversion_index)
        Q = range_finder(F, omega, q, F_sketch)
    W = F @ Q
    C = Q.T @ W
    C = 0.5 * (C + C.T)
    lam, P = jacobi_eig(C)
    U = sign_normalize(Q @ P[:, :r])
    D = lam[:r].copy()
    if return_all:
        return U, D, {"Q": Q, "C": C, "lam": lam, "P": P}
    return U, D


def rsvd(F: np.ndarray, r: int, p: int, q: int, seed: int, stream_id: int = 0,
         inversion_index: int = 0, return_all: bool = False, F_sketch: np.ndarray = None):
    """Randomized SVD of a symmetric PSD factor, Alg. 2, returning (V~, Sigma~).

    B = Q^T F (l x d); the SVD of B^T = F Q (d x l) gives B = U_B Sigma_B V_B^T; the
    returned factor is V~ = V_B[:, :r] (the more accurate one for symmetric PSD
    matrices, Sec. 2.2.2) with D = Sigma_B[:r].  F_sketch: see range_finder."""
    F = np.asarray(F, dtype=np.float64)
    d = F.shape[0]
    l = _sketch_width(d, r, p)
    if l == d:
        Q = np.eye(d)
    else:
        omega = gaussian_test_matrix(d, l, seed, stream_id, inversion_index)
        Q = range_finder(F, omega, q, F_sketch)
    Bt = F @ Q
    Vb, s, Ub = jacobi_svd(Bt)
    V = sign_normalize(Vb[:, :r])
    D = s[:r].copy()
    if return_all:
        return V, D, {"Q": Q, "sigma": s, "U_B": Ub}
    return V, D


# ----------------------------------------------------------------------------------------
# Damped low-rank inverse application (Sec. 4.1 identity; Alg. 4 M and S lines).
# ----------------------------------------------------------------------------------------
def damping_weights(D: np.ndarray, lam: float) -> np.ndarray:
    """f_i = 1/(D_i + lam) - 1/lam: the diagonal [(D + lam I)^{-1} - I/lam]."""
    D = np.asarray(D, dtype=np.float64)
    return 1.0 / (D + lam) - 1.0 / lam


def precondition(J: np.ndarray, U_a: np.ndarray, D_a: np.ndarray, U_g: np.ndarray,
                 D_g: np.ndarray, lam: float) -> np.ndarray:
    """S = (U_g D_g U_g^T + lam I)^{-1} J (U_a D_a U_a^T + lam I)^{-1} via the identity:
    M = J U_a diag(f_a) U_a^T + J/lam;  S = U_g diag(f_g) U_g^T M + M/lam.
    J = Mat(g) is d_g x d_a (rows: output/backward side, columns: input/forward side)."""
    J = np.asarray(J, dtype=np.float64)
    U_a = np.asarray(U_a, dtype=np.float64)
    U_g = np.asarray(U_g, dtype=np.float64)
    f_a = damping_weights(D_a, lam)
    f_g = damping_weights(D_g, lam)
    M = ((J @ U_a) * f_a[None, :]) @ U_a.T + J / lam
    S = U_g @ ((U_g.T @ M) * f_g[:, None]) + M / lam
    return S


def exact_precondition(J: np.ndarray, A: np.ndarray, G: np.ndarray, lam: float) -> np.ndarray:
    """S* = (G + lam I)^{-1} J (A + lam I)^{-1} by Cholesky solves (Kronecker inverse
    identity of Sec. 2.1 with both factors damped as in Alg. 1)."""
    from scipy.linalg import cho_factor, cho_solve
    J = np.asarray(J, dtype=np.float64)
    Ga = cho_factor(np.asarray(G, dtype=np.float64) + lam * np.eye(G.shape[0]))
    Aa = cho_factor(np.asarray(A, dtype=np.float64) + lam * np.eye(A.shape[0]))
    left = cho_solve(Ga, J)                 # (G + lam I)^{-1} J
    return cho_solve(Aa, left.T).T          # ... (A + lam I)^{-1}  (A symmetric)


# ----------------------------------------------------------------------------------------
# Proposition 3.1 (Sec. 3).
# ----------------------------------------------------------------------------------------
def prop31_r_eps(rho: float, alpha: float, eps: float) -> int:
    """r_eps = ceil(log(alpha * eps) / log(rho))."""
    return int(math.ceil(math.log(alpha * eps) / math.log(rho)))


def prop31_max_modes(rho: float, alpha: float, eps: float, n_M: int, d_M: int) -> int:
    """At most min(r_eps * n_M, d_M) eigenvalues exceed eps * lambda_max."""
    return min(prop31_r_eps(rho, alpha, eps) * n_M, d_M)


# ----------------------------------------------------------------------------------------
# One K-factor step over a set of layers (Alg. 1 EA lines, then Alg. 5 per layer).
# ----------------------------------------------------------------------------------------
def kfactor_step(layers, rho: float, lam: float, r_cap: int, p: int, q: int, seed: int,
                 inversion_index: int = 0):
    """layers: list of dicts with keys A (d_a x d_a), G (d_g x d_g), a (n x d_a_in),
    g (n x d_g), bias (bool), J (d_g x d_a).  Factor stream ids are 2l (A side) and
    2l+1 (G side).  Returns a list of dicts (A, G, U_a, D_a, U_g, D_g, S)."""
    out = []
    for li, L in enumerate(layers):
        n = L["a"].shape[0]
        A = ea_update(L["A"], L["a"], rho, 1.0 / n, append_ones=L["bias"])
        G = ea_update(L["G"], L["g"], rho, 1.0 / L["g"].shape[0], append_ones=False)
        ra, rg = min(r_cap, A.shape[0]), min(r_cap, G.shape[0])
        U_a, D_a = srevd(A, ra, p, q, seed, 2 * li, inversion_index)
        U_g, D_g = srevd(G, rg, p, q, seed, 2 * li + 1, inversion_index)
        S = precondition(L["J"], U_a, D_a, U_g, D_g, lam)
        out.append({"A": A, "G": G, "U_a": U_a, "D_a": D_a, "U_g": U_g, "D_g": D_g, "S": S})
    return out


def linear_forward(x: np.ndarray, W: np.ndarray, b: np.ndarray = None) -> np.ndarray:
    """Forward pass of a fully-connected layer over a batch (rows are samples): s = a W^T + b
    (Alg. 1 forward pass, whose inputs a feed the forward factor)."""
    y = x @ W.T
    if b is not None:
        y = y + b[None, :]
    return y


def linear_backward(x: np.ndarray, W: np.ndarray, g: np.ndarray):
    """Backward pass of s = a W^T + b for a batch, given g = dL/ds (rows are samples):
    dL/da = g W, dL/dW = g^T a, dL/db = sum over rows of g (Alg. 1 backward pass: Mat(g) of
    the layer and the back-propagated gradients that feed the backward factor)."""
    return g @ W, g.T @ x, g.sum(axis=0)
