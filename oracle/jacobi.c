/*
 * FP64 reference eigensolvers for the K-factor oracle.  TEST INFRASTRUCTURE ONLY:
 * nothing in the GPU product path may link or call this file.
 *
 *  - oracle_jacobi_eig: cyclic-by-row two-sided Jacobi for a dense symmetric matrix
 *    (Golub & Van Loan, "Matrix Computations", cyclic Jacobi, sec. 8.5).  It plays the
 *    role of the full eigendecomposition eig(.) of Algorithm 1 and of
 *    Eigen_decomp(C) in Algorithm 3 (SREVD).
 *  - oracle_jacobi_svd: one-sided (Hestenes) Jacobi for the thin SVD of a tall matrix,
 *    used for the SVD of B^T in Algorithm 2 (RSVD).
 *
 * Plain C99, no BLAS, row-major storage, everything in double.
 */
#include <math.h>
#include <string.h>

/* Symmetric Schur decomposition of the 2x2 block (p,q): the rotation J = [c s; -s c]
 * (rows/cols p,q) such that (J^T A J)_pq = 0.  tau = (a_qq - a_pp)/(2 a_pq); t is the
 * root of t^2 + 2 tau t - 1 = 0 of smaller magnitude. */
static void sym_schur2(double app, double aqq, double apq, double* c, double* s) {
  if (apq == 0.0) { *c = 1.0; *s = 0.0; return; }
  double tau = (aqq - app) / (2.0 * apq);
  double t;
  if (tau >= 0.0) t = 1.0 / (tau + sqrt(1.0 + tau * tau));
  else            t = -1.0 / (-tau + sqrt(1.0 + tau * tau));
  *c = 1.0 / sqrt(1.0 + t * t);
  *s = t * (*c);
}

static double off_norm2(const double* A, int n) {
  double s = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      if (i != j) s += A[(long)i * n + j] * A[(long)i * n + j];
  return s;
}

/* A (n x n, symmetric, row-major) is overwritten; on exit its diagonal holds the
 * eigenvalues (unsorted).  V (n x n) receives the eigenvectors as columns.
 * Returns the number of sweeps used, or -1 if 60 sweeps did not converge. */
int oracle_jacobi_eig(double* A, double* V, int n, double tol) {
  memset(V, 0, sizeof(double) * (size_t)n * (size_t)n);
  for (int i = 0; i < n; ++i) V[(long)i * n + i] = 1.0;
  double fro2 = 0.0;
  for (long i = 0; i < (long)n * n; ++i) fro2 += A[i] * A[i];
  if (fro2 == 0.0) return 0;
  for (int sweep = 1; sweep <= 60; ++sweep) {
    for (int p = 0; p < n - 1; ++p) {
      for (int q = p + 1; q < n; ++q) {
        double apq = A[(long)p * n + q];
        double app = A[(long)p * n + p], aqq = A[(long)q * n + q];
        if (fabs(apq) <= 1e-300) continue;
        double c, s;
        sym_schur2(app, aqq, apq, &c, &s);
        /* A <- A J  (columns p, q) */
        for (int k = 0; k < n; ++k) {
          double akp = A[(long)k * n + p], akq = A[(long)k * n + q];
          A[(long)k * n + p] = c * akp - s * akq;
          A[(long)k * n + q] = s * akp + c * akq;
        }
        /* A <- J^T A  (rows p, q) */
        for (int k = 0; k < n; ++k) {
          double apk = A[(long)p * n + k], aqk = A[(long)q * n + k];
          A[(long)p * n + k] = c * apk - s * aqk;
          A[(long)q * n + k] = s * apk + c * aqk;
        }
        A[(long)p * n + q] = 0.0;
        A[(long)q * n + p] = 0.0;
        /* V <- V J */
        for (int k = 0; k < n; ++k) {
          double vkp = V[(long)k * n + p], vkq = V[(long)k * n + q];
          V[(long)k * n + p] = c * vkp - s * vkq;
          V[(long)k * n + q] = s * vkp + c * vkq;
        }
      }
    }
    if (off_norm2(A, n) <= tol * tol * fro2) return sweep;
  }
  return -1;
}

/* One-sided Jacobi SVD of a tall m x n matrix W (m >= n, row-major): columns of W are
 * rotated pairwise until mutually orthogonal, W J = U Sigma.  On exit W holds U*Sigma
 * (unnormalised left vectors), sig the column norms (unsorted), and Vr (n x n) the
 * accumulated rotation J (right singular vectors as columns).
 * Returns sweeps used, or -1 without convergence. */
int oracle_jacobi_svd(double* W, double* sig, double* Vr, int m, int n, double tol) {
  memset(Vr, 0, sizeof(double) * (size_t)n * (size_t)n);
  for (int i = 0; i < n; ++i) Vr[(long)i * n + i] = 1.0;
  for (int sweep = 1; sweep <= 60; ++sweep) {
    int rotated = 0;
    for (int p = 0; p < n - 1; ++p) {
      for (int q = p + 1; q < n; ++q) {
        double alpha = 0.0, beta = 0.0, gamma = 0.0;
        for (int k = 0; k < m; ++k) {
          double wp = W[(long)k * n + p], wq = W[(long)k * n + q];
          alpha += wp * wp; beta += wq * wq; gamma += wp * wq;
        }
        if (gamma == 0.0 || fabs(gamma) <= tol * sqrt(alpha * beta)) continue;
        rotated = 1;
        /* Rotation diagonalising the 2x2 Gram [alpha gamma; gamma beta]. */
        double c, s;
        sym_schur2(alpha, beta, gamma, &c, &s);
        for (int k = 0; k < m; ++k) {
          double wp = W[(long)k * n + p], wq = W[(long)k * n + q];
          W[(long)k * n + p] = c * wp - s * wq;
          W[(long)k * n + q] = s * wp + c * wq;
        }
        for (int k = 0; k < n; ++k) {
          double vp = Vr[(long)k * n + p], vq = Vr[(long)k * n + q];
          Vr[(long)k * n + p] = c * vp - s * vq;
          Vr[(long)k * n + q] = s * vp + c * vq;
        }
      }
    }
    if (!rotated) {
      for (int j = 0; j < n; ++j) {
        double ss = 0.0;
        for (int k = 0; k < m; ++k) ss += W[(long)k * n + j] * W[(long)k * n + j];
        sig[j] = sqrt(ss);
      }
      return sweep;
    }
  }
  return -1;
}
