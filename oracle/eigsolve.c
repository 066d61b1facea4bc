/*
 * Oracle dense symmetric eigensolver (test infrastructure only).
 *
 * This file belongs to the CPU oracle.  Only tests, the smoke check and the
 * CPU-baseline leg of the benchmark load it; the product library never does,
 * and it shares no code with the product library.
 *
 * What it computes: all eigenvalues (optionally eigenvectors) of a dense real
 * symmetric matrix, the "direct diagonalization" that the paper delegates to
 * LAPACK for the projected problem (Sec. II.C, App. C) and that, applied to the
 * full Hamiltonian, is the plain definition the central eigenvalues must match.
 *
 * Algorithms (textbook, written out plainly, FP64):
 *   - Householder tridiagonalisation (Golub & Van Loan, "Matrix Computations",
 *     symmetric Householder reduction): for each column k a reflector
 *     P = I - beta v v^T zeroes A[k+2:, k]; the trailing block is updated as
 *     A <- A - v w^T - w v^T with p = beta A v, w = p - (beta p^T v / 2) v.
 *   - Implicit QL with a Wilkinson-type shift on the tridiagonal (the
 *     Wilkinson-Reinsch algorithm), optionally accumulating the rotations into
 *     the Householder Q so that columns of Z are eigenvectors.
 *   - Cyclic Jacobi (classical two-sided rotations), an independent algorithm
 *     used only to cross-check the QL path in the oracle's own pins.
 *
 * OpenMP parallelises the O(n^2) loops of each step (row ranges); the
 * arithmetic of every element is the plain formula above.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define A_(i, j) a[(size_t)(i) * (size_t)n + (size_t)(j)]

/* Householder reduction of the symmetric n x n row-major matrix a (full
 * storage, overwritten).  On return d[0..n-1] is the diagonal, e[0..n-2] the
 * sub-diagonal (e[n-1] = 0).  If q != NULL it receives the orthogonal Q
 * (row-major n x n) with A_original = Q T Q^T. */
int orc_tridiagonalize(int n, double *a, double *d, double *e, double *q) {
  if (n <= 0) return 0;
  double *v = (double *)malloc(sizeof(double) * (size_t)n);
  double *p = (double *)malloc(sizeof(double) * (size_t)n);
  /* Householder vectors are kept (scaled) for Q accumulation. */
  double *vs = q ? (double *)calloc((size_t)n * (size_t)n, sizeof(double)) : NULL;
  double *betas = q ? (double *)calloc((size_t)n, sizeof(double)) : NULL;
  if (!v || !p || (q && (!vs || !betas))) {
    free(v); free(p); free(vs); free(betas);
    return -1;
  }
  for (int k = 0; k < n - 2; ++k) {
    const int m = n - k - 1; /* length of x = A[k+1:n, k] */
    double sigma = 0.0;
    for (int i = 1; i < m; ++i) sigma += A_(k + 1 + i, k) * A_(k + 1 + i, k);
    const double x0 = A_(k + 1, k);
    double beta = 0.0;
    if (sigma == 0.0) {
      /* already tridiagonal in this column */
      d[k] = A_(k, k);
      e[k] = x0;
      if (betas) betas[k] = 0.0;
      continue;
    }
    const double mu = sqrt(x0 * x0 + sigma);
    /* v = x - alpha e1 with alpha = -sign(x0) mu, so no cancellation */
    const double alpha = (x0 >= 0.0) ? -mu : mu;
    v[0] = x0 - alpha;
    for (int i = 1; i < m; ++i) v[i] = A_(k + 1 + i, k);
    double vtv = 0.0;
    for (int i = 0; i < m; ++i) vtv += v[i] * v[i];
    beta = 2.0 / vtv;
    /* p = beta * A22 v */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < m; ++i) {
      const double *row = &A_(k + 1 + i, k + 1);
      double s = 0.0;
      for (int j = 0; j < m; ++j) s += row[j] * v[j];
      p[i] = beta * s;
    }
    double ptv = 0.0;
    for (int i = 0; i < m; ++i) ptv += p[i] * v[i];
    const double half = 0.5 * beta * ptv;
    for (int i = 0; i < m; ++i) p[i] -= half * v[i]; /* p now holds w */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < m; ++i) {
      double *row = &A_(k + 1 + i, k + 1);
      const double vi = v[i], wi = p[i];
      for (int j = 0; j < m; ++j) row[j] -= vi * p[j] + wi * v[j];
    }
    d[k] = A_(k, k);
    e[k] = alpha;
    if (vs) {
      for (int i = 0; i < m; ++i) vs[(size_t)k * n + k + 1 + i] = v[i];
      betas[k] = beta;
    }
  }
  if (n >= 2) {
    d[n - 2] = A_(n - 2, n - 2);
    e[n - 2] = A_(n - 1, n - 2);
  }
  d[n - 1] = A_(n - 1, n - 1);
  e[n - 1] = 0.0;
  if (q) {
    /* Q = P_0 P_1 ... P_{n-3}; accumulate backwards on the identity. */
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) q[(size_t)i * n + j] = (i == j) ? 1.0 : 0.0;
    for (int k = n - 3; k >= 0; --k) {
      const double beta = betas[k];
      if (beta == 0.0) continue;
      const double *vk = &vs[(size_t)k * n];
      /* Q <- P_k Q = Q - beta v (v^T Q); only rows/cols k+1.. are touched */
#pragma omp parallel for schedule(static)
      for (int j = k + 1; j < n; ++j) {
        double s = 0.0;
        for (int i = k + 1; i < n; ++i) s += vk[i] * q[(size_t)i * n + j];
        s *= beta;
        for (int i = k + 1; i < n; ++i) q[(size_t)i * n + j] -= s * vk[i];
      }
    }
  }
  free(v); free(p); free(vs); free(betas);
  return 0;
}

/* Implicit QL on the symmetric tridiagonal (d, e) with e[i] coupling d[i] and
 * d[i+1].  Eigenvalues overwrite d (unsorted).  If z != NULL (row-major n x n)
 * the rotations are applied to its columns: pass Q from the tridiagonalisation
 * to obtain eigenvectors of the original matrix (column j <-> d[j]).
 * Returns 0, or -1 when an eigenvalue fails to converge in 60 iterations. */
int orc_tridiag_ql(int n, double *d, double *e, double *z) {
  if (n <= 0) return 0;
  e[n - 1] = 0.0;
  /* An off-diagonal element is negligible once it is below eps times the scale of the matrix seen
   * so far, the running maximum of |d_l| + |e_l| (the Wilkinson-Reinsch test).  A test against
   * the two neighbouring diagonal entries alone never deflates a cluster of eigenvalues at zero,
   * as in the singular overlap matrix of the projected problem. */
  double tst1 = 0.0;
  for (int l = 0; l < n; ++l) {
    int iter = 0;
    int mm;
    tst1 = fmax(tst1, fabs(d[l]) + fabs(e[l]));
    for (;;) {
      for (mm = l; mm < n - 1; ++mm) {
        if (fabs(e[mm]) <= 2.220446049250313e-16 * tst1) break;
      }
      if (mm == l) break;
      if (++iter > 60) return -1;
      /* shift from the leading 2x2 block: eigenvalue of it closest to d[l] */
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = hypot(g, 1.0);
      g = d[mm] - d[l] + e[l] / (g + (g >= 0.0 ? fabs(r) : -fabs(r)));
      double s = 1.0, c = 1.0, p = 0.0;
      int i;
      int early = 0;
      for (i = mm - 1; i >= l; --i) {
        const double f = s * e[i];
        const double bb = c * e[i];
        r = hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= p;
          e[mm] = 0.0;
          early = 1;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0 * c * bb;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - bb;
        if (z) {
#pragma omp parallel for schedule(static) if (n > 512)
          for (int k = 0; k < n; ++k) {
            double *zr = &z[(size_t)k * n];
            const double zf = zr[i + 1];
            zr[i + 1] = s * zr[i] + c * zf;
            zr[i] = c * zr[i] - s * zf;
          }
        }
      }
      if (early) continue;
      d[l] -= p;
      e[l] = g;
      e[mm] = 0.0;
    }
  }
  return 0;
}

/* Full symmetric eigen-decomposition: a (row-major, destroyed) -> w (ascending),
 * optional z (row-major n x n, column j = eigenvector of w[j]). */
int orc_syev(int n, double *a, double *w, double *z) {
  double *e = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  if (!e) return -1;
  int rc = orc_tridiagonalize(n, a, w, e, z);
  if (rc == 0) rc = orc_tridiag_ql(n, w, e, z);
  free(e);
  if (rc != 0) return rc;
  /* selection sort of eigenvalues (and matching columns), ascending */
  for (int i = 0; i < n - 1; ++i) {
    int k = i;
    for (int j = i + 1; j < n; ++j)
      if (w[j] < w[k]) k = j;
    if (k != i) {
      const double t = w[i]; w[i] = w[k]; w[k] = t;
      if (z)
        for (int r = 0; r < n; ++r) {
          const double u = z[(size_t)r * n + i];
          z[(size_t)r * n + i] = z[(size_t)r * n + k];
          z[(size_t)r * n + k] = u;
        }
    }
  }
  return 0;
}

/* Eigenvalues of a symmetric tridiagonal given directly (used for the
 * Jordan-Wigner single-particle problem).  w ascending on return. */
int orc_tridiag_eigvals(int n, const double *d, const double *e, double *w) {
  double *ee = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  if (!ee) return -1;
  for (int i = 0; i < n; ++i) { w[i] = d[i]; ee[i] = (i < n - 1) ? e[i] : 0.0; }
  int rc = orc_tridiag_ql(n, w, ee, NULL);
  free(ee);
  if (rc) return rc;
  for (int i = 1; i < n; ++i) { /* insertion sort */
    const double t = w[i];
    int j = i - 1;
    while (j >= 0 && w[j] > t) { w[j + 1] = w[j]; --j; }
    w[j + 1] = t;
  }
  return 0;
}

/* Cyclic Jacobi eigenvalue algorithm (independent cross-check).  a row-major,
 * destroyed; w ascending; v (row-major, may be NULL) eigenvectors by column. */
int orc_jacobi(int n, double *a, double *w, double *v, int max_sweeps) {
  if (v)
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) v[(size_t)i * n + j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const double x = A_(i, j) * A_(i, j);
        tot += x;
        if (i != j) off += x;
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A_(p, q);
        if (apq == 0.0) continue;
        const double theta = (A_(q, q) - A_(p, p)) / (2.0 * apq);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0);
        const double s = t * c;
        /* A <- J^T A J with J the rotation in the (p, q) plane */
        for (int k = 0; k < n; ++k) {
          const double akp = A_(k, p), akq = A_(k, q);
          A_(k, p) = c * akp - s * akq;
          A_(k, q) = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A_(p, k), aqk = A_(q, k);
          A_(p, k) = c * apk - s * aqk;
          A_(q, k) = s * apk + c * aqk;
        }
        if (v)
          for (int k = 0; k < n; ++k) {
            const double vkp = v[(size_t)k * n + p], vkq = v[(size_t)k * n + q];
            v[(size_t)k * n + p] = c * vkp - s * vkq;
            v[(size_t)k * n + q] = s * vkp + c * vkq;
          }
      }
  }
  for (int i = 0; i < n; ++i) w[i] = A_(i, i);
  for (int i = 0; i < n - 1; ++i) {
    int k = i;
    for (int j = i + 1; j < n; ++j)
      if (w[j] < w[k]) k = j;
    if (k != i) {
      const double t = w[i]; w[i] = w[k]; w[k] = t;
      if (v)
        for (int r = 0; r < n; ++r) {
          const double u = v[(size_t)r * n + i];
          v[(size_t)r * n + i] = v[(size_t)r * n + k];
          v[(size_t)r * n + k] = u;
        }
    }
  }
  return 0;
}
