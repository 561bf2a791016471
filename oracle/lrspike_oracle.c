/*
 * LR-SPIKE oracle: plain, slow, FP64 CPU reference for the banded LR-SPIKE
 * solver of Spring, Polizzi and Sameh, "Low-Rank SPIKE Framework for Solving
 * Large Sparse Linear Systems with Applications" (arXiv 2504.11167).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the GPU path: no BLAS, no LAPACK,
 * no headers of the product.
 *
 * Conventions
 *   bands  band-major input, bands[(d + k) * n + i] = A[i, i + d], d in [-k, k];
 *          entries with i + d outside [0, n) are ignored.
 *   f, x   row-major n x m (column c of row i at i * m + c).
 *   Partitions j = 0 .. p-1 (the paper numbers them 1 .. p).
 *
 * Every routine is written out in the order of the paper's equations, with
 * no blocking and no fusion, so that it can be read against the paper.
 * Return codes: 0 ok, >0 a zero pivot (1-based position), <0 bad argument.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* General band matrix with kl sub- and ku super-diagonals, stored column by */
/* column with kl extra rows for the fill that row interchanges create (the  */
/* classic layout of band Gaussian elimination with partial pivoting).       */
/* ------------------------------------------------------------------------ */
typedef struct {
  int64_t n;
  int kl, ku, ld; /* ld = 2 kl + ku + 1 */
  double *ab;
  int64_t *ipiv;
} gband;

static double *gb_at(gband *M, int64_t i, int64_t j) {
  return &M->ab[j * (int64_t)M->ld + (M->kl + M->ku + i - j)];
}

static int gb_alloc(gband *M, int64_t n, int kl, int ku) {
  M->n = n;
  M->kl = kl;
  M->ku = ku;
  M->ld = 2 * kl + ku + 1;
  M->ab = (double *)calloc((size_t)(n * M->ld), sizeof(double));
  M->ipiv = (int64_t *)calloc((size_t)n, sizeof(int64_t));
  return (M->ab && M->ipiv) ? 0 : -100;
}

static void gb_free(gband *M) {
  free(M->ab);
  free(M->ipiv);
  M->ab = NULL;
  M->ipiv = NULL;
}

static int64_t imin64(int64_t a, int64_t b) { return a < b ? a : b; }
static int64_t imax64(int64_t a, int64_t b) { return a > b ? a : b; }

/* A[i, j] of the input band (zero outside the band or the matrix). */
static double band_entry(int64_t n, int k, const double *bands, int64_t i,
                         int64_t j) {
  int64_t d = j - i;
  if (i < 0 || j < 0 || i >= n || j >= n || d < -k || d > k) return 0.0;
  return bands[(d + k) * n + i];
}

/* Copy the square block A[s : s + len, s : s + len] of the input band. */
static int gb_from_input(gband *M, int64_t n, int k, const double *bands,
                         int64_t s, int64_t len) {
  if (gb_alloc(M, len, k, k)) return -100;
  for (int64_t i = 0; i < len; ++i)
    for (int64_t j = imax64(0, i - k); j <= imin64(len - 1, i + k); ++j)
      *gb_at(M, i, j) = band_entry(n, k, bands, s + i, s + j);
  return 0;
}

/*
 * Band Gaussian elimination with row partial pivoting, column by column.
 * The pivot of column j is the first row of largest magnitude among rows
 * j .. j + kl.  Returns 0, or j + 1 for the first exactly zero pivot.
 */
static int64_t gb_factor(gband *M) {
  int64_t n = M->n, info = 0;
  int kl = M->kl, ku = M->ku;
  for (int64_t j = 0; j < n; ++j) {
    int64_t last = imin64(n - 1, j + kl);
    int64_t piv = j;
    double best = fabs(*gb_at(M, j, j));
    for (int64_t i = j + 1; i <= last; ++i)
      if (fabs(*gb_at(M, i, j)) > best) {
        best = fabs(*gb_at(M, i, j));
        piv = i;
      }
    M->ipiv[j] = piv;
    int64_t cend = imin64(n - 1, j + kl + ku);
    if (piv != j)
      for (int64_t c = j; c <= cend; ++c) {
        double t = *gb_at(M, j, c);
        *gb_at(M, j, c) = *gb_at(M, piv, c);
        *gb_at(M, piv, c) = t;
      }
    double d = *gb_at(M, j, j);
    if (d == 0.0) {
      if (!info) info = j + 1;
      continue;
    }
    for (int64_t i = j + 1; i <= last; ++i) {
      double l = *gb_at(M, i, j) / d;
      *gb_at(M, i, j) = l;
      for (int64_t c = j + 1; c <= cend; ++c) *gb_at(M, i, c) -= l * *gb_at(M, j, c);
    }
  }
  return info;
}

/* Solve A x = b in place with the factors of gb_factor; b is len x m row-major. */
static void gb_solve(gband *M, int m, double *b) {
  int64_t n = M->n;
  int kl = M->kl, ku = M->ku;
  for (int c = 0; c < m; ++c) {
    for (int64_t j = 0; j < n; ++j) {
      int64_t p = M->ipiv[j];
      if (p != j) {
        double t = b[j * m + c];
        b[j * m + c] = b[p * m + c];
        b[p * m + c] = t;
      }
      for (int64_t i = j + 1; i <= imin64(n - 1, j + kl); ++i)
        b[i * m + c] -= *gb_at(M, i, j) * b[j * m + c];
    }
    for (int64_t j = n - 1; j >= 0; --j) {
      b[j * m + c] /= *gb_at(M, j, j);
      for (int64_t i = imax64(0, j - kl - ku); i < j; ++i)
        b[i * m + c] -= *gb_at(M, i, j) * b[j * m + c];
    }
  }
}

/* Solve A^T x = b in place: U^T first, then the multipliers and interchanges
 * in reverse order (the transpose of the sequence applied by gb_solve). */
static void gb_solve_t(gband *M, int m, double *b) {
  int64_t n = M->n;
  int kl = M->kl, ku = M->ku;
  for (int c = 0; c < m; ++c) {
    for (int64_t j = 0; j < n; ++j) {
      double s = b[j * m + c];
      for (int64_t i = imax64(0, j - kl - ku); i < j; ++i)
        s -= *gb_at(M, i, j) * b[i * m + c];
      b[j * m + c] = s / *gb_at(M, j, j);
    }
    for (int64_t j = n - 1; j >= 0; --j) {
      double s = b[j * m + c];
      for (int64_t i = j + 1; i <= imin64(n - 1, j + kl); ++i)
        s -= *gb_at(M, i, j) * b[i * m + c];
      b[j * m + c] = s;
      int64_t p = M->ipiv[j];
      if (p != j) {
        double t = b[j * m + c];
        b[j * m + c] = b[p * m + c];
        b[p * m + c] = t;
      }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* R0: the plain definition x* = A^{-1} f (and A^{-T} g).                    */
/* ------------------------------------------------------------------------ */
int orc_band_solve(int64_t n, int k, const double *bands, int m, const double *f,
                   double *x, int transpose) {
  if (n < 1 || k < 0 || m < 1) return -1;
  gband M;
  if (gb_from_input(&M, n, k, bands, 0, n)) return -100;
  int64_t info = gb_factor(&M);
  if (info) {
    gb_free(&M);
    return (int)imin64(info, 2147483647);
  }
  memcpy(x, f, sizeof(double) * (size_t)(n * m));
  if (transpose)
    gb_solve_t(&M, m, x);
  else
    gb_solve(&M, m, x);
  gb_free(&M);
  return 0;
}

/* y = A x (transpose = 0) or y = A^T x (transpose = 1), x and y n x m. */
void orc_band_matvec(int64_t n, int k, const double *bands, int m, const double *x,
                     double *y, int transpose) {
  for (int64_t i = 0; i < n; ++i)
    for (int c = 0; c < m; ++c) {
      double s = 0.0;
      for (int64_t j = imax64(0, i - k); j <= imin64(n - 1, i + k); ++j) {
        double a = transpose ? band_entry(n, k, bands, j, i) : band_entry(n, k, bands, i, j);
        s += a * x[j * m + c];
      }
      y[i * m + c] = s;
    }
}

/*
 * x* in FP64 made accurate to about one rounding independently of the
 * condition number: R0 followed by `steps` corrections whose residual
 * f - A x is accumulated in long double.  transpose = 1: the same for
 * A^T x = f (residual f - A^T x, corrections by the transposed solve).
 */
int orc_band_solve_refined(int64_t n, int k, const double *bands, int m,
                           const double *f, double *x, int steps, int transpose) {
  gband M;
  if (gb_from_input(&M, n, k, bands, 0, n)) return -100;
  int64_t info = gb_factor(&M);
  if (info) {
    gb_free(&M);
    return (int)imin64(info, 2147483647);
  }
  memcpy(x, f, sizeof(double) * (size_t)(n * m));
  if (transpose)
    gb_solve_t(&M, m, x);
  else
    gb_solve(&M, m, x);
  double *r = (double *)malloc(sizeof(double) * (size_t)(n * m));
  for (int s = 0; s < steps; ++s) {
    for (int64_t i = 0; i < n; ++i)
      for (int c = 0; c < m; ++c) {
        long double acc = (long double)f[i * m + c];
        for (int64_t j = imax64(0, i - k); j <= imin64(n - 1, i + k); ++j) {
          const double a = transpose ? band_entry(n, k, bands, j, i) : band_entry(n, k, bands, i, j);
          acc -= (long double)a * (long double)x[j * m + c];
        }
        r[i * m + c] = (double)acc;
      }
    if (transpose)
      gb_solve_t(&M, m, r);
    else
      gb_solve(&M, m, r);
    for (int64_t i = 0; i < n * m; ++i) x[i] += r[i];
  }
  free(r);
  gb_free(&M);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Partitioning (paper: SPIKE partitioning).  Partition j has               */
/* floor(n/p) + [j < n mod p] rows; offs has p + 1 entries.                  */
/* ------------------------------------------------------------------------ */
void orc_partition(int64_t n, int p, int64_t *offs) {
  int64_t base = n / p, extra = n % p;
  offs[0] = 0;
  for (int j = 0; j < p; ++j) offs[j + 1] = offs[j] + base + (j < extra ? 1 : 0);
}

/* ------------------------------------------------------------------------ */
/* Thin SVD of a tall rows x cols matrix (row-major): Householder QR, then   */
/* one-sided (Hestenes) Jacobi on the cols x cols factor R.  Returns the     */
/* singular values in descending order and the right singular vectors as the */
/* columns of vr (cols x cols, row-major).                                   */
/* ------------------------------------------------------------------------ */
int orc_thin_svd(int64_t rows, int cols, const double *a, double *sigma, double *vr) {
  double *w = (double *)malloc(sizeof(double) * (size_t)(rows * cols));
  double *R = (double *)calloc((size_t)(cols * cols), sizeof(double));
  double *v = (double *)malloc(sizeof(double) * (size_t)rows);
  if (!w || !R || !v) return -100;
  memcpy(w, a, sizeof(double) * (size_t)(rows * cols));
  int64_t steps = imin64(rows, cols);
  /* Householder QR: w := Q^T a, R = upper triangle of w. */
  for (int64_t c = 0; c < steps; ++c) {
    double nrm = 0.0;
    for (int64_t i = c; i < rows; ++i) nrm += w[i * cols + c] * w[i * cols + c];
    nrm = sqrt(nrm);
    if (nrm == 0.0) continue;
    double alpha = w[c * cols + c] > 0 ? -nrm : nrm;
    for (int64_t i = c; i < rows; ++i) v[i] = w[i * cols + c];
    v[c] -= alpha;
    double vv = 0.0;
    for (int64_t i = c; i < rows; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    for (int64_t cc = c; cc < cols; ++cc) {
      double s = 0.0;
      for (int64_t i = c; i < rows; ++i) s += v[i] * w[i * cols + cc];
      s = 2.0 * s / vv;
      for (int64_t i = c; i < rows; ++i) w[i * cols + cc] -= s * v[i];
    }
  }
  for (int64_t i = 0; i < steps; ++i)
    for (int64_t c = i; c < cols; ++c) R[i * cols + c] = w[i * cols + c];
  /* One-sided Jacobi on R: rotate column pairs until they are orthogonal. */
  for (int i = 0; i < cols; ++i)
    for (int c = 0; c < cols; ++c) vr[i * cols + c] = (i == c) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 80; ++sweep) {
    int rotated = 0;
    for (int a1 = 0; a1 < cols - 1; ++a1)
      for (int b1 = a1 + 1; b1 < cols; ++b1) {
        double al = 0, be = 0, ga = 0;
        for (int i = 0; i < cols; ++i) {
          al += R[i * cols + a1] * R[i * cols + a1];
          be += R[i * cols + b1] * R[i * cols + b1];
          ga += R[i * cols + a1] * R[i * cols + b1];
        }
        if (ga == 0.0 || fabs(ga) <= 1e-15 * sqrt(al * be)) continue;
        rotated = 1;
        double zeta = (be - al) / (2.0 * ga);
        double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
        for (int i = 0; i < cols; ++i) {
          double ra = R[i * cols + a1], rb = R[i * cols + b1];
          R[i * cols + a1] = cs * ra - sn * rb;
          R[i * cols + b1] = sn * ra + cs * rb;
          double va = vr[i * cols + a1], vb = vr[i * cols + b1];
          vr[i * cols + a1] = cs * va - sn * vb;
          vr[i * cols + b1] = sn * va + cs * vb;
        }
      }
    if (!rotated) break;
  }
  for (int c = 0; c < cols; ++c) {
    double s = 0.0;
    for (int i = 0; i < cols; ++i) s += R[i * cols + c] * R[i * cols + c];
    sigma[c] = sqrt(s);
  }
  /* Sort descending (selection sort keeps ties in their original order). */
  for (int c = 0; c < cols; ++c) {
    int best = c;
    for (int d = c + 1; d < cols; ++d)
      if (sigma[d] > sigma[best]) best = d;
    if (best != c) {
      double t = sigma[c];
      sigma[c] = sigma[best];
      sigma[best] = t;
      for (int i = 0; i < cols; ++i) {
        t = vr[i * cols + c];
        vr[i * cols + c] = vr[i * cols + best];
        vr[i * cols + best] = t;
      }
    }
  }
  free(w);
  free(R);
  free(v);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Randomized SVD of a spike (section "SVD representation of the spikes":    */
/* the proto-algorithm of Halko, Martinsson and Tropp with a few passes over  */
/* the matrix and oversampling).  For the tall rows x cols matrix a and the  */
/* Gaussian test matrix omega (cols x ell, row-major, drawn by the caller):  */
/*   Y = (a a^T)^q a omega          (q power steps, 2 + 2q passes over a)    */
/*   Q = orthonormal basis of range(Y)  (Householder QR of Y)                */
/*   B = Q^T a,   a ~ Q B = Q Q^T a                                          */
/* The SVD of B gives the approximate singular triplets of a: Q U_B, S_B and */
/* V_B.  Q B has the same singular values and right singular vectors as B,   */
/* so a is replaced here by Q Q^T a (written to proj, rows x cols) and the   */
/* caller takes the thin SVD of that, exactly as for the whole spike.        */
/* ------------------------------------------------------------------------ */
int orc_rsvd_project(int64_t rows, int cols, const double *a, int ell, int q, const double *omega,
                     double *proj) {
  if (rows < 1 || cols < 1 || ell < 1 || ell > cols || ell > rows || q < 0) return -1;
  double *Y = (double *)calloc((size_t)(rows * ell), sizeof(double));
  double *Z = (double *)calloc((size_t)cols * ell, sizeof(double));
  double *H = (double *)calloc((size_t)(rows * ell), sizeof(double)); /* reflectors */
  double *hv = (double *)calloc((size_t)ell, sizeof(double));         /* v^T v of each */
  double *Q = (double *)calloc((size_t)(rows * ell), sizeof(double));
  if (!Y || !Z || !H || !hv || !Q) return -100;
  /* Y = a omega */
  for (int64_t i = 0; i < rows; ++i)
    for (int c = 0; c < ell; ++c) {
      double acc = 0.0;
      for (int b = 0; b < cols; ++b) acc += a[i * cols + b] * omega[b * ell + c];
      Y[i * ell + c] = acc;
    }
  /* power steps: Z = a^T Y, Y = a Z */
  for (int it = 0; it < q; ++it) {
    for (int b = 0; b < cols; ++b)
      for (int c = 0; c < ell; ++c) {
        double acc = 0.0;
        for (int64_t i = 0; i < rows; ++i) acc += a[i * cols + b] * Y[i * ell + c];
        Z[b * ell + c] = acc;
      }
    for (int64_t i = 0; i < rows; ++i)
      for (int c = 0; c < ell; ++c) {
        double acc = 0.0;
        for (int b = 0; b < cols; ++b) acc += a[i * cols + b] * Z[b * ell + c];
        Y[i * ell + c] = acc;
      }
  }
  /* Householder QR of Y: reflector c zeroes column c below the diagonal */
  for (int c = 0; c < ell; ++c) {
    double nrm = 0.0;
    for (int64_t i = c; i < rows; ++i) nrm += Y[i * ell + c] * Y[i * ell + c];
    nrm = sqrt(nrm);
    hv[c] = 0.0;
    if (nrm == 0.0) continue; /* column already zero: H_c = I */
    double alpha = Y[c * ell + c] > 0 ? -nrm : nrm;
    for (int64_t i = c; i < rows; ++i) H[i * ell + c] = Y[i * ell + c];
    H[c * ell + c] -= alpha;
    double vv = 0.0;
    for (int64_t i = c; i < rows; ++i) vv += H[i * ell + c] * H[i * ell + c];
    hv[c] = vv;
    if (vv == 0.0) continue;
    for (int cc = c; cc < ell; ++cc) {
      double t = 0.0;
      for (int64_t i = c; i < rows; ++i) t += H[i * ell + c] * Y[i * ell + cc];
      t = 2.0 * t / vv;
      for (int64_t i = c; i < rows; ++i) Y[i * ell + cc] -= t * H[i * ell + c];
    }
  }
  /* Q = H_0 H_1 ... H_{ell-1} [I_ell; 0] (orthonormal columns in every case) */
  for (int c = 0; c < ell; ++c) Q[c * ell + c] = 1.0;
  for (int c = ell - 1; c >= 0; --c) {
    if (hv[c] == 0.0) continue;
    for (int cc = 0; cc < ell; ++cc) {
      double t = 0.0;
      for (int64_t i = c; i < rows; ++i) t += H[i * ell + c] * Q[i * ell + cc];
      t = 2.0 * t / hv[c];
      for (int64_t i = c; i < rows; ++i) Q[i * ell + cc] -= t * H[i * ell + c];
    }
  }
  /* B = Q^T a (ell x cols, in Z's storage), proj = Q B */
  for (int c = 0; c < ell; ++c)
    for (int b = 0; b < cols; ++b) {
      double acc = 0.0;
      for (int64_t i = 0; i < rows; ++i) acc += Q[i * ell + c] * a[i * cols + b];
      Z[c * cols + b] = acc;
    }
  for (int64_t i = 0; i < rows; ++i)
    for (int b = 0; b < cols; ++b) {
      double acc = 0.0;
      for (int c = 0; c < ell; ++c) acc += Q[i * ell + c] * Z[c * cols + b];
      proj[i * cols + b] = acc;
    }
  free(Y);
  free(Z);
  free(H);
  free(hv);
  free(Q);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Literal LR-SPIKE (paper: SPIKE partitioning, the DS factorization, the    */
/* spikes, the reduced system, recovery; low-rank SVD representation of the  */
/* spikes).                                                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
  int64_t n;
  int k, p, r;
  int64_t *offs;   /* p + 1 */
  gband *A;        /* per-partition factors of A_j */
  double *Bc, *Cc; /* per-partition k x k coupling blocks */
  double *Vt, *Vb, *Wt, *Wb; /* per-partition truncated tips, k x k each */
  double *sv;      /* singular values, p x 2 x k (V then W); zero when absent */
  gband S;         /* the assembled reduced system, order 2 k p */
} orc_plan;

static void plan_free(orc_plan *P) {
  if (P->A)
    for (int j = 0; j < P->p; ++j) gb_free(&P->A[j]);
  free(P->A);
  free(P->offs);
  free(P->Bc);
  free(P->Cc);
  free(P->Vt);
  free(P->Vb);
  free(P->Wt);
  free(P->Wb);
  free(P->sv);
  if (P->S.ab) gb_free(&P->S);
  memset(P, 0, sizeof(*P));
}

/* tip := tip * Pi * Pi^T with Pi the first r columns of vr (k x k). */
static void project_tip(int k, int r, const double *vr, double *tip) {
  double *t1 = (double *)calloc((size_t)(k * k), sizeof(double));
  for (int i = 0; i < k; ++i)
    for (int q = 0; q < r; ++q) {
      double s = 0.0;
      for (int c = 0; c < k; ++c) s += tip[i * k + c] * vr[c * k + q];
      t1[i * k + q] = s;
    }
  for (int i = 0; i < k; ++i)
    for (int c = 0; c < k; ++c) {
      double s = 0.0;
      for (int q = 0; q < r; ++q) s += t1[i * k + q] * vr[c * k + q];
      tip[i * k + c] = s;
    }
  free(t1);
}

/* Factorization stage.  Returns 0, >0 on a zero pivot, <0 on bad input. */
static int plan_build(orc_plan *P, int64_t n, int k, const double *bands, int p,
                      int r, int variant, int nthreads, int ell, int q, const double *omega) {
  memset(P, 0, sizeof(*P));
  if (n < 1 || k < 1 || p < 1 || r < 0 || r > k) return -1;
  P->n = n;
  P->k = k;
  P->p = p;
  P->r = r;
  P->offs = (int64_t *)malloc(sizeof(int64_t) * (size_t)(p + 1));
  orc_partition(n, p, P->offs);
  for (int j = 0; j < p; ++j)
    if (p > 1 && P->offs[j + 1] - P->offs[j] < 2 * k) {
      plan_free(P);
      return -4;
    }
  size_t kk = (size_t)k * k;
  P->A = (gband *)calloc((size_t)p, sizeof(gband));
  P->Bc = (double *)calloc(kk * p, sizeof(double));
  P->Cc = (double *)calloc(kk * p, sizeof(double));
  P->Vt = (double *)calloc(kk * p, sizeof(double));
  P->Vb = (double *)calloc(kk * p, sizeof(double));
  P->Wt = (double *)calloc(kk * p, sizeof(double));
  P->Wb = (double *)calloc(kk * p, sizeof(double));
  P->sv = (double *)calloc((size_t)p * 2 * k, sizeof(double));
  int bad = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic) reduction(| : bad)
#endif
  for (int j = 0; j < p; ++j) {
    int64_t s = P->offs[j], nj = P->offs[j + 1] - P->offs[j];
    double *Bj = P->Bc + kk * j, *Cj = P->Cc + kk * j;
    /* Coupling blocks: B_j = A[s_{j+1}-k : s_{j+1}, s_{j+1} : s_{j+1}+k],
     *                  C_j = A[s_j : s_j+k, s_j-k : s_j]. */
    for (int a = 0; a < k; ++a)
      for (int b = 0; b < k; ++b) {
        if (j < p - 1) Bj[a * k + b] = band_entry(n, k, bands, s + nj - k + a, s + nj + b);
        if (j > 0) Cj[a * k + b] = band_entry(n, k, bands, s + a, s - k + b);
      }
    if (gb_from_input(&P->A[j], n, k, bands, s, nj)) {
      bad |= 1;
      continue;
    }
    if (gb_factor(&P->A[j])) {
      bad |= 2;
      continue;
    }
    /* Spikes V_j = A_j^{-1} [0; B_j] (j < p-1) and W_j = A_j^{-1} [C_j; 0] (j > 0). */
    double *sp = (double *)malloc(sizeof(double) * (size_t)(nj * k));
    double *vr = (double *)malloc(sizeof(double) * kk);
    for (int which = 0; which < 2; ++which) {
      if (which == 0 && j == p - 1) continue;
      if (which == 1 && j == 0) continue;
      memset(sp, 0, sizeof(double) * (size_t)(nj * k));
      for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) {
          if (which == 0)
            sp[(nj - k + a) * k + b] = Bj[a * k + b];
          else
            sp[a * k + b] = Cj[a * k + b];
        }
      gb_solve(&P->A[j], k, sp);
      if (omega && r < k) {
        /* randomized SVD: the spike is replaced by its projection Q Q^T sp
         * onto the sketched range, whose thin SVD below is that of B */
        double *pr = (double *)malloc(sizeof(double) * (size_t)(nj * k));
        if (orc_rsvd_project(nj, k, sp, ell, q, omega + ((size_t)j * 2 + which) * k * ell, pr)) bad |= 4;
        memcpy(sp, pr, sizeof(double) * (size_t)(nj * k));
        free(pr);
      }
      double *top = (which == 0 ? P->Vt : P->Wt) + kk * j;
      double *bot = (which == 0 ? P->Vb : P->Wb) + kk * j;
      memcpy(top, sp, sizeof(double) * kk);
      memcpy(bot, sp + (nj - k) * k, sizeof(double) * kk);
      /* Rank-r truncation of the whole spike (low-rank SVD representation):
       * the tips of u~ Sigma~ v~ equal tip * Pi Pi^T, Pi = leading right
       * singular vectors (of Q Q^T sp with the randomized SVD). */
      orc_thin_svd(nj, k, sp, P->sv + (size_t)j * 2 * k + (size_t)which * k, vr);
      if (r < k) {
        project_tip(k, r, vr, top);
        project_tip(k, r, vr, bot);
      }
    }
    free(sp);
    free(vr);
  }
  if (bad) {
    plan_free(P);
    return 1;
  }
  /* Reduced system, order 2kp, unknowns ordered [x_{0,t}; x_{0,b}; x_{1,t}; ...],
   * identity on the diagonal, truncated V tips in the column block of
   * x_{j+1,t} and truncated W tips in the column block of x_{j-1,b}.
   * variant 1 (LR-SPIKE-T, the truncated-SPIKE form of eqs. truncated_redsys
   * and red_sys_prec_mid_1): the blocks V~_{j,t} and W~_{j,b} that couple the
   * interfaces are left out, so only the 2 x 2 blocks
   * [[I, V~_{j,b}], [W~_{j+1,t}, I]] on x_{j,b}, x_{j+1,t} remain. */
  if (p > 1) {
    int64_t N = 2 * (int64_t)k * p;
    int hb = 3 * k - 1;
    if (gb_alloc(&P->S, N, hb, hb)) {
      plan_free(P);
      return -100;
    }
    for (int64_t i = 0; i < N; ++i) *gb_at(&P->S, i, i) = 1.0;
    for (int j = 0; j < p; ++j) {
      int64_t rt = 2 * (int64_t)j * k, rb = rt + k;
      for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) {
          if (j < p - 1) {
            int64_t col = 2 * (int64_t)(j + 1) * k + b; /* x_{j+1,t} */
            if (variant == 0) *gb_at(&P->S, rt + a, col) = P->Vt[kk * j + a * k + b];
            *gb_at(&P->S, rb + a, col) = P->Vb[kk * j + a * k + b];
          }
          if (j > 0) {
            int64_t col = (2 * (int64_t)(j - 1) + 1) * k + b; /* x_{j-1,b} */
            *gb_at(&P->S, rt + a, col) = P->Wt[kk * j + a * k + b];
            if (variant == 0) *gb_at(&P->S, rb + a, col) = P->Wb[kk * j + a * k + b];
          }
        }
    }
    if (gb_factor(&P->S)) {
      plan_free(P);
      return 2;
    }
  }
  return 0;
}

/* D-stage: y_j = A_j^{-1} f_j; the tips form the reduced right-hand side
 * yr (order 2kp: [y_{0,t}; y_{0,b}; y_{1,t}; ...], k x m each). */
static void plan_dstage(orc_plan *P, int m, const double *f, double *yr) {
  int k = P->k, p = P->p;
  for (int j = 0; j < p; ++j) {
    int64_t s = P->offs[j], nj = P->offs[j + 1] - s;
    double *y = (double *)malloc(sizeof(double) * (size_t)(nj * m));
    memcpy(y, f + s * m, sizeof(double) * (size_t)(nj * m));
    gb_solve(&P->A[j], m, y);
    memcpy(yr + 2 * (int64_t)j * k * m, y, sizeof(double) * (size_t)k * m);
    memcpy(yr + (2 * (int64_t)j + 1) * k * m, y + (nj - k) * m, sizeof(double) * (size_t)k * m);
    free(y);
  }
}

static void plan_recover(orc_plan *P, int m, const double *f, const double *yr, double *x);

/* Solve stage: D-stage, reduced system, solve-based recovery. */
static void plan_solve(orc_plan *P, int m, const double *f, double *x) {
  int k = P->k, p = P->p;
  int64_t n = P->n;
  if (p == 1) {
    memcpy(x, f, sizeof(double) * (size_t)(n * m));
    gb_solve(&P->A[0], m, x);
    return;
  }
  int64_t N = 2 * (int64_t)k * p;
  double *yr = (double *)malloc(sizeof(double) * (size_t)(N * m));
  plan_dstage(P, m, f, yr);
  /* Reduced system: x_red = S_red^{-1} y_red. */
  gb_solve(&P->S, m, yr);
  plan_recover(P, m, f, yr, x);
  free(yr);
}

/* Recovery from the interface tips yr (eqs. recovery1/2):
 * x_j = A_j^{-1} (f_j - [C_j x_{j-1,b}; 0; B_j x_{j+1,t}]). */
static void plan_recover(orc_plan *P, int m, const double *f, const double *yr, double *x) {
  int k = P->k, p = P->p;
  size_t kk = (size_t)k * k;
  for (int j = 0; j < p; ++j) {
    int64_t s = P->offs[j], nj = P->offs[j + 1] - s;
    double *g = x + s * m;
    memcpy(g, f + s * m, sizeof(double) * (size_t)(nj * m));
    if (j > 0) {
      const double *xb = yr + (2 * (int64_t)(j - 1) + 1) * k * m;
      for (int a = 0; a < k; ++a)
        for (int c = 0; c < m; ++c) {
          double acc = 0.0;
          for (int b = 0; b < k; ++b) acc += P->Cc[kk * j + a * k + b] * xb[b * m + c];
          g[a * m + c] -= acc;
        }
    }
    if (j < p - 1) {
      const double *xt = yr + 2 * (int64_t)(j + 1) * k * m;
      for (int a = 0; a < k; ++a)
        for (int c = 0; c < m; ++c) {
          double acc = 0.0;
          for (int b = 0; b < k; ++b) acc += P->Bc[kk * j + a * k + b] * xt[b * m + c];
          g[(nj - k + a) * m + c] -= acc;
        }
    }
    gb_solve(&P->A[j], m, g);
  }
}

/* Adjoint: lambda = D^{-T} (g - E w), w = S_red^{-T} K^T D^{-T} g, the exact
 * transpose of plan_solve for every rank r. */
static void plan_solve_t(orc_plan *P, int m, const double *g, double *lam) {
  int k = P->k, p = P->p;
  int64_t n = P->n;
  size_t kk = (size_t)k * k;
  if (p == 1) {
    memcpy(lam, g, sizeof(double) * (size_t)(n * m));
    gb_solve_t(&P->A[0], m, lam);
    return;
  }
  int64_t N = 2 * (int64_t)k * p;
  double *h = (double *)calloc((size_t)(N * m), sizeof(double));
  /* nu_j = A_j^{-T} g_j; h(j+1,t) += B_j^T nu_{j,b}; h(j-1,b) += C_j^T nu_{j,t}. */
  for (int j = 0; j < p; ++j) {
    int64_t s = P->offs[j], nj = P->offs[j + 1] - s;
    double *nu = (double *)malloc(sizeof(double) * (size_t)(nj * m));
    memcpy(nu, g + s * m, sizeof(double) * (size_t)(nj * m));
    gb_solve_t(&P->A[j], m, nu);
    if (j < p - 1) {
      double *ht = h + 2 * (int64_t)(j + 1) * k * m;
      for (int b = 0; b < k; ++b)
        for (int c = 0; c < m; ++c) {
          double acc = 0.0;
          for (int a = 0; a < k; ++a) acc += P->Bc[kk * j + a * k + b] * nu[(nj - k + a) * m + c];
          ht[b * m + c] += acc;
        }
    }
    if (j > 0) {
      double *hb = h + (2 * (int64_t)(j - 1) + 1) * k * m;
      for (int b = 0; b < k; ++b)
        for (int c = 0; c < m; ++c) {
          double acc = 0.0;
          for (int a = 0; a < k; ++a) acc += P->Cc[kk * j + a * k + b] * nu[a * m + c];
          hb[b * m + c] += acc;
        }
    }
    free(nu);
  }
  gb_solve_t(&P->S, m, h);
  for (int j = 0; j < p; ++j) {
    int64_t s = P->offs[j], nj = P->offs[j + 1] - s;
    double *o = lam + s * m;
    memcpy(o, g + s * m, sizeof(double) * (size_t)(nj * m));
    const double *wt = h + 2 * (int64_t)j * k * m, *wb = h + (2 * (int64_t)j + 1) * k * m;
    for (int a = 0; a < k; ++a)
      for (int c = 0; c < m; ++c) {
        o[a * m + c] -= wt[a * m + c];
        o[(nj - k + a) * m + c] -= wb[a * m + c];
      }
    gb_solve_t(&P->A[j], m, o);
  }
  free(h);
}

/*
 * R1 (transpose = 0): x = M_r^{-1} f, the LR-SPIKE solution at rank r.
 * R3 (transpose = 1): x = M_r^{-T} f.
 * variant 0: the whole truncated reduced system S~_red; variant 1: LR-SPIKE-T,
 * its truncated-SPIKE form S~~_red (table solver-list), with the same
 * solve-based recovery.
 * sv (nullable) receives the singular values of every spike, p x 2 x k
 * (V_j then W_j, descending; zeros for the absent V_{p-1} and W_0).
 * orc_lrspike_rsvd: with omega (p x 2 x k x ell Gaussian test matrices, V_j
 * then W_j of every partition) and r < k, every spike is truncated through
 * the randomized SVD (orc_rsvd_project, ell columns, q power steps) instead
 * of its exact SVD; sv then holds the singular values of Q Q^T spike.
 */
int orc_lrspike_rsvd(int64_t n, int k, const double *bands, int p, int r, int m,
                     const double *f, double *x, int transpose, double *sv, int nthreads,
                     int variant, int ell, int q, const double *omega) {
  if (m < 1) return -6;
  if (variant != 0 && variant != 1) return -12;
  if (omega && (ell < 1 || ell > k)) return -13;
  if (omega && q < 0) return -14;
  orc_plan P;
  int rc = plan_build(&P, n, k, bands, p, r, variant, nthreads, ell, q, omega);
  if (rc) return rc;
  if (sv) memcpy(sv, P.sv, sizeof(double) * (size_t)p * 2 * k);
  if (transpose)
    plan_solve_t(&P, m, f, x);
  else
    plan_solve(&P, m, f, x);
  plan_free(&P);
  return 0;
}

int orc_lrspike(int64_t n, int k, const double *bands, int p, int r, int m,
                const double *f, double *x, int transpose, double *sv, int nthreads,
                int variant) {
  return orc_lrspike_rsvd(n, k, bands, p, r, m, f, x, transpose, sv, nthreads, variant, 0, 0, NULL);
}

/*
 * BiCGStab preconditioned on the right by the LR-SPIKE operator M_r^{-1}
 * (variant 0 LR-SPIKE, 1 LR-SPIKE-T), the outer Krylov solver the paper pairs
 * with its preconditioners (table solver-list; the BiCGStab experiments with
 * SuiteSparse matrices).  The textbook recurrence (van der Vorst), each column
 * on its own, starting from x_0 = M^{-1} f:
 *   r = f - A x, rh = r, p = v = 0, rho_old = alpha = omega = 1;
 *   repeat: rho = (rh, r); beta = (rho / rho_old)(alpha / omega);
 *           p = r + beta (p - omega v); ph = M^{-1} p; v = A ph;
 *           alpha = rho / (rh, v); s = r - alpha v; sh = M^{-1} s; t = A sh;
 *           omega = (t, s) / (t, t)  (0 when t = 0);
 *           x += alpha ph + omega sh; r = s - omega t; rho_old = rho
 *   until ||r||_2 <= tol ||f||_2 or max_it iterations.  transpose = 1 solves
 *   A^T x = f with M_r^{-T}.  iters[c] receives the iterations of column c
 *   and relres[c] its final ||r|| / ||f|| (the recursively updated residual).
 */
static double col_dot(int64_t n, int m, int c, const double *a, const double *b) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += a[i * m + c] * b[i * m + c];
  return s;
}

int orc_bicgstab(int64_t n, int k, const double *bands, int p, int r, int variant, int m,
                 const double *f, double *x, double tol, int max_it, int transpose,
                 int *iters, double *relres, int nthreads) {
  if (m < 1 || max_it < 0) return -7;
  if (variant != 0 && variant != 1) return -6;
  orc_plan P;
  int rc = plan_build(&P, n, k, bands, p, r, variant, nthreads, 0, 0, NULL);
  if (rc) return rc;
  size_t nm = (size_t)(n * m);
  double *rv = (double *)malloc(sizeof(double) * nm), *rh = (double *)malloc(sizeof(double) * nm);
  double *pv = (double *)calloc(nm, sizeof(double)), *vv = (double *)calloc(nm, sizeof(double));
  double *ph = (double *)malloc(sizeof(double) * nm), *sv = (double *)malloc(sizeof(double) * nm);
  double *sh = (double *)malloc(sizeof(double) * nm), *tv = (double *)malloc(sizeof(double) * nm);
  double *col = (double *)malloc(sizeof(double) * (size_t)n);
  double *col2 = (double *)malloc(sizeof(double) * (size_t)n);
  /* the preconditioner and the matrix are applied column by column */
  void (*Msolve)(orc_plan *, int, const double *, double *) = transpose ? plan_solve_t : plan_solve;
#define APPLY_M(src, dst, c)                                               \
  do {                                                                     \
    for (int64_t i_ = 0; i_ < n; ++i_) col[i_] = (src)[i_ * m + (c)];      \
    Msolve(&P, 1, col, col2);                                              \
    for (int64_t i_ = 0; i_ < n; ++i_) (dst)[i_ * m + (c)] = col2[i_];     \
  } while (0)
#define APPLY_A(src, dst, c)                                               \
  do {                                                                     \
    for (int64_t i_ = 0; i_ < n; ++i_) col[i_] = (src)[i_ * m + (c)];      \
    orc_band_matvec(n, k, bands, 1, col, col2, transpose);                 \
    for (int64_t i_ = 0; i_ < n; ++i_) (dst)[i_ * m + (c)] = col2[i_];     \
  } while (0)
  for (int c = 0; c < m; ++c) {
    APPLY_M(f, x, c);
    APPLY_A(x, rv, c);
    for (int64_t i = 0; i < n; ++i) {
      rv[i * m + c] = f[i * m + c] - rv[i * m + c];
      rh[i * m + c] = rv[i * m + c];
    }
    double nf = sqrt(col_dot(n, m, c, f, f));
    double rho_old = 1.0, alpha = 1.0, omega = 1.0;
    int it = 0;
    double nr = sqrt(col_dot(n, m, c, rv, rv));
    while (it < max_it && !(nr <= tol * nf)) {
      double rho = col_dot(n, m, c, rh, rv);
      double beta = (rho / rho_old) * (alpha / omega);
      for (int64_t i = 0; i < n; ++i) {
        size_t o = (size_t)(i * m + c);
        pv[o] = rv[o] + beta * (pv[o] - omega * vv[o]);
      }
      APPLY_M(pv, ph, c);
      APPLY_A(ph, vv, c);
      alpha = rho / col_dot(n, m, c, rh, vv);
      for (int64_t i = 0; i < n; ++i) {
        size_t o = (size_t)(i * m + c);
        sv[o] = rv[o] - alpha * vv[o];
      }
      APPLY_M(sv, sh, c);
      APPLY_A(sh, tv, c);
      double tt = col_dot(n, m, c, tv, tv);
      omega = tt > 0.0 ? col_dot(n, m, c, tv, sv) / tt : 0.0;
      for (int64_t i = 0; i < n; ++i) {
        size_t o = (size_t)(i * m + c);
        x[o] += alpha * ph[o] + omega * sh[o];
        rv[o] = sv[o] - omega * tv[o];
      }
      rho_old = rho;
      ++it;
      nr = sqrt(col_dot(n, m, c, rv, rv));
      if (!(rho != 0.0 && omega != 0.0) && !(nr <= tol * nf)) break; /* breakdown */
    }
    if (iters) iters[c] = it;
    if (relres) relres[c] = nf > 0.0 ? nr / nf : 0.0;
  }
#undef APPLY_M
#undef APPLY_A
  free(rv); free(rh); free(pv); free(vv); free(ph); free(sv); free(sh); free(tv); free(col); free(col2);
  plan_free(&P);
  return 0;
}

/*
 * Iterative reduced solves (table solver-list):
 *   kind 0, LR-SPIKE-I:   S~_red (the spikes' rank-r representation) solved
 *                         by BiCGStab;
 *   kind 1, LR-SPIKE-OTF: the true S_red (eq. spikered, whole spikes) solved
 *                         by BiCGStab; the paper multiplies by it on the fly
 *                         through partition solves (eqs. OTF-1/2), which is
 *                         the same product as the one with the whole spikes'
 *                         tips written out here;
 * both right-preconditioned by S~~_red at rank r (the LR-SPIKE-T system),
 * then the solve-based recovery (eqs. recovery1/2) from the iterated tips.
 * The BiCGStab recurrence is orc_bicgstab's, per column, on vectors of order
 * 2kp, from x_0 = S~~_red^{-1} y_red; iters[c] / relres[c] (nullable) receive
 * the inner iterations and the final ||r|| / ||y_red|| of column c.  With
 * kind 1 the result is A^{-1} f to the inner tolerance for every r.
 */
static void red_matvec(const orc_plan *P, const double *x, double *y) {
  /* y = S x for the plan's tips, one column of order 2kp */
  int k = P->k, p = P->p;
  size_t kk = (size_t)k * k;
  for (int j = 0; j < p; ++j)
    for (int a = 0; a < k; ++a) {
      int64_t rt = 2 * (int64_t)j * k + a, rb = rt + k;
      double yt = x[rt], yb = x[rb];
      for (int b = 0; b < k; ++b) {
        if (j < p - 1) {
          double xn = x[2 * (int64_t)(j + 1) * k + b]; /* x_{j+1,t} */
          yt += P->Vt[kk * j + a * k + b] * xn;
          yb += P->Vb[kk * j + a * k + b] * xn;
        }
        if (j > 0) {
          double xp = x[(2 * (int64_t)(j - 1) + 1) * k + b]; /* x_{j-1,b} */
          yt += P->Wt[kk * j + a * k + b] * xp;
          yb += P->Wb[kk * j + a * k + b] * xp;
        }
      }
      y[rt] = yt;
      y[rb] = yb;
    }
}

int orc_lrspike_iter(int64_t n, int k, const double *bands, int p, int r, int m, const double *f,
                     double *x, int kind, double tol, int max_it, int *iters, double *relres,
                     int nthreads) {
  if (m < 1 || max_it < 0) return -7;
  if (kind != 0 && kind != 1) return -8;
  if (p < 2) return -4;
  orc_plan Pm, Pt;
  /* the operator: truncated tips (I) or whole spikes' tips (OTF) */
  int rc = plan_build(&Pm, n, k, bands, p, kind == 0 ? r : k, 0, nthreads, 0, 0, NULL);
  if (rc) return rc;
  rc = plan_build(&Pt, n, k, bands, p, r, 1, nthreads, 0, 0, NULL);
  if (rc) {
    plan_free(&Pm);
    return rc;
  }
  int64_t N = 2 * (int64_t)k * p;
  size_t Nm = (size_t)(N * m);
  double *yr = (double *)malloc(sizeof(double) * Nm), *xr = (double *)malloc(sizeof(double) * Nm);
  plan_dstage(&Pm, m, f, yr);
  double *rv = (double *)malloc(sizeof(double) * Nm), *rh = (double *)malloc(sizeof(double) * Nm);
  double *pv = (double *)calloc(Nm, sizeof(double)), *vv = (double *)calloc(Nm, sizeof(double));
  double *ph = (double *)malloc(sizeof(double) * Nm), *sv = (double *)malloc(sizeof(double) * Nm);
  double *sh = (double *)malloc(sizeof(double) * Nm), *tv = (double *)malloc(sizeof(double) * Nm);
  double *col = (double *)malloc(sizeof(double) * (size_t)N), *col2 = (double *)malloc(sizeof(double) * (size_t)N);
#define APPLY_M(src, dst, c)                                           \
  do {                                                                 \
    for (int64_t i_ = 0; i_ < N; ++i_) col[i_] = (src)[i_ * m + (c)];  \
    gb_solve(&Pt.S, 1, col);                                           \
    for (int64_t i_ = 0; i_ < N; ++i_) (dst)[i_ * m + (c)] = col[i_];  \
  } while (0)
#define APPLY_S(src, dst, c)                                           \
  do {                                                                 \
    for (int64_t i_ = 0; i_ < N; ++i_) col[i_] = (src)[i_ * m + (c)];  \
    red_matvec(&Pm, col, col2);                                        \
    for (int64_t i_ = 0; i_ < N; ++i_) (dst)[i_ * m + (c)] = col2[i_]; \
  } while (0)
  for (int c = 0; c < m; ++c) {
    APPLY_M(yr, xr, c);
    APPLY_S(xr, rv, c);
    for (int64_t i = 0; i < N; ++i) {
      rv[i * m + c] = yr[i * m + c] - rv[i * m + c];
      rh[i * m + c] = rv[i * m + c];
    }
    double nf = sqrt(col_dot(N, m, c, yr, yr));
    double rho_old = 1.0, alpha = 1.0, omega = 1.0;
    int it = 0;
    double nr = sqrt(col_dot(N, m, c, rv, rv));
    while (it < max_it && !(nr <= tol * nf)) {
      double rho = col_dot(N, m, c, rh, rv);
      double beta = (rho / rho_old) * (alpha / omega);
      for (int64_t i = 0; i < N; ++i) {
        size_t o = (size_t)(i * m + c);
        pv[o] = rv[o] + beta * (pv[o] - omega * vv[o]);
      }
      APPLY_M(pv, ph, c);
      APPLY_S(ph, vv, c);
      alpha = rho / col_dot(N, m, c, rh, vv);
      for (int64_t i = 0; i < N; ++i) {
        size_t o = (size_t)(i * m + c);
        sv[o] = rv[o] - alpha * vv[o];
      }
      APPLY_M(sv, sh, c);
      APPLY_S(sh, tv, c);
      double tt = col_dot(N, m, c, tv, tv);
      omega = tt > 0.0 ? col_dot(N, m, c, tv, sv) / tt : 0.0;
      for (int64_t i = 0; i < N; ++i) {
        size_t o = (size_t)(i * m + c);
        xr[o] += alpha * ph[o] + omega * sh[o];
        rv[o] = sv[o] - omega * tv[o];
      }
      rho_old = rho;
      ++it;
      nr = sqrt(col_dot(N, m, c, rv, rv));
      if (!(rho != 0.0 && omega != 0.0) && !(nr <= tol * nf)) break; /* breakdown */
    }
    if (iters) iters[c] = it;
    if (relres) relres[c] = nf > 0.0 ? nr / nf : 0.0;
  }
#undef APPLY_M
#undef APPLY_S
  plan_recover(&Pm, m, f, xr, x);
  free(yr); free(xr); free(rv); free(rh); free(pv); free(vv); free(ph); free(sv); free(sh); free(tv);
  free(col); free(col2);
  plan_free(&Pm);
  plan_free(&Pt);
  return 0;
}

/* The dense reduced system S~_red (order 2kp, row-major) at rank r. */
int orc_reduced_dense(int64_t n, int k, const double *bands, int p, int r, double *S) {
  orc_plan P;
  int rc = plan_build(&P, n, k, bands, p, r, 0, 1, 0, 0, NULL);
  if (rc) return rc;
  int64_t N = 2 * (int64_t)k * p;
  memset(S, 0, sizeof(double) * (size_t)(N * N));
  for (int64_t i = 0; i < N; ++i) S[i * N + i] = 1.0;
  size_t kk = (size_t)k * k;
  for (int j = 0; j < p; ++j) {
    int64_t rt = 2 * (int64_t)j * k, rb = rt + k;
    for (int a = 0; a < k; ++a)
      for (int b = 0; b < k; ++b) {
        if (j < p - 1) {
          int64_t col = 2 * (int64_t)(j + 1) * k + b;
          S[(rt + a) * N + col] = P.Vt[kk * j + a * k + b];
          S[(rb + a) * N + col] = P.Vb[kk * j + a * k + b];
        }
        if (j > 0) {
          int64_t col = (2 * (int64_t)(j - 1) + 1) * k + b;
          S[(rt + a) * N + col] = P.Wt[kk * j + a * k + b];
          S[(rb + a) * N + col] = P.Wb[kk * j + a * k + b];
        }
      }
  }
  plan_free(&P);
  return 0;
}

/* The full spikes of partition j (nj x k each, row-major); a spike that does
 * not exist (V of the last partition, W of the first) is returned as zeros. */
int orc_partition_spikes(int64_t n, int k, const double *bands, int p, int j,
                         double *V, double *W) {
  if (j < 0 || j >= p) return -5;
  int64_t *offs = (int64_t *)malloc(sizeof(int64_t) * (size_t)(p + 1));
  orc_partition(n, p, offs);
  int64_t s = offs[j], nj = offs[j + 1] - s;
  free(offs);
  gband A;
  if (gb_from_input(&A, n, k, bands, s, nj)) return -100;
  if (gb_factor(&A)) {
    gb_free(&A);
    return 1;
  }
  memset(V, 0, sizeof(double) * (size_t)(nj * k));
  memset(W, 0, sizeof(double) * (size_t)(nj * k));
  for (int a = 0; a < k; ++a)
    for (int b = 0; b < k; ++b) {
      if (j < p - 1) V[(nj - k + a) * k + b] = band_entry(n, k, bands, s + nj - k + a, s + nj + b);
      if (j > 0) W[a * k + b] = band_entry(n, k, bands, s + a, s - k + b);
    }
  gb_solve(&A, k, V);
  gb_solve(&A, k, W);
  gb_free(&A);
  return 0;
}

/* grad[(d+k) n + i] = - sum_c lam[i, c] x[i+d, c] on the band, zero outside. */
void orc_band_grad(int64_t n, int k, int m, const double *lam, const double *x,
                   double *grad) {
  for (int d = -k; d <= k; ++d)
    for (int64_t i = 0; i < n; ++i) {
      double s = 0.0;
      if (i + d >= 0 && i + d < n)
        for (int c = 0; c < m; ++c) s -= lam[i * m + c] * x[(i + d) * m + c];
      grad[(d + k) * n + i] = s;
    }
}
