// Rank-r form of the spike tips and the reduced interface system.
//
// Truncation (section "SVD representation of the spikes"): the rank-r SVD of
// a whole spike V_j = u Sigma v keeps the leading r right singular vectors
// Pi_j (k x r); its tips are V_{j,t} Pi_j Pi_j^T and V_{j,b} Pi_j Pi_j^T.  Pi_j
// is taken here from the eigen-decomposition of the Gram matrix V_j^T V_j
// (cyclic Jacobi), which has the same leading eigenvectors; at r = k the
// truncation is the identity and no decomposition is done.
//
// Reduced system (eq. spikered with the truncated tips; the SVD-accelerated
// products of eqs. per-partition_1/2).  With the compressed unknowns
//   a_j = Pi_j^T x_{j+1,t},  c_{j+1} = Psi_{j+1}^T x_{j,b}   (interface j = 0..p-2)
// and the projected tips P_{j,t/b} = V_{j,t/b} Pi_j, Q_{j,t/b} = W_{j,t/b} Psi_j,
// the truncated reduced system is equivalent to the block-tridiagonal system
// Z z = g of order 2 r (p - 1), z_j = [a_j; c_{j+1}]:
//   D_j = [[I, Pi_j^T Q_{j+1,t}], [Psi_{j+1}^T P_{j,b}, I]]        (diagonal)
//   E_j = [[Pi_j^T P_{j+1,t}, 0], [0, 0]]    couples z_{j+1}       (j + 1 <= p - 2)
//   F_j = [[0, 0], [0, Psi_{j+1}^T Q_{j,b}]] couples z_{j-1}       (j >= 1)
//   g_j = [Pi_j^T y_{j+1,t}; Psi_{j+1}^T y_{j,b}]
// and the tips follow as x_{j,t/b} = y_{j,t/b} - P_{j,t/b} a_j - Q_{j,t/b} c_j.
// Z is factored by block cyclic reduction (log2(p) levels, every level fully
// parallel) in FP64 for every precision.
#include "common.h"
#include "layout.h"

namespace lrs {

struct RedArgs {
  char* ws;
  Layout L;
  int level;      // cyclic-reduction level
  int m;          // solve columns
  int transpose;  // solve with Z^T
};

template <typename T>
__device__ inline T* rws(char* ws, size_t off) {
  return reinterpret_cast<T*>(ws + off);
}

// ------------------------------------------------------------------ Jacobi
// One wave per (partition, spike): eigen-decomposition of the K x K Gram
// matrix by cyclic Jacobi with a round-robin (parallel) pair ordering; writes
// the eigenvectors of the r largest eigenvalues as the columns of Pi (K x r).
template <int K>
__global__ __launch_bounds__(LRS_NT) void eigen_kernel(RedArgs a) {
  constexpr int LD = K + 1;
  constexpr int KE = (K % 2) ? K + 1 : K;  // players in the tournament
  __shared__ double G[K * LD], V[K * LD];
  __shared__ double cs[KE / 2], sn[KE / 2];
  __shared__ int pa[KE / 2], pb[KE / 2];
  __shared__ int order[K];
  __shared__ int s_done;
  const Layout& L = a.L;
  const int j = blockIdx.x, which = blockIdx.y;  // which: 0 = V (Pi), 1 = W (Psi)
  const int tid = threadIdx.x, r = L.r;
  double* Pi = rws<double>(a.ws, L.proj) + ((size_t)j * 2 + which) * K * r;
  const double* gram = rws<double>(a.ws, L.gram) + ((size_t)j * 2 + which) * K * K;
  for (int o = tid; o < K * K; o += blockDim.x) {
    int i = o / K, c = o % K;
    G[i * LD + c] = gram[o];
    V[i * LD + c] = (i == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 20; ++sweep) {
    // convergence: off-diagonal mass against the diagonal mass (Frobenius,
    // relative 1e-14: below that the entries are rounding noise of the Gram)
    {
      double off = 0.0, dia = 0.0;
      for (int o = tid; o < K * K; o += blockDim.x) {
        int i = o / K, c = o % K;
        double v = G[i * LD + c] * G[i * LD + c];
        if (i == c)
          dia += v;
        else
          off += v;
      }
      for (int w = 32; w >= 1; w >>= 1) {
        off += __shfl_xor(off, w);
        dia += __shfl_xor(dia, w);
      }
      if (tid == 0) s_done = (off <= 1e-28 * dia) ? 1 : 0;
    }
    __syncthreads();
    if (s_done) break;
    for (int step = 0; step < KE - 1; ++step) {
      if (tid < KE / 2) {
        // round-robin: player 0 fixed, the others rotate
        int q = tid;
        int x = (q == 0) ? 0 : 1 + (q - 1 + step) % (KE - 1);
        int y = 1 + (KE - 2 - q + step) % (KE - 1);
        int p1 = x < y ? x : y, p2 = x < y ? y : x;
        pa[q] = p1;
        pb[q] = p2;
        double c = 1.0, s = 0.0;
        if (p2 < K) {
          double apq = G[p1 * LD + p2];
          if (apq != 0.0) {
            double app = G[p1 * LD + p1], aqq = G[p2 * LD + p2];
            double theta = (aqq - app) / (2.0 * apq);
            double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
          }
        }
        cs[q] = c;
        sn[q] = s;
      }
      __syncthreads();
      // columns: G <- G J, V <- V J
      for (int o = tid; o < K * (KE / 2); o += blockDim.x) {
        int i = o / (KE / 2), q = o % (KE / 2);
        int p1 = pa[q], p2 = pb[q];
        if (p2 >= K) continue;
        double c = cs[q], s = sn[q];
        double g1 = G[i * LD + p1], g2 = G[i * LD + p2];
        G[i * LD + p1] = c * g1 - s * g2;
        G[i * LD + p2] = s * g1 + c * g2;
        double v1 = V[i * LD + p1], v2 = V[i * LD + p2];
        V[i * LD + p1] = c * v1 - s * v2;
        V[i * LD + p2] = s * v1 + c * v2;
      }
      __syncthreads();
      // rows: G <- J^T G
      for (int o = tid; o < K * (KE / 2); o += blockDim.x) {
        int i = o / (KE / 2), q = o % (KE / 2);
        int p1 = pa[q], p2 = pb[q];
        if (p2 >= K) continue;
        double c = cs[q], s = sn[q];
        double g1 = G[p1 * LD + i], g2 = G[p2 * LD + i];
        G[p1 * LD + i] = c * g1 - s * g2;
        G[p2 * LD + i] = s * g1 + c * g2;
      }
      __syncthreads();
    }
  }
  // order eigenvalues descending (stable: ties keep the lower index first)
  if (tid == 0) {
    for (int i = 0; i < K; ++i) order[i] = i;
    for (int i = 0; i < K; ++i) {
      int best = i;
      for (int c = i + 1; c < K; ++c)
        if (G[order[c] * LD + order[c]] > G[order[best] * LD + order[best]]) best = c;
      int t = order[i];
      order[i] = order[best];
      order[best] = t;
    }
  }
  __syncthreads();
  for (int o = tid; o < K * r; o += blockDim.x) {
    int i = o / r, q = o % r;
    Pi[i * r + q] = V[i * LD + order[q]];
  }
}

// Identity projectors (r = k): Pi = Psi = I.
template <int K>
__global__ void identity_proj_kernel(RedArgs a) {
  const Layout& L = a.L;
  const int j = blockIdx.x, r = L.r;
  double* Pi = rws<double>(a.ws, L.proj) + (size_t)j * 2 * K * r;
  for (int o = threadIdx.x; o < 2 * K * r; o += blockDim.x) {
    int e = o % (K * r), i = e / r, q = e % r;
    Pi[o] = (i == q) ? 1.0 : 0.0;
  }
}

// Projected tips P_t = V_t Pi, P_b = V_b Pi, Q_t = W_t Psi, Q_b = W_b Psi.
template <int K>
__global__ void project_kernel(RedArgs a) {
  const Layout& L = a.L;
  const int j = blockIdx.x, r = L.r;
  const double* tips = rws<double>(a.ws, L.tips) + (size_t)j * 4 * K * K;  // Vt Vb Wt Wb
  const double* proj = rws<double>(a.ws, L.proj) + (size_t)j * 2 * K * r;  // Pi Psi
  double* pt = rws<double>(a.ws, L.ptip) + (size_t)j * 4 * K * r;         // Pt Pb Qt Qb
  for (int o = threadIdx.x; o < 4 * K * r; o += blockDim.x) {
    int w = o / (K * r), e = o % (K * r), i = e / r, q = e % r;
    const double* tip = tips + (size_t)w * K * K;
    const double* P = proj + (size_t)(w / 2) * K * r;
    double s = 0.0;
    for (int l = 0; l < K; ++l) s += tip[i * K + l] * P[l * r + q];
    pt[o] = s;
  }
}

// ------------------------------------------------------------------ assembly
// One block per interface i: D_i, and level-0 F_i / E_i.
template <int K>
__global__ void zassemble_kernel(RedArgs a) {
  const Layout& L = a.L;
  const int i = blockIdx.x, r = L.r, R2 = L.R2, p = L.p;
  const double* proj = rws<double>(a.ws, L.proj);
  const double* ptip = rws<double>(a.ws, L.ptip);
  auto Pi = [&](int j) { return proj + (size_t)j * 2 * K * r; };
  auto Psi = [&](int j) { return proj + ((size_t)j * 2 + 1) * K * r; };
  auto PT = [&](int j, int w) { return ptip + ((size_t)j * 4 + w) * K * r; };  // 0 Pt 1 Pb 2 Qt 3 Qb
  double* D = rws<double>(a.ws, L.zD) + (size_t)i * R2 * R2;
  double* FE = rws<double>(a.ws, L.zFE) + (size_t)(L.lvl_off[0] + i) * 2 * R2 * R2;
  double* F = FE;
  double* E = FE + R2 * R2;
  for (int o = threadIdx.x; o < R2 * R2; o += blockDim.x) {
    int row = o / R2, col = o % R2;
    double d = 0.0, e = 0.0, f = 0.0;
    const int ra = row < r ? row : row - r, ca = col < r ? col : col - r;
    // proj^T tip: sum_l X[l][ra] * Y[l][ca]
    auto dot = [&](const double* X, const double* Y) {
      double s = 0.0;
      for (int l = 0; l < K; ++l) s += X[l * r + ra] * Y[l * r + ca];
      return s;
    };
    if (row < r && col < r) {
      d = (row == col) ? 1.0 : 0.0;
      if (i + 1 <= p - 2) e = dot(Pi(i), PT(i + 1, 0));  // Pi_i^T P_{i+1,t}
    } else if (row < r && col >= r) {
      d = dot(Pi(i), PT(i + 1, 2));  // Pi_i^T Q_{i+1,t}
    } else if (row >= r && col < r) {
      d = dot(Psi(i + 1), PT(i, 1));  // Psi_{i+1}^T P_{i,b}
    } else {
      d = (row == col) ? 1.0 : 0.0;
      if (i >= 1) f = dot(Psi(i + 1), PT(i, 3));  // Psi_{i+1}^T Q_{i,b}
    }
    D[o] = d;
    E[o] = e;
    F[o] = f;
  }
}

// ------------------------------------------------------------------ small dense LU
// Partial-pivoting LU of the R2 x R2 matrix M (LDS, pitch ld) by one workgroup.
__device__ inline void dense_lu(double* M, int ld, int R2, int* piv, int* latch, int part) {
  const int tid = threadIdx.x;
  for (int c = 0; c < R2; ++c) {
    if (tid == 0) {
      int best = c;
      double bv = fabs(M[c * ld + c]);
      for (int i = c + 1; i < R2; ++i)
        if (fabs(M[i * ld + c]) > bv) {
          bv = fabs(M[i * ld + c]);
          best = i;
        }
      piv[c] = best;
      if (bv == 0.0) latch_error(latch, 2, part, c);
    }
    __syncthreads();
    int pv = piv[c];
    if (pv != c)
      for (int col = tid; col < R2; col += blockDim.x) {
        double t = M[c * ld + col];
        M[c * ld + col] = M[pv * ld + col];
        M[pv * ld + col] = t;
      }
    __syncthreads();
    double d = M[c * ld + c];
    for (int i = c + 1 + tid; i < R2; i += blockDim.x) M[i * ld + c] /= d;
    __syncthreads();
    int w = R2 - c - 1;
    for (int o = tid; o < w * w; o += blockDim.x) {
      int i = c + 1 + o / w, col = c + 1 + o % w;
      M[i * ld + col] -= M[i * ld + c] * M[c * ld + col];
    }
    __syncthreads();
  }
}

// Solve (LU) X = B in place for B (R2 x nc, pitch ldb), LU in global or LDS.
// transpose: solve (LU)^T-form, i.e. D^T X = B for D = P L U.
// Columns are independent: one thread per column.
__device__ inline void lu_solve_cols(const double* LU, int ld, const int* piv, int R2, double* B,
                                     int ldb, int nc, bool transpose) {
  for (int c = threadIdx.x; c < nc; c += blockDim.x) {
    if (!transpose) {
      for (int i = 0; i < R2; ++i) {
        int pv = piv[i];
        if (pv != i) {
          double t = B[i * ldb + c];
          B[i * ldb + c] = B[pv * ldb + c];
          B[pv * ldb + c] = t;
        }
      }
      for (int i = 0; i < R2; ++i) {
        double s = B[i * ldb + c];
        for (int l = 0; l < i; ++l) s -= LU[i * ld + l] * B[l * ldb + c];
        B[i * ldb + c] = s;
      }
      for (int i = R2 - 1; i >= 0; --i) {
        double s = B[i * ldb + c];
        for (int l = i + 1; l < R2; ++l) s -= LU[i * ld + l] * B[l * ldb + c];
        B[i * ldb + c] = s / LU[i * ld + i];
      }
    } else {
      for (int i = 0; i < R2; ++i) {  // U^T y = b
        double s = B[i * ldb + c];
        for (int l = 0; l < i; ++l) s -= LU[l * ld + i] * B[l * ldb + c];
        B[i * ldb + c] = s / LU[i * ld + i];
      }
      for (int i = R2 - 1; i >= 0; --i) {  // L^T w = y
        double s = B[i * ldb + c];
        for (int l = i + 1; l < R2; ++l) s -= LU[l * ld + i] * B[l * ldb + c];
        B[i * ldb + c] = s;
      }
      for (int i = R2 - 1; i >= 0; --i) {
        int pv = piv[i];
        if (pv != i) {
          double t = B[i * ldb + c];
          B[i * ldb + c] = B[pv * ldb + c];
          B[pv * ldb + c] = t;
        }
      }
    }
  }
}

// ------------------------------------------------------------------ CR factorization
// Level l (stride s = 2^l), active rows i = 0, s, 2s, ... < NI.
// Odd rows (i/s odd) are eliminated: Dinv_i = D_i^{-1} (partial-pivoting LU,
// then solves against the identity), X^F_i = Dinv_i F_i, X^E_i = Dinv_i E_i
// replace (F_i, E_i) in the row's level slot.  Even rows survive:
//   D_i -= F_i X^E_{i-s} + E_i X^F_{i+s},  F_i' = -F_i X^F_{i-s},  E_i' = -E_i X^E_{i+s},
// and their level slot is overwritten by M^F_i = F_i Dinv_{i-s}, M^E_i = E_i Dinv_{i+s}.
// With these the four solves (Z, Z^T, forward and back substitution) are
// products of small dense blocks only.
__global__ __launch_bounds__(LRS_NT) void cr_odd_kernel(RedArgs a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double* M = reinterpret_cast<double*>(lds_raw);
  __shared__ int piv[128];
  const Layout& L = a.L;
  const int R2 = L.R2, s = 1 << a.level;
  const bool top = a.level >= L.levels;
  const int i = top ? 0 : (2 * blockIdx.x + 1) * s;
  if (i >= L.NI) return;
  const int ld = R2 + 1, ldx = 3 * R2 + 1;
  double* X = M + R2 * ld;
  int* latch = rws<int>(a.ws, L.latch);
  const double* D = rws<double>(a.ws, L.zD) + (size_t)i * R2 * R2;
  for (int o = threadIdx.x; o < R2 * R2; o += blockDim.x) M[o / R2 * ld + o % R2] = D[o];
  double* FE = top ? nullptr : rws<double>(a.ws, L.zFE) + (size_t)(L.lvl_off[a.level] + i / s) * 2 * R2 * R2;
  // right-hand sides [I | F | E]
  for (int o = threadIdx.x; o < R2 * 3 * R2; o += blockDim.x) {
    int row = o / (3 * R2), col = o % (3 * R2);
    double v;
    if (col < R2)
      v = (row == col) ? 1.0 : 0.0;
    else if (top)
      v = 0.0;
    else
      v = FE[(col < 2 * R2 ? 0 : R2 * R2) + row * R2 + (col < 2 * R2 ? col - R2 : col - 2 * R2)];
    X[row * ldx + col] = v;
  }
  __syncthreads();
  dense_lu(M, ld, R2, piv, latch, i);
  lu_solve_cols(M, ld, piv, R2, X, ldx, top ? R2 : 3 * R2, false);
  __syncthreads();
  double* Dinv = rws<double>(a.ws, L.zLU) + (size_t)i * R2 * R2;
  for (int o = threadIdx.x; o < R2 * R2; o += blockDim.x) Dinv[o] = X[o / R2 * ldx + o % R2];
  if (top) return;
  for (int o = threadIdx.x; o < 2 * R2 * R2; o += blockDim.x) {
    int which = o / (R2 * R2), e = o % (R2 * R2), row = e / R2, col = e % R2;
    FE[o] = X[row * ldx + R2 + which * R2 + col];  // [X^F | X^E]
  }
}

__global__ __launch_bounds__(LRS_NT) void cr_even_kernel(RedArgs a) {
  const Layout& L = a.L;
  const int R2 = L.R2, s = 1 << a.level;
  const int i = 2 * blockIdx.x * s;
  if (i >= L.NI) return;
  const bool hasL = i - s >= 0, hasR = i + s < L.NI;
  double* D = rws<double>(a.ws, L.zD) + (size_t)i * R2 * R2;
  double* FE = rws<double>(a.ws, L.zFE) + (size_t)(L.lvl_off[a.level] + i / s) * 2 * R2 * R2;
  double* FEn = rws<double>(a.ws, L.zFE) + (size_t)(L.lvl_off[a.level + 1] + i / (2 * s)) * 2 * R2 * R2;
  const double* F = FE;
  const double* E = FE + R2 * R2;
  auto slot = [&](int row) { return rws<double>(a.ws, L.zFE) + (size_t)(L.lvl_off[a.level] + row / s) * 2 * R2 * R2; };
  const double* XL = hasL ? slot(i - s) : nullptr;  // [X^F | X^E] of row i - s
  const double* XR = hasR ? slot(i + s) : nullptr;
  const double* DL = hasL ? rws<double>(a.ws, L.zLU) + (size_t)(i - s) * R2 * R2 : nullptr;
  const double* DR = hasR ? rws<double>(a.ws, L.zLU) + (size_t)(i + s) * R2 * R2 : nullptr;
  // pass 1: next-level blocks and the new D (reads F, E); M^F, M^E staged in
  // the row's scratch block until every thread is done reading F, E
  double* MS = rws<double>(a.ws, L.zX) + (size_t)i * 2 * R2 * R2;
  for (int o = threadIdx.x; o < R2 * R2; o += blockDim.x) {
    int row = o / R2, col = o % R2;
    double dd = 0.0, fn = 0.0, en = 0.0, mf = 0.0, me = 0.0;
    for (int l = 0; l < R2; ++l) {
      if (hasL) {
        double fl = F[row * R2 + l];
        dd += fl * XL[R2 * R2 + l * R2 + col];  // F X^E_{i-s}
        fn += fl * XL[l * R2 + col];            // F X^F_{i-s}
        mf += fl * DL[l * R2 + col];            // F Dinv_{i-s}
      }
      if (hasR) {
        double el = E[row * R2 + l];
        dd += el * XR[l * R2 + col];            // E X^F_{i+s}
        en += el * XR[R2 * R2 + l * R2 + col];  // E X^E_{i+s}
        me += el * DR[l * R2 + col];            // E Dinv_{i+s}
      }
    }
    D[o] -= dd;
    FEn[o] = -fn;
    FEn[R2 * R2 + o] = -en;
    MS[o] = mf;
    MS[R2 * R2 + o] = me;
  }
  __syncthreads();
  for (int o = threadIdx.x; o < 2 * R2 * R2; o += blockDim.x) FE[o] = MS[o];  // [M^F | M^E]
}

// ------------------------------------------------------------------ CR solves
// g (compressed vectors, [NI][R2][mmax]) is solved in place.
// Forward reduction at level l, even rows:
//   Z:    g_i -= M^F_i g_{i-s} + M^E_i g_{i+s}
//   Z^T:  g_i -= (X^E_{i-s})^T g_{i-s} + (X^F_{i+s})^T g_{i+s}
__global__ __launch_bounds__(LRS_NT) void crs_forward_kernel(RedArgs a) {
  const Layout& L = a.L;
  const int R2 = L.R2, s = 1 << a.level, m = a.m, mm = L.mmax;
  const int i = 2 * blockIdx.x * s;
  if (i >= L.NI) return;
  const bool hasL = i - s >= 0, hasR = i + s < L.NI;
  double* g = rws<double>(a.ws, L.zg);
  auto slot = [&](int row) { return rws<double>(a.ws, L.zFE) + (size_t)(L.lvl_off[a.level] + row / s) * 2 * R2 * R2; };
  const double* own = slot(i);
  for (int o = threadIdx.x; o < R2 * m; o += blockDim.x) {
    int row = o / m, c = o % m;
    double acc = 0.0;
    if (hasL) {
      const double* gl = g + (size_t)(i - s) * R2 * mm;
      if (!a.transpose) {
        for (int l = 0; l < R2; ++l) acc += own[row * R2 + l] * gl[l * mm + c];
      } else {
        const double* XE = slot(i - s) + R2 * R2;
        for (int l = 0; l < R2; ++l) acc += XE[l * R2 + row] * gl[l * mm + c];
      }
    }
    if (hasR) {
      const double* gr = g + (size_t)(i + s) * R2 * mm;
      if (!a.transpose) {
        for (int l = 0; l < R2; ++l) acc += own[R2 * R2 + row * R2 + l] * gr[l * mm + c];
      } else {
        const double* XF = slot(i + s);
        for (int l = 0; l < R2; ++l) acc += XF[l * R2 + row] * gr[l * mm + c];
      }
    }
    g[((size_t)i * R2 + row) * mm + c] -= acc;
  }
}

// Top (row 0 alone) and back substitution of the odd rows of level l:
//   Z:    g_i = Dinv_i g_i - X^F_i g_{i-s} - X^E_i g_{i+s}
//   Z^T:  g_i = Dinv_i^T g_i - (M^E_{i-s})^T g_{i-s} - (M^F_{i+s})^T g_{i+s}
__global__ __launch_bounds__(LRS_NT) void crs_backward_kernel(RedArgs a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double* Tg = reinterpret_cast<double*>(lds_raw);
  const Layout& L = a.L;
  const int R2 = L.R2, s = 1 << a.level, m = a.m, mm = L.mmax;
  const bool top = a.level >= L.levels;
  const int i = top ? 0 : (2 * blockIdx.x + 1) * s;
  if (i >= L.NI) return;
  double* g = rws<double>(a.ws, L.zg);
  auto slot = [&](int row) { return rws<double>(a.ws, L.zFE) + (size_t)(L.lvl_off[a.level] + row / s) * 2 * R2 * R2; };
  const bool hasL = !top && i - s >= 0, hasR = !top && i + s < L.NI;
  const double* Dinv = rws<double>(a.ws, L.zLU) + (size_t)i * R2 * R2;
  for (int o = threadIdx.x; o < R2 * m; o += blockDim.x) Tg[o] = g[((size_t)i * R2 + o / m) * mm + o % m];
  __syncthreads();
  for (int o = threadIdx.x; o < R2 * m; o += blockDim.x) {
    int row = o / m, c = o % m;
    double v = 0.0;
    for (int l = 0; l < R2; ++l) v += (a.transpose ? Dinv[l * R2 + row] : Dinv[row * R2 + l]) * Tg[l * m + c];
    if (hasL) {
      const double* gl = g + (size_t)(i - s) * R2 * mm;
      if (!a.transpose) {
        const double* XF = slot(i);
        for (int l = 0; l < R2; ++l) v -= XF[row * R2 + l] * gl[l * mm + c];
      } else {
        const double* ME = slot(i - s) + R2 * R2;
        for (int l = 0; l < R2; ++l) v -= ME[l * R2 + row] * gl[l * mm + c];
      }
    }
    if (hasR) {
      const double* gr = g + (size_t)(i + s) * R2 * mm;
      if (!a.transpose) {
        const double* XE = slot(i) + R2 * R2;
        for (int l = 0; l < R2; ++l) v -= XE[row * R2 + l] * gr[l * mm + c];
      } else {
        const double* MF = slot(i + s);
        for (int l = 0; l < R2; ++l) v -= MF[l * R2 + row] * gr[l * mm + c];
      }
    }
    g[((size_t)i * R2 + row) * mm + c] = v;
  }
}

// ------------------------------------------------------------------ compressed rhs
// Z:   g_j = [Pi_j^T y_{j+1,t}; Psi_{j+1}^T y_{j,b}]
// Z^T: g_j = L^T h with h_{(j,t)} = B_{j-1}^T nu_{j-1,b}, h_{(j,b)} = C_{j+1}^T nu_{j+1,t}:
//   (a_j)     = P_{j,t}^T h_{(j,t)} + P_{j,b}^T h_{(j,b)}
//   (c_{j+1}) = Q_{j+1,t}^T h_{(j+1,t)} + Q_{j+1,b}^T h_{(j+1,b)}
template <int K>
__global__ void zrhs_kernel(RedArgs a, const double* bands) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double* H = reinterpret_cast<double*>(lds_raw);  // up to 4 vectors K x m
  const Layout& L = a.L;
  const int i = blockIdx.x, r = L.r, m = a.m, mm = L.mmax, p = L.p, k = L.k;
  const double* ytip = rws<double>(a.ws, L.ytip);
  const double* proj = rws<double>(a.ws, L.proj);
  const double* ptip = rws<double>(a.ws, L.ptip);
  double* g = rws<double>(a.ws, L.zg) + (size_t)i * L.R2 * mm;
  auto yt = [&](int j, int w) { return ytip + ((size_t)j * 2 + w) * K * mm; };
  if (!a.transpose) {
    for (int o = threadIdx.x; o < 2 * r * m; o += blockDim.x) {
      int row = o / m, c = o % m;
      double s = 0.0;
      if (row < r) {
        const double* Pi = proj + (size_t)i * 2 * K * r;
        const double* y = yt(i + 1, 0);
        for (int l = 0; l < K; ++l) s += Pi[l * r + row] * y[l * mm + c];
      } else {
        const double* Psi = proj + ((size_t)(i + 1) * 2 + 1) * K * r;
        const double* y = yt(i, 1);
        for (int l = 0; l < K; ++l) s += Psi[l * r + row - r] * y[l * mm + c];
      }
      g[row * mm + c] = s;
    }
    return;
  }
  // h vectors: H0 = h_{(i,t)}, H1 = h_{(i,b)}, H2 = h_{(i+1,t)}, H3 = h_{(i+1,b)}
  auto hvec = [&](int jj, bool top, double* out) {
    // h_{(jj,t)} = B_{jj-1}^T nu_{jj-1,b} (jj >= 1);  h_{(jj,b)} = C_{jj+1}^T nu_{jj+1,t} (jj <= p-2)
    Geom gj = part_geom(L.n, p, jj, K);
    for (int o = threadIdx.x; o < K * m; o += blockDim.x) {
      int row = o / m, c = o % m;
      double s = 0.0;
      if (top && jj >= 1) {
        const double* nu = yt(jj - 1, 1);
        for (int l = 0; l < K; ++l) s += band_at(bands, L.n, k, gj.s - K + l, gj.s + row) * nu[l * mm + c];
      } else if (!top && jj <= p - 2) {
        const double* nu = yt(jj + 1, 0);
        const int64_t s1 = gj.s + gj.nj;
        for (int l = 0; l < K; ++l) s += band_at(bands, L.n, k, s1 + l, s1 - K + row) * nu[l * mm + c];
      }
      out[row * m + c] = s;
    }
  };
  hvec(i, true, H);
  hvec(i, false, H + K * m);
  hvec(i + 1, true, H + 2 * K * m);
  hvec(i + 1, false, H + 3 * K * m);
  __syncthreads();
  auto PT = [&](int j, int w) { return ptip + ((size_t)j * 4 + w) * K * r; };
  for (int o = threadIdx.x; o < 2 * r * m; o += blockDim.x) {
    int row = o / m, c = o % m;
    double s = 0.0;
    if (row < r) {
      const double* Pt = PT(i, 0);
      const double* Pb = PT(i, 1);
      for (int l = 0; l < K; ++l) s += Pt[l * r + row] * H[l * m + c] + Pb[l * r + row] * H[K * m + l * m + c];
    } else {
      const double* Qt = PT(i + 1, 2);
      const double* Qb = PT(i + 1, 3);
      int q = row - r;
      for (int l = 0; l < K; ++l)
        s += Qt[l * r + q] * H[2 * K * m + l * m + c] + Qb[l * r + q] * H[3 * K * m + l * m + c];
    }
    g[row * mm + c] = s;
  }
}

}  // namespace lrs
