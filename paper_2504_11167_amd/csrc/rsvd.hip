// Randomized SVD of the spikes (section "SVD representation of the spikes":
// the proto-algorithm of Halko, Martinsson and Tropp, a few passes over the
// spike, oversampled sketch).  For the spike V_j = A_j^{-1} [0; B_j] (and W_j
// = A_j^{-1} [C_j; 0] alike) and a caller-drawn Gaussian Omega (k x ell):
//   Y = (V V^T)^q V Omega:  solves with ell columns instead of k
//       (V X = A_j^{-1} [0; B_j X]: a block-diagonal solve of a right-hand
//        side that is nonzero in the coupling rows only),
//   V^T Y = B_j^T (A_j^{-T} Y)_bottom:  an adjoint solve of which only the
//       tips are kept,
//   Q = Y_S R^{-1} with Y_S^T Y_S = R^T R (Cholesky of the Gram Y^T Y with
//       diagonal pivoting; sketch directions whose residual norm falls below
//       1e-6 of the largest column are dropped as numerically dependent),
//   B = Q^T V = R^{-T} (V^T Y_S)^T,  Q Q^T V = Y_S T with T = R^{-1} B  (ell' x k).
// The truncation then proceeds as for the whole spike, on Q Q^T V: its tips
// Y_{S,t} T, Y_{S,b} T go to the tip slots; its Gram (Q Q^T V)^T (Q Q^T V) =
// B^T B has rank ell' only, so instead of that K x K matrix (whose K - ell'
// zero eigenvalues would only slow the Jacobi sweeps) the eigensolver takes
// R_h R_h^T from the thin QR B^T = Q_b R_h (ell' x ell'), and the right
// singular vectors of B are Q_b times its eigenvectors (rsvd_lift_kernel).
//
// Column conventions: the oracle-style k columns of a spike map to the
// K-padded spike columns b (V) and K - k + b (W), as in the spike sweeps.
#pragma once
#include "common.h"
#include "layout.h"

namespace lrs {

struct RsvdArgs {
  const double* bands;
  char* ws;
  Layout L;
  const double* om;  // [p][2][k][ell]: Omega on the first pass, V^T Y (W^T Y) on a power step
};

template <typename T>
__device__ inline T* rsw(char* ws, size_t off) {
  return reinterpret_cast<T*>(ws + off);
}

// Sketch right-hand side, row-major n x 2 ell: rows of partition j carry
// B_j Om_{j,V} in its last k rows (columns [0, ell)) and C_j Om_{j,W} in its
// first k rows (columns [ell, 2 ell)); every other entry is zero.
// Grid (p, chunks), rows of a partition in chunks of 64.
__global__ __launch_bounds__(256) void rsvd_rhs_kernel(RsvdArgs a) {
  const Layout& L = a.L;
  const int j = blockIdx.x, ell = L.ell, w = 2 * ell, k = L.k;
  const Geom g = part_geom(L, j, L.K);
  double* Y = rsw<double>(a.ws, L.ysk);
  const double* omv = a.om + ((size_t)j * 2 + 0) * k * ell;
  const double* omw = a.om + ((size_t)j * 2 + 1) * k * ell;
  constexpr int ROWS = 64;
  for (int r0 = blockIdx.y * ROWS; r0 < g.nj; r0 += gridDim.y * ROWS)
    for (int o = threadIdx.x; o < ROWS * w; o += blockDim.x) {
      const int li = r0 + o / w, c = o % w;
      if (li >= g.nj) continue;
      const int64_t i = g.s + li;
      double v = 0.0;
      if (c < ell) {
        if (j < L.p - 1 && li >= g.nj - k)
          for (int b = 0; b < k; ++b) v += band_at(a.bands, L.n, k, i, g.s + g.nj + b) * omv[b * ell + c];
      } else if (j > 0 && li < k) {
        for (int b = 0; b < k; ++b) v += band_at(a.bands, L.n, k, i, g.s - k + b) * omw[b * ell + c - ell];
      }
      Y[i * w + c] = v;
    }
}

// Gram Y_s^T Y_s of one partition's sketch (s = 0: V, 1: W), ell x ell,
// over 64-row chunks staged in LDS: thread t accumulates the 4 x 4 block
// t mod nblk of the Gram (nblk = ceil(ell / 4)^2 <= 256) over every
// (256 / nblk)-th row of a chunk, and the row groups are summed at the end.
// Grid (p, 2), 256 threads.
__global__ __launch_bounds__(256) void rsvd_gram_kernel(RsvdArgs a) {
  constexpr int ROWS = 64, LP = 65;
  __shared__ double ys[ROWS * LP];
  const Layout& L = a.L;
  const int j = blockIdx.x, s = blockIdx.y, ell = L.ell, w = 2 * ell, tid = threadIdx.x;
  const int nbk = (ell + 3) / 4, nblk = nbk * nbk, groups = 256 / nblk;
  const int blk = tid % nblk, grp = tid / nblk, bi = 4 * (blk / nbk), bj = 4 * (blk % nbk);
  const bool active = grp < groups;
  const Geom g = part_geom(L, j, L.K);
  const double* Y = rsw<double>(a.ws, L.ysk) + (size_t)g.s * w + s * ell;
  double acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
  for (int r0 = 0; r0 < g.nj; r0 += ROWS) {
    const int nr = min(ROWS, g.nj - r0);
    for (int o = tid; o < ROWS * 4 * nbk; o += blockDim.x) {
      const int rr = o / (4 * nbk), c = o % (4 * nbk);
      ys[rr * LP + c] = (rr < nr && c < ell) ? Y[(size_t)(r0 + rr) * w + c] : 0.0;
    }
    __syncthreads();
    if (active)
      for (int rr = grp; rr < ROWS; rr += groups) {
        double x[4], y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          x[u] = ys[rr * LP + bi + u];
          y[u] = ys[rr * LP + bj + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[u][v] = fma(x[u], y[v], acc[u][v]);
      }
    __syncthreads();
  }
  // sum the row groups (fixed order) through the staging buffer
  double* red = ys;  // groups x nblk x 16 <= 256 x 16 doubles
  if (active)
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) red[(grp * nblk + blk) * 16 + u * 4 + v] = acc[u][v];
  __syncthreads();
  double* G = rsw<double>(a.ws, L.rgy) + ((size_t)j * 2 + s) * ell * ell;
  for (int o = tid; o < nblk * 16; o += blockDim.x) {
    const int bb = o / 16, e = o % 16, row = 4 * (bb / nbk) + e / 4, col = 4 * (bb % nbk) + e % 4;
    double sum = 0.0;
    for (int q = 0; q < groups; ++q) sum += red[(q * nblk + bb) * 16 + e];
    if (row < ell && col < ell) G[row * ell + col] = sum;
  }
}

// V^T Y = B_j^T nu_b and W^T Y = C_j^T nu_t from the adjoint solve's tips
// nu = A_j^{-T} Y (tip buffer: first and last K real rows, row stride mmax),
// k x ell each, to the [p][2][k][ell] buffer (zero for the absent V_{p-1},
// W_0).  Grid (p, 2).
__global__ __launch_bounds__(256) void rsvd_vty_kernel(RsvdArgs a) {
  const Layout& L = a.L;
  const int j = blockIdx.x, s = blockIdx.y, ell = L.ell, k = L.k, K = L.K;
  const Geom g = part_geom(L, j, K);
  const double* yt = rsw<double>(a.ws, L.ytip) + (size_t)j * 2 * K * L.mmax;
  double* M = rsw<double>(a.ws, L.rmv) + ((size_t)j * 2 + s) * k * ell;
  const bool present = s == 0 ? j < L.p - 1 : j > 0;
  for (int o = threadIdx.x; o < k * ell; o += blockDim.x) {
    const int b = o / ell, c = o % ell;
    double v = 0.0;
    if (present) {
      if (s == 0) {  // B_j[a][b] = A[s_j + nj - K + a, s_j + nj + b], nu_b rows a, columns [0, ell)
        const int64_t r0 = g.s + g.nj - K, c0 = g.s + g.nj;
        for (int q = 0; q < K; ++q)
          v += band_at(a.bands, L.n, k, r0 + q, c0 + b) * yt[((size_t)K + q) * L.mmax + c];
      } else {       // C_j[a][b] = A[s_j + a, s_j - k + b], nu_t rows a, columns [ell, 2 ell)
        for (int q = 0; q < K; ++q)
          v += band_at(a.bands, L.n, k, g.s + q, g.s - k + b) * yt[(size_t)q * L.mmax + ell + c];
      }
    }
    M[o] = v;
  }
}

// Order of the small eigenproblem: the smallest power of two >= ell.
__host__ __device__ constexpr int rsvd_ke(int ell) { return ell <= 1 ? 1 : (ell <= 2 ? 2 : (ell <= 4 ? 4 : (ell <= 8 ? 8 : (ell <= 16 ? 16 : (ell <= 32 ? 32 : 64))))); }

// Per (partition, spike): pivoted Cholesky Y_S^T Y_S = R^T R, B = Q^T V =
// R^{-T} M_S^T and T = R^{-1} B; the thin QR B^T = Q_b R_h by Gram-Schmidt
// with reorthogonalization (Q_b, k x ell, over the consumed V^T Y slot;
// R_h R_h^T, KE x KE with KE = rsvd_ke(ell), zero-padded, into the Gram
// slot), and the tips Y_{S,t/b} T of Q Q^T V into the tip slots (K x K,
// padded columns).  Grid (p, 2), 256 threads; dynamic LDS of
// rsvd_small_lds(ell, k) bytes.
__host__ __device__ constexpr size_t rsvd_small_lds(int ell, int k) {
  return ((size_t)ell * (ell + 1) + (size_t)ell * ell + 2 * (size_t)ell * (k + 1) + 64 + 64) * sizeof(double);
}

__global__ __launch_bounds__(256) void rsvd_small_kernel(RsvdArgs a) {
  extern __shared__ __align__(16) double rs_lds[];
  __shared__ int perm[64];
  __shared__ int s_go, s_best;
  __shared__ double s_dmax;
  const Layout& L = a.L;
  const int j = blockIdx.x, s = blockIdx.y, ell = L.ell, k = L.k, K = L.K, tid = threadIdx.x;
  const int LG = ell + 1, LM = k + 1, w = 2 * ell;
  double* G = rs_lds;          // ell x LG, the sketch Gram
  double* R = G + ell * LG;    // ell x ell: R[t * ell + u], row t, pivot position u (upper triangle)
  double* Tm = R + ell * ell;  // ell x LM: M_S^T, then Z = R^{-T} M_S^T, then T = R^{-1} Z
  double* d = Tm + ell * LM;   // residual diagonal by sketch column
  double* Qb = d + 64;         // ell x LM: rows of Q_b^T (orthonormal rows spanning those of B)
  double* Rh = G;              // ell x ell: R_h[v * ell + u] (upper triangle; over G, free after the Cholesky)
  double* cf = Qb + ell * LM;  // 64 Gram-Schmidt coefficients
  __shared__ double s_inv, s_bn;
  const Geom g = part_geom(L, j, K);
  const double* Gg = rsw<double>(a.ws, L.rgy) + ((size_t)j * 2 + s) * ell * ell;
  const double* M = rsw<double>(a.ws, L.rmv) + ((size_t)j * 2 + s) * k * ell;
  const double* Y = rsw<double>(a.ws, L.ysk) + s * ell;
  for (int o = tid; o < ell * ell; o += blockDim.x) {
    G[(o / ell) * LG + o % ell] = Gg[o];
    R[o] = 0.0;
  }
  if (tid < ell) perm[tid] = tid;
  __syncthreads();
  if (tid < ell) d[tid] = G[tid * LG + tid];
  __syncthreads();
  if (tid == 0) {
    double dm = 0.0;
    for (int i = 0; i < ell; ++i) dm = fmax(dm, d[i]);
    s_dmax = dm;
  }
  __syncthreads();
  int lp = 0;
  for (int t = 0; t < ell; ++t) {
    if (tid == 0) {
      int best = t;
      for (int u = t + 1; u < ell; ++u)
        if (d[perm[u]] > d[perm[best]]) best = u;
      s_go = d[perm[best]] > 1e-12 * s_dmax;  // false for a zero (absent) spike and for NaN
      if (s_go) {
        const int tp = perm[t];
        perm[t] = perm[best];
        perm[best] = tp;
      }
      s_best = best;
    }
    __syncthreads();
    if (!s_go) break;
    const int best = s_best;
    if (best != t)  // the rows above t follow the column swap
      for (int v = tid; v < t; v += blockDim.x) {
        const double x = R[v * ell + t];
        R[v * ell + t] = R[v * ell + best];
        R[v * ell + best] = x;
      }
    __syncthreads();
    const int pi = perm[t];
    const double rt = sqrt(d[pi]);
    for (int u = t + 1 + tid; u < ell; u += blockDim.x) {
      const int i = perm[u];
      double sum = G[pi * LG + i];
      for (int v = 0; v < t; ++v) sum -= R[v * ell + t] * R[v * ell + u];
      const double e = sum / rt;
      R[t * ell + u] = e;
      d[i] -= e * e;
    }
    if (tid == 0) R[t * ell + t] = rt;
    __syncthreads();
    lp = t + 1;
  }
  // T = (R^T R)^{-1} M_S^T, one column b per thread
  for (int o = tid; o < lp * k; o += blockDim.x) {
    const int u = o / k, b = o % k;
    Tm[u * LM + b] = M[b * ell + perm[u]];
  }
  __syncthreads();
  for (int b = tid; b < k; b += blockDim.x)
    for (int u = 0; u < lp; ++u) {  // Z = R^{-T} M_S^T = Q^T V = B
      double z = Tm[u * LM + b];
      for (int v = 0; v < u; ++v) z -= R[v * ell + u] * Tm[v * LM + b];
      Tm[u * LM + b] = z / R[u * ell + u];
    }
  __syncthreads();
  // thin QR of B^T: Gram-Schmidt over the rows b_u of B, each projection
  // pass done twice; a row whose remaining norm falls below 1e-13 of the
  // largest row norm is dependent and leaves a zero row of Q_b^T
  for (int o = tid; o < ell * ell; o += blockDim.x) Rh[o] = 0.0;
  if (tid == 0) {
    double bm = 0.0;
    for (int u = 0; u < lp; ++u) {
      double nn = 0.0;
      for (int b = 0; b < k; ++b) nn += Tm[u * LM + b] * Tm[u * LM + b];
      bm = fmax(bm, nn);
    }
    s_bn = sqrt(bm);
  }
  for (int u = 0; u < lp; ++u) {
    for (int b = tid; b < k; b += blockDim.x) Qb[u * LM + b] = Tm[u * LM + b];
    for (int pass = 0; pass < 2; ++pass) {
      __syncthreads();
      for (int v = tid; v < u; v += blockDim.x) {
        double c = 0.0;
        for (int b = 0; b < k; ++b) c += Qb[v * LM + b] * Qb[u * LM + b];
        cf[v] = c;
      }
      __syncthreads();
      for (int b = tid; b < k; b += blockDim.x) {
        double x = Qb[u * LM + b];
        for (int v = 0; v < u; ++v) x -= cf[v] * Qb[v * LM + b];
        Qb[u * LM + b] = x;
      }
      for (int v = tid; v < u; v += blockDim.x) Rh[v * ell + u] += cf[v];
    }
    __syncthreads();
    if (tid == 0) {
      double nn = 0.0;
      for (int b = 0; b < k; ++b) nn += Qb[u * LM + b] * Qb[u * LM + b];
      const double nr = sqrt(nn);
      const bool ok = nr > 1e-13 * s_bn;
      Rh[u * ell + u] = ok ? nr : 0.0;
      s_inv = ok ? 1.0 / nr : 0.0;
    }
    __syncthreads();
    for (int b = tid; b < k; b += blockDim.x) Qb[u * LM + b] *= s_inv;
  }
  __syncthreads();
  // R_h R_h^T (the nonzero eigenvalues of B^T B), zero-padded to KE x KE,
  // and Q_b (k x ell, row b = spike column b) over M, which is consumed
  {
    const int KE = rsvd_ke(ell);
    double* gram = rsw<double>(a.ws, L.gram) + ((size_t)j * 2 + s) * KE * KE;
    for (int o = tid; o < KE * KE; o += blockDim.x) {
      const int u1 = o / KE, u2 = o % KE;
      double gv = 0.0;
      if (u1 < lp && u2 < lp)
        for (int u = max(u1, u2); u < lp; ++u) gv += Rh[u1 * ell + u] * Rh[u2 * ell + u];
      gram[o] = gv;
    }
    double* qm = rsw<double>(a.ws, L.rmv) + ((size_t)j * 2 + s) * k * ell;
    for (int o = tid; o < k * ell; o += blockDim.x) {
      const int b = o / ell, u = o % ell;
      qm[o] = u < lp ? Qb[u * LM + b] : 0.0;
    }
  }
  __syncthreads();
  for (int b = tid; b < k; b += blockDim.x)
    for (int u = lp - 1; u >= 0; --u) {  // T = R^{-1} Z
      double z = Tm[u * LM + b];
      for (int v = u + 1; v < lp; ++v) z -= R[u * ell + v] * Tm[v * LM + b];
      Tm[u * LM + b] = z / R[u * ell + u];
    }
  __syncthreads();
  // tips of Q Q^T V: Y_{S,t} T, Y_{S,b} T
  const int cof = s == 0 ? 0 : K - k;  // padded column of spike column 0
  double* tt = rsw<double>(a.ws, L.tips) + ((size_t)j * 4 + 2 * s) * K * K;
  double* tb = tt + (size_t)K * K;
  for (int o = tid; o < K * K; o += blockDim.x) {
    const int i = o / K, b2 = o % K - cof;
    double vt = 0.0, vb = 0.0;
    if (b2 >= 0 && b2 < k)
      for (int u = 0; u < lp; ++u) {
        const double tv = Tm[u * LM + b2];
        const int col = perm[u];
        vt += Y[(size_t)(g.s + i) * w + col] * tv;
        vb += Y[(size_t)(g.s + g.nj - K + i) * w + col] * tv;
      }
    tt[o] = vt;
    tb[o] = vb;
  }
}

// Projectors of the randomized truncation: Pi (K x r, padded rows) = Q_b W,
// W (KE x r) the eigenvectors of R_h R_h^T for the r largest eigenvalues
// (written by the eigensolver at W, KE x r per (partition, spike)); rows
// outside the spike's k columns are zero.  Grid (p, 2), 256 threads.
__global__ __launch_bounds__(256) void rsvd_lift_kernel(RsvdArgs a, const double* W) {
  const Layout& L = a.L;
  const int j = blockIdx.x, s = blockIdx.y, ell = L.ell, k = L.k, K = L.K, r = L.r, KE = rsvd_ke(ell);
  const int cof = s == 0 ? 0 : K - k;
  const double* qm = rsw<double>(a.ws, L.rmv) + ((size_t)j * 2 + s) * k * ell;
  const double* w = W + ((size_t)j * 2 + s) * KE * r;
  double* pi = rsw<double>(a.ws, L.proj) + ((size_t)j * 2 + s) * K * r;
  for (int o = threadIdx.x; o < K * r; o += blockDim.x) {
    const int i = o / r, q = o % r, b = i - cof;
    double v = 0.0;
    if (b >= 0 && b < k)
      for (int u = 0; u < ell; ++u) v += qm[b * ell + u] * w[u * r + q];
    pi[o] = v;
  }
}

}  // namespace lrs
