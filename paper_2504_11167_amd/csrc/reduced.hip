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
//
// LR-SPIKE-T (the truncated-SPIKE system S~~_red of eqs. truncated_redsys,
// red_sys_prec_mid_1/2, red_sys_1, red_sys_mid, red_sys_3) drops V~_{j,t} and
// W~_{j,b}: in the compressed form that removes E_j and F_j, so every
// interface j is the independent system D_j z_j = g_j (solved here by the
// inverse of D_j: the 2r x 2r counterpart of the block inversion the paper
// writes with the Schur complement M_i), and the tips keep only their own
// interface's term: x_{j,b} = y_{j,b} - P_{j,b} a_j, x_{j+1,t} = y_{j+1,t} -
// Q_{j+1,t} c_{j+1}.
#include "common.h"
#include "layout.h"

namespace lrs {

struct RedArgs {
  char* ws;
  Layout L;
  int level;      // cyclic-reduction level; -1 = LR-SPIKE-T: every interface block on its own
  int m;          // solve columns
  int transpose;  // solve with Z^T
  const int* gate;  // refinement: nonzero *gate = no-op (null = always run)
};

template <typename T>
__device__ inline T* rws(char* ws, size_t off) {
  return reinterpret_cast<T*>(ws + off);
}

// ------------------------------------------------------------------ Jacobi
// One wave per (partition, spike): eigen-decomposition of the K x K Gram
// matrix by cyclic Jacobi with a round-robin (parallel) pair ordering; writes
// the eigenvectors of the r largest eigenvalues as the columns of Pi (K x r).
// Launched with LRS_NT threads.
template <int K>
__global__ __launch_bounds__(LRS_NT) __attribute__((aligned(4096))) void eigen_kernel(RedArgs a) {
  constexpr int LD = K + 1;
  constexpr int KE = (K % 2) ? K + 1 : K;  // players in the tournament
  extern __shared__ __align__(16) double eig_lds[];  // G and V, K x LD each (dynamic: 66.5 KB at K = 64)
  double* G = eig_lds;
  double* V = eig_lds + K * LD;
  __shared__ double cs[KE / 2], sn[KE / 2];
  __shared__ int pa[KE / 2], pb[KE / 2];
  __shared__ int order[K];
  __shared__ int s_done;
  __shared__ double s_red[2 * (LRS_NT / 64)];
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
      if ((tid & 63) == 0) {
        s_red[2 * (tid >> 6)] = off;
        s_red[2 * (tid >> 6) + 1] = dia;
      }
      __syncthreads();
      if (tid == 0) {
        double so = 0.0, sd = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
          so += s_red[2 * w];
          sd += s_red[2 * w + 1];
        }
        s_done = (so <= 1e-28 * sd) ? 1 : 0;
      }
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
      // G <- J^T G J one 2 x 2 block (rows of pair qa, columns of pair qb) per
      // item: the column rotation of pair qb, then the row rotation of pair qa,
      // in registers (one pass over G per step); V <- V J alongside
      for (int o = tid; o < (KE / 2) * (KE / 2); o += blockDim.x) {
        const int qa = o / (KE / 2), qb = o % (KE / 2);
        const int r1 = pa[qa], r2 = pb[qa], c1 = pa[qb], c2 = pb[qb];
        const bool hr = r2 < K, hc = c2 < K;  // false only for the idle player of odd K
        const double cr = cs[qa], sr = sn[qa], cc = cs[qb], sc = sn[qb];
        const double g11 = G[r1 * LD + c1], g12 = hc ? G[r1 * LD + c2] : 0.0;
        const double g21 = hr ? G[r2 * LD + c1] : 0.0, g22 = (hr && hc) ? G[r2 * LD + c2] : 0.0;
        const double a11 = cc * g11 - sc * g12, a12 = sc * g11 + cc * g12;
        const double a21 = cc * g21 - sc * g22, a22 = sc * g21 + cc * g22;
        G[r1 * LD + c1] = cr * a11 - sr * a21;
        if (hc) G[r1 * LD + c2] = cr * a12 - sr * a22;
        if (hr) G[r2 * LD + c1] = sr * a11 + cr * a21;
        if (hr && hc) G[r2 * LD + c2] = sr * a12 + cr * a22;
      }
      for (int o = tid; o < K * (KE / 2); o += blockDim.x) {
        int i = o / (KE / 2), q = o % (KE / 2);
        int p1 = pa[q], p2 = pb[q];
        if (p2 >= K) continue;
        double c = cs[q], s = sn[q];
        double v1 = V[i * LD + p1], v2 = V[i * LD + p2];
        V[i * LD + p1] = c * v1 - s * v2;
        V[i * LD + p2] = s * v1 + c * v2;
      }
      __syncthreads();
    }
  }
  // order eigenvalues descending (stable: ties keep the lower index first):
  // lane i places itself at its rank
  if (tid < K) {
    // a NaN eigenvalue (non-finite spike; latched later in the reduced
    // system) ranks last, so that the ranks stay a permutation
    auto eig = [&](int c) {
      const double v = G[c * LD + c];
      return v == v ? v : -INFINITY;
    };
    const double di = eig(tid);
    int rank = 0;
    for (int c = 0; c < K; ++c) {
      const double dc = eig(c);
      rank += (dc > di || (dc == di && c < tid)) ? 1 : 0;
    }
    order[rank] = tid;
  }
  __syncthreads();
  // diagnostic: relative singular-value gap at the truncation,
  // (sigma_r - sigma_{r+1}) / sigma_1 with sigma = sqrt(eigenvalue); a spike
  // that is zero (no coupling block) has none
  if (tid == 0 && r > 0 && r < K) {
    auto sig = [&](int q) { return sqrt(fmax(G[order[q] * LD + order[q]], 0.0)); };
    const double s1 = sig(0);
    if (s1 > 0.0) state_min(rws<int>(a.ws, L.latch), S_GAPMIN, fmax((sig(r - 1) - sig(r)) / s1, 0.0));
  }
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
  double zmax = 0.0;
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
    if (L.variant) e = f = 0.0;  // LR-SPIKE-T: no coupling between interfaces
    D[o] = d;
    E[o] = e;
    F[o] = f;
    zmax = fmax(zmax, fmax(fabs(d), fmax(fabs(e), fabs(f))));
  }
  zmax = wave_max(zmax);
  if ((threadIdx.x & 63) == 0) state_max(rws<int>(a.ws, L.latch), S_ZMAX, zmax);
}

// ------------------------------------------------------------------ block products
// C (R x N) from sum_l a(i, l) b(l, j) over l < Kd, by one 256-thread
// workgroup: every thread owns TS x TS register tiles of C; a and b read LDS.
// `out(i, j, v)` receives each finished element.
template <int TS, typename FA, typename FB, typename FO>
__device__ inline void block_mm_ts(int R, int N, int Kd, FA a, FB b, FO out) {
  const int ntj = (N + TS - 1) / TS, nt = ((R + TS - 1) / TS) * ntj;
  for (int t = threadIdx.x; t < nt; t += blockDim.x) {
    const int i0 = (t / ntj) * TS, j0 = (t % ntj) * TS;
    double acc[TS][TS];
#pragma unroll
    for (int u = 0; u < TS; ++u)
#pragma unroll
      for (int v = 0; v < TS; ++v) acc[u][v] = 0.0;
    for (int l = 0; l < Kd; ++l) {
      double av[TS], bv[TS];
#pragma unroll
      for (int u = 0; u < TS; ++u) av[u] = (i0 + u < R) ? a(i0 + u, l) : 0.0;
#pragma unroll
      for (int v = 0; v < TS; ++v) bv[v] = (j0 + v < N) ? b(l, j0 + v) : 0.0;
#pragma unroll
      for (int u = 0; u < TS; ++u)
#pragma unroll
        for (int v = 0; v < TS; ++v) acc[u][v] = fma(av[u], bv[v], acc[u][v]);
    }
#pragma unroll
    for (int u = 0; u < TS; ++u)
#pragma unroll
      for (int v = 0; v < TS; ++v)
        if (i0 + u < R && j0 + v < N) out(i0 + u, j0 + v, acc[u][v]);
  }
}
// Matrix cores for R, N multiples of 16 up to 64 and Kd a multiple of 4: wave
// w takes the 16-row tile w (and every 16-column tile), the A fragment
// a(16 tr + lane mod 16, 4s + lane / 16) shared by the column tiles.
template <typename FA, typename FB, typename FO>
__device__ inline void block_mm_mfma(int R, int N, int Kd, FA a, FB b, FO out) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int ntr = R / 16, ntc = N / 16;
  for (int tr = w; tr < ntr; tr += nw) {
    lrs_d4 acc[4] = {lrs_d4{0, 0, 0, 0}, lrs_d4{0, 0, 0, 0}, lrs_d4{0, 0, 0, 0}, lrs_d4{0, 0, 0, 0}};
    for (int s = 0; s < Kd / 4; ++s) {
      const int kk = 4 * s + (lane >> 4);
      const double av = a(16 * tr + (lane & 15), kk);
#pragma unroll
      for (int ct = 0; ct < 4; ++ct)
        if (ct < ntc) acc[ct] = mfma_step(av, (double)b(kk, 16 * ct + (lane & 15)), acc[ct]);
    }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
      if (ct < ntc)
#pragma unroll
        for (int v = 0; v < 4; ++v) out(16 * tr + acc_row<double>(lane, v), 16 * ct + (lane & 15), acc[ct][v]);
  }
}
// register tile chosen so that the tiles cover about one workgroup
template <typename FA, typename FB, typename FO>
__device__ inline void block_mm(int R, int N, int Kd, FA a, FB b, FO out) {
  const int rn = R * N;
  if (R % 16 == 0 && N % 16 == 0 && Kd % 4 == 0 && R <= 64 && N <= 64)
    block_mm_mfma(R, N, Kd, a, b, out);
  else if (rn <= 256)
    block_mm_ts<1>(R, N, Kd, a, b, out);
  else if (rn <= 1024)
    block_mm_ts<2>(R, N, Kd, a, b, out);
  else
    block_mm_ts<4>(R, N, Kd, a, b, out);
}

// rows x cols block from global (row-major, pitch gl) into LDS (pitch pl); zero if src is null
__device__ inline void stage(double* dst, int pl, const double* src, int gl, int rows, int cols) {
  for (int o = threadIdx.x; o < rows * cols; o += blockDim.x) {
    const int i = o / cols, j = o % cols;
    dst[i * pl + j] = src ? src[(size_t)i * gl + j] : 0.0;
  }
}

// In-place Gauss-Jordan inversion with partial pivoting (first maximum wins)
// of the R x R left half of W = [D | I] (LDS, pitch pw = 2R + 1): on return
// the right half holds D^{-1}.  colc (R) and rowc (2R) are LDS scratch.
// Latches REDUCED_SINGULAR on an exactly zero pivot.  Needs R <= 64 and 256 threads.
__device__ inline void gauss_jordan(double* W, int pw, int R, double* colc, double* rowc, int* s_piv,
                                    int* latch, int part) {
  const int tid = threadIdx.x, lane = tid & 63;
  for (int c = 0; c < R; ++c) {
    if (tid < 64) {  // one wave finds the pivot row
      double bv = -1.0;
      int bi = R;
      bool nonfinite = false;
      for (int i = c + lane; i < R; i += 64) {
        const double v = fabs(W[i * pw + c]);
        nonfinite |= !(v <= 1.7976931348623157e308);
        if (v > bv) {
          bv = v;
          bi = i;
        }
      }
      nonfinite = __any(nonfinite);
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(bv, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ov > bv || (ov == bv && oi < bi)) {
          bv = ov;
          bi = oi;
        }
      }
      if (lane == 0) {
        *s_piv = bi;
        if (nonfinite)
          latch_error(latch, 4, part, c);
        else if (!(bv > 0.0))
          latch_error(latch, 2, part, c);
      }
    }
    __syncthreads();
    const int pv = *s_piv;
    if (pv != c && pv < R)
      for (int j = tid; j < 2 * R; j += blockDim.x) {
        const double t = W[c * pw + j];
        W[c * pw + j] = W[pv * pw + j];
        W[pv * pw + j] = t;
      }
    __syncthreads();
    const double inv = 1.0 / W[c * pw + c];
    for (int i = tid; i < R; i += blockDim.x) colc[i] = W[i * pw + c];
    for (int j = tid; j < 2 * R; j += blockDim.x) rowc[j] = W[c * pw + j] * inv;
    __syncthreads();
    // columns that still matter: c+1 .. R-1 of the left half, all of the right
    // half; a thread keeps its columns (tid mod 64) and rows tid/64 + 4q, whose
    // entries are all loaded before any is stored (R <= 64, 256 threads)
    const int wl = R - c - 1, w = wl + R, i0 = tid >> 6;
    double cc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) cc[q] = (i0 + 4 * q < R) ? colc[i0 + 4 * q] : 0.0;
    for (int jj = lane; jj < w; jj += 64) {
      const int j = jj < wl ? c + 1 + jj : R + (jj - wl);
      const double rj = rowc[j];
      double wv[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) wv[q] = (i0 + 4 * q < R) ? W[(i0 + 4 * q) * pw + j] : 0.0;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int i = i0 + 4 * q;
        if (i < R) W[i * pw + j] = (i == c) ? rj : fma(-cc[q], rj, wv[q]);
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ CR factorization
// Level l (stride s = 2^l), active rows i = 0, s, 2s, ... < NI.
// Odd rows (i/s odd) are eliminated: Dinv_i = D_i^{-1} (Gauss-Jordan with
// partial pivoting), X^F_i = Dinv_i F_i, X^E_i = Dinv_i E_i replace (F_i, E_i)
// in the row's level slot.  Even rows survive:
//   D_i -= F_i X^E_{i-s} + E_i X^F_{i+s},  F_i' = -F_i X^F_{i-s},  E_i' = -E_i X^E_{i+s},
// and their level slot is overwritten by M^F_i = F_i Dinv_{i-s}, M^E_i = E_i Dinv_{i+s}.
// With these the four solves (Z, Z^T, forward and back substitution) are
// products of small dense blocks only.
// LDS: W = R2 x (2 R2 + 1), then column and row scratch (3 R2).
__global__ __launch_bounds__(LRS_NT) void cr_odd_kernel(RedArgs a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double* W = reinterpret_cast<double*>(lds_raw);
  __shared__ int s_piv;
  const Layout& L = a.L;
  const bool tmode = a.level < 0;  // LR-SPIKE-T: invert every diagonal block, nothing else
  const int R = L.R2, s = tmode ? 1 : 1 << a.level, pw = 2 * R + 1;
  const bool top = tmode || a.level >= L.levels;
  const int i = tmode ? blockIdx.x : (top ? 0 : (2 * blockIdx.x + 1) * s);
  if (i >= L.NI) return;
  double* colc = W + R * pw;
  double* rowc = colc + R;
  const double* D = rws<double>(a.ws, L.zD) + (size_t)i * R * R;
  double dmax = 0.0;  // largest entry of the block being inverted (a Schur complement above level 0)
  for (int o = threadIdx.x; o < R * 2 * R; o += blockDim.x) {
    const int row = o / (2 * R), col = o % (2 * R);
    const double v = col < R ? D[row * R + col] : (col - R == row ? 1.0 : 0.0);
    W[row * pw + col] = v;
    dmax = fmax(dmax, fabs(v));
  }
  dmax = wave_max(dmax);
  if ((threadIdx.x & 63) == 0) state_max(rws<int>(a.ws, L.latch), S_ZGROW, dmax);
  __syncthreads();
  gauss_jordan(W, pw, R, colc, rowc, &s_piv, rws<int>(a.ws, L.latch), i);
  double* Dinv = rws<double>(a.ws, L.zLU) + (size_t)i * R * R;
  for (int o = threadIdx.x; o < R * R; o += blockDim.x) Dinv[o] = W[(o / R) * pw + R + o % R];
  if (top) return;
  double* FE = rws<double>(a.ws, L.zFE) + (size_t)(L.lvl_off[a.level] + i / s) * 2 * R * R;
  for (int which = 0; which < 2; ++which) {  // X^F = Dinv F, then X^E = Dinv E
    double* slot = FE + which * R * R;
    stage(W, pw, slot, R, R, R);  // into the (now free) left half
    __syncthreads();
    block_mm(R, R, R, [&](int r, int l) { return W[r * pw + R + l]; }, [&](int l, int c) { return W[l * pw + c]; },
             [&](int r, int c, double v) { slot[r * R + c] = v; });
    __syncthreads();
  }
}

// LDS: A and B blocks, R2 x (R2 + 1) each.
__global__ __launch_bounds__(LRS_NT) void cr_even_kernel(RedArgs a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const Layout& L = a.L;
  const int R = L.R2, s = 1 << a.level, pl = R + 1;
  const int i = 2 * blockIdx.x * s;
  if (i >= L.NI) return;
  double* A = reinterpret_cast<double*>(lds_raw);
  double* B = A + R * pl;
  const bool hasL = i - s >= 0, hasR = i + s < L.NI;
  double* D = rws<double>(a.ws, L.zD) + (size_t)i * R * R;
  double* FE = rws<double>(a.ws, L.zFE) + (size_t)(L.lvl_off[a.level] + i / s) * 2 * R * R;
  double* FEn = rws<double>(a.ws, L.zFE) + (size_t)(L.lvl_off[a.level + 1] + i / (2 * s)) * 2 * R * R;
  auto slot = [&](int row) { return rws<double>(a.ws, L.zFE) + (size_t)(L.lvl_off[a.level] + row / s) * 2 * R * R; };
  auto dinv = [&](int row) { return rws<double>(a.ws, L.zLU) + (size_t)row * R * R; };
  auto fa = [&](int r, int l) { return A[r * pl + l]; };
  auto fb = [&](int l, int c) { return B[l * pl + c]; };
  // side 0: A = F with the row i - s;  side 1: A = E with the row i + s
  for (int side = 0; side < 2; ++side) {
    const bool has = side == 0 ? hasL : hasR;
    double* own = FE + side * R * R;  // F_i or E_i, replaced by M^F_i or M^E_i
    double* nxt = FEn + side * R * R;
    if (!has) {
      for (int o = threadIdx.x; o < R * R; o += blockDim.x) {
        own[o] = 0.0;
        nxt[o] = 0.0;
      }
      continue;
    }
    const double* X = slot(side == 0 ? i - s : i + s);  // [X^F | X^E] of the neighbour
    __syncthreads();
    stage(A, pl, own, R, R, R);
    stage(B, pl, X + (side == 0 ? R * R : 0), R, R, R);  // X^E_{i-s} or X^F_{i+s}
    __syncthreads();
    block_mm(R, R, R, fa, fb, [&](int r, int c, double v) { D[r * R + c] -= v; });
    __syncthreads();
    stage(B, pl, X + (side == 0 ? 0 : R * R), R, R, R);  // X^F_{i-s} or X^E_{i+s}
    __syncthreads();
    block_mm(R, R, R, fa, fb, [&](int r, int c, double v) { nxt[r * R + c] = -v; });
    __syncthreads();
    stage(B, pl, dinv(side == 0 ? i - s : i + s), R, R, R);
    __syncthreads();
    block_mm(R, R, R, fa, fb, [&](int r, int c, double v) { own[r * R + c] = v; });
  }
}

// ------------------------------------------------------------------ CR solves
// g (compressed vectors, [NI][R2][mmax]) is solved in place, in chunks of up
// to CRS_MC columns (grid y).  Every product stages its R2 x R2 block and the
// R2 x mc vector block in LDS.
// LDS: R2 x (R2 + 1) block, R2 x (mc + 1) vectors, R2 x mc own vector copy.
#define CRS_MC 32
struct CrsLds {
  double *A, *G, *O;
  int pa, pg;
};
__device__ inline CrsLds crs_lds(int R, int m) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  CrsLds c;
  c.A = reinterpret_cast<double*>(lds_raw);
  c.pa = R + 1;
  c.G = c.A + R * c.pa;
  c.pg = m + 1;
  c.O = c.G + R * c.pg;
  return c;
}
// out(i, c) op= op(Mblk) x gblk with op = transpose or not
template <typename FO>
__device__ inline void crs_product(const CrsLds& w, int R, int m, int mm, const double* Mblk, bool tr,
                                   const double* gblk, FO out) {
  __syncthreads();
  stage(w.A, w.pa, Mblk, R, R, R);
  stage(w.G, w.pg, gblk, mm, R, m);
  __syncthreads();
  if (tr)
    block_mm(R, m, R, [&](int r, int l) { return w.A[l * w.pa + r]; }, [&](int l, int c) { return w.G[l * w.pg + c]; },
             out);
  else
    block_mm(R, m, R, [&](int r, int l) { return w.A[r * w.pa + l]; }, [&](int l, int c) { return w.G[l * w.pg + c]; },
             out);
}

// Forward reduction at level l, even rows:
//   Z:    g_i -= M^F_i g_{i-s} + M^E_i g_{i+s}
//   Z^T:  g_i -= (X^E_{i-s})^T g_{i-s} + (X^F_{i+s})^T g_{i+s}
__global__ __launch_bounds__(LRS_NT) void crs_forward_kernel(RedArgs a) {
  if (a.gate && *a.gate) return;
  const Layout& L = a.L;
  const int R = L.R2, s = 1 << a.level, c0 = blockIdx.y * CRS_MC, m = min(CRS_MC, a.m - c0), mm = L.mmax;
  const int i = 2 * blockIdx.x * s;
  if (i >= L.NI) return;
  const CrsLds w = crs_lds(R, m);
  double* g = rws<double>(a.ws, L.zg) + c0;
  double* gi = g + (size_t)i * R * mm;
  auto slot = [&](int row) { return rws<double>(a.ws, L.zFE) + (size_t)(L.lvl_off[a.level] + row / s) * 2 * R * R; };
  auto sub = [&](int r, int c, double v) { gi[r * mm + c] -= v; };
  if (i - s >= 0) {
    const double* Mb = a.transpose ? slot(i - s) + R * R : slot(i);
    crs_product(w, R, m, mm, Mb, a.transpose, g + (size_t)(i - s) * R * mm, sub);
  }
  if (i + s < L.NI) {
    const double* Mb = a.transpose ? slot(i + s) : slot(i) + R * R;
    crs_product(w, R, m, mm, Mb, a.transpose, g + (size_t)(i + s) * R * mm, sub);
  }
}

// Top (row 0 alone) and back substitution of the odd rows of level l:
//   Z:    g_i = Dinv_i g_i - X^F_i g_{i-s} - X^E_i g_{i+s}
//   Z^T:  g_i = Dinv_i^T g_i - (M^E_{i-s})^T g_{i-s} - (M^F_{i+s})^T g_{i+s}
__global__ __launch_bounds__(LRS_NT) void crs_backward_kernel(RedArgs a) {
  if (a.gate && *a.gate) return;
  const Layout& L = a.L;
  const bool tmode = a.level < 0;  // LR-SPIKE-T: g_i = Dinv_i g_i for every interface
  const int R = L.R2, s = tmode ? 1 : 1 << a.level, c0 = blockIdx.y * CRS_MC, m = min(CRS_MC, a.m - c0),
            mm = L.mmax;
  const bool top = tmode || a.level >= L.levels;
  const int i = tmode ? blockIdx.x : (top ? 0 : (2 * blockIdx.x + 1) * s);
  if (i >= L.NI) return;
  const CrsLds w = crs_lds(R, m);
  double* g = rws<double>(a.ws, L.zg) + c0;
  double* gi = g + (size_t)i * R * mm;
  auto slot = [&](int row) { return rws<double>(a.ws, L.zFE) + (size_t)(L.lvl_off[a.level] + row / s) * 2 * R * R; };
  const bool hasL = !top && i - s >= 0, hasR = !top && i + s < L.NI;
  // own vector first (it is overwritten by the first product)
  crs_product(w, R, m, mm, rws<double>(a.ws, L.zLU) + (size_t)i * R * R, a.transpose, gi,
              [&](int r, int c, double v) { w.O[r * m + c] = v; });
  auto sub = [&](int r, int c, double v) { w.O[r * m + c] -= v; };
  if (hasL) {
    const double* Mb = a.transpose ? slot(i - s) + R * R : slot(i);
    crs_product(w, R, m, mm, Mb, a.transpose, g + (size_t)(i - s) * R * mm, sub);
  }
  if (hasR) {
    const double* Mb = a.transpose ? slot(i + s) : slot(i) + R * R;
    crs_product(w, R, m, mm, Mb, a.transpose, g + (size_t)(i + s) * R * mm, sub);
  }
  __syncthreads();
  for (int o = threadIdx.x; o < R * m; o += blockDim.x) gi[(o / m) * mm + o % m] = w.O[o];
}

// ------------------------------------------------------------------ compressed rhs
// Z:   g_j = [Pi_j^T y_{j+1,t}; Psi_{j+1}^T y_{j,b}]
// Z^T: g_j = L^T h with h_{(j,t)} = B_{j-1}^T nu_{j-1,b}, h_{(j,b)} = C_{j+1}^T nu_{j+1,t}:
//   (a_j)     = P_{j,t}^T h_{(j,t)} + P_{j,b}^T h_{(j,b)}
//   (c_{j+1}) = Q_{j+1,t}^T h_{(j+1,t)} + Q_{j+1,b}^T h_{(j+1,b)}
template <int K>
__global__ void zrhs_kernel(RedArgs a, const double* bands) {
  if (a.gate && *a.gate) return;
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
    Geom gj = part_geom(L, jj, K);
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
  // LR-SPIKE-T keeps only P_{i,b} in (a_i) and Q_{i+1,t} in (c_{i+1}): the
  // transpose of the tip corrections it applies
  const bool tv = L.variant != 0;
  if (!tv) hvec(i, true, H);
  hvec(i, false, H + K * m);
  hvec(i + 1, true, H + 2 * K * m);
  if (!tv) hvec(i + 1, false, H + 3 * K * m);
  __syncthreads();
  auto PT = [&](int j, int w) { return ptip + ((size_t)j * 4 + w) * K * r; };
  for (int o = threadIdx.x; o < 2 * r * m; o += blockDim.x) {
    int row = o / m, c = o % m;
    double s = 0.0;
    if (row < r) {
      const double* Pt = PT(i, 0);
      const double* Pb = PT(i, 1);
      for (int l = 0; l < K; ++l) {
        if (!tv) s += Pt[l * r + row] * H[l * m + c];
        s += Pb[l * r + row] * H[K * m + l * m + c];
      }
    } else {
      const double* Qt = PT(i + 1, 2);
      const double* Qb = PT(i + 1, 3);
      int q = row - r;
      for (int l = 0; l < K; ++l) {
        s += Qt[l * r + q] * H[2 * K * m + l * m + c];
        if (!tv) s += Qb[l * r + q] * H[3 * K * m + l * m + c];
      }
    }
    g[row * mm + c] = s;
  }
}

}  // namespace lrs
