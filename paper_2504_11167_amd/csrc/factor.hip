// Factorization stage of LR-SPIKE, one workgroup per partition.
//
// Pass 1 (top -> bottom over the K-row blocks of partition j): block LU of A_j
// with partial pivoting inside the band (section "SPIKE partitioning": the
// diagonal blocks A_j of the DS factorization), fused with
//   * the forward sweeps of both spike right-hand sides (eq. Veqn):
//       W_j = A_j^{-1} [C_j; 0],   V_j = A_j^{-1} [0; B_j],
//   * the forward substitution G = U_j^{-T} E_t, which turns "top K rows of
//     U_j^{-1} y" into the dot product G^T y accumulated in any top -> bottom
//     sweep; it gives the top tips V_{j,t}, W_{j,t} here and y_{j,t} in the
//     D-stage without a second sweep,
//   * the bottom tips V_{j,b}, W_{j,b} from the last block's back substitution.
// For every block it stores the factors in the packed form the sweeps read:
//   LP = strict lower part of L11^{-1}  +  upper part of L21      (K x K)
//   UP = upper part of U11^{-1}          +  strict lower part of U12 (K x K)
//   UD = diagonal of U12                                           (K)
// plus, for the (rare) blocks touched by row interchanges, the full L21 and
// U13 (this block interchanged) and the full U12 (this or the previous block
// interchanged: the fill lands in the coupling block).  Without interchanges
// L21 is upper and U12 lower triangular and U13 = 0.
//
// Pass 2 (only for r < k; bottom -> top): the back substitution of both
// spikes, accumulating the Gram matrices V^T V and W^T W whose leading
// eigenvectors are the leading right singular vectors used by the rank-r
// truncation (section "SVD representation of the spikes").
#include "sweep.h"

namespace lrs {

struct FactorArgs {
  const double* bands;
  char* ws;
  Layout L;
  int only_flagged;  // factor only the partitions flagged in the npv array
};

template <typename T>
__device__ inline T* wsT(char* ws, size_t off) {
  return reinterpret_cast<T*>(ws + off);
}

// LDS plan of pass 1 (element offsets in T units)
template <int K>
struct P1Lds {
  static constexpr int LDW = 3 * K + 1;  // window pitch
  static constexpr int LDK = K + 1;      // K-wide tiles
  static constexpr int LD2 = 2 * K + 1;  // 2K-wide tiles
  static constexpr int oWn = 0;                    // [2K][LDW]  window
  static constexpr int oT1 = oWn + 2 * K * LDW;    // [K][LD2]   U12|U13, later Y_b
  static constexpr int oLi = oT1 + K * LD2;        // [K][LDK]
  static constexpr int oUi = oLi + K * LDK;        // [K][LDK]
  static constexpr int oWv = oUi + K * LDK;        // [2K][LD2] spike rhs window [W | V]
  static constexpr int oGa = oWv + 2 * K * LD2;    // [K][LDK]  G accumulator A
  static constexpr int oGb2 = oGa + K * LDK;       // [K][LDK]  G accumulator B
  static constexpr int oG = oGb2 + K * LDK;        // [K][LDK]  g_b
  static constexpr int total = oG + K * LDK;
};

template <typename T, int K>
__global__ __launch_bounds__(LRS_NT) void factor_pass1(FactorArgs a) {
  using LD = P1Lds<K>;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* lds = reinterpret_cast<T*>(lds_raw);
  __shared__ int s_ipiv[K];
  __shared__ int s_flag;
  __shared__ T s_dinv[K];
  T* Wn = lds + LD::oWn;
  T* T1 = lds + LD::oT1;
  T* Li = lds + LD::oLi;
  T* Ui = lds + LD::oUi;
  T* Wv = lds + LD::oWv;
  T* Ga = lds + LD::oGa;
  T* Gb2 = lds + LD::oGb2;
  T* G = lds + LD::oG;
  constexpr int LDW = LD::LDW, LDK = LD::LDK, LD2 = LD::LD2;

  const Layout& L = a.L;
  const int j = blockIdx.x;
  const int tid = threadIdx.x;
  if (a.only_flagged && wsT<int>(a.ws, L.npv)[j] == 0) return;
  const Geom g = part_geom(L, j, K);
  const int k = L.k;
  const int nb = g.nb;
  int* latch = wsT<int>(a.ws, L.latch);

  T* fac = wsT<T>(a.ws, L.fac) + (size_t)j * L.nbmax * L.rec;
  T* swx = wsT<T>(a.ws, L.swx) + (size_t)j * L.nbmax * 3 * K * K;
  T* gm = wsT<T>(a.ws, L.gmat) + (size_t)j * L.nbmax * K * K;
  T* ym = (L.r < K) ? wsT<T>(a.ws, L.ymat) + (size_t)j * L.nbmax * 2 * K * K : nullptr;
  int* ipv = wsT<int>(a.ws, L.ipiv) + (size_t)j * L.nbmax * K;
  int* flg = wsT<int>(a.ws, L.flag) + (size_t)j * L.nbmax;
  double* tips = wsT<double>(a.ws, L.tips) + (size_t)j * 4 * K * K;  // Vt, Vb, Wt, Wb

  // accumulated top tips [W_t | V_t] = sum_b G_b^T Y_b: matrix-core tiles held
  // in registers by their owning wave (K >= 16), else thread-owned entries
  constexpr bool MF = (K >= 16);
  constexpr int NACC = MF ? 1 : (2 * K * K + LRS_NT - 1) / LRS_NT;
  double tacc[NACC];
#pragma unroll
  for (int t = 0; t < NACC; ++t) tacc[t] = 0.0;
  constexpr int TT = MF ? (K / 16) * (2 * K / 16) : 1;  // accumulator tiles
  constexpr int TPW = (TT + 3) / 4;                     // tiles per wave
  using AccV = typename AccVec<T>::type;
  AccV macc[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) macc[t] = AccV{0, 0, 0, 0};
  const int lane = tid & 63, wave = tid >> 6;

  // Load row block R (padded rows R K .. R K + K - 1) into window rows
  // [wrow0, wrow0 + K), window column = padded column - colbase, reading the
  // band diagonal by diagonal so that consecutive lanes read consecutive rows.
  // Band values of row block R, diagonal-major so that consecutive lanes read
  // consecutive rows; issued one step ahead into registers (pre[]) and written
  // into the window after the shift.
  constexpr int NPRE = ((2 * K + 1) * K + LRS_NT - 1) / LRS_NT;
  T pre[NPRE];
  T amax_run = T(0), pmin_run = T(INFINITY);  // diagnostics: largest band entry read, smallest pivot (wave 0)
  auto prefetch_rowblock = [&](int R) {
#pragma unroll
    for (int t = 0; t < NPRE; ++t) {
      const int o = tid + t * LRS_NT;
      T v = T(0);
      if (o < (2 * k + 1) * K) {
        const int d = o / K - k, i = o % K;
        const int q = R * K + i, lr = q - g.pad;
        if (lr < 0) {
          v = (d == 0) ? T(1) : T(0);
        } else if (lr < g.nj) {
          const int lc = lr + d;
          if (lc >= 0 && lc < g.nj) v = (T)a.bands[(int64_t)(d + k) * L.n + g.s + lr];
        }
      }
      pre[t] = v;
      amax_run = fmax(amax_run, fabs(v));
    }
  };
  // write the prefetched row block R into window rows K..2K-1 (zeroed first)
  auto store_prefetched = [&](int R, int colbase) {
#pragma unroll
    for (int t = 0; t < NPRE; ++t) {
      const int o = tid + t * LRS_NT;
      if (o < (2 * k + 1) * K) {
        const int d = o / K - k, i = o % K;
        const int wc = R * K + i + d - colbase;
        if (wc >= 0 && wc < 3 * K) Wn[(K + i) * LDW + wc] = pre[t];
      }
    }
  };
  auto load_rowblock = [&](int R, int wrow0, int colbase, int wcols) {
    for (int o = tid; o < K * wcols; o += LRS_NT) Wn[(wrow0 + o / wcols) * LDW + o % wcols] = T(0);
    __syncthreads();
    for (int o = tid; o < (2 * k + 1) * K; o += LRS_NT) {
      const int d = o / K - k, i = o % K;
      const int q = R * K + i, lr = q - g.pad;
      const int wc = q + d - colbase;
      if (lr < 0) {
        if (d == 0) Wn[(wrow0 + i) * LDW + wc] = T(1);
      } else if (lr < g.nj) {
        const int lc = lr + d;
        if (lc >= 0 && lc < g.nj && wc >= 0 && wc < wcols) {
          const T v = (T)a.bands[(int64_t)(d + k) * L.n + g.s + lr];
          Wn[(wrow0 + i) * LDW + wc] = v;
          amax_run = fmax(amax_run, fabs(v));
        }
      }
    }
  };
  // spike right-hand sides of row block R into Wv rows [wrow0, wrow0 + K):
  // columns 0..K-1 = [C_j; 0] (first K real rows), K..2K-1 = [0; B_j] (last K real rows)
  auto load_spike_rhs = [&](int R, int wrow0) {
    const int lr0 = R * K - g.pad;
    const bool any = (lr0 < K) || (lr0 + K > g.nj - K);
    for (int o = tid; o < K * 2 * K; o += LRS_NT) {
      int i = o / (2 * K), c = o % (2 * K);
      int lr = lr0 + i;
      double v = 0.0;
      if (any && lr >= 0 && lr < g.nj) {
        if (c < K) {
          if (lr < K) v = band_at(a.bands, L.n, k, g.s + lr, g.s - K + c);
        } else {
          int a2 = lr - (g.nj - K);
          if (a2 >= 0) v = band_at(a.bands, L.n, k, g.s + lr, g.s + g.nj + (c - K));
        }
      }
      Wv[(wrow0 + i) * LD2 + c] = (T)v;
    }
  };

  // initial window: row block 0 in rows 0..K-1 (block columns 0, 1), row block 1 below
  for (int o = tid; o < 2 * K * LDW; o += LRS_NT) Wn[o] = T(0);
  for (int o = tid; o < K * LDK; o += LRS_NT) {
    Ga[o] = T(0);
    Gb2[o] = T(0);
  }
  load_rowblock(0, 0, 0, 2 * K);
  __syncthreads();
  if (nb > 1) load_rowblock(1, K, 0, 3 * K);
  load_spike_rhs(0, 0);
  if (nb > 1)
    load_spike_rhs(1, K);
  else
    for (int o = tid; o < K * LD2; o += LRS_NT) Wv[K * LD2 + o] = T(0);
  __syncthreads();

  T* Gcur = Ga;   // pending accumulator for block b
  T* Gnext = Gb2; // pending accumulator for block b+1
  int nswapped = 0;
  bool prev_sw = false;

  for (int b = 0; b < nb; ++b) {
    const bool last = (b == nb - 1);
    const int nr = last ? K : 2 * K;
    const int64_t row0 = (int64_t)b * K - g.pad;
    // spike columns in play: W always; V only once its right-hand side (the
    // last block) is inside the window
    const int ncs = (b >= nb - 2) ? 2 * K : K;
    if (b + 2 < nb) prefetch_rowblock(b + 2);
    if (tid < 64) {
      bool sw = panel_lu_wave<T, K>(Wn, LDW, nr, last ? K : 3 * K, Wv, LD2, 2 * K, s_ipiv, latch, j, row0, pmin_run);
      if (tid == 0) s_flag = sw ? 1 : 0;
    }
    __syncthreads();
    const bool swapped = s_flag != 0;
    nswapped += swapped ? 1 : 0;
    const bool prev_swapped = prev_sw;
    prev_sw = swapped;
    if (tid < 64)
      tri_inv_lower_wave<T, K>(Wn, LDW, Li, LDK);
    else if (tid < 128)
      tri_inv_upper_wave<T, K>(Wn, LDW, Ui, LDK, s_dinv);
    __syncthreads();

    T* rec = fac + (size_t)b * L.rec;
    if (!last) {
      // [U12 | U13] = L11^{-1} R1  (U13 = 0 unless this block interchanged rows)
      const int nu = swapped ? 2 * K : K;
      gemm<T, false>(K, nu, K, T(1), Li, LDK, Wn + K, LDW, T(0), T1, LD2);
      if (!swapped)
        for (int o = tid; o < K * K; o += LRS_NT) T1[(o / K) * LD2 + K + o % K] = T(0);
      __syncthreads();
      // trailing rows: R2 -= L21 [U12 | U13]
      gemm<T, false>(K, nu, K, T(-1), Wn + K * LDW, LDW, T1, LD2, T(1), Wn + K * LDW + K, LDW);
    }
    // G step: g_b = U11^{-T} (e_b + pending)
    for (int i = tid; i < K; i += LRS_NT) {
      int col = b * K + i - g.pad;
      if (col >= 0 && col < K) Gcur[i * LDK + col] += T(1);
    }
    __syncthreads();
    gemm<T, true>(K, K, K, T(1), Ui, LDK, Gcur, LDK, T(0), G, LDK);
    __syncthreads();
    if (!last) {
      // pending(b+1) -= U12^T g_b ; pending(b+2) = -U13^T g_b
      gemm<T, true>(K, K, K, T(-1), T1, LD2, G, LDK, T(1), Gnext, LDK);
      if (swapped)
        gemm<T, true>(K, K, K, T(-1), T1 + K, LD2, G, LDK, T(0), Gcur, LDK);
      else
        for (int o = tid; o < K * LDK; o += LRS_NT) Gcur[o] = T(0);
    }
    // store factors of this block
    for (int o = tid; o < K * K; o += LRS_NT) {
      int i, c;
      fidx_inv<T, K>(o, i, c);  // element (i, c) lives at storage position o
      T lp = (i > c) ? Li[i * LDK + c] : (last ? T(0) : Wn[(K + i) * LDW + c]);
      T up = (i <= c) ? Ui[i * LDK + c] : (last ? T(0) : T1[i * LD2 + c]);
      const int fo = o;
      rec[fo] = lp;
      rec[K * K + fo] = up;
      gm[(size_t)b * K * K + o] = G[c * LDK + i];  // G^T in operand order
      if (!last && (swapped || prev_swapped)) {
        T* sx = swx + (size_t)b * 3 * K * K;
        if (swapped) {
          sx[fo] = Wn[(K + i) * LDW + c];
          sx[2 * K * K + fo] = T1[i * LD2 + K + c];
        }
        sx[K * K + fo] = T1[i * LD2 + c];
      }
    }
    for (int i = tid; i < K; i += LRS_NT) {
      rec[2 * K * K + i] = last ? T(0) : T1[i * LD2 + i];
      ipv[(size_t)b * K + i] = s_ipiv[i];
    }
    // bit 0: this block interchanged rows (full L21, U13 != 0);
    // bit 1: U12 is full (fill from an interchange in this or the previous block)
    if (tid == 0) flg[b] = (swapped ? 1 : 0) | ((!last && (swapped || prev_swapped)) ? 2 : 0);
    __syncthreads();
    // spike forward step: Y_b = L11^{-1} Wv[0:K] (into T1); Wv[K:2K] -= L21 Y_b
    gemm<T, false>(K, ncs, K, T(1), Li, LDK, Wv, LD2, T(0), T1, LD2);
    if (ncs == K)
      for (int o = tid; o < K * K; o += LRS_NT) T1[(o / K) * LD2 + K + o % K] = T(0);
    __syncthreads();
    if (!last) gemm<T, false>(K, ncs, K, T(-1), Wn + K * LDW, LDW, T1, LD2, T(1), Wv + K * LD2, LD2);
    // top tips accumulate G_b^T Y_b
    if constexpr (MF) {
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        const int tile = wave + 4 * t;
        const int i0 = (tile / (2 * K / 16)) * 16, j0 = (tile % (2 * K / 16)) * 16;
        if (tile < TT && j0 < ncs)
#pragma unroll
          for (int k0 = 0; k0 < K; k0 += 4)
            macc[t] = mfma_step(G[(k0 + (lane >> 4)) * LDK + i0 + (lane & 15)],
                                T1[(k0 + (lane >> 4)) * LD2 + j0 + (lane & 15)], macc[t]);
      }
    } else {
#pragma unroll
      for (int t = 0; t < NACC; ++t) {
        int o = tid + t * LRS_NT;
        if (o < 2 * K * K) {
          int i = o / (2 * K), c = o % (2 * K);
          if (c < ncs) {
            double sacc = 0.0;
            for (int l = 0; l < K; ++l) sacc += (double)G[l * LDK + i] * (double)T1[l * LD2 + c];
            tacc[t] += sacc;
          }
        }
      }
    }
    if (ym)
      for (int o = tid; o < 2 * K * K; o += LRS_NT) ym[(size_t)b * 2 * K * K + o] = T1[o / (2 * K) * LD2 + o % (2 * K)];
    if (last) {
      // bottom tips: [W_b | V_b] = U11^{-1} Y_last (the last block has nothing below)
      for (int o = tid; o < 2 * K * K; o += LRS_NT) {
        int i = o / (2 * K), c = o % (2 * K);
        double sacc = 0.0;
        for (int l = i; l < K; ++l) sacc += (double)Ui[i * LDK + l] * (double)T1[l * LD2 + c];
        if (c < K)
          tips[3 * K * K + i * K + c] = (j > 0) ? sacc : 0.0;  // W_b
        else
          tips[1 * K * K + i * K + (c - K)] = (j < L.p - 1) ? sacc : 0.0;  // V_b
      }
    }
    __syncthreads();
    if (!last) {
      // shift: trailing rows become the current row block; load row block b+2
      for (int o = tid; o < K * 3 * K; o += LRS_NT) {
        int i = o / (3 * K), c = o % (3 * K);
        Wn[i * LDW + c] = (c < 2 * K) ? Wn[(K + i) * LDW + K + c] : T(0);
      }
      for (int o = tid; o < K * 2 * K; o += LRS_NT) {
        int i = o / (2 * K), c = o % (2 * K);
        Wv[i * LD2 + c] = Wv[(K + i) * LD2 + c];
      }
      __syncthreads();
      if (b + 2 < nb) {
        for (int o = tid; o < K * LDW; o += LRS_NT) Wn[K * LDW + o] = T(0);
        load_spike_rhs(b + 2, K);
        __syncthreads();
        store_prefetched(b + 2, (b + 1) * K);
      } else {
        for (int o = tid; o < K * LDW; o += LRS_NT) Wn[K * LDW + o] = T(0);
        for (int o = tid; o < K * LD2; o += LRS_NT) Wv[K * LD2 + o] = T(0);
      }
      T* t = Gcur;
      Gcur = Gnext;
      Gnext = t;
      __syncthreads();
    }
  }
  // top tips
  auto put_top = [&](int i, int c, double v) {
    if (c < K)
      tips[2 * K * K + i * K + c] = (j > 0) ? v : 0.0;  // W_t
    else
      tips[0 * K * K + i * K + (c - K)] = (j < L.p - 1) ? v : 0.0;  // V_t
  };
  if constexpr (MF) {
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int tile = wave + 4 * t;
      const int i0 = (tile / (2 * K / 16)) * 16, j0 = (tile % (2 * K / 16)) * 16;
      if (tile < TT)
#pragma unroll
        for (int v = 0; v < 4; ++v) put_top(i0 + acc_row<T>(lane, v), j0 + (lane & 15), (double)macc[t][v]);
    }
  } else {
#pragma unroll
    for (int t = 0; t < NACC; ++t) {
      int o = tid + t * LRS_NT;
      if (o < 2 * K * K) put_top(o / (2 * K), o % (2 * K), tacc[t]);
    }
  }
  if (tid == 0 && nswapped) atomicAdd(latch + S_SWAPPED, nswapped);
  const T am = wave_max(amax_run);
  if (lane == 0) state_max(latch, S_AMAX, (double)am);
  if (tid == 0) state_min(latch, S_PIVMIN, (double)pmin_run);
}

// ------------------------------------------------------------------------
// Pass 2: back substitution of both spikes (bottom -> top) with Gram
// accumulation.  z_b = U11^{-1} (Y_b - U12 z_{b+1} - U13 z_{b+2}).
// ------------------------------------------------------------------------
template <int K>
struct P2Lds {
  static constexpr int LDK = K + 1, LD2 = 2 * K + 1;
  static constexpr int oUi = 0;
  static constexpr int oU12 = oUi + K * LDK;
  static constexpr int oU13 = oU12 + K * LDK;
  static constexpr int oZ0 = oU13 + K * LDK;   // z_b (and Y_b staging)
  static constexpr int oZ1 = oZ0 + K * LD2;    // z_{b+1}
  static constexpr int oZ2 = oZ1 + K * LD2;    // z_{b+2}
  static constexpr int oY = oZ2 + K * LD2;
  static constexpr int total = oY + K * LD2;
};

template <typename T, int K>
__global__ __launch_bounds__(LRS_NT) void factor_pass2(FactorArgs a) {
  using LD = P2Lds<K>;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* lds = reinterpret_cast<T*>(lds_raw);
  constexpr int LDK = LD::LDK, LD2 = LD::LD2;
  T* Ui = lds + LD::oUi;
  T* U12 = lds + LD::oU12;
  T* U13 = lds + LD::oU13;
  T* Zb[3] = {lds + LD::oZ0, lds + LD::oZ1, lds + LD::oZ2};
  T* Y = lds + LD::oY;
  const Layout& L = a.L;
  const int j = blockIdx.x, tid = threadIdx.x;
  const Geom g = part_geom(L, j, K);
  const T* fac = wsT<T>(a.ws, L.fac) + (size_t)j * L.nbmax * L.rec;
  const T* swx = wsT<T>(a.ws, L.swx) + (size_t)j * L.nbmax * 3 * K * K;
  const T* ym = wsT<T>(a.ws, L.ymat) + (size_t)j * L.nbmax * 2 * K * K;
  const int* flg = wsT<int>(a.ws, L.flag) + (size_t)j * L.nbmax;
  double* gram = wsT<double>(a.ws, L.gram) + (size_t)j * 2 * K * K;  // GV, GW

  constexpr int NACC = (2 * K * K + LRS_NT - 1) / LRS_NT;
  double acc[NACC];
#pragma unroll
  for (int t = 0; t < NACC; ++t) acc[t] = 0.0;
  for (int o = tid; o < K * LD2; o += LRS_NT) {
    Zb[1][o] = T(0);
    Zb[2][o] = T(0);
  }
  __syncthreads();
  for (int b = g.nb - 1; b >= 0; --b) {
    const T* rec = fac + (size_t)b * L.rec;
    const int fl = flg[b];
    const bool sw = (fl & 1) != 0;
    const bool last = (b == g.nb - 1);
    load_ufac<T, K>(rec, swx + (size_t)b * 3 * K * K, fl, last, Ui, U12, U13);
    for (int o = tid; o < 2 * K * K; o += LRS_NT) Y[o / (2 * K) * LD2 + o % (2 * K)] = ym[(size_t)b * 2 * K * K + o];
    __syncthreads();
    gemm<T, false>(K, 2 * K, K, T(-1), U12, LDK, Zb[1], LD2, T(1), Y, LD2);
    __syncthreads();
    if (sw) {
      gemm<T, false>(K, 2 * K, K, T(-1), U13, LDK, Zb[2], LD2, T(1), Y, LD2);
      __syncthreads();
    }
    gemm<T, false>(K, 2 * K, K, T(1), Ui, LDK, Y, LD2, T(0), Zb[0], LD2);
    __syncthreads();
    // Grams: GV += z_V^T z_V (columns K..2K-1), GW += z_W^T z_W (columns 0..K-1)
#pragma unroll
    for (int t = 0; t < NACC; ++t) {
      int o = tid + t * LRS_NT;
      if (o < 2 * K * K) {
        int which = o / (K * K), e = o % (K * K), i = e / K, c = e % K;
        int off = (which == 0) ? K : 0;
        double s = 0.0;
        for (int l = 0; l < K; ++l) s += (double)Zb[0][l * LD2 + off + i] * (double)Zb[0][l * LD2 + off + c];
        acc[t] += s;
      }
    }
    __syncthreads();
    T* t2 = Zb[2];
    Zb[2] = Zb[1];
    Zb[1] = Zb[0];
    Zb[0] = t2;
  }
#pragma unroll
  for (int t = 0; t < NACC; ++t) {
    int o = tid + t * LRS_NT;
    if (o < 2 * K * K) gram[o] = acc[t];
  }
  (void)g;
}

}  // namespace lrs
