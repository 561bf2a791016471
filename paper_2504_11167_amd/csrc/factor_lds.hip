// Factorization for K = 64: one 256-thread workgroup per partition with every
// K x K block resident in LDS (the single-wave kernels keep a 2K-row panel in
// one wave's registers, which does not fit at this width).
//
// Per K-row block b (the same block formulation as the other factor kernels):
//   panel [Dc_b; Lo_{b+1}] eliminated in place without interchanges; a
//   multiplier above 1 in magnitude means partial pivoting would interchange
//   rows, which this width does not support: NOT_SUPPORTED is latched for the
//   partition;
//   L11^{-1} and U11^{-1} in place by row sweeps;  U12 = L11^{-1} Up_b;
//   G step g_b = U11^{-T}(e_b + pending), pending = -U12^T g_b;
//   records in the fragment order the sweeps read;  Dc_{b+1} = D_{b+1} - L21 U12.
// The spikes are formed afterwards from the records (spike_lds_kernel) and,
// for r < k, swept back with their Gram matrices (pass2_lds_kernel).
// Block products: every thread owns one 4 x 4 tile of a 64 x 64 result.
#include "sweep.h"

namespace lrs {

template <int K>
struct LdsTile {
  static_assert(K == 64, "one 4 x 4 tile per thread of a 256-thread workgroup");
  static __device__ __forceinline__ int i0() { return 4 * (threadIdx.x >> 4); }
  static __device__ __forceinline__ int j0() { return 4 * (threadIdx.x & 15); }
};

// acc (4 x 4, this thread's tile) += sum_l a(i, l) b(l, j)
template <int K, typename FA, typename FB>
__device__ __forceinline__ void tile_mm(double (&acc)[4][4], FA a, FB b) {
  const int i0 = LdsTile<K>::i0(), j0 = LdsTile<K>::j0();
  for (int l = 0; l < K; ++l) {
    double av[4], bv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) av[u] = (double)a(i0 + u, l);
#pragma unroll
    for (int v = 0; v < 4; ++v) bv[v] = (double)b(l, j0 + v);
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] = fma(av[u], bv[v], acc[u][v]);
  }
}
__device__ __forceinline__ void tile_zero(double (&acc)[4][4]) {
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
}

template <typename T, int K>
struct FLds {
  static constexpr int PT = K + 1;
  static constexpr int oP = 0;               // [2K][PT] panel
  static constexpr int oU = oP + 2 * K * PT; // [K][PT]  Up_b -> U12
  static constexpr int oG = oU + K * PT;     // [K][PT]  pending G / g_b
  static constexpr int total = oG + K * PT;
};

template <typename T, int K>
__global__ __launch_bounds__(LRS_NT) void factor_lds_kernel(FactorArgs a) {
  using F = FLds<T, K>;
  constexpr int PT = F::PT;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* P = reinterpret_cast<T*>(lds_raw) + F::oP;
  T* U = reinterpret_cast<T*>(lds_raw) + F::oU;
  T* Gp = reinterpret_cast<T*>(lds_raw) + F::oG;
  __shared__ int s_bad;
  __shared__ int s_row;
  const Layout& L = a.L;
  const int j = blockIdx.x, tid = threadIdx.x, k = L.k;
  const Geom g = part_geom(L, j, K);
  const int nb = g.nb;
  T* fac = wsT<T>(a.ws, L.fac) + (size_t)j * L.nbmax * L.rec;
  T* gm = wsT<T>(a.ws, L.gmat) + (size_t)j * L.nbmax * K * K;
  int* ipv = wsT<int>(a.ws, L.ipiv) + (size_t)j * L.nbmax * K;
  int* flg = wsT<int>(a.ws, L.flag) + (size_t)j * L.nbmax;
  int* latch = wsT<int>(a.ws, L.latch);
  // A_j(lr, lc) in partition-local rows/columns (identity on the padding rows)
  auto Aj = [&](int lr, int lc) -> T {
    if (lr < 0 || lc < 0) return (lr == lc) ? T(1) : T(0);
    if (lr >= g.nj || lc >= g.nj) return T(0);
    const int d = lc - lr;
    if (d < -k || d > k) return T(0);
    return (T)a.bands[(int64_t)(d + k) * L.n + g.s + lr];
  };
  auto blk = [&](int R, int C, int i, int c) { return Aj(R * K + i - g.pad, C * K + c - g.pad); };
  for (int o = tid; o < K * K; o += LRS_NT) {
    const int i = o / K, c = o % K;
    P[i * PT + c] = blk(0, 0, i, c);
    Gp[i * PT + c] = T(0);
  }
  if (tid == 0) s_bad = 0;
  const int i0 = LdsTile<K>::i0(), j0 = LdsTile<K>::j0();
  for (int b = 0; b < nb; ++b) {
    const bool last = (b == nb - 1);
    const int nr = last ? K : 2 * K;
    if (!last)
      for (int o = tid; o < K * K; o += LRS_NT) {
        const int i = o / K, c = o % K;
        P[(K + i) * PT + c] = blk(b + 1, b, i, c);
        U[i * PT + c] = blk(b, b + 1, i, c);
      }
    __syncthreads();
    // ---- elimination without interchanges: lane = column, wave w rows w + 4q
    {
      const int lane = tid & 63, w = tid >> 6;
      for (int C = 0; C < K; ++C) {
        const T piv = P[C * PT + C];
        if (tid == 0 && !(piv != T(0))) {
          s_bad = 1;
          s_row = b * K + C - g.pad;
        }
        for (int i = C + 1 + tid; i < nr; i += LRS_NT) {
          const T l = P[i * PT + C] / piv;
          if (!(fabs(l) <= T(1)) && s_bad == 0) {
            s_bad = 2;
            s_row = b * K + C - g.pad;
          }
          P[i * PT + C] = l;
        }
        __syncthreads();
        const int c = C + 1 + lane;
        if (c < K) {
          const T pc = P[C * PT + c];
          T v[32], l[32];
#pragma unroll
          for (int q = 0; q < 32; ++q) {
            const int i = C + 1 + w + 4 * q;
            v[q] = i < nr ? P[i * PT + c] : T(0);
            l[q] = i < nr ? P[i * PT + C] : T(0);
          }
#pragma unroll
          for (int q = 0; q < 32; ++q) {
            const int i = C + 1 + w + 4 * q;
            if (i < nr) P[i * PT + c] = fma(-l[q], pc, v[q]);
          }
        }
        __syncthreads();
      }
    }
    if (s_bad) {
      if (tid == 0) latch_error(latch, s_bad == 1 ? LRSPIKE_ERR_ZERO_PIVOT : LRSPIKE_ERR_NOT_SUPPORTED, j, s_row);
      return;
    }
    // ---- in-place inverses: L11^{-1} (strict lower, unit diagonal) by rows
    // top-down and U11^{-1} (upper) by rows bottom-up, both in one loop (the
    // two touch disjoint triangles); a column is split over four threads of
    // one wave that reduce with lane shuffles.
    //   L row i:   X[i][c] = -(L[i][c] + sum_{l=c+1}^{i-1} L[i][l] X[l][c]),  c < i
    //   U row iu:  X[iu][c] = -(sum_{l=iu+1}^{c} U[iu][l] X[l][c]) / U[iu][iu], c > iu,
    //              X[iu][iu] = 1 / U[iu][iu]
    {
      const int c = tid >> 2, part = tid & 3;
      if (tid == 0) P[(K - 1) * PT + (K - 1)] = T(1) / P[(K - 1) * PT + (K - 1)];
      __syncthreads();
      for (int s = 1; s < K; ++s) {
        const int i = s, iu = K - 1 - s;
        T accl = T(0), accu = T(0);
        if (c < i)
          for (int l = c + 1 + part; l < i; l += 4) accl = fma(P[i * PT + l], P[l * PT + c], accl);
        if (c > iu)
          for (int l = iu + 1 + part; l <= c; l += 4) accu = fma(P[iu * PT + l], P[l * PT + c], accu);
        accl += __shfl_xor(accl, 1);
        accl += __shfl_xor(accl, 2);
        accu += __shfl_xor(accu, 1);
        accu += __shfl_xor(accu, 2);
        const T dinv = T(1) / P[iu * PT + iu];
        __syncthreads();
        if (part == 0) {
          if (c < i) P[i * PT + c] = -(P[i * PT + c] + accl);
          if (c > iu) P[iu * PT + c] = -accu * dinv;
          if (c == iu) P[iu * PT + iu] = dinv;
        }
        __syncthreads();
      }
    }
    auto Li = [&](int r, int l) -> T { return r > l ? P[r * PT + l] : (r == l ? T(1) : T(0)); };
    auto Ui = [&](int r, int l) -> T { return r <= l ? P[r * PT + l] : T(0); };
    double acc[4][4];
    // ---- U12 = L11^{-1} Up_b (in place in U)
    if (!last) {
      tile_zero(acc);
      tile_mm<K>(acc, Li, [&](int l, int c) { return U[l * PT + c]; });
      __syncthreads();
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) U[(i0 + u) * PT + j0 + v] = (T)acc[u][v];
      __syncthreads();
    }
    // ---- G step: g_b = U11^{-T} (e_b + pending); G^T record; pending = -U12^T g_b
    for (int o = tid; o < K * K; o += LRS_NT) {
      const int i = o / K, c = o % K;
      if (c == b * K + i - g.pad) Gp[i * PT + c] += T(1);
    }
    __syncthreads();
    tile_zero(acc);
    tile_mm<K>(acc, [&](int r, int l) { return Ui(l, r); }, [&](int l, int c) { return Gp[l * PT + c]; });
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        Gp[(i0 + u) * PT + j0 + v] = (T)acc[u][v];
        gm[(size_t)b * K * K + fidx<T, K>(j0 + v, i0 + u)] = (T)acc[u][v];  // G^T in operand order
      }
    __syncthreads();
    if (!last) {
      tile_zero(acc);
      tile_mm<K>(acc, [&](int r, int l) { return U[l * PT + r]; }, [&](int l, int c) { return Gp[l * PT + c]; });
      __syncthreads();
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) Gp[(i0 + u) * PT + j0 + v] = (T)(-acc[u][v]);
    }
    // ---- records: LP = L11^{-1} strict lower | L21 upper;  UP = U11^{-1} upper | U12 strict lower; UD
    T* rec = fac + (size_t)b * L.rec;
    for (int o = tid; o < K * K; o += LRS_NT) {
      const int i = o / K, c = o % K, f = fidx<T, K>(i, c);
      rec[f] = (i > c) ? P[i * PT + c] : (last ? T(0) : P[(K + i) * PT + c]);
      rec[K * K + f] = (i <= c) ? P[i * PT + c] : (last ? T(0) : U[i * PT + c]);
    }
    if (tid < K) {
      rec[2 * K * K + tid] = last ? T(0) : U[tid * PT + tid];
      ipv[(size_t)b * K + tid] = tid;
    }
    if (tid == 0) flg[b] = 0;
    __syncthreads();
    // ---- Dc_{b+1} = D_{b+1} - L21 U12 into the panel top
    if (!last) {
      tile_zero(acc);
      tile_mm<K>(acc, [&](int r, int l) { return r <= l ? P[(K + r) * PT + l] : T(0); },
                 [&](int l, int c) { return U[l * PT + c]; });
      __syncthreads();
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          P[(i0 + u) * PT + j0 + v] = blk(b + 1, b + 1, i0 + u, j0 + v) - (T)acc[u][v];
      __syncthreads();
    }
  }
}

// Spikes from the records, one workgroup per (partition, spike, chunk of MS
// columns):  W (spike 0): rhs [C_j; 0] swept forward (z_b = L11^{-1} r_b,
// r_{b+1} -= L21 z_b), W_t = sum_b G_b^T z_b, W_b = U11^{-1} z_last, z kept in
// the Y array for the back-sweep when r < k;  V (spike 1): rhs [0; B_j] lives in
// the last block only: z = L11^{-1} B_j there, V_b = U11^{-1} z, V_t = G_last^T z.
template <typename T, int K>
struct SLds {
  static constexpr int MS = 16, PT = K + 1, PM = MS + 1;
  static constexpr int oA = 0;             // [K][PT] L11^{-1} / U11^{-1}
  static constexpr int oB = oA + K * PT;   // [K][PT] L21
  static constexpr int oG = oB + K * PT;   // [K][PT] G_b (block rows x columns)
  static constexpr int oR = oG + K * PT;   // [2K][PM] rhs window
  static constexpr int oZ = oR + 2 * K * PM;  // [K][PM] z_b
  static constexpr int total = oZ + K * PM;
};

template <typename T, int K>
__global__ __launch_bounds__(LRS_NT) void spike_lds_kernel(FactorArgs a) {
  using S = SLds<T, K>;
  constexpr int PT = S::PT, PM = S::PM, MS = S::MS;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* A = reinterpret_cast<T*>(lds_raw) + S::oA;
  T* B = reinterpret_cast<T*>(lds_raw) + S::oB;
  T* Gb = reinterpret_cast<T*>(lds_raw) + S::oG;
  T* Rw = reinterpret_cast<T*>(lds_raw) + S::oR;
  T* Z = reinterpret_cast<T*>(lds_raw) + S::oZ;
  const Layout& L = a.L;
  const int j = blockIdx.x, spike = blockIdx.y, c0 = blockIdx.z * MS, tid = threadIdx.x, k = L.k;
  const Geom g = part_geom(L, j, K);
  const int nb = g.nb;
  const T* fac = wsT<T>(a.ws, L.fac) + (size_t)j * L.nbmax * L.rec;
  const T* gm = wsT<T>(a.ws, L.gmat) + (size_t)j * L.nbmax * K * K;
  T* ym = (L.r < K) ? wsT<T>(a.ws, L.ymat) + (size_t)j * L.nbmax * 2 * K * K : nullptr;
  double* tips = wsT<double>(a.ws, L.tips) + (size_t)j * 4 * K * K;  // Vt, Vb, Wt, Wb
  const int coff = spike == 0 ? 0 : K;
  auto bandv = [&](int64_t gi, int64_t gc) -> T { return (T)band_at(a.bands, L.n, k, gi, gc); };
  // rhs of block R (K rows of the chunk)
  auto rhs = [&](int R, int i, int c) -> T {
    const int lr = R * K + i - g.pad;
    if (lr < 0) return T(0);
    if (spike == 0) return (j > 0 && lr < K) ? bandv(g.s + lr, g.s - K + c0 + c) : T(0);  // [C_j; 0]
    return (j < L.p - 1 && R == nb - 1) ? bandv(g.s + lr, g.s + g.nj + c0 + c) : T(0);   // [0; B_j]
  };
  auto load_L = [&](int b, bool with_l21) {
    const T* rec = fac + (size_t)b * L.rec;
    for (int o = tid; o < K * K; o += LRS_NT) {
      const int i = o / K, c = o % K;
      const T x = rec[fidx<T, K>(i, c)];
      A[i * PT + c] = i > c ? x : (i == c ? T(1) : T(0));
      if (with_l21) B[i * PT + c] = i <= c ? x : T(0);
      Gb[c * PT + i] = gm[(size_t)b * K * K + fidx<T, K>(i, c)];  // stored G^T(i, c) = G(c, i)
    }
  };
  // out (K x MS) = M (K x K, pitch PT) x X (K x MS, pitch PM), 4 rows x 1 column per thread
  auto mm = [&](const T* M, bool trans, const T* X, T* out, T sign, bool accumulate) {
    const int col = tid & 15, r0 = 4 * (tid >> 4);
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int l = 0; l < K; ++l) {
      const double x = (double)X[l * PM + col];
#pragma unroll
      for (int u = 0; u < 4; ++u) s[u] = fma((double)(trans ? M[l * PT + r0 + u] : M[(r0 + u) * PT + l]), x, s[u]);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u)
      out[(r0 + u) * PM + col] = (T)((accumulate ? (double)out[(r0 + u) * PM + col] : 0.0) + sign * s[u]);
    __syncthreads();
  };
  double acc[4] = {0.0, 0.0, 0.0, 0.0};  // top tip: rows r0..r0+3 of column col
  const int col = tid & 15, r0 = 4 * (tid >> 4);
  auto put_tip = [&](int which, const T* X, bool dbl_acc) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
      tips[(size_t)which * K * K + (r0 + u) * K + c0 + col] = dbl_acc ? acc[u] : (double)X[(r0 + u) * PM + col];
  };
  auto store_y = [&](int b) {
    if (!ym) return;
    for (int o = tid; o < K * MS; o += LRS_NT) {
      const int i = o / MS, c = o % MS;
      ym[(size_t)b * 2 * K * K + i * 2 * K + coff + c0 + c] = Z[i * PM + c];
    }
  };
  if (spike == 0) {
    for (int o = tid; o < 2 * K * MS; o += LRS_NT) {
      const int i = o / MS, c = o % MS;
      Rw[i * PM + c] = (i < K) ? rhs(0, i, c) : (nb > 1 ? rhs(1, i - K, c) : T(0));
    }
    for (int b = 0; b < nb; ++b) {
      const bool last = (b == nb - 1);
      load_L(b, !last);
      __syncthreads();
      mm(A, false, Rw, Z, T(1), false);  // z_b
      if (!last) mm(B, false, Z, Rw + K * PM, T(-1), true);
      // W_t += G_b^T z_b
      for (int l = 0; l < K; ++l) {
        const double z = (double)Z[l * PM + col];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] = fma((double)Gb[l * PT + r0 + u], z, acc[u]);
      }
      store_y(b);
      if (last) {
        const T* up = fac + (size_t)b * L.rec + K * K;
        for (int o = tid; o < K * K; o += LRS_NT) {
          const int i = o / K, c = o % K;
          A[i * PT + c] = i <= c ? up[fidx<T, K>(i, c)] : T(0);
        }
        __syncthreads();
        mm(A, false, Z, Rw, T(1), false);  // W_b = U11^{-1} z_last
        put_tip(3, Rw, false);
        put_tip(2, nullptr, true);
      } else {
        for (int o = tid; o < K * MS; o += LRS_NT) {
          const int i = o / MS, c = o % MS;
          Rw[i * PM + c] = Rw[(K + i) * PM + c];
          Rw[(K + i) * PM + c] = (b + 2 < nb) ? rhs(b + 2, i, c) : T(0);
        }
        __syncthreads();
      }
    }
  } else {
    const int b = nb - 1;
    for (int o = tid; o < K * MS; o += LRS_NT) Rw[(o / MS) * PM + o % MS] = rhs(b, o / MS, o % MS);
    load_L(b, false);
    __syncthreads();
    mm(A, false, Rw, Z, T(1), false);  // z = L11^{-1} B_j (last block)
    for (int l = 0; l < K; ++l) {
      const double z = (double)Z[l * PM + col];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] = fma((double)Gb[l * PT + r0 + u], z, acc[u]);
    }
    store_y(b);
    const T* up = fac + (size_t)b * L.rec + K * K;
    for (int o = tid; o < K * K; o += LRS_NT) {
      const int i = o / K, c = o % K;
      A[i * PT + c] = i <= c ? up[fidx<T, K>(i, c)] : T(0);
    }
    __syncthreads();
    mm(A, false, Z, Rw, T(1), false);  // V_b = U11^{-1} z
    put_tip(1, Rw, false);
    put_tip(0, nullptr, true);
  }
}

// Back-sweeps of both spikes with their Gram matrices (r < k), one workgroup
// per (partition, spike):  z_b = U11^{-1}(Y_b - U12 z_{b+1}),  Gram += z_b^T z_b.
// V's forward result is zero above the last block (no interchanges at this width).
template <typename T, int K>
__global__ __launch_bounds__(LRS_NT) void pass2_lds_kernel(FactorArgs a) {
  constexpr int PT = K + 1;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* Ui = reinterpret_cast<T*>(lds_raw);
  T* U12 = Ui + K * PT;
  T* Zn = U12 + K * PT;  // z_{b+1}, then z_b
  T* Tm = Zn + K * PT;
  const Layout& L = a.L;
  const int j = blockIdx.x, spike = blockIdx.y, tid = threadIdx.x;
  const Geom g = part_geom(L, j, K);
  const T* fac = wsT<T>(a.ws, L.fac) + (size_t)j * L.nbmax * L.rec;
  const T* ym = wsT<T>(a.ws, L.ymat) + (size_t)j * L.nbmax * 2 * K * K;
  const int coff = spike == 0 ? 0 : K;
  const int i0 = LdsTile<K>::i0(), j0 = LdsTile<K>::j0();
  double gr[4][4], acc[4][4];
  tile_zero(gr);
  for (int o = tid; o < K * PT; o += LRS_NT) Zn[o] = T(0);
  for (int b = g.nb - 1; b >= 0; --b) {
    const bool last = (b == g.nb - 1);
    const T* rec = fac + (size_t)b * L.rec;
    for (int o = tid; o < K * K; o += LRS_NT) {
      const int i = o / K, c = o % K;
      const T x = rec[K * K + fidx<T, K>(i, c)];
      Ui[i * PT + c] = i <= c ? x : T(0);
      U12[i * PT + c] = last ? T(0) : (i > c ? x : (i == c ? rec[2 * K * K + i] : T(0)));
    }
    __syncthreads();
    // Tm = Y_b - U12 z_{b+1}
    tile_zero(acc);
    if (!last) tile_mm<K>(acc, [&](int r, int l) { return U12[r * PT + l]; }, [&](int l, int c) { return Zn[l * PT + c]; });
    const bool ynz = spike == 0 || last;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double y = ynz ? (double)ym[(size_t)b * 2 * K * K + (i0 + u) * 2 * K + coff + j0 + v] : 0.0;
        Tm[(i0 + u) * PT + j0 + v] = (T)(y - acc[u][v]);
      }
    __syncthreads();
    tile_zero(acc);
    tile_mm<K>(acc, [&](int r, int l) { return Ui[r * PT + l]; }, [&](int l, int c) { return Tm[l * PT + c]; });
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) Zn[(i0 + u) * PT + j0 + v] = (T)acc[u][v];
    __syncthreads();
    tile_mm<K>(gr, [&](int r, int l) { return Zn[l * PT + r]; }, [&](int l, int c) { return Zn[l * PT + c]; });
    __syncthreads();
  }
  double* gram = wsT<double>(a.ws, L.gram) + ((size_t)j * 2 + (spike == 0 ? 1 : 0)) * K * K;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) gram[(i0 + u) * K + j0 + v] = gr[u][v];
}

}  // namespace lrs
