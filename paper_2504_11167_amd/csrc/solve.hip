// Solve stage of LR-SPIKE (summary of the SPIKE solve: D-stage, reduced
// system, recovery), and its exact transpose.
//
//   D-stage    y_j = A_j^{-1} f_j, keeping only the tips: one top -> bottom
//              pass; y_{j,t} = G^T (L^{-1} P^T f_j) with G = U^{-T} E_t from the
//              factorization, y_{j,b} from the last block's back substitution.
//   recovery   x_j = A_j^{-1} (f_j - [C_j x_{j-1,b}; 0; B_j x_{j+1,t}])
//              (eqs. recovery1, recovery2 with the signs restored), in place.
//   adjoint    nu_j = A_j^{-T} g_j (tips), and
//              lambda_j = A_j^{-T} (g_j - [w_{j,t}; 0; w_{j,b}]).
// One workgroup per (partition, chunk of <= mc_of<K>() right-hand-side columns).
#include "sweep.h"

namespace lrs {

struct SolveArgs {
  const double* bands;
  char* ws;
  Layout L;
  const double* src;  // right-hand side read (n x ld, row-major)
  double* dst;        // output written (may equal src)
  int ld;             // row stride of src / dst
  int m;              // columns
  const int* gate;    // refinement: nonzero *gate = the iteration has stopped, the kernel is a no-op (null = always run)
  int only_flagged;   // workgroup adjoint kernels: only the partitions factored with interchanges
  int block_only;     // retrieval kernels: x_j = A_j^{-1} f_j, no coupling terms (block-diagonal solve)
};

__device__ __forceinline__ bool gated(const int* gate) { return gate && *gate != 0; }

template <int K>
struct SwLds {
  static constexpr int LDK = K + 1, LDM = mc_of<K>() + 1;
  static constexpr int oW = 0;                  // [2K][LDM] window / x_b, x_{b+1}
  static constexpr int oW2 = oW + 2 * K * LDM;  // [K][LDM]  x_{b+2} / z_b
  static constexpr int oTmp = oW2 + K * LDM;    // [2K][LDM]
  static constexpr int oA = oTmp + 2 * K * LDM; // [K][LDK]  Li / Ui
  static constexpr int oB = oA + K * LDK;       // [K][LDK]  L21 / U12
  static constexpr int oC = oB + K * LDK;       // [K][LDK]  G / U13
  static constexpr int oCt = oC + K * LDK;      // [K][LDM]  top correction
  static constexpr int oCb = oCt + K * LDM;     // [K][LDM]  bottom correction
  static constexpr int total = oCb + K * LDM;
};

// ---------------------------------------------------------------- helpers

// rhs value of padded row q of partition g, column c (minus corrections)
template <typename T, int K>
__device__ inline T rhs_at(const SolveArgs& a, const Geom& g, int q, int c, int c0, const T* Ct,
                           const T* Cb) {
  constexpr int LDM = mc_of<K>() + 1;
  int lr = q - g.pad;
  if (lr < 0 || lr >= g.nj) return T(0);
  T v = (T)a.src[(g.s + lr) * (int64_t)a.ld + c0 + c];
  if (Ct && lr < K) v -= Ct[lr * LDM + c];
  if (Cb && lr >= g.nj - K) v -= Cb[(lr - (g.nj - K)) * LDM + c];
  return v;
}

// Interface tips of the reduced solution: x_{i,t} (top = true) or x_{i,b} of
// partition i, written as T into X (K x mc, pitch LDM):
//   x_{i,t} = y_{i,t} - Q_{i,t} c_i - P_{i,t} a_i,   x_{i,b} likewise,
// with a_i = z_i[0:r] (i <= p-2) and c_i = z_{i-1}[r:2r] (i >= 1).  LR-SPIKE-T
// drops the terms of the other interface (P_{i,t} a_i and Q_{i,b} c_i).
template <typename T, int K>
__device__ inline void interface_tip(const SolveArgs& a, int i, bool top, int c0, int mc, T* X) {
  constexpr int LDM = mc_of<K>() + 1;
  const Layout& L = a.L;
  const int r = L.r;
  const double* yt = wsp<double>(a.ws, L.ytip) + ((size_t)i * 2 + (top ? 0 : 1)) * K * L.mmax;
  const double* pt = wsp<double>(a.ws, L.ptip) + (size_t)i * 4 * K * r;  // Pt, Pb, Qt, Qb
  const double* P = pt + (top ? 0 : 1) * K * r;
  const double* Q = pt + (top ? 2 : 3) * K * r;
  const double* zg = wsp<double>(a.ws, L.zg);
  for (int o = threadIdx.x; o < K * mc; o += blockDim.x) {
    int row = o / mc, c = o % mc;
    double v = yt[row * L.mmax + c0 + c];
    if (r > 0) {
      if (i <= L.p - 2 && !(L.variant && top)) {
        const double* av = zg + (size_t)i * L.R2 * L.mmax;  // a_i = first r entries of z_i
        for (int q = 0; q < r; ++q) v -= P[row * r + q] * av[q * L.mmax + c0 + c];
      }
      if (i >= 1 && !(L.variant && !top)) {
        const double* cv = zg + ((size_t)(i - 1) * L.R2 + r) * L.mmax;  // c_i
        for (int q = 0; q < r; ++q) v -= Q[row * r + q] * cv[q * L.mmax + c0 + c];
      }
    }
    X[row * LDM + c] = (T)v;
  }
}

// ---------------------------------------------------------------- forward pass
// Runs L^{-1} P^T over the partition's rhs (minus optional corrections).
// If dstage: accumulates y_t = G^T z, writes y_t and y_b = U11^{-1} z_last into
// the tip buffer.  Otherwise writes z into a.dst rows (real rows only).
template <typename T, int K, bool DSTAGE>
__device__ void forward_pass(const SolveArgs& a, const Geom& g, int j, int c0, int mc, T* lds,
                             const T* Ct, const T* Cb, int* s_perm) {
  using LD = SwLds<K>;
  constexpr int LDK = LD::LDK, LDM = LD::LDM;
  T* Zw = lds + LD::oW;
  T* Zt = lds + LD::oW2;
  T* Tmp = lds + LD::oTmp;
  T* Li = lds + LD::oA;
  T* L21 = lds + LD::oB;
  T* Gt = lds + LD::oC;
  const Layout& L = a.L;
  const int tid = threadIdx.x;
  const T* fac = wsp<T>(a.ws, L.fac) + (size_t)j * L.nbmax * L.rec;
  const T* swx = wsp<T>(a.ws, L.swx) + (size_t)j * L.nbmax * 3 * K * K;
  const T* gm = wsp<T>(a.ws, L.gmat) + (size_t)j * L.nbmax * K * K;
  const int* ipv = wsp<int>(a.ws, L.ipiv) + (size_t)j * L.nbmax * K;
  const int* flg = wsp<int>(a.ws, L.flag) + (size_t)j * L.nbmax;
  constexpr int NACC = (K * mc_of<K>() + LRS_NT - 1) / LRS_NT;
  double acc[NACC];
#pragma unroll
  for (int t = 0; t < NACC; ++t) acc[t] = 0.0;

  for (int o = tid; o < 2 * K * mc; o += LRS_NT) {
    int i = o / mc, c = o % mc;
    Zw[i * LDM + c] = (i < K || g.nb > 1) ? rhs_at<T, K>(a, g, i, c, c0, Ct, Cb) : T(0);
  }
  __syncthreads();
  for (int b = 0; b < g.nb; ++b) {
    const bool last = (b == g.nb - 1);
    const int fl = flg[b];
    const bool sw = (fl & 1) != 0;
    const T* rec = fac + (size_t)b * L.rec;
    load_lfac<T, K>(rec, swx + (size_t)b * 3 * K * K, fl, last, Li, L21);
    if (DSTAGE)
      for (int o = tid; o < K * K; o += LRS_NT) Gt[o / K * LDK + o % K] = gm[(size_t)b * K * K + fidx<T, K>(o % K, o / K)];
    if (sw) permute_rows<T, K>(Zw, LDM, last ? K : 2 * K, mc, ipv + (size_t)b * K, s_perm, Tmp);
    __syncthreads();
    gemm<T, false>(K, mc, K, T(1), Li, LDK, Zw, LDM, T(0), Zt, LDM);
    __syncthreads();
    if (!last) gemm<T, false>(K, mc, K, T(-1), L21, LDK, Zt, LDM, T(1), Zw + K * LDM, LDM);
    if (DSTAGE) {
#pragma unroll
      for (int t = 0; t < NACC; ++t) {
        int o = tid + t * LRS_NT;
        if (o < K * mc) {
          int i = o / mc, c = o % mc;
          double s = 0.0;
          for (int l = 0; l < K; ++l) s += (double)Gt[l * LDK + i] * (double)Zt[l * LDM + c];
          acc[t] += s;
        }
      }
    } else {
      for (int o = tid; o < K * mc; o += LRS_NT) {
        int i = o / mc, c = o % mc;
        int lr = b * K + i - g.pad;
        if (lr >= 0) a.dst[(g.s + lr) * (int64_t)a.ld + c0 + c] = (double)Zt[i * LDM + c];
      }
    }
    if (last && DSTAGE) {
      // y_b = U11^{-1} z_last
      const T* up = rec + K * K;
      double* yb = wsp<double>(a.ws, L.ytip) + ((size_t)j * 2 + 1) * K * L.mmax;
      for (int o = tid; o < K * mc; o += LRS_NT) {
        int i = o / mc, c = o % mc;
        double s = 0.0;
        for (int l = i; l < K; ++l) s += (double)up[fidx<T, K>(i, l)] * (double)Zt[l * LDM + c];
        yb[i * L.mmax + c0 + c] = s;
      }
    }
    __syncthreads();
    if (!last) {
      for (int o = tid; o < K * mc; o += LRS_NT) {
        int i = o / mc, c = o % mc;
        Zw[i * LDM + c] = Zw[(K + i) * LDM + c];
      }
      __syncthreads();
      for (int o = tid; o < K * mc; o += LRS_NT) {
        int i = o / mc, c = o % mc;
        Zw[(K + i) * LDM + c] = (b + 2 < g.nb) ? rhs_at<T, K>(a, g, (b + 2) * K + i, c, c0, Ct, Cb) : T(0);
      }
      __syncthreads();
    }
  }
  if (DSTAGE) {
    double* yt = wsp<double>(a.ws, L.ytip) + ((size_t)j * 2 + 0) * K * L.mmax;
#pragma unroll
    for (int t = 0; t < NACC; ++t) {
      int o = tid + t * LRS_NT;
      if (o < K * mc) {
        int i = o / mc, c = o % mc;
        yt[i * L.mmax + c0 + c] = acc[t];
      }
    }
  }
}

// ---------------------------------------------------------------- backward pass
// x_b = U11^{-1}(z_b - U12 x_{b+1} - U13 x_{b+2}), z read from and x written
// to a.dst (real rows).
template <typename T, int K>
__device__ void backward_pass(const SolveArgs& a, const Geom& g, int j, int c0, int mc, T* lds) {
  using LD = SwLds<K>;
  constexpr int LDK = LD::LDK, LDM = LD::LDM;
  T* X[3] = {lds + LD::oW, lds + LD::oW + K * LDM, lds + LD::oW2};
  T* Zb = lds + LD::oTmp;
  T* Ui = lds + LD::oA;
  T* U12 = lds + LD::oB;
  T* U13 = lds + LD::oC;
  const Layout& L = a.L;
  const int tid = threadIdx.x;
  const T* fac = wsp<T>(a.ws, L.fac) + (size_t)j * L.nbmax * L.rec;
  const T* swx = wsp<T>(a.ws, L.swx) + (size_t)j * L.nbmax * 3 * K * K;
  const int* flg = wsp<int>(a.ws, L.flag) + (size_t)j * L.nbmax;
  for (int o = tid; o < K * LDM; o += LRS_NT) {
    X[1][o] = T(0);
    X[2][o] = T(0);
  }
  __syncthreads();
  for (int b = g.nb - 1; b >= 0; --b) {
    const bool last = (b == g.nb - 1);
    const int fl = flg[b];
    const bool sw = (fl & 1) != 0;
    load_ufac<T, K>(fac + (size_t)b * L.rec, swx + (size_t)b * 3 * K * K, fl, last, Ui, U12, U13);
    for (int o = tid; o < K * mc; o += LRS_NT) {
      int i = o / mc, c = o % mc;
      int lr = b * K + i - g.pad;
      Zb[i * LDM + c] = (lr >= 0) ? (T)a.dst[(g.s + lr) * (int64_t)a.ld + c0 + c] : T(0);
    }
    __syncthreads();
    if (!last) {
      gemm<T, false>(K, mc, K, T(-1), U12, LDK, X[1], LDM, T(1), Zb, LDM);
      __syncthreads();
      if (sw) {
        gemm<T, false>(K, mc, K, T(-1), U13, LDK, X[2], LDM, T(1), Zb, LDM);
        __syncthreads();
      }
    }
    gemm<T, false>(K, mc, K, T(1), Ui, LDK, Zb, LDM, T(0), X[0], LDM);
    __syncthreads();
    for (int o = tid; o < K * mc; o += LRS_NT) {
      int i = o / mc, c = o % mc;
      int lr = b * K + i - g.pad;
      if (lr >= 0) a.dst[(g.s + lr) * (int64_t)a.ld + c0 + c] = (double)X[0][i * LDM + c];
    }
    __syncthreads();
    T* t2 = X[2];
    X[2] = X[1];
    X[1] = X[0];
    X[0] = t2;
  }
}

// ---------------------------------------------------------------- kernels

template <typename T, int K>
__global__ __launch_bounds__(LRS_NT) void dstage_kernel(SolveArgs a) {
  if (gated(a.gate)) return;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ int s_perm[2 * K];
  T* lds = reinterpret_cast<T*>(lds_raw);
  const int j = blockIdx.x, c0 = blockIdx.y * mc_of<K>();
  const int mc = min(mc_of<K>(), a.m - c0);
  const Geom g = part_geom(a.L, j, K);
  forward_pass<T, K, true>(a, g, j, c0, mc, lds, nullptr, nullptr, s_perm);
}

// Recovery: corrections from the neighbours' interface tips, then both passes.
template <typename T, int K>
__global__ __launch_bounds__(LRS_NT) void retrieve_kernel(SolveArgs a) {
  if (gated(a.gate)) return;
  using LD = SwLds<K>;
  constexpr int LDM = LD::LDM;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ int s_perm[2 * K];
  T* lds = reinterpret_cast<T*>(lds_raw);
  const Layout& L = a.L;
  const int j = blockIdx.x, c0 = blockIdx.y * mc_of<K>();
  const int mc = min(mc_of<K>(), a.m - c0);
  const Geom g = part_geom(L, j, K);
  T* Ct = lds + LD::oCt;
  T* Cb = lds + LD::oCb;
  T* Xn = lds + LD::oTmp;  // neighbour tip staging
  const int tid = threadIdx.x;
  const int k = L.k;
  const bool top = j > 0 && !a.block_only, bot = j < L.p - 1 && !a.block_only;
  if (top) {
    interface_tip<T, K>(a, j - 1, false, c0, mc, Xn);  // x_{j-1,b}
    __syncthreads();
    // Ct = C_j x_{j-1,b}, C_j[i][l] = A[s_j + i, s_j - K + l]
    for (int o = tid; o < K * mc; o += LRS_NT) {
      int i = o / mc, c = o % mc;
      double s = 0.0;
      for (int l = 0; l < K; ++l) s += band_at(a.bands, L.n, k, g.s + i, g.s - K + l) * (double)Xn[l * LDM + c];
      Ct[i * LDM + c] = (T)s;
    }
    __syncthreads();
  }
  if (bot) {
    interface_tip<T, K>(a, j + 1, true, c0, mc, Xn);  // x_{j+1,t}
    __syncthreads();
    // Cb = B_j x_{j+1,t}, B_j[i][l] = A[s_{j+1} - K + i, s_{j+1} + l]
    const int64_t s1 = g.s + g.nj;
    for (int o = tid; o < K * mc; o += LRS_NT) {
      int i = o / mc, c = o % mc;
      double s = 0.0;
      for (int l = 0; l < K; ++l) s += band_at(a.bands, L.n, k, s1 - K + i, s1 + l) * (double)Xn[l * LDM + c];
      Cb[i * LDM + c] = (T)s;
    }
    __syncthreads();
  }
  forward_pass<T, K, false>(a, g, j, c0, mc, lds, top ? Ct : nullptr, bot ? Cb : nullptr, s_perm);
  __syncthreads();
  backward_pass<T, K>(a, g, j, c0, mc, lds);
}

// ---------------------------------------------------------------- transposed passes
// Transposed forward: w_b = U11^{-T} (src_b - corrections + pending_b),
// pending_{b+1} -= U12^T w_b, pending_{b+2} = -U13^T w_b; w written to dst.
template <typename T, int K>
__device__ void tforward_pass(const SolveArgs& a, const Geom& g, int j, int c0, int mc, T* lds,
                              const T* Ct, const T* Cb) {
  using LD = SwLds<K>;
  constexpr int LDK = LD::LDK, LDM = LD::LDM;
  T* P0 = lds + LD::oW;            // pending for b
  T* P1 = lds + LD::oW + K * LDM;  // pending for b+1
  T* Wb = lds + LD::oW2;
  T* Rb = lds + LD::oTmp;
  T* Ui = lds + LD::oA;
  T* U12 = lds + LD::oB;
  T* U13 = lds + LD::oC;
  const Layout& L = a.L;
  const int tid = threadIdx.x;
  const T* fac = wsp<T>(a.ws, L.fac) + (size_t)j * L.nbmax * L.rec;
  const T* swx = wsp<T>(a.ws, L.swx) + (size_t)j * L.nbmax * 3 * K * K;
  const int* flg = wsp<int>(a.ws, L.flag) + (size_t)j * L.nbmax;
  for (int o = tid; o < K * LDM; o += LRS_NT) {
    P0[o] = T(0);
    P1[o] = T(0);
  }
  __syncthreads();
  for (int b = 0; b < g.nb; ++b) {
    const bool last = (b == g.nb - 1);
    const int fl = flg[b];
    const bool sw = (fl & 1) != 0;
    load_ufac<T, K>(fac + (size_t)b * L.rec, swx + (size_t)b * 3 * K * K, fl, last, Ui, U12, U13);
    for (int o = tid; o < K * mc; o += LRS_NT) {
      int i = o / mc, c = o % mc;
      Rb[i * LDM + c] = rhs_at<T, K>(a, g, b * K + i, c, c0, Ct, Cb) + P0[i * LDM + c];
    }
    __syncthreads();
    gemm<T, true>(K, mc, K, T(1), Ui, LDK, Rb, LDM, T(0), Wb, LDM);
    __syncthreads();
    if (!last) {
      gemm<T, true>(K, mc, K, T(-1), U12, LDK, Wb, LDM, T(1), P1, LDM);
      if (sw)
        gemm<T, true>(K, mc, K, T(-1), U13, LDK, Wb, LDM, T(0), P0, LDM);
      else
        for (int o = tid; o < K * LDM; o += LRS_NT) P0[o] = T(0);
    }
    for (int o = tid; o < K * mc; o += LRS_NT) {
      int i = o / mc, c = o % mc;
      int lr = b * K + i - g.pad;
      if (lr >= 0) a.dst[(g.s + lr) * (int64_t)a.ld + c0 + c] = (double)Wb[i * LDM + c];
    }
    __syncthreads();
    T* t = P0;
    P0 = P1;
    P1 = t;
  }
}

// Transposed backward: for b = last .. 0 on the window [u_b; u_{b+1}]:
// u_b = L11^{-T}(u_b - L21^T u_{b+1}), then the block's interchanges in
// reverse order; u_{b+1} is then final.  Reads and writes a.dst.
template <typename T, int K>
__device__ void tbackward_pass(const SolveArgs& a, const Geom& g, int j, int c0, int mc, T* lds,
                               int* s_perm) {
  using LD = SwLds<K>;
  constexpr int LDK = LD::LDK, LDM = LD::LDM;
  T* Uw = lds + LD::oW;  // [2K] window
  T* Ut = lds + LD::oW2;
  T* Tmp = lds + LD::oTmp;
  T* Li = lds + LD::oA;
  T* L21 = lds + LD::oB;
  const Layout& L = a.L;
  const int tid = threadIdx.x;
  const T* fac = wsp<T>(a.ws, L.fac) + (size_t)j * L.nbmax * L.rec;
  const T* swx = wsp<T>(a.ws, L.swx) + (size_t)j * L.nbmax * 3 * K * K;
  const int* ipv = wsp<int>(a.ws, L.ipiv) + (size_t)j * L.nbmax * K;
  const int* flg = wsp<int>(a.ws, L.flag) + (size_t)j * L.nbmax;
  auto store_block = [&](int b, const T* src) {
    for (int o = tid; o < K * mc; o += LRS_NT) {
      int i = o / mc, c = o % mc;
      int lr = b * K + i - g.pad;
      if (lr >= 0) a.dst[(g.s + lr) * (int64_t)a.ld + c0 + c] = (double)src[i * LDM + c];
    }
  };
  for (int b = g.nb - 1; b >= 0; --b) {
    const bool last = (b == g.nb - 1);
    const int fl = flg[b];
    const bool sw = (fl & 1) != 0;
    load_lfac<T, K>(fac + (size_t)b * L.rec, swx + (size_t)b * 3 * K * K, fl, last, Li, L21);
    for (int o = tid; o < K * mc; o += LRS_NT) {
      int i = o / mc, c = o % mc;
      int lr = b * K + i - g.pad;
      Ut[i * LDM + c] = (lr >= 0) ? (T)a.dst[(g.s + lr) * (int64_t)a.ld + c0 + c] : T(0);
    }
    __syncthreads();
    if (!last) {
      gemm<T, true>(K, mc, K, T(-1), L21, LDK, Uw + K * LDM, LDM, T(1), Ut, LDM);
      __syncthreads();
    }
    gemm<T, true>(K, mc, K, T(1), Li, LDK, Ut, LDM, T(0), Uw, LDM);
    __syncthreads();
    if (sw) permute_rows_t<T, K>(Uw, LDM, last ? K : 2 * K, mc, ipv + (size_t)b * K, s_perm, Tmp);
    if (!last) store_block(b + 1, Uw + K * LDM);
    __syncthreads();
    // carry u_b down to the window's second half
    for (int o = tid; o < K * mc; o += LRS_NT) {
      int i = o / mc, c = o % mc;
      Uw[(K + i) * LDM + c] = Uw[i * LDM + c];
    }
    __syncthreads();
  }
  store_block(0, Uw + K * LDM);
  __syncthreads();
}

// Adjoint D-stage: nu_j = A_j^{-T} g_j into the scratch (full), tips into ytip.
template <typename T, int K>
__global__ __launch_bounds__(LRS_NT) void adj_dstage_kernel(SolveArgs a) {
  if (gated(a.gate)) return;
  if (a.only_flagged && wsp<int>(a.ws, a.L.npv)[blockIdx.x] == 0) return;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ int s_perm[2 * K];
  T* lds = reinterpret_cast<T*>(lds_raw);
  const Layout& L = a.L;
  const int j = blockIdx.x, c0 = blockIdx.y * mc_of<K>();
  const int mc = min(mc_of<K>(), a.m - c0);
  const Geom g = part_geom(L, j, K);
  tforward_pass<T, K>(a, g, j, c0, mc, lds, nullptr, nullptr);
  __syncthreads();
  tbackward_pass<T, K>(a, g, j, c0, mc, lds, s_perm);
  // tips nu_t (first K real rows) and nu_b (last K rows)
  double* yt = wsp<double>(a.ws, L.ytip) + (size_t)j * 2 * K * L.mmax;
  for (int o = threadIdx.x; o < 2 * K * mc; o += LRS_NT) {
    int which = o / (K * mc), e = o % (K * mc), i = e / mc, c = e % mc;
    int lr = which == 0 ? i : g.nj - K + i;
    yt[((size_t)which * K + i) * L.mmax + c0 + c] = a.dst[(g.s + lr) * (int64_t)a.ld + c0 + c];
  }
}

// Adjoint recovery: lambda_j = A_j^{-T}(g_j - [w_{j,t}; 0; w_{j,b}]) with
//   w_{j,t} = B_{j-1}^T nu_{j-1,b} - Pi_{j-1} u_a(j-1)      (j >= 1)
//   w_{j,b} = C_{j+1}^T nu_{j+1,t} - Psi_{j+1} u_c(j+1)      (j <= p-2)
// where u = Z^{-T} L^T h sits in the compressed vector.
template <typename T, int K>
__global__ __launch_bounds__(LRS_NT) void adj_retrieve_kernel(SolveArgs a) {
  if (gated(a.gate)) return;
  if (a.only_flagged && wsp<int>(a.ws, a.L.npv)[blockIdx.x] == 0) return;
  using LD = SwLds<K>;
  constexpr int LDM = LD::LDM;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ int s_perm[2 * K];
  T* lds = reinterpret_cast<T*>(lds_raw);
  const Layout& L = a.L;
  const int j = blockIdx.x, c0 = blockIdx.y * mc_of<K>();
  const int mc = min(mc_of<K>(), a.m - c0);
  const Geom g = part_geom(L, j, K);
  T* Ct = lds + LD::oCt;
  T* Cb = lds + LD::oCb;
  const int tid = threadIdx.x, k = L.k, r = L.r;
  const double* ytip = wsp<double>(a.ws, L.ytip);
  const double* proj = wsp<double>(a.ws, L.proj);  // Pi, Psi per partition (K x r)
  const double* zg = wsp<double>(a.ws, L.zg);
  if (j > 0) {
    // w_{j,t}[i] = sum_l B_{j-1}[l][i] nu_{j-1,b}[l] - sum_q Pi_{j-1}[i][q] u_a(j-1)[q]
    const double* nub = ytip + ((size_t)(j - 1) * 2 + 1) * K * L.mmax;
    const double* Pi = proj + (size_t)(j - 1) * 2 * K * r;
    const double* ua = zg + (size_t)(j - 1) * L.R2 * L.mmax;
    for (int o = tid; o < K * mc; o += LRS_NT) {
      int i = o / mc, c = o % mc;
      double s = 0.0;
      for (int l = 0; l < K; ++l) s += band_at(a.bands, L.n, k, g.s - K + l, g.s + i) * nub[l * L.mmax + c0 + c];
      for (int q = 0; q < r; ++q) s -= Pi[i * r + q] * ua[q * L.mmax + c0 + c];
      Ct[i * LDM + c] = (T)s;
    }
  }
  if (j < L.p - 1) {
    const double* nut = ytip + ((size_t)(j + 1) * 2 + 0) * K * L.mmax;
    const double* Psi = proj + ((size_t)(j + 1) * 2 + 1) * K * r;
    const double* uc = zg + ((size_t)j * L.R2 + r) * L.mmax;
    const int64_t s1 = g.s + g.nj;
    for (int o = tid; o < K * mc; o += LRS_NT) {
      int i = o / mc, c = o % mc;
      double s = 0.0;
      // C_{j+1}[l][i] = A[s_{j+1} + l, s_{j+1} - K + i]
      for (int l = 0; l < K; ++l) s += band_at(a.bands, L.n, k, s1 + l, s1 - K + i) * nut[l * L.mmax + c0 + c];
      for (int q = 0; q < r; ++q) s -= Psi[i * r + q] * uc[q * L.mmax + c0 + c];
      Cb[i * LDM + c] = (T)s;
    }
  }
  __syncthreads();
  tforward_pass<T, K>(a, g, j, c0, mc, lds, j > 0 ? Ct : nullptr, j < L.p - 1 ? Cb : nullptr);
  __syncthreads();
  tbackward_pass<T, K>(a, g, j, c0, mc, lds, s_perm);
}

// ---------------------------------------------------------------- FP64 band kernels

// r = f - op(A) x (op(A) = A or A^T), FP64, for RES_ROWS rows per workgroup in
// chunks of RES_MC columns: the x rows a block needs (RES_ROWS + 2k) are staged
// in LDS once per chunk, each thread owns one row and the chunk's columns (every
// band entry is read once, coalesced along the diagonal), and f and r pass
// through LDS so that their global accesses are coalesced too.
#define RES_ROWS 256
#define RES_MC 16
__global__ __launch_bounds__(RES_ROWS) void residual_kernel(const double* __restrict__ bands, int64_t n, int k,
                                                            const double* __restrict__ f,
                                                            const double* __restrict__ x,
                                                            double* __restrict__ out, int ld, int m,
                                                            int transpose, const int* gate) {
  if (gated(gate)) return;
  extern __shared__ double xs[];  // (RES_ROWS + 2k) x PX
  // odd pitch: the rows the lanes of a wave read lie in different LDS banks
  constexpr int PX = RES_MC + 1;
  const int t = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * RES_ROWS, i = i0 + t;
  const int rows = RES_ROWS + 2 * k;
  for (int c0 = 0; c0 < m; c0 += RES_MC) {
    const int mc = min(RES_MC, m - c0);
    __syncthreads();
    for (int o = t; o < rows * mc; o += RES_ROWS) {
      const int rr = o / mc, cc = o % mc;
      const int64_t gi = i0 - k + rr;
      xs[rr * PX + cc] = (gi >= 0 && gi < n) ? x[gi * ld + c0 + cc] : 0.0;
    }
    __syncthreads();
    double acc[RES_MC];
#pragma unroll
    for (int cc = 0; cc < RES_MC; ++cc) acc[cc] = 0.0;
    if (i < n) {
      // band entries in groups of RES_DG diagonals: the group's loads are
      // issued together (unconditional, from clamped addresses) before use
      constexpr int RES_DG = 8;
      for (int d0 = -k; d0 <= k; d0 += RES_DG) {
        double av[RES_DG];
#pragma unroll
        for (int u = 0; u < RES_DG; ++u) {
          const int d = min(d0 + u, k);
          const int64_t jj = min(max(i + d, (int64_t)0), n - 1);
          av[u] = transpose ? bands[(int64_t)(-d + k) * n + jj] : bands[(int64_t)(d + k) * n + i];
        }
#pragma unroll
        for (int u = 0; u < RES_DG; ++u) {
          const int d = d0 + u;
          const int64_t jj = i + d;
          const double a = (d <= k && jj >= 0 && jj < n) ? av[u] : 0.0;
          const double* xr = xs + (t + min(d, k) + k) * PX;
#pragma unroll
          for (int cc = 0; cc < RES_MC; ++cc) acc[cc] = fma(-a, xr[cc], acc[cc]);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int cc = 0; cc < RES_MC; ++cc) xs[t * PX + cc] = acc[cc];
    __syncthreads();
    for (int o = t; o < RES_ROWS * mc; o += RES_ROWS) {
      const int rr = o / mc, cc = o % mc;
      const int64_t gi = i0 + rr;
      if (gi < n) out[gi * ld + c0 + cc] = f[gi * ld + c0 + cc] + xs[rr * PX + cc];
    }
  }
}

// grad[(d+k) n + i] = - sum_c lam[i, c] x[i+d, c]
__global__ void band_grad_kernel(int64_t n, int k, const double* __restrict__ lam,
                                 const double* __restrict__ x, int ld, int m,
                                 double* __restrict__ grad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int d = (int)blockIdx.y - k;
  if (i >= n) return;
  double s = 0.0;
  int64_t jj = i + d;
  if (jj >= 0 && jj < n)
    for (int c = 0; c < m; ++c) s -= lam[i * ld + c] * x[jj * ld + c];
  grad[(int64_t)(d + k) * n + i] = s;
}

}  // namespace lrs
