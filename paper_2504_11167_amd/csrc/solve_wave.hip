// Matrix-core sweeps for K >= 16: one wave per (partition, chunk of up to
// 16 * MCT right-hand-side columns), no workgroup barriers.
//
// The right-hand-side strip of a block (K rows x 16 columns per column tile)
// lives in 16x16 accumulator tiles.  With the k permutation of fidx, the
// accumulator element v of tile t is exactly the B operand of k-step 4t + v,
// so a product's result feeds the next product without leaving registers.
// The A operands (L11^{-1}, L21, G^T, U11^{-1}, U12, U13) are loaded as whole
// fragments from the fragment-ordered factor records, one block ahead.
//
// D-stage  (eq. D-stage of the solve summary): forward L^{-1} P^T over f,
//          y_t = G^T z accumulated, y_b = U11^{-1} z_last.
// Recovery (eqs. recovery1/2): forward over f minus the interface
//          corrections with z stored in x, then x_b = U11^{-1}(z_b - U12 x_{b+1} - U13 x_{b+2}).
#include "sweep.h"

namespace lrs {

template <typename T, int K, int MCT>
struct WaveSweep {
  static constexpr int RT = K / 16;  // 16-row tiles per block
  static constexpr int KS = K / 4;   // k-steps per block product
  static constexpr int NC = 16 * MCT;
  using V = typename AccVec<T>::type;
  // LDS: row-major staging for interchanges (2K x NC), interface corrections
  // (2 x K x NC), neighbour tip (K x NC), permutation (2K ints)
  static constexpr int oStage = 0;
  static constexpr int oCt = oStage + 2 * K * NC;
  static constexpr int oCb = oCt + K * NC;
  static constexpr int oXn = oCb + K * NC;
  static constexpr int total = oXn + K * NC;
};

// Masked A-operand element for lane `lane` of fragment (t, step).
//   kind 0: L11^{-1} from LP (strict lower + unit diagonal)
//   kind 1: L21 from LP (upper incl. diagonal)
//   kind 2: U11^{-1} from UP (upper incl. diagonal)
//   kind 3: U12 from UP (strict lower) + its diagonal, passed per fragment in dg
template <typename T, int kind>
__device__ __forceinline__ T fmask(T v, int t, int step, int lane, T dg) {
  const int i = 16 * t + (lane & 15);
  const int kk = frag_k<T>(step, lane >> 4);
  if constexpr (kind == 0) return i > kk ? v : (i == kk ? T(1) : T(0));
  if constexpr (kind == 1) return i <= kk ? v : T(0);
  if constexpr (kind == 2) return i <= kk ? v : T(0);
  if constexpr (kind == 3) return i > kk ? v : dg;
  // transposed operands, v = M(kk, i) gathered by load_tfrags:
  if constexpr (kind == 4) return i < kk ? v : (i == kk ? T(1) : T(0));  // (L11^{-1})^T, unit upper
  if constexpr (kind == 5) return i >= kk ? v : T(0);                    // L21^T, (U11^{-1})^T: lower
  if constexpr (kind == 7) return kk > i ? v : T(0);                     // U12^T without its diagonal
  return v;
}

// strip (K rows x NC columns) <-> global rows of the partition
template <typename T, int K, int MCT>
__device__ __forceinline__ void load_strip(typename WaveSweep<T, K, MCT>::V (&st)[K / 16][MCT],
                                           const double* src, int64_t ld, const Geom& g, int R,
                                           int c0, int m, const T* Ct, const T* Cb) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < K / 16; ++t)
#pragma unroll
    for (int ct = 0; ct < MCT; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * t + acc_row<T>(lane, v), col = 16 * ct + (lane & 15);
        const int lr = R * K + row - g.pad;
        T x = T(0);
        if (lr >= 0 && lr < g.nj && c0 + col < m) {
          x = (T)src[(g.s + lr) * ld + c0 + col];
          if (Ct && lr < K) x -= Ct[lr * (16 * MCT) + col];
          if (Cb && lr >= g.nj - K) x -= Cb[(lr - (g.nj - K)) * (16 * MCT) + col];
        }
        st[t][ct][v] = x;
      }
}

// strip -= the interface corrections of its rows (rows in the first K and the
// last K real rows of the partition); callers skip blocks without such rows
template <typename T, int K, int MCT>
__device__ __forceinline__ void sub_corr(typename WaveSweep<T, K, MCT>::V (&st)[K / 16][MCT], const Geom& g, int R,
                                         const T* Ct, const T* Cb) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < K / 16; ++t)
#pragma unroll
    for (int ct = 0; ct < MCT; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * t + acc_row<T>(lane, v), col = 16 * ct + (lane & 15);
        const int lr = R * K + row - g.pad;
        if (lr >= 0 && lr < g.nj) {
          if (Ct && lr < K) st[t][ct][v] -= Ct[lr * (16 * MCT) + col];
          if (Cb && lr >= g.nj - K) st[t][ct][v] -= Cb[(lr - (g.nj - K)) * (16 * MCT) + col];
        }
      }
}

// does block R hold rows that take an interface correction?
__device__ __forceinline__ bool corr_block(const Geom& g, int K, int R) {
  const int lo = R * K - g.pad, hi = lo + K - 1;
  return lo < K || hi >= g.nj - K;
}

template <typename T, int K, int MCT>
__device__ __forceinline__ void store_strip(const typename WaveSweep<T, K, MCT>::V (&st)[K / 16][MCT],
                                            double* dst, int64_t ld, const Geom& g, int R, int c0,
                                            int m) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < K / 16; ++t)
#pragma unroll
    for (int ct = 0; ct < MCT; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * t + acc_row<T>(lane, v), col = 16 * ct + (lane & 15);
        const int lr = R * K + row - g.pad;
        if (lr >= 0 && c0 + col < m) dst[(g.s + lr) * ld + c0 + col] = (double)st[t][ct][v];
      }
}

// Interchanges of a block applied to the window strips (rows of w0 then w1),
// through LDS (rare: only blocks whose factorization interchanged rows).
template <typename T, int K, int MCT>
__device__ void permute_strips(typename WaveSweep<T, K, MCT>::V (&w0)[K / 16][MCT],
                               typename WaveSweep<T, K, MCT>::V (&w1)[K / 16][MCT], bool two,
                               const int* ipiv_g, T* stage, int* perm) {
  constexpr int NC = 16 * MCT;
  const int lane = threadIdx.x & 63;
  const int nr = two ? 2 * K : K;
  if (lane == 0) {
    for (int q = 0; q < nr; ++q) perm[q] = q;
    for (int c = 0; c < K; ++c) {
      int pv = ipiv_g[c];
      int t = perm[c];
      perm[c] = perm[pv];
      perm[pv] = t;
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int t = 0; t < K / 16; ++t)
#pragma unroll
      for (int ct = 0; ct < MCT; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = h * K + 16 * t + acc_row<T>(lane, v), col = 16 * ct + (lane & 15);
          stage[row * NC + col] = h ? w1[t][ct][v] : w0[t][ct][v];
        }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int t = 0; t < K / 16; ++t)
#pragma unroll
      for (int ct = 0; ct < MCT; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = h * K + 16 * t + acc_row<T>(lane, v), col = 16 * ct + (lane & 15);
          if (row < nr) {
            T x = stage[perm[row] * NC + col];
            if (h)
              w1[t][ct][v] = x;
            else
              w0[t][ct][v] = x;
          }
        }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// out[t][ct] (+)= sign * A(kind) * in  for one K x K block; A fragments from frag[].
// The 16 x 16 tiles a triangular operand leaves zero are skipped (k-steps 4q..4q+3
// cover columns 16q..16q+15): lower operands (kinds 0, 3) right of the row tile,
// upper ones (kinds 1, 2) left of it.
template <typename T, int K, int MCT, int kind>
__device__ __forceinline__ void blk_mul(const T (&frag)[(K / 16) * (K / 4)], const T* dg, T sign,
                                        const typename WaveSweep<T, K, MCT>::V (&in)[K / 16][MCT],
                                        typename WaveSweep<T, K, MCT>::V (&out)[K / 16][MCT]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < K / 16; ++t)
#pragma unroll
    for (int step = 0; step < K / 4; ++step) {
      if (((kind == 0 || kind == 3 || kind == 5) && (step >> 2) > t) ||
          ((kind == 1 || kind == 2 || kind == 4 || kind == 7) && (step >> 2) < t))
        continue;
      const T av = sign * fmask<T, kind>(frag[t * (K / 4) + step], t, step, lane,
                                         kind == 3 ? dg[t * (K / 4) + step] : T(0));
#pragma unroll
      for (int ct = 0; ct < MCT; ++ct) out[t][ct] = mfma_step(av, in[step >> 2][ct][step & 3], out[t][ct]);
    }
}

template <typename T, int K>
__device__ __forceinline__ void load_frags(T (&dst)[(K / 16) * (K / 4)], const T* src) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int f = 0; f < (K / 16) * (K / 4); ++f) dst[f] = src[(f << 6) + lane];
}

// Fragments of M^T as the A operand: lane holds M(kk, i) for (i, kk) =
// (16 t + lane mod 16, frag_k(step, lane / 16)), gathered inside the K x K
// record block (a few cache lines); blk_mul's transposed kinds mask them.
template <typename T, int K>
__device__ __forceinline__ void load_tfrags(T (&dst)[(K / 16) * (K / 4)], const T* blk) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < K / 16; ++t)
#pragma unroll
    for (int step = 0; step < K / 4; ++step)
      dst[t * (K / 4) + step] = blk[fidx<T, K>(frag_k<T>(step, lane >> 4), 16 * t + (lane & 15))];
}

// Diagonal of U12 (UD vector of the record) at the strip rows a lane holds.
template <typename T, int K>
__device__ __forceinline__ void load_udrows(T (&dst)[K / 16][4], const T* ud) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < K / 16; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) dst[t][v] = ud[16 * t + acc_row<T>(lane, v)];
}

// out -= U12 x with U12 = strict lower part of UP + diag(UD) (no side slot)
template <typename T, int K, int MCT>
__device__ __forceinline__ void u12_mul(const T (&up)[(K / 16) * (K / 4)], const T (&udr)[K / 16][4],
                                        const typename WaveSweep<T, K, MCT>::V (&x)[K / 16][MCT],
                                        typename WaveSweep<T, K, MCT>::V (&out)[K / 16][MCT]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < K / 16; ++t)
#pragma unroll
    for (int step = 0; step < K / 4; ++step) {
      if ((step >> 2) > t) continue;  // strictly lower: zero right of the row tile
      const int i = 16 * t + (lane & 15), kk = frag_k<T>(step, lane >> 4);
      const T av = (i > kk) ? -up[t * (K / 4) + step] : T(0);
#pragma unroll
      for (int ct = 0; ct < MCT; ++ct) out[t][ct] = mfma_step(av, x[step >> 2][ct][step & 3], out[t][ct]);
    }
#pragma unroll
  for (int t = 0; t < K / 16; ++t)
#pragma unroll
    for (int ct = 0; ct < MCT; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) out[t][ct][v] -= udr[t][v] * x[t][ct][v];
}

template <typename T, int K, int MCT>
__device__ __forceinline__ void zero_strip(typename WaveSweep<T, K, MCT>::V (&st)[K / 16][MCT]) {
#pragma unroll
  for (int t = 0; t < K / 16; ++t)
#pragma unroll
    for (int ct = 0; ct < MCT; ++ct) st[t][ct] = typename WaveSweep<T, K, MCT>::V{0, 0, 0, 0};
}

// Prefetch distance of the sweeps in blocks: the records and right-hand-side
// rows of block b + PD are requested while block b is processed.  With one
// wave per partition the chain of one block does not cover the memory
// latency; the short blocks at K = 16 take the deeper ring (at most 63 loads
// may be outstanding per wave; a K = 16 block issues about a dozen).
template <int K, int MCT>
constexpr int sweep_pd() { return (K <= 16 && MCT == 1) ? 4 : 2; }

// Calls f(std::integral_constant<int, u>) for u = 0 .. N-1.
template <int N, int U = 0, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (U < N) {
    f(std::integral_constant<int, U>{});
    static_for<N, U + 1>(f);
  }
}

// Right-hand-side rows of one partition through a buffer descriptor whose
// range is the partition's rows: an element outside the partition or the
// column range gets an offset past the range, so its load returns 0 and its
// store is dropped by the hardware.  No element needs a branch, every load is
// issued unconditionally, and the wait counts stay exact across the
// unrolled block loop.  (The host keeps rows x ld x 8 below 2^31.)
typedef unsigned int lrs_u32x2 __attribute__((ext_vector_type(2)));
struct RowBuf {
  __amdgpu_buffer_rsrc_t rs;
  int ld, nj, pad, mcol;  // mcol: columns of this chunk (c < mcol valid)
};
__device__ __forceinline__ RowBuf row_buf(const double* base, const Geom& g, int64_t ld, int c0, int m) {
  RowBuf rb;
  rb.rs = __builtin_amdgcn_make_buffer_rsrc((void*)(base + g.s * ld + c0), 0, (int)((int64_t)g.nj * ld * 8),
                                            0x00020000);
  rb.ld = (int)ld;
  rb.nj = g.nj;
  rb.pad = g.pad;
  rb.mcol = m - c0;
  return rb;
}
__device__ __forceinline__ int row_off(const RowBuf& rb, int lr, int col) {
  return (lr >= 0 && lr < rb.nj && col < rb.mcol) ? (lr * rb.ld + col) * 8 : 0x7FFFFFF8;
}
template <typename T, int K, int MCT>
__device__ __forceinline__ void buf_load_strip(typename WaveSweep<T, K, MCT>::V (&st)[K / 16][MCT], const RowBuf& rb,
                                               int R) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < K / 16; ++t)
#pragma unroll
    for (int ct = 0; ct < MCT; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * t + acc_row<T>(lane, v), col = 16 * ct + (lane & 15);
        const lrs_u32x2 raw = __builtin_amdgcn_raw_buffer_load_b64(rb.rs, row_off(rb, R * K + row - rb.pad, col), 0, 0);
        st[t][ct][v] = (T)__builtin_bit_cast(double, raw);
      }
}
template <typename T, int K, int MCT>
__device__ __forceinline__ void buf_store_strip(const typename WaveSweep<T, K, MCT>::V (&st)[K / 16][MCT],
                                                const RowBuf& rb, int R) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < K / 16; ++t)
#pragma unroll
    for (int ct = 0; ct < MCT; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * t + acc_row<T>(lane, v), col = 16 * ct + (lane & 15);
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(lrs_u32x2, (double)st[t][ct][v]), rb.rs,
                                              row_off(rb, R * K + row - rb.pad, col), 0, 0);
      }
}

// Forward pass L^{-1} P^T over the partition (rhs minus optional corrections).
// DSTAGE: accumulate y_t = G^T z and write y_b, y_t to the tip buffer;
// otherwise z is written to a.dst.  The per-block data live in rings of
// NS = PD + 1 register slots, block b in slot b mod NS; the block loop is
// unrolled NS times so that every slot index is a compile-time constant, and
// every prefetch is issued unconditionally (a block past the end re-reads the
// last one).  SWP: the partition was factored with interchanges (block
// flags, permutations and side-slot factors are read); without it no flag is
// read at all.
template <typename T, int K, int MCT, bool DSTAGE, bool SWP>
__device__ void fwd_wave_impl(const SolveArgs& a, const Geom& g, int j, int c0, T* lds, const T* Ct, const T* Cb) {
  using W = WaveSweep<T, K, MCT>;
  using V = typename W::V;
  constexpr int NF = W::RT * W::KS, PD = sweep_pd<K, MCT>(), NS = PD + 1;
  const Layout& L = a.L;
  const int lane = threadIdx.x & 63, nb = g.nb;
  const T* fac = wsp<T>(a.ws, L.fac) + (size_t)j * L.nbmax * L.rec;
  const T* swx = wsp<T>(a.ws, L.swx) + (size_t)j * L.nbmax * 3 * K * K;
  const T* gm = wsp<T>(a.ws, L.gmat) + (size_t)j * L.nbmax * K * K;
  const int* ipv = wsp<int>(a.ws, L.ipiv) + (size_t)j * L.nbmax * K;
  const int* flg = wsp<int>(a.ws, L.flag) + (size_t)j * L.nbmax;
  int* perm = reinterpret_cast<int*>(lds + W::total);
  const RowBuf src = row_buf(a.src, g, a.ld, c0, a.m);
  const RowBuf dst = row_buf(a.dst, g, a.ld, c0, a.m);
  V z[W::RT][MCT], acc[W::RT][MCT], rows[NS][W::RT][MCT];  // rows[b mod NS]: r_b, updated in place
  T lpq[NS][NF], gtq[NS][NF];
  zero_strip<T, K, MCT>(acc);
  auto fetch_rec = [&](int q, T (&lp)[NF], T (&gt)[NF]) __attribute__((always_inline)) {
    const int qc = min(q, nb - 1);
    load_frags<T, K>(lp, fac + (size_t)qc * L.rec);
    if (DSTAGE) load_frags<T, K>(gt, gm + (size_t)qc * K * K);
  };
  // block 0 with its interface corrections, then the first PD records and rows
  buf_load_strip<T, K, MCT>(rows[0], src, 0);
  if (Ct || Cb) sub_corr<T, K, MCT>(rows[0], g, 0, Ct, Cb);
  static_for<PD>([&](auto U) __attribute__((always_inline)) {
    constexpr int u = decltype(U)::value;
    fetch_rec(u, lpq[u], gtq[u]);
    buf_load_strip<T, K, MCT>(rows[u + 1], src, u + 1);
  });
  auto body = [&](auto U, int b) __attribute__((always_inline)) {
    constexpr int u = decltype(U)::value;  // slot of block b
    constexpr int u1 = (u + 1) % NS;       // rows of block b + 1
    constexpr int uf = (u + PD) % NS;      // slot that receives the records of block b + PD
    const bool last = (b == nb - 1);
    fetch_rec(b + PD, lpq[uf], gtq[uf]);
    T (&lp)[NF] = lpq[u];
    V (&w0)[W::RT][MCT] = rows[u];
    V (&w1)[W::RT][MCT] = rows[u1];
    if ((Ct || Cb) && !last && corr_block(g, K, b + 1)) sub_corr<T, K, MCT>(w1, g, b + 1, Ct, Cb);
    int fl = 0;
    if constexpr (SWP) {
      fl = flg[b];
      if (fl & 1) permute_strips<T, K, MCT>(w0, w1, !last, ipv + (size_t)b * K, lds + W::oStage, perm);
    }
    zero_strip<T, K, MCT>(z);
    blk_mul<T, K, MCT, 0>(lp, nullptr, T(1), w0, z);  // z_b = L11^{-1} r_b
    buf_load_strip<T, K, MCT>(rows[u], src, b + 1 + PD);  // slot (b + 1 + PD) mod NS = u, free once z_b is formed
    if (!last) {
      if (SWP && (fl & 1)) {
        T l21[NF];
        load_frags<T, K>(l21, swx + (size_t)b * 3 * K * K);
        blk_mul<T, K, MCT, 9>(l21, nullptr, T(-1), z, w1);
      } else {
        blk_mul<T, K, MCT, 1>(lp, nullptr, T(-1), z, w1);  // r_{b+1} -= L21 z_b
      }
    }
    if (DSTAGE)
      blk_mul<T, K, MCT, 9>(gtq[u], nullptr, T(1), z, acc);  // y_t += G^T z_b
    else
      buf_store_strip<T, K, MCT>(z, dst, b);
  };
  int b0 = 0;
  for (; b0 + NS <= nb; b0 += NS)
    static_for<NS>([&](auto U) __attribute__((always_inline)) { body(U, b0 + decltype(U)::value); });
  static_for<NS>([&](auto U) __attribute__((always_inline)) {
    if (b0 + decltype(U)::value < nb) body(U, b0 + decltype(U)::value);
  });
  if (DSTAGE) {
    // y_b = U11^{-1} z_last; y_t and y_b to the tip buffer
    T up[NF];
    load_frags<T, K>(up, fac + (size_t)(nb - 1) * L.rec + K * K);
    V yb[W::RT][MCT];
    zero_strip<T, K, MCT>(yb);
    blk_mul<T, K, MCT, 2>(up, nullptr, T(1), z, yb);
    double* yt = wsp<double>(a.ws, L.ytip) + (size_t)j * 2 * K * L.mmax;
#pragma unroll
    for (int t = 0; t < W::RT; ++t)
#pragma unroll
      for (int ct = 0; ct < MCT; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 16 * t + acc_row<T>(lane, v), col = 16 * ct + (lane & 15);
          if (c0 + col < a.m) {
            yt[(size_t)row * L.mmax + c0 + col] = (double)acc[t][ct][v];
            yt[(size_t)(K + row) * L.mmax + c0 + col] = (double)yb[t][ct][v];
          }
        }
  }
}

template <typename T, int K, int MCT, bool DSTAGE>
__device__ void fwd_wave(const SolveArgs& a, const Geom& g, int j, int c0, T* lds, const T* Ct, const T* Cb) {
  if (wsp<int>(a.ws, a.L.npv)[j] != 0)
    fwd_wave_impl<T, K, MCT, DSTAGE, true>(a, g, j, c0, lds, Ct, Cb);
  else
    fwd_wave_impl<T, K, MCT, DSTAGE, false>(a, g, j, c0, lds, Ct, Cb);
}

// Backward pass x_b = U11^{-1}(z_b - U12 x_{b+1} - U13 x_{b+2}) over a.dst,
// blocks from the last to the first; the q-th block visited (b = nb - 1 - q)
// lives in ring slot q mod NS (same ring as the forward pass).
template <typename T, int K, int MCT, bool SWP>
__device__ void bwd_wave_impl(const SolveArgs& a, const Geom& g, int j, int c0) {
  using W = WaveSweep<T, K, MCT>;
  using V = typename W::V;
  constexpr int NF = W::RT * W::KS, PD = sweep_pd<K, MCT>(), NS = PD + 1;
  const Layout& L = a.L;
  const int nb = g.nb;
  const T* fac = wsp<T>(a.ws, L.fac) + (size_t)j * L.nbmax * L.rec;
  const T* swx = wsp<T>(a.ws, L.swx) + (size_t)j * L.nbmax * 3 * K * K;
  const int* flg = wsp<int>(a.ws, L.flag) + (size_t)j * L.nbmax;
  const RowBuf xb_buf = row_buf(a.dst, g, a.ld, c0, a.m);
  V x1[W::RT][MCT], x2[W::RT][MCT], xb[W::RT][MCT], zq[NS][W::RT][MCT];
  T upq[NS][NF], udq[NS][W::RT][4];
  zero_strip<T, K, MCT>(x1);
  zero_strip<T, K, MCT>(x2);
  auto fetch = [&](int q, T (&up)[NF], T (&ud)[W::RT][4], V (&zs)[W::RT][MCT]) __attribute__((always_inline)) {
    const int b = max(nb - 1 - q, 0);
    load_frags<T, K>(up, fac + (size_t)b * L.rec + K * K);
    load_udrows<T, K>(ud, fac + (size_t)b * L.rec + 2 * K * K);
    buf_load_strip<T, K, MCT>(zs, xb_buf, nb - 1 - q);  // rows before the partition read as 0
  };
  static_for<PD>([&](auto U) __attribute__((always_inline)) {
    constexpr int u = decltype(U)::value;
    fetch(u, upq[u], udq[u], zq[u]);
  });
  auto body = [&](auto U, int q) __attribute__((always_inline)) {
    constexpr int u = decltype(U)::value, uf = (u + PD) % NS;
    const int b = nb - 1 - q;
    const bool last = (q == 0);
    fetch(q + PD, upq[uf], udq[uf], zq[uf]);
    T (&up)[NF] = upq[u];
    V (&zb)[W::RT][MCT] = zq[u];
    if (!last) {
      int fl = 0;
      if constexpr (SWP) fl = flg[b];
      if (SWP && (fl & 2)) {
        T u12[NF];
        load_frags<T, K>(u12, swx + (size_t)b * 3 * K * K + K * K);
        blk_mul<T, K, MCT, 9>(u12, nullptr, T(-1), x1, zb);
      } else {
        u12_mul<T, K, MCT>(up, udq[u], x1, zb);  // z_b -= U12 x_{b+1}
      }
      if (SWP && (fl & 1)) {
        T u13[NF];
        load_frags<T, K>(u13, swx + (size_t)b * 3 * K * K + 2 * K * K);
        blk_mul<T, K, MCT, 9>(u13, nullptr, T(-1), x2, zb);
      }
    }
    zero_strip<T, K, MCT>(xb);
    blk_mul<T, K, MCT, 2>(up, nullptr, T(1), zb, xb);  // x_b = U11^{-1} (...)
    buf_store_strip<T, K, MCT>(xb, xb_buf, b);
#pragma unroll
    for (int t = 0; t < W::RT; ++t)
#pragma unroll
      for (int ct = 0; ct < MCT; ++ct) {
        x2[t][ct] = x1[t][ct];
        x1[t][ct] = xb[t][ct];
      }
  };
  int q0 = 0;
  for (; q0 + NS <= nb; q0 += NS)
    static_for<NS>([&](auto U) __attribute__((always_inline)) { body(U, q0 + decltype(U)::value); });
  static_for<NS>([&](auto U) __attribute__((always_inline)) {
    if (q0 + decltype(U)::value < nb) body(U, q0 + decltype(U)::value);
  });
}

template <typename T, int K, int MCT>
__device__ void bwd_wave(const SolveArgs& a, const Geom& g, int j, int c0) {
  if (wsp<int>(a.ws, a.L.npv)[j] != 0)
    bwd_wave_impl<T, K, MCT, true>(a, g, j, c0);
  else
    bwd_wave_impl<T, K, MCT, false>(a, g, j, c0);
}

template <typename T, int K, int MCT>
__global__ __launch_bounds__(64) __attribute__((aligned(4096))) void dstage_wave_kernel(SolveArgs a) {
  if (gated(a.gate)) return;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* lds = reinterpret_cast<T*>(lds_raw);
  const int j = blockIdx.x, c0 = blockIdx.y * 16 * MCT;
  const Geom g = part_geom(a.L, j, K);
  fwd_wave<T, K, MCT, true>(a, g, j, c0, lds, nullptr, nullptr);
}

template <typename T, int K, int MCT>
__global__ __launch_bounds__(64) __attribute__((aligned(4096))) void retrieve_wave_kernel(SolveArgs a) {
  if (gated(a.gate)) return;
  using W = WaveSweep<T, K, MCT>;
  constexpr int NC = W::NC;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* lds = reinterpret_cast<T*>(lds_raw);
  const Layout& L = a.L;
  const int j = blockIdx.x, c0 = blockIdx.y * NC;
  const int mc = min(NC, a.m - c0);
  const Geom g = part_geom(L, j, K);
  const int lane = threadIdx.x & 63, k = L.k;
  T* Ct = lds + W::oCt;
  T* Cb = lds + W::oCb;
  T* Xn = lds + W::oXn;
  auto sync = [] {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  };
  // Xn uses the generic interface-tip routine with its pitch MC + 1; keep a
  // local copy of the logic at pitch NC instead.
  auto tip = [&](int i, bool top) {
    const int r = L.r;
    const double* yt = wsp<double>(a.ws, L.ytip) + ((size_t)i * 2 + (top ? 0 : 1)) * K * L.mmax;
    const double* pt = wsp<double>(a.ws, L.ptip) + (size_t)i * 4 * K * r;
    const double* P = pt + (top ? 0 : 1) * K * r;
    const double* Q = pt + (top ? 2 : 3) * K * r;
    const double* zg = wsp<double>(a.ws, L.zg);
    for (int o = lane; o < K * mc; o += 64) {
      int row = o / mc, c = o % mc;
      double v = yt[row * L.mmax + c0 + c];
      if (r > 0) {
        if (i <= L.p - 2 && !(L.variant && top)) {  // (LR-SPIKE-T: own interface only)
          const double* av = zg + (size_t)i * L.R2 * L.mmax;
          for (int q = 0; q < r; ++q) v -= P[row * r + q] * av[q * L.mmax + c0 + c];
        }
        if (i >= 1 && !(L.variant && !top)) {
          const double* cv = zg + ((size_t)(i - 1) * L.R2 + r) * L.mmax;
          for (int q = 0; q < r; ++q) v -= Q[row * r + q] * cv[q * L.mmax + c0 + c];
        }
      }
      Xn[row * NC + c] = (T)v;
    }
  };
  const bool top = j > 0 && !a.block_only, bot = j < L.p - 1 && !a.block_only;
  if (top) {
    tip(j - 1, false);  // x_{j-1,b}
    sync();
    for (int o = lane; o < K * mc; o += 64) {
      int i = o / mc, c = o % mc;
      double s = 0.0;
      for (int l = 0; l < K; ++l) s += band_at(a.bands, L.n, k, g.s + i, g.s - K + l) * (double)Xn[l * NC + c];
      Ct[i * NC + c] = (T)s;
    }
    sync();
  }
  if (bot) {
    tip(j + 1, true);  // x_{j+1,t}
    sync();
    const int64_t s1 = g.s + g.nj;
    for (int o = lane; o < K * mc; o += 64) {
      int i = o / mc, c = o % mc;
      double s = 0.0;
      for (int l = 0; l < K; ++l) s += band_at(a.bands, L.n, k, s1 - K + i, s1 + l) * (double)Xn[l * NC + c];
      Cb[i * NC + c] = (T)s;
    }
    sync();
  }
  fwd_wave<T, K, MCT, false>(a, g, j, c0, lds, top ? Ct : nullptr, bot ? Cb : nullptr);
  bwd_wave<T, K, MCT>(a, g, j, c0);
}


// ------------------------------------------------------------------ adjoint
// Transposed sweeps for partitions factored without interchanges (A_j = L U,
// A_j^{-T} = L^{-T} U^{-T}), with the prefetch ring of the forward sweeps.
// Transposed forward (U^T, top to bottom): W_b = U11^{-T} R_b, then
// R_{b+1} -= U12^T W_b; W is written to a.dst.  One gather of the UP record
// serves (U11^{-1})^T (its lower part) and U12^T (its strict upper part; the
// diagonal UD is applied elementwise).
template <typename T, int K, int MCT>
__device__ void tfwd_wave(const SolveArgs& a, const Geom& g, int j, int c0, const T* Ct, const T* Cb) {
  using W = WaveSweep<T, K, MCT>;
  using V = typename W::V;
  constexpr int NF = W::RT * W::KS, PD = sweep_pd<K, MCT>(), NS = PD + 1;
  const Layout& L = a.L;
  const int nb = g.nb;
  const T* fac = wsp<T>(a.ws, L.fac) + (size_t)j * L.nbmax * L.rec;
  const RowBuf src = row_buf(a.src, g, a.ld, c0, a.m);
  const RowBuf dst = row_buf(a.dst, g, a.ld, c0, a.m);
  V wb[W::RT][MCT], rows[NS][W::RT][MCT];
  T upq[NS][NF], udq[NS][W::RT][4];
  auto fetch_rec = [&](int q, T (&up)[NF], T (&ud)[W::RT][4]) __attribute__((always_inline)) {
    const int qc = min(q, nb - 1);
    load_tfrags<T, K>(up, fac + (size_t)qc * L.rec + K * K);
    load_udrows<T, K>(ud, fac + (size_t)qc * L.rec + 2 * K * K);
  };
  buf_load_strip<T, K, MCT>(rows[0], src, 0);
  if (Ct || Cb) sub_corr<T, K, MCT>(rows[0], g, 0, Ct, Cb);
  static_for<PD>([&](auto U) __attribute__((always_inline)) {
    constexpr int u = decltype(U)::value;
    fetch_rec(u, upq[u], udq[u]);
    buf_load_strip<T, K, MCT>(rows[u + 1], src, u + 1);
  });
  auto body = [&](auto U, int b) __attribute__((always_inline)) {
    constexpr int u = decltype(U)::value, u1 = (u + 1) % NS, uf = (u + PD) % NS;
    const bool last = (b == nb - 1);
    fetch_rec(b + PD, upq[uf], udq[uf]);
    V (&w0)[W::RT][MCT] = rows[u];
    V (&w1)[W::RT][MCT] = rows[u1];
    if ((Ct || Cb) && !last && corr_block(g, K, b + 1)) sub_corr<T, K, MCT>(w1, g, b + 1, Ct, Cb);
    zero_strip<T, K, MCT>(wb);
    blk_mul<T, K, MCT, 5>(upq[u], nullptr, T(1), w0, wb);  // W_b = U11^{-T} R_b
    buf_load_strip<T, K, MCT>(rows[u], src, b + 1 + PD);
    if (!last) {
      blk_mul<T, K, MCT, 7>(upq[u], nullptr, T(-1), wb, w1);  // R_{b+1} -= U12^T W_b (off the diagonal)
#pragma unroll
      for (int t = 0; t < W::RT; ++t)
#pragma unroll
        for (int ct = 0; ct < MCT; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) w1[t][ct][v] -= udq[u][t][v] * wb[t][ct][v];
    }
    buf_store_strip<T, K, MCT>(wb, dst, b);
  };
  int b0 = 0;
  for (; b0 + NS <= nb; b0 += NS)
    static_for<NS>([&](auto U) __attribute__((always_inline)) { body(U, b0 + decltype(U)::value); });
  static_for<NS>([&](auto U) __attribute__((always_inline)) {
    if (b0 + decltype(U)::value < nb) body(U, b0 + decltype(U)::value);
  });
}

// Transposed backward (L^T, bottom to top) over a.dst: u_b = L11^{-T}(W_b -
// L21^T u_{b+1}); one gather of the LP record serves L21^T (its lower part)
// and (L11^{-1})^T (its strict upper part, unit diagonal).  TIPS: u is not
// stored; the rows of its first and last K real rows go to the tip buffer
// (the adjoint D-stage).  Otherwise u overwrites a.dst.
template <typename T, int K, int MCT, bool TIPS>
__device__ void tbwd_wave(const SolveArgs& a, const Geom& g, int j, int c0) {
  using W = WaveSweep<T, K, MCT>;
  using V = typename W::V;
  constexpr int NF = W::RT * W::KS, PD = sweep_pd<K, MCT>(), NS = PD + 1;
  const Layout& L = a.L;
  const int nb = g.nb, lane = threadIdx.x & 63;
  const T* fac = wsp<T>(a.ws, L.fac) + (size_t)j * L.nbmax * L.rec;
  const RowBuf buf = row_buf(a.dst, g, a.ld, c0, a.m);
  double* yt = wsp<double>(a.ws, L.ytip) + (size_t)j * 2 * K * L.mmax;
  V x1[W::RT][MCT], ub[W::RT][MCT], zq[NS][W::RT][MCT];
  T lpq[NS][NF];
  zero_strip<T, K, MCT>(x1);
  auto fetch = [&](int q, T (&lp)[NF], V (&zs)[W::RT][MCT]) __attribute__((always_inline)) {
    const int b = max(nb - 1 - q, 0);
    load_tfrags<T, K>(lp, fac + (size_t)b * L.rec);
    buf_load_strip<T, K, MCT>(zs, buf, nb - 1 - q);
  };
  static_for<PD>([&](auto U) __attribute__((always_inline)) {
    constexpr int u = decltype(U)::value;
    fetch(u, lpq[u], zq[u]);
  });
  auto body = [&](auto U, int q) __attribute__((always_inline)) {
    constexpr int u = decltype(U)::value, uf = (u + PD) % NS;
    const int b = nb - 1 - q;
    fetch(q + PD, lpq[uf], zq[uf]);
    V (&zb)[W::RT][MCT] = zq[u];
    if (q != 0) blk_mul<T, K, MCT, 5>(lpq[u], nullptr, T(-1), x1, zb);  // W_b - L21^T u_{b+1}
    zero_strip<T, K, MCT>(ub);
    blk_mul<T, K, MCT, 4>(lpq[u], nullptr, T(1), zb, ub);  // u_b = L11^{-T} (...)
    if constexpr (TIPS) {
      if (corr_block(g, K, b)) {
#pragma unroll
        for (int t = 0; t < W::RT; ++t)
#pragma unroll
          for (int ct = 0; ct < MCT; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int row = 16 * t + acc_row<T>(lane, v), col = 16 * ct + (lane & 15);
              const int lr = b * K + row - g.pad;
              if (lr >= 0 && c0 + col < a.m) {
                if (lr < K) yt[(size_t)lr * L.mmax + c0 + col] = (double)ub[t][ct][v];
                if (lr >= g.nj - K) yt[(size_t)(K + lr - (g.nj - K)) * L.mmax + c0 + col] = (double)ub[t][ct][v];
              }
            }
      }
    } else {
      buf_store_strip<T, K, MCT>(ub, buf, b);
    }
#pragma unroll
    for (int t = 0; t < W::RT; ++t)
#pragma unroll
      for (int ct = 0; ct < MCT; ++ct) x1[t][ct] = ub[t][ct];
  };
  int q0 = 0;
  for (; q0 + NS <= nb; q0 += NS)
    static_for<NS>([&](auto U) __attribute__((always_inline)) { body(U, q0 + decltype(U)::value); });
  static_for<NS>([&](auto U) __attribute__((always_inline)) {
    if (q0 + decltype(U)::value < nb) body(U, q0 + decltype(U)::value);
  });
}

// Adjoint D-stage on the matrix cores: nu_j = A_j^{-T} g_j (U^T sweep with
// W into a.dst, then L^T sweep), tips nu_t, nu_b to the tip buffer.
// Partitions factored with interchanges are left to adj_dstage_kernel.
template <typename T, int K>
__global__ __launch_bounds__(64) __attribute__((aligned(4096))) void adj_dstage_wave_kernel(SolveArgs a) {
  if (gated(a.gate)) return;
  const int j = blockIdx.x, c0 = blockIdx.y * 16;
  if (wsp<int>(a.ws, a.L.npv)[j]) return;
  const Geom g = part_geom(a.L, j, K);
  tfwd_wave<T, K, 1>(a, g, j, c0, nullptr, nullptr);
  tbwd_wave<T, K, 1, true>(a, g, j, c0);
}

// Adjoint recovery on the matrix cores: lambda_j = A_j^{-T}(g_j - [w_{j,t};
// 0; w_{j,b}]) in place, with
//   w_{j,t} = B_{j-1}^T nu_{j-1,b} - Pi_{j-1} u_a(j-1)      (j >= 1)
//   w_{j,b} = C_{j+1}^T nu_{j+1,t} - Psi_{j+1} u_c(j+1)      (j <= p-2)
// (u = Z^{-T} L^T h in the compressed vector); LR-SPIKE-T needs no change here.
template <typename T, int K>
__global__ __launch_bounds__(64) __attribute__((aligned(4096))) void adj_retrieve_wave_kernel(SolveArgs a) {
  if (gated(a.gate)) return;
  using W = WaveSweep<T, K, 1>;
  constexpr int NC = W::NC;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* lds = reinterpret_cast<T*>(lds_raw);
  const Layout& L = a.L;
  const int j = blockIdx.x, c0 = blockIdx.y * NC;
  if (wsp<int>(a.ws, L.npv)[j]) return;
  const int mc = min(NC, a.m - c0);
  const Geom g = part_geom(L, j, K);
  const int lane = threadIdx.x & 63, k = L.k, r = L.r;
  T* Ct = lds + W::oCt;
  T* Cb = lds + W::oCb;
  const double* ytip = wsp<double>(a.ws, L.ytip);
  const double* proj = wsp<double>(a.ws, L.proj);
  const double* zg = wsp<double>(a.ws, L.zg);
  if (j > 0) {
    const double* nub = ytip + ((size_t)(j - 1) * 2 + 1) * K * L.mmax;
    const double* Pi = proj + (size_t)(j - 1) * 2 * K * r;
    const double* ua = zg + (size_t)(j - 1) * L.R2 * L.mmax;
    for (int o = lane; o < K * mc; o += 64) {
      const int i = o / mc, c = o % mc;
      double s = 0.0;
      for (int l = 0; l < K; ++l) s += band_at(a.bands, L.n, k, g.s - K + l, g.s + i) * nub[l * L.mmax + c0 + c];
      for (int q = 0; q < r; ++q) s -= Pi[i * r + q] * ua[q * L.mmax + c0 + c];
      Ct[i * NC + c] = (T)s;
    }
  }
  if (j < L.p - 1) {
    const double* nut = ytip + ((size_t)(j + 1) * 2 + 0) * K * L.mmax;
    const double* Psi = proj + ((size_t)(j + 1) * 2 + 1) * K * r;
    const double* uc = zg + ((size_t)j * L.R2 + r) * L.mmax;
    const int64_t s1 = g.s + g.nj;
    for (int o = lane; o < K * mc; o += 64) {
      const int i = o / mc, c = o % mc;
      double s = 0.0;
      for (int l = 0; l < K; ++l) s += band_at(a.bands, L.n, k, s1 + l, s1 - K + i) * nut[l * L.mmax + c0 + c];
      for (int q = 0; q < r; ++q) s -= Psi[i * r + q] * uc[q * L.mmax + c0 + c];
      Cb[i * NC + c] = (T)s;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  tfwd_wave<T, K, 1>(a, g, j, c0, j > 0 ? Ct : nullptr, j < L.p - 1 ? Cb : nullptr);
  tbwd_wave<T, K, 1, false>(a, g, j, c0);
}

// Pass-2 back substitution of one spike (kernel below).  The q-th block
// visited (b = nb - 1 - q) lives in ring slot q mod NS, as in the solve's
// backward pass: records, U12 diagonals and Y strips are prefetched PD blocks
// ahead with unconditional (clamped) loads.
template <typename T, int K, bool SWP>
__device__ void pass2_wave_impl(const FactorArgs& a, const Geom& g, int j, int spike) {
  constexpr int MCT = K / 16;
  using W = WaveSweep<T, K, MCT>;
  using V = typename W::V;
  // no prefetch at K = 32: the kernel then fits two waves per SIMD (the grid
  // has a wave per partition and spike, twice the SIMDs at p = 1024), and the
  // second wave hides the loads of the first (0.84 -> 0.72 ms at n = 2^22)
  constexpr int NF = W::RT * W::KS, PD = (K == 32 ? 0 : sweep_pd<K, MCT>()), NS = PD + 1;
  const Layout& L = a.L;
  const int lane = threadIdx.x & 63, nb = g.nb;
  const T* fac = wsT<T>(a.ws, L.fac) + (size_t)j * L.nbmax * L.rec;
  const T* swx = wsT<T>(a.ws, L.swx) + (size_t)j * L.nbmax * 3 * K * K;
  const T* ym = wsT<T>(a.ws, L.ymat) + (size_t)j * L.nbmax * 2 * K * K;
  const int* flg = wsT<int>(a.ws, L.flag) + (size_t)j * L.nbmax;
  const int coff = spike == 0 ? 0 : K;  // Y columns [W | V]
  // V's right-hand side lives in the last k rows: its forward result is zero
  // above the last two blocks (interchanges act within a block pair) and is
  // not stored there; those blocks read the strip of block nb - 2 (cached)
  // and take zero instead
  const int ymin = spike == 0 ? 0 : max(nb - 2, 0);
  V x1[W::RT][MCT], x2[W::RT][MCT], xb[W::RT][MCT], zq[NS][W::RT][MCT], gr[W::RT][W::RT];
  T upq[NS][NF], udq[NS][W::RT][4];
  zero_strip<T, K, MCT>(x1);
  zero_strip<T, K, MCT>(x2);
#pragma unroll
  for (int ti = 0; ti < W::RT; ++ti)
#pragma unroll
    for (int tj = 0; tj < W::RT; ++tj) gr[ti][tj] = V{0, 0, 0, 0};
  auto fetch = [&](int q, T (&up)[NF], T (&ud)[W::RT][4], V (&zs)[W::RT][MCT]) __attribute__((always_inline)) {
    const int b = max(nb - 1 - q, 0), by = max(b, ymin);
    load_frags<T, K>(up, fac + (size_t)b * L.rec + K * K);
    load_udrows<T, K>(ud, fac + (size_t)b * L.rec + 2 * K * K);
    const T* yb = ym + (size_t)by * 2 * K * K + coff;
#pragma unroll
    for (int t = 0; t < W::RT; ++t)
#pragma unroll
      for (int ct = 0; ct < MCT; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          zs[t][ct][v] = yb[(16 * t + acc_row<T>(lane, v)) * 2 * K + 16 * ct + (lane & 15)];
  };
  static_for<PD>([&](auto U) __attribute__((always_inline)) {
    constexpr int u = decltype(U)::value;
    fetch(u, upq[u], udq[u], zq[u]);
  });
  auto body = [&](auto U, int q) __attribute__((always_inline)) {
    constexpr int u = decltype(U)::value, uf = (u + PD) % NS;
    const int b = nb - 1 - q;
    fetch(q + PD, upq[uf], udq[uf], zq[uf]);
    T (&up)[NF] = upq[u];
    V (&zb)[W::RT][MCT] = zq[u];
    if (b < ymin) zero_strip<T, K, MCT>(zb);
    if (q > 0) {
      int fl = 0;
      if constexpr (SWP) fl = flg[b];
      if (SWP && (fl & 2)) {
        T u12[NF];
        load_frags<T, K>(u12, swx + (size_t)b * 3 * K * K + K * K);
        blk_mul<T, K, MCT, 9>(u12, nullptr, T(-1), x1, zb);
      } else {
        u12_mul<T, K, MCT>(up, udq[u], x1, zb);
      }
      if (SWP && (fl & 1)) {
        T u13[NF];
        load_frags<T, K>(u13, swx + (size_t)b * 3 * K * K + 2 * K * K);
        blk_mul<T, K, MCT, 9>(u13, nullptr, T(-1), x2, zb);
      }
    }
    zero_strip<T, K, MCT>(xb);
    blk_mul<T, K, MCT, 2>(up, nullptr, T(1), zb, xb);
    // Gram += z_b^T z_b (tiles on and above the diagonal; mirrored when stored)
#pragma unroll
    for (int ti = 0; ti < W::RT; ++ti)
#pragma unroll
      for (int tj = ti; tj < W::RT; ++tj)
#pragma unroll
        for (int step = 0; step < W::KS; ++step)
          gr[ti][tj] = mfma_step(xb[step >> 2][ti][step & 3], xb[step >> 2][tj][step & 3], gr[ti][tj]);
#pragma unroll
    for (int t = 0; t < W::RT; ++t)
#pragma unroll
      for (int ct = 0; ct < MCT; ++ct) {
        x2[t][ct] = x1[t][ct];
        x1[t][ct] = xb[t][ct];
      }
  };
  int q0 = 0;
  for (; q0 + NS <= nb; q0 += NS)
    static_for<NS>([&](auto U) __attribute__((always_inline)) { body(U, q0 + decltype(U)::value); });
  static_for<NS>([&](auto U) __attribute__((always_inline)) {
    if (q0 + decltype(U)::value < nb) body(U, q0 + decltype(U)::value);
  });
  // gram layout [GV | GW], K x K row-major each
  double* gram = wsT<double>(a.ws, L.gram) + ((size_t)j * 2 + (spike == 0 ? 1 : 0)) * K * K;
#pragma unroll
  for (int ti = 0; ti < W::RT; ++ti)
#pragma unroll
    for (int tj = 0; tj < W::RT; ++tj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (tj < ti) continue;
        const int row = 16 * ti + acc_row<T>(lane, v), col = 16 * tj + (lane & 15);
        gram[row * K + col] = (double)gr[ti][tj][v];
        if (tj > ti) gram[col * K + row] = (double)gr[ti][tj][v];
      }
}

// Factorization pass 2 for K >= 16 (r < k): back substitution of one spike
// (blockIdx.y = 0: W, 1: V) over the stored forward intermediate Y,
//   z_b = U11^{-1} (Y_b - U12 z_{b+1} - U13 z_{b+2}),
// accumulating the Gram matrix z^T z on the matrix cores: the accumulator
// tiles of z are at once the B operand and (tile-transposed) the A operand.
// The interchange flags are read only for partitions factored with
// interchanges (a compile-time variant: elsewhere they are all zero).
template <typename T, int K>
__global__ __launch_bounds__(64) __attribute__((aligned(4096))) __attribute__((amdgpu_waves_per_eu(2))) void pass2_wave_kernel(FactorArgs a) {
  const int j = blockIdx.x, spike = blockIdx.y;
  const Geom g = part_geom(a.L, j, K);
  if (wsT<int>(a.ws, a.L.npv)[j] != 0)
    pass2_wave_impl<T, K, true>(a, g, j, spike);
  else
    pass2_wave_impl<T, K, false>(a, g, j, spike);
}

}  // namespace lrs
