// Factorization for K = 64: one 256-thread workgroup per partition with every
// K x K block resident in LDS (the single-wave kernels keep a 2K-row panel in
// one wave's registers, which does not fit at this width).  Uses the register
// elimination steps FwdElim / BwdElim of the single-wave factor kernel.
//
// Per K-row block b (the same block formulation as the other factor kernels):
//   panel [Dc_b; Lo_{b+1}] factored without interchanges, the diagonal block
//   as 2 x 2 blocks of K/2 (register elimination of the K/2-column panels by
//   one wave, block products by the workgroup), giving L11^{-1}, U11^{-1} and
//   L21 = Lo_{b+1} U11^{-1}; a multiplier above 1 in magnitude means partial
//   pivoting would interchange rows, which this width does not support:
//   NOT_SUPPORTED is latched for the partition;  U12 = L11^{-1} Up_b;
//   G step g_b = U11^{-T}(e_b + pending), pending = -U12^T g_b;
//   records in the fragment order the sweeps read;  Dc_{b+1} = D_{b+1} - L21 U12.
// The spikes are formed afterwards from the records (spike_lds_kernel) and,
// for r < k, swept back with their Gram matrices (pass2_lds_kernel).
// Every block product runs on the matrix cores from LDS operands (mm64, mm32,
// and the 64 x 16 products of the spike sweeps).
#include "sweep.h"

namespace lrs {

// Matrix-core block products from LDS operands for the 256-thread workgroup.
// mm64: C (64 x 64) += A B, wave w owns rows 16w..16w+15 (four 16-column
// tiles); per k-step s the A fragment is A(16w + lane mod 16, 4s + lane / 16)
// and the B fragment B(4s + lane / 16, 16ct + lane mod 16).  TRI skips the
// 16 x 16 tiles a triangular operand leaves zero: 1 A lower, 2 A upper,
// 3 B upper, 4 B lower.
// The thread index is re-read opaquely at every call, so that the operand
// addresses are formed next to their use instead of being hoisted out of the
// callers' block loops (where they would occupy registers for the whole loop);
// the wave index is made uniform, so the triangular skips are scalar branches.
__device__ __forceinline__ void lds_lane_wave(int& lane, int& w) {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  lane = t & 63;
  w = __builtin_amdgcn_readfirstlane(t >> 6);
}
template <typename T, int TRI, typename FA, typename FB>
__device__ __forceinline__ void mm64(typename AccVec<T>::type (&acc)[4], FA a, FB b) {
  int lane, w;
  lds_lane_wave(lane, w);
  const int i = 16 * w + (lane & 15), kq = lane >> 4, jl = lane & 15;
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    if (TRI == 1 && s >= 4 * (w + 1)) break;
    if (TRI == 2 && s < 4 * w) continue;
    const int kk = 4 * s + kq;
    const T av = a(i, kk);
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      if (TRI == 3 && s >= 4 * (ct + 1)) continue;
      if (TRI == 4 && s < 4 * ct) continue;
      acc[ct] = mfma_step(av, b(kk, 16 * ct + jl), acc[ct]);
    }
  }
}
// mm32: C (32 x 32) += A B, wave w owns the 16 x 16 tile (w / 2, w mod 2).
template <typename T, typename FA, typename FB>
__device__ __forceinline__ void mm32(typename AccVec<T>::type& acc, FA a, FB b) {
  int lane, w;
  lds_lane_wave(lane, w);
  const int i = 16 * (w >> 1) + (lane & 15), j = 16 * (w & 1) + (lane & 15), kq = lane >> 4;
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int kk = 4 * s + kq;
    acc = mfma_step(a(i, kk), b(kk, j), acc);
  }
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
  // diagnostics in LDS (registers are spent on the products): per thread the
  // largest band entry it loaded, and the smallest pivot (wave 0)
  __shared__ double s_amax[LRS_NT];
  __shared__ double s_pmin;
  __shared__ double s_dinv[K];  // reciprocal pivots of the block's two register passes
  s_amax[tid] = 0.0;
  if (tid == 0) s_pmin = INFINITY;
  // A_j(lr, lc) in partition-local rows/columns (identity on the padding rows)
  auto Aj = [&](int lr, int lc) -> T {
    if (lr < 0 || lc < 0) return (lr == lc) ? T(1) : T(0);
    if (lr >= g.nj || lc >= g.nj) return T(0);
    const int d = lc - lr;
    if (d < -k || d > k) return T(0);
    return (T)a.bands[(int64_t)(d + k) * L.n + g.s + lr];
  };
  (void)Aj;
  // K x K block (rows of block R, columns of block C) into dst (pitch PT)
  // by the last NW waves of the workgroup (fetched into registers, then put).  Lane = block row, so a wave reads
  // one diagonal segment (coalesced); the waves take every NW-th diagonal
  // offset e = c - i; every load is issued (from a clamped, always valid
  // address) before any store.
  auto block_fetch = [&](auto& vals, int R, int C, auto nw) {
    constexpr int NW = decltype(nw)::value;
    constexpr int NI = (2 * K - 1 + NW - 1) / NW;
    int i = tid & 63;  // opaque: keeps the per-diagonal addresses from being hoisted out of the block loop
    asm volatile("" : "+v"(i));
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6) - (LRS_NT / 64 - NW);
    const int lr = R * K + i - g.pad;
#pragma unroll
    for (int t = 0; t < NI; ++t) {
      // bitwise conjunction: a select of the index, not a branch per load
      const int e = w + NW * t - (K - 1), c = i + e, lc = C * K + c - g.pad, d = lc - lr;
      const bool inb = (e <= K - 1) & (c >= 0) & (c < K) & (lr >= 0) & (lr < g.nj) & (lc >= 0) & (lc < g.nj) &
                       (d >= -k) & (d <= k);
      const int64_t idx = (int64_t)(d + k) * L.n + g.s + lr;
      vals[t] = (T)a.bands[inb ? idx : 0];
    }
  };
  auto block_put = [&](T* dst, const auto& vals, int R, int C, auto nw) {
    constexpr int NW = decltype(nw)::value;
    constexpr int NI = (2 * K - 1 + NW - 1) / NW;
    int i = tid & 63;
    asm volatile("" : "+v"(i));
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6) - (LRS_NT / 64 - NW);
    const int lr = R * K + i - g.pad;
    T am = T(0);
#pragma unroll
    for (int t = 0; t < NI; ++t) {
      const int e = w + NW * t - (K - 1), c = i + e, lc = C * K + c - g.pad, d = lc - lr;
      const bool inb = e <= K - 1 && c >= 0 && c < K && lr >= 0 && lr < g.nj && lc >= 0 && lc < g.nj &&
                       d >= -k && d <= k;
      const bool ident = (lr < 0 || lc < 0) && lr == lc;
      if (e <= K - 1 && c >= 0 && c < K) dst[i * PT + c] = inb ? vals[t] : (ident ? T(1) : T(0));
      if (inb) am = fmax(am, fabs(vals[t]));
    }
    s_amax[tid] = fmax(s_amax[tid], (double)am);
  };
  auto load_block = [&](T* dst, int R, int C, auto nw) {
    T vals[(2 * K - 1 + decltype(nw)::value - 1) / decltype(nw)::value];
    block_fetch(vals, R, C, nw);
    block_put(dst, vals, R, C, nw);
  };
  using W4 = std::integral_constant<int, LRS_NT / 64>;
  using W3 = std::integral_constant<int, LRS_NT / 64 - 1>;
  load_block(P, 0, 0, W4{});
  for (int o = tid; o < K * K; o += LRS_NT) Gp[(o / K) * PT + o % K] = T(0);
  if (tid == 0) s_bad = 0;
  __syncthreads();
  for (int b = 0; b < nb; ++b) {
    // the thread index re-read opaquely per block (see lds_lane_wave)
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const bool last = (b == nb - 1);
    // ---- the diagonal block D (panel top) as 2 x 2 blocks of H = K/2 columns:
    //   [D11; D21] = [L1; L2'] U1 by the register elimination of one wave
    //   (lane = row, no interchanges), with L1^{-1} riding along and U1^{-1}
    //   by the upward Gauss-Jordan pass;  U1' = L1^{-1} D12;  S = D22 - L2' U1';
    //   S = L2 U2 the same way;  then
    //   L11^{-1} = [L1^{-1} 0; -L2^{-1} L2' L1^{-1}  L2^{-1}],
    //   U11^{-1} = [U1^{-1}  -U1^{-1} U1' U2^{-1}; 0  U2^{-1}],
    //   L21 = Lo U11^{-1}.
    // These are the factors column-by-column elimination of [Dc_b; Lo_{b+1}]
    // gives; each multiplier (L1, L2', L2 in the register passes, L21 after its
    // product) is compared with 1 in magnitude, the same interchange test.
    // The result is packed in place: L11^{-1} strictly below the diagonal of
    // the panel top, U11^{-1} on and above it, L21 in the panel bottom.
    {
      constexpr int H = K / 2;
      const int lane = tid & 63;
      // register LU of the H x H block at (r0, r0) and the rows below it
      // (nrow rows in all), wave 0 only
      auto reg_lu = [&](int r0, int nrow) {
        T pa[H], iv[H];
        const int lr = lane < nrow ? lane : nrow - 1;
#pragma unroll
        for (int c = 0; c < H; ++c) {
          pa[c] = P[(r0 + lr) * PT + r0 + c];
          iv[c] = T(0);
        }
        T mx = T(0), dmin = T(INFINITY), dinv = T(0);
        int ln1 = lane;  // opaque lane index (see factor_pass1_wave_kernel)
        asm volatile("" : "+v"(ln1));
        // the L1^{-1} ride-along and the U1^{-1} pass cover the 16 x 16
        // diagonal blocks; their off-diagonal blocks come from block products
        FwdElim<T, H, 0, 16>::run(pa, iv, ln1, nrow, mx, dmin, dinv);
        // a zero pivot leaves an infinite reciprocal in its lane, a non-finite
        // one a NaN or zero reciprocal; the first failing pivot decides the
        // code (ZERO_PIVOT for a zero one even though the steps after it turn
        // NaN); a multiplier above 1 would need an interchange
        // (the reciprocals go through LDS: no extra registers while the panel is live)
        if (lane < H) s_dinv[r0 + lane] = (double)dinv;
        wave_fence();
        const unsigned long long zb = __ballot(lane < H && !(isfinite(dinv) && dinv != T(0)));
        const unsigned long long bb = __ballot(lane < nrow && !(mx <= T(1)));
        if (lane == 0 && s_bad == 0 && (zb || bb || !(dmin > T(0)))) {
          s_bad = zb ? (isinf(s_dinv[r0 + __ffsll(zb) - 1]) ? 1 : 3) : (!(dmin > T(0)) ? 1 : 2);
          s_row = b * K + r0 + (zb ? __ffsll(zb) - 1 : (bb ? __ffsll(bb) - 1 : 0)) - g.pad;
        }
        if (lane < H) {
#pragma unroll
          for (int c = 0; c < H; ++c)
            if (c < lane) P[(r0 + lane) * PT + r0 + c] = (c >= (lane & ~15)) ? iv[c] : pa[c];
        } else if (lane < nrow) {
#pragma unroll
          for (int c = 0; c < H; ++c) P[(r0 + lane) * PT + r0 + c] = pa[c];
        }
        lower_offdiag_inverse<T>(P + r0 * PT + r0, PT, lane);
        int ln2 = lane;
        asm volatile("" : "+v"(ln2));
#pragma unroll
        for (int c = 0; c < H; ++c) iv[c] = (c == ln2) ? T(1) : T(0);
        BwdElim<T, H, H - 1, 16>::run(pa, iv, ln2, dinv);
        if (lane < H)
#pragma unroll
          for (int c = 0; c < H; ++c)
            if (c >= lane) P[(r0 + lane) * PT + r0 + c] = (c < (lane | 15) + 1) ? iv[c] : pa[c];
        upper_offdiag_inverse<T>(P + r0 * PT + r0, PT, lane);
      };
      // unit lower / upper parts of a packed H x H block at (r0, r0); loads
      // are unconditional (valid addresses) so the products stay branch-free
      auto lo = [&](int r0, int i, int l) -> T {
        const T x = P[(r0 + i) * PT + r0 + l];
        return l < i ? x : (l == i ? T(1) : T(0));
      };
      auto up = [&](int r0, int i, int l) -> T {
        const T x = P[(r0 + i) * PT + r0 + l];
        return l >= i ? x : T(0);
      };
      auto blk = [&](int r0, int c0, int i, int l) -> T { return P[(r0 + i) * PT + c0 + l]; };
      using AV = typename AccVec<T>::type;
      const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
      // 32 x 32 results: element v of wave w's tile at (row, col) of the quadrant
      auto put32 = [&](const AV& acc, int r0, int c0, T sg) {
#pragma unroll
        for (int v = 0; v < 4; ++v)
          P[(r0 + 16 * (w >> 1) + acc_row<T>(lane, v)) * PT + c0 + 16 * (w & 1) + (lane & 15)] = sg * acc[v];
      };
      AV a1, a2;
      // wave 0 factors the left half of the panel top while the other waves
      // bring in Lo_{b+1} (panel bottom) and Up_b (free since the last block)
      if (tid < 64)
        reg_lu(0, K);
      else if (!last) {
        load_block(P + K * PT, b + 1, b, W3{});
        load_block(U, b, b + 1, W3{});
      }
      __syncthreads();
      // U1' = L1^{-1} D12 (in place)
      a1 = AV{0, 0, 0, 0};
      mm32<T>(a1, [&](int i, int l) { return lo(0, i, l); }, [&](int l, int c) { return blk(0, H, l, c); });
      __syncthreads();
      put32(a1, 0, H, T(1));
      __syncthreads();
      // S = D22 - L2' U1' (reads other quadrants than it writes)
      a1 = AV{0, 0, 0, 0};
      mm32<T>(a1, [&](int i, int l) { return blk(H, 0, i, l); }, [&](int l, int c) { return blk(0, H, l, c); });
#pragma unroll
      for (int v = 0; v < 4; ++v)
        P[(H + 16 * (w >> 1) + acc_row<T>(lane, v)) * PT + H + 16 * (w & 1) + (lane & 15)] -= a1[v];
      __syncthreads();
      if (tid < 64) reg_lu(H, H);
      __syncthreads();
      // T1 = L2' L1^{-1},  T2 = U1^{-1} U1'
      a1 = AV{0, 0, 0, 0};
      a2 = AV{0, 0, 0, 0};
      mm32<T>(a1, [&](int i, int l) { return blk(H, 0, i, l); }, [&](int l, int c) { return lo(0, l, c); });
      mm32<T>(a2, [&](int i, int l) { return up(0, i, l); }, [&](int l, int c) { return blk(0, H, l, c); });
      __syncthreads();
      put32(a1, H, 0, T(1));
      put32(a2, 0, H, T(1));
      __syncthreads();
      // lower-left of L11^{-1}: -L2^{-1} T1;  upper-right of U11^{-1}: -T2 U2^{-1}
      a1 = AV{0, 0, 0, 0};
      a2 = AV{0, 0, 0, 0};
      mm32<T>(a1, [&](int i, int l) { return lo(H, i, l); }, [&](int l, int c) { return blk(H, 0, l, c); });
      mm32<T>(a2, [&](int i, int l) { return blk(0, H, i, l); }, [&](int l, int c) { return up(H, l, c); });
      __syncthreads();
      put32(a1, H, 0, T(-1));
      put32(a2, 0, H, T(-1));
      __syncthreads();
      // L21 = Lo U11^{-1} (in place in the panel bottom)
      if (!last) {
        AV acc[4] = {AV{0, 0, 0, 0}, AV{0, 0, 0, 0}, AV{0, 0, 0, 0}, AV{0, 0, 0, 0}};
        mm64<T, 3>(acc, [&](int r, int l) { return P[(K + r) * PT + l]; }, [&](int l, int c) {
          const T x = P[l * PT + c];
          return l <= c ? x : T(0);
        });
        __syncthreads();
        bool big = false;
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            P[(K + 16 * w + acc_row<T>(lane, v)) * PT + 16 * ct + (lane & 15)] = acc[ct][v];
            big |= !(fabs(acc[ct][v]) <= T(1));
          }
        if (big && s_bad == 0) {  // every writer stores the same values
          s_bad = 2;
          s_row = (b + 1) * K - g.pad;
        }
      }
      __syncthreads();
    }
    if (s_bad) {
      if (tid == 0)
        latch_error(latch,
                    s_bad == 1 ? LRSPIKE_ERR_ZERO_PIVOT : (s_bad == 3 ? LRSPIKE_ERR_NONFINITE : LRSPIKE_ERR_NOT_SUPPORTED),
                    j, s_row);
      return;
    }
    if (tid < 64) {  // smallest pivot of the block's real rows (block 0 may start with virtual unit rows)
      const double pinv = wave_max((tid < K && b * K + tid >= g.pad) ? fabs(s_dinv[tid]) : 0.0);
      if (tid == 0 && pinv > 0.0) s_pmin = fmin(s_pmin, 1.0 / pinv);
    }
    auto Li = [&](int r, int l) -> T {
      const T x = P[r * PT + l];
      return r > l ? x : (r == l ? T(1) : T(0));
    };
    auto Ui = [&](int r, int l) -> T {
      const T x = P[r * PT + l];
      return r <= l ? x : T(0);
    };
    using AV = typename AccVec<T>::type;
    const int lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    // (row, col) of element v of accumulator tile ct
    auto each = [&](auto&& fn) {
#pragma unroll
      for (int ct = 0; ct < 4; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) fn(ct, v, 16 * w + acc_row<T>(lane, v), 16 * ct + (lane & 15));
    };
    AV acc[4];
    auto zero = [&]() {
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) acc[ct] = AV{0, 0, 0, 0};
    };
    // ---- U12 = L11^{-1} Up_b (in place in U)
    if (!last) {
      zero();
      mm64<T, 1>(acc, Li, [&](int l, int c) { return U[l * PT + c]; });
      __syncthreads();
      each([&](int ct, int v, int row, int col) { U[row * PT + col] = acc[ct][v]; });
      __syncthreads();
    }
    // ---- G step: g_b = U11^{-T} (e_b + pending); G^T record; pending = -U12^T g_b
    for (int o = tid; o < K * K; o += LRS_NT) {
      const int i = o / K, c = o % K;
      if (c == b * K + i - g.pad) Gp[i * PT + c] += T(1);
    }
    __syncthreads();
    zero();
    mm64<T, 1>(acc, [&](int r, int l) { return Ui(l, r); }, [&](int l, int c) { return Gp[l * PT + c]; });
    __syncthreads();
    each([&](int ct, int v, int row, int col) {
      Gp[row * PT + col] = acc[ct][v];
      gm[(size_t)b * K * K + fidx<T, K>(col, row)] = acc[ct][v];  // G^T in operand order
    });
    __syncthreads();
    if (!last) {
      zero();
      mm64<T, 2>(acc, [&](int r, int l) { return U[l * PT + r]; }, [&](int l, int c) { return Gp[l * PT + c]; });
      __syncthreads();
      each([&](int ct, int v, int row, int col) { Gp[row * PT + col] = -acc[ct][v]; });
    }
    // ---- records: LP = L11^{-1} strict lower | L21 upper;  UP = U11^{-1} upper | U12 strict lower; UD
    // (written in storage order: coalesced stores)
    T* rec = fac + (size_t)b * L.rec;
    for (int o = tid; o < K * K; o += LRS_NT) {
      int i, c;
      fidx_inv<T, K>(o, i, c);
      rec[o] = (i > c) ? P[i * PT + c] : (last ? T(0) : P[(K + i) * PT + c]);
      rec[K * K + o] = (i <= c) ? P[i * PT + c] : (last ? T(0) : U[i * PT + c]);
    }
    if (tid < K) {
      rec[2 * K * K + tid] = last ? T(0) : U[tid * PT + tid];
      ipv[(size_t)b * K + tid] = tid;
    }
    if (tid == 0) flg[b] = 0;
    __syncthreads();
    // ---- Dc_{b+1} = D_{b+1} - L21 U12 into the panel top
    if (!last) {
      zero();
      mm64<T, 2>(acc, [&](int r, int l) {
        const T x = P[(K + r) * PT + l];
        return r <= l ? x : T(0);
      },
                 [&](int l, int c) { return U[l * PT + c]; });
      load_block(P, b + 1, b + 1, W4{});  // D_{b+1} (the panel top is free once the records are out)
      __syncthreads();
      each([&](int ct, int v, int row, int col) { P[row * PT + col] -= acc[ct][v]; });
      __syncthreads();
    }
  }
  __syncthreads();
  const double am = wave_max(s_amax[tid]);
  if ((tid & 63) == 0) state_max(latch, S_AMAX, am);
  if (tid == 0) state_min(latch, S_PIVMIN, s_pmin);  // the register passes run on wave 0
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
  // out (K x MS) = sign M X (+ out), M K x K (pitch PT, or its transpose),
  // X K x MS (pitch PM): matrix cores, wave w computes rows 16w..16w+15
  using AV = typename AccVec<T>::type;
  const int lane = tid & 63, w = tid >> 6, col = lane & 15;
  auto mm = [&](const T* M, bool trans, const T* X, T* out, T sign, bool accumulate) {
    AV acc = AV{0, 0, 0, 0};
    const int i = 16 * w + (lane & 15);
#pragma unroll
    for (int s2 = 0; s2 < K / 4; ++s2) {
      const int kk = 4 * s2 + (lane >> 4);
      acc = mfma_step(trans ? M[kk * PT + i] : M[i * PT + kk], X[kk * PM + col], acc);
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * w + acc_row<T>(lane, v);
      out[row * PM + col] = (accumulate ? out[row * PM + col] : T(0)) + sign * acc[v];
    }
    __syncthreads();
  };
  AV tacc = AV{0, 0, 0, 0};  // top tip: rows 16w.., the chunk's 16 columns
  auto gt_acc = [&]() {  // tacc += G_b^T z_b (Gb holds G_b^T transposed: Gb[l][r] = G_b(l, r))
    const int i = 16 * w + (lane & 15);
#pragma unroll
    for (int s2 = 0; s2 < K / 4; ++s2) {
      const int kk = 4 * s2 + (lane >> 4);
      tacc = mfma_step(Gb[kk * PT + i], Z[kk * PM + col], tacc);
    }
  };
  auto put_tip = [&](int which, const T* X, bool from_acc) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * w + acc_row<T>(lane, v);
      tips[(size_t)which * K * K + row * K + c0 + col] = from_acc ? (double)tacc[v] : (double)X[row * PM + col];
    }
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
      gt_acc();  // W_t += G_b^T z_b
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
    gt_acc();
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
  using AV = typename AccVec<T>::type;
  const int lane = tid & 63, w = tid >> 6;
  auto each = [&](auto&& fn) {  // (tile, element, row, col) of this wave's accumulators
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) fn(ct, v, 16 * w + acc_row<T>(lane, v), 16 * ct + (lane & 15));
  };
  AV gr[4], acc[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) gr[ct] = AV{0, 0, 0, 0};
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
    // Tm = Y_b - U12 z_{b+1}  (U12 lower triangular)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[ct] = AV{0, 0, 0, 0};
    if (!last) mm64<T, 1>(acc, [&](int r, int l) { return U12[r * PT + l]; }, [&](int l, int c) { return Zn[l * PT + c]; });
    const bool ynz = spike == 0 || last;
    each([&](int ct, int v, int row, int col) {
      const T y = ynz ? ym[(size_t)b * 2 * K * K + row * 2 * K + coff + col] : T(0);
      Tm[row * PT + col] = y - acc[ct][v];
    });
    __syncthreads();
    // z_b = U11^{-1} Tm  (upper triangular)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[ct] = AV{0, 0, 0, 0};
    mm64<T, 2>(acc, [&](int r, int l) { return Ui[r * PT + l]; }, [&](int l, int c) { return Tm[l * PT + c]; });
    each([&](int ct, int v, int row, int col) { Zn[row * PT + col] = acc[ct][v]; });
    __syncthreads();
    // Gram += z_b^T z_b
    mm64<T, 0>(gr, [&](int r, int l) { return Zn[l * PT + r]; }, [&](int l, int c) { return Zn[l * PT + c]; });
    __syncthreads();
  }
  double* gram = wsT<double>(a.ws, L.gram) + ((size_t)j * 2 + (spike == 0 ? 1 : 0)) * K * K;
  each([&](int ct, int v, int row, int col) { gram[row * K + col] = (double)gr[ct][v]; });
}

}  // namespace lrs
