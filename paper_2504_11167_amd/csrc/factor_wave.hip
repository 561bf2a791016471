// Factorization pass 1 for K >= 16, one wave per partition (no workgroup
// barriers; every partition of a 1024-partition problem resident at once).
//
// Per K-row block b (see factor.hip for the block formulation):
//   panel [Dc_b; Lo_{b+1}] eliminated in registers (lane = row, the pivot row
//   reaching the other lanes by lane reads) WITHOUT row interchanges, an
//   identity block riding along so that the first K lanes end with the rows of
//   L11^{-1} (its 16 x 16 diagonal blocks; at K = 32 the block below them by
//   two matrix-core products);  if any multiplier exceeds 1 in magnitude (or a
//   pivot is zero) partial pivoting would have interchanged rows: the
//   partition is flagged and refactored by the interchanging kernel, so the
//   result is always the partial-pivoting factorization;
//   U11^{-1} by an upward Gauss-Jordan pass over the same registers (again on
//   the 16 x 16 diagonal blocks, the block right of them by products), with
//   U12 = L11^{-1} Up_b and Dc_{b+1} = D_{b+1} - L21 U12 issued on the matrix
//   cores alongside it;
//   G step:    g_b = U11^{-T} (e_b + pending), pending' = -U12^T g_b (matrix cores)
// The spike forward sweeps run afterwards in spike_wave_kernel over the
// stored factors (same structure as the D-stage of the solve).
// Block products keep their operands in accumulator tiles (the accumulator
// layout is the B operand layout, and tile-transposed the A operand of the
// transposed product); LDS holds only the band slab of the next row block,
// the packed L11^{-1}\U11 (later U11^{-1}) and L21 (later U12) blocks.
#include <limits>

#include "solve_wave.hip"

namespace lrs {

template <typename T, int K>
struct FWave {
  static constexpr int RT = K / 16, KS = K / 4, PT = K + 1;
  using V = typename AccVec<T>::type;
  static constexpr int oSlab = 0;                    // (2K+1) x K, diagonal-major
  static constexpr int oLib = oSlab + (2 * K + 1) * K;  // K x PT
  static constexpr int oL21 = oLib + K * PT;         // K x PT
  static constexpr int oDiag = oL21 + K * PT;        // per lane: max |1 / pivot|, max |a_ij| (diagnostics)
  static constexpr int total = oDiag + 128;
};

__device__ __forceinline__ void wave_fence() {  // order LDS accesses of one wave
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Forward elimination step C of the 2K x K panel without interchanges, lane =
// row, row held in pa[] (U part / multipliers) and iv[] (the row of L11^{-1}
// being formed, implicit 1 at the lane's own column).  The pivot row (lane C)
// reaches the other lanes by lane reads into scalar registers (no LDS traffic,
// so the waves sharing a CU do not contend); a scheduling barrier per step
// keeps those reads next to their use.
// BW < K restricts the ride-along to the BW x BW diagonal blocks of L11^{-1}
// (columns [BW floor(C / BW), C) at step C); the blocks below the diagonal are
// then formed by block products.
// mx and dmin collect max |multiplier| and min |pivot| (NaN operands are
// ignored there: a non-finite pivot shows as a non-finite or zero reciprocal
// dinv in its lane, which the callers test once per panel).
template <typename T, int K, int C, int BW = K>
struct FwdElimLA {
  // d, inv: this step's pivot and its reciprocal, formed during the previous
  // step as soon as the pivot's own entry was final (look-ahead: the division
  // overlaps the rest of that step's updates instead of heading this one)
  static __device__ __forceinline__ void run(T (&pa)[K], T (&iv)[K], int lane, int nr, T& mx, T& dmin, T& dinv,
                                             T d, T inv) {
    if constexpr (C < K) {
      __builtin_amdgcn_sched_barrier(0);
      if (lane == C) dinv = inv;
      dmin = fmin(dmin, fabs(d));
      const bool act = lane > C && lane < nr;
      const T l = act ? pa[C] * inv : T(0);
      mx = fmax(mx, fabs(l));
      if (act) pa[C] = l;
      T dn = T(1), invn = T(1);
      if constexpr (C + 1 < K) {
        pa[C + 1] = fma(-l, bcast(pa[C + 1], C), pa[C + 1]);
        dn = bcast(pa[C + 1], C + 1);
        invn = T(1) / dn;
      }
#pragma unroll
      for (int c = C + 2; c < K; ++c) pa[c] = fma(-l, bcast(pa[c], C), pa[c]);
#pragma unroll
      for (int c = (C / BW) * BW; c < C; ++c) iv[c] = fma(-l, bcast(iv[c], C), iv[c]);
      iv[C] -= l;
      FwdElimLA<T, K, C + 1, BW>::run(pa, iv, lane, nr, mx, dmin, dinv, dn, invn);
    }
  }
};
template <typename T, int K, int C, int BW = K>
struct FwdElim {
  static __device__ __forceinline__ void run(T (&pa)[K], T (&iv)[K], int lane, int nr, T& mx, T& dmin, T& dinv) {
    const T d0 = bcast(pa[0], 0);
    FwdElimLA<T, K, 0, BW>::run(pa, iv, lane, nr, mx, dmin, dinv, d0, T(1) / d0);
  }
};

// Upward Gauss-Jordan step C (counting down): lane i < K holds in uv[] the row
// i of U11^{-1} being formed; U11 itself is read from pa[] (upper part) and
// lane C scales its finished row by 1/U_CC (its dinv from the forward pass).
// The same pass with a hook called at the start of every step (with the step
// count as a compile-time constant), so that independent matrix-core work can
// be issued between the lane reads and the updates of the step.
// BW < K restricts the pass to the BW x BW diagonal blocks of U11^{-1}
// (columns [C, BW (floor(C / BW) + 1)) at step C).
template <typename T, int K, int C, int BW = K>
struct BwdElimH {
  template <typename H>
  static __device__ __forceinline__ void run(const T (&pa)[K], T (&uv)[K], int lane, T dinv, H& hook) {
    if constexpr (C >= 0) {
      constexpr int CE = (C / BW + 1) * BW;
      __builtin_amdgcn_sched_barrier(0);
      hook(std::integral_constant<int, K - 1 - C>{});
      if (lane == C) {
#pragma unroll
        for (int c = C; c < CE; ++c) uv[c] *= dinv;
      }
      const T m = lane < C ? pa[C] : T(0);
#pragma unroll
      for (int c = C; c < CE; ++c) uv[c] = fma(-m, bcast(uv[c], C), uv[c]);
      BwdElimH<T, K, C - 1, BW>::run(pa, uv, lane, dinv, hook);
    }
  }
};

template <typename T, int K, int C, int BW = K>
struct BwdElim {
  static __device__ __forceinline__ void run(const T (&pa)[K], T (&uv)[K], int lane, T dinv) {
    if constexpr (C >= 0) {
      constexpr int CE = (C / BW + 1) * BW;
      __builtin_amdgcn_sched_barrier(0);
      if (lane == C) {
#pragma unroll
        for (int c = C; c < CE; ++c) uv[c] *= dinv;
      }
      const T m = lane < C ? pa[C] : T(0);
#pragma unroll
      for (int c = C; c < CE; ++c) uv[c] = fma(-m, bcast(uv[c], C), uv[c]);
      BwdElim<T, K, C - 1, BW>::run(pa, uv, lane, dinv);
    }
  }
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Off-diagonal 16 x 16 blocks of the inverses of a 32 x 32 packed block M
// (pitch pm) whose passes covered only the 16 x 16 diagonal blocks; one wave,
// two matrix-core products each (the accumulator layout of a tile is the B
// operand layout of the next product).
//   lower: M holds L11^{-1} (strict lower) in the diagonal blocks and the block
//   L_{21} of L11 below them; it becomes X = -L_{22}^{-1} (L_{21} L_{11}^{-1}).
//   upper: M holds U11^{-1} (upper) in the diagonal blocks and the block U_{12}
//   of U11 right of them; it becomes Y = -U_{11}^{-1} (U_{12} U_{22}^{-1}).
template <typename T>
__device__ __forceinline__ void lower_offdiag_inverse(T* M, int pm, int lane) {
  using V = typename AccVec<T>::type;
  wave_fence();
  V ai, t1 = V{0, 0, 0, 0}, x = V{0, 0, 0, 0};
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = acc_row<T>(lane, v), col = lane & 15;
    const T e = M[row * pm + col];
    ai[v] = row > col ? e : (row == col ? T(1) : T(0));
  }
#pragma unroll
  for (int step = 0; step < 4; ++step)
    t1 = mfma_step(M[(16 + (lane & 15)) * pm + frag_k<T>(step, lane >> 4)], ai[step], t1);
#pragma unroll
  for (int step = 0; step < 4; ++step) {
    const int i = lane & 15, kk = frag_k<T>(step, lane >> 4);
    const T e = M[(16 + i) * pm + 16 + kk];
    x = mfma_step(-(kk < i ? e : (kk == i ? T(1) : T(0))), t1[step], x);
  }
  wave_fence();
#pragma unroll
  for (int v = 0; v < 4; ++v) M[(16 + acc_row<T>(lane, v)) * pm + (lane & 15)] = x[v];
}
template <typename T>
__device__ __forceinline__ void upper_offdiag_inverse(T* M, int pm, int lane) {
  using V = typename AccVec<T>::type;
  wave_fence();
  V u2, t2 = V{0, 0, 0, 0}, y = V{0, 0, 0, 0};
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = acc_row<T>(lane, v), col = lane & 15;
    const T e = M[(16 + row) * pm + 16 + col];
    u2[v] = col >= row ? e : T(0);
  }
#pragma unroll
  for (int step = 0; step < 4; ++step)
    t2 = mfma_step(M[(lane & 15) * pm + 16 + frag_k<T>(step, lane >> 4)], u2[step], t2);
#pragma unroll
  for (int step = 0; step < 4; ++step) {
    const int i = lane & 15, kk = frag_k<T>(step, lane >> 4);
    const T e = M[i * pm + kk];
    y = mfma_step(-(kk >= i ? e : T(0)), t2[step], y);
  }
  wave_fence();
#pragma unroll
  for (int v = 0; v < 4; ++v) M[acc_row<T>(lane, v) * pm + 16 + (lane & 15)] = y[v];
}

// The hot kernels (this one, the wave sweeps, the eigensolver) start on 4 KB
// boundaries: with the code otherwise packed, changes elsewhere in the library
// moved this kernel and changed its time by up to 5 % with identical
// instructions (measured on one device, alternating the two library versions).
template <typename T, int K>
__global__ __launch_bounds__(64) __attribute__((aligned(4096))) void factor_wave_kernel(FactorArgs a) {
  using F = FWave<T, K>;
  using V = typename F::V;
  constexpr int RT = F::RT, KS = F::KS, PT = F::PT;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* lds = reinterpret_cast<T*>(lds_raw);
  T* slab = lds + F::oSlab;
  T* lib = lds + F::oLib;
  T* l21b = lds + F::oL21;
  const Layout& L = a.L;
  const int j = blockIdx.x, k = L.k;
  int lane = threadIdx.x & 63;
  const Geom g = part_geom(L, j, K);
  const int nb = g.nb;
  T* fac = wsT<T>(a.ws, L.fac) + (size_t)j * L.nbmax * L.rec;
  T* gm = wsT<T>(a.ws, L.gmat) + (size_t)j * L.nbmax * K * K;
  int* ipv = wsT<int>(a.ws, L.ipiv) + (size_t)j * L.nbmax * K;
  int* flg = wsT<int>(a.ws, L.flag) + (size_t)j * L.nbmax;
  int* npv = wsT<int>(a.ws, L.npv);
  // diagnostics, kept per lane in LDS (not in registers, which the panel
  // and the products need): max |1 / pivot| over the lane's pivots and max
  // |a_ij| over the band entries the lane stored
  T* diag = lds + F::oDiag;
  diag[lane] = T(0);
  diag[64 + lane] = T(0);

  // band slab of row block R: slab[(d + K) K + i] = A(R K + i, R K + i + d)
  // (partition-local, identity on the virtual rows, zero outside)
  // (loads issued in groups of SG before their LDS stores, so that the
  // latency is paid once per group rather than once per element)
  auto slab_load = [&](int R) {
    constexpr int NS = ((2 * K + 1) * K + 63) / 64, SG = NS < 17 ? NS : 17;
    // the lane index made opaque: the per-element offsets are cheap to
    // recompute, and hoisting them out of the block loop only spills them
    int ln = lane;
    asm volatile("" : "+v"(ln));
    for (int it0 = 0; it0 < NS; it0 += SG) {
      T v[SG];
#pragma unroll
      for (int u = 0; u < SG; ++u) {
        const int o = ln + 64 * (it0 + u);
        const int d = o / K - k, i = o % K;
        const int lr = R * K + i - g.pad;
        T x = T(0);
        if (o < (2 * k + 1) * K) {
          if (lr < 0) {
            x = (d == 0) ? T(1) : T(0);
          } else if (lr < g.nj) {
            const int lc = lr + d;
            if (lc >= 0 && lc < g.nj) x = (T)a.bands[(int64_t)(d + k) * L.n + g.s + lr];
          }
        }
        v[u] = x;
      }
      T am = diag[64 + ln];
#pragma unroll
      for (int u = 0; u < SG; ++u) {
        const int o = ln + 64 * (it0 + u);
        if (o < (2 * k + 1) * K) {
          slab[o + (K - k) * K] = v[u];
          am = fmax(am, fabs(v[u]));
        }
      }
      diag[64 + ln] = am;
    }
  };
  // The same slab through registers: fetched early, stored late.  With
  // K >= 16 one pass of 64 lanes covers DPI = 64 / K whole diagonals, so a
  // lane keeps one row i = lane mod K and walks the diagonals lane / K + DPI it.
  // The loads are unconditional from clamped (always valid) addresses, so
  // that they issue back to back; the identity rows, the entries outside the
  // partition and the padding diagonals are applied when the slab is stored.
  constexpr int NS = ((2 * K + 1) * K + 63) / 64, DPI = 64 / K;
  auto slab_fetch = [&](int R, T (&nx)[NS]) {
    int ln = lane;
    asm volatile("" : "+v"(ln));
    const int i = ln % K, dd0 = ln / K;
    const int lr = min(max(R * K + i - g.pad, 0), g.nj - 1);
    const double* src = a.bands + g.s + lr;
#pragma unroll
    for (int it = 0; it < NS; ++it) nx[it] = (T)src[(int64_t)min(dd0 + DPI * it, 2 * k) * L.n];
  };
  auto slab_put = [&](int R, const T (&nx)[NS]) {
    int ln = lane;
    asm volatile("" : "+v"(ln));
    const int i = ln % K, dd0 = ln / K, lr = R * K + i - g.pad;
    T* dst = slab + (K - k) * K + ln;
    T am = diag[64 + ln];
#pragma unroll
    for (int it = 0; it < NS; ++it) {
      const int dd = dd0 + DPI * it, d = dd - k, lc = lr + d;
      const T v = lr < 0 ? ((d == 0) ? T(1) : T(0)) : ((lr < g.nj && lc >= 0 && lc < g.nj) ? nx[it] : T(0));
      if (dd < 2 * k + 1) {
        dst[64 * it] = v;
        am = fmax(am, fabs(v));
      }
    }
    diag[64 + ln] = am;
  };
  auto sl = [&](int i, int d) -> T { return (d >= -K && d <= K) ? slab[(d + K) * K + i] : T(0); };
  auto for_elems = [&](auto&& fn) {  // (t, ct, v, row, col) of the lane's accumulator elements
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int ct = 0; ct < RT; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) fn(t, ct, v, 16 * t + acc_row<T>(lane, v), 16 * ct + (lane & 15));
  };
  auto zero = [&](V (&x)[RT][RT]) {
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int ct = 0; ct < RT; ++ct) x[t][ct] = V{0, 0, 0, 0};
  };
  // out (+)= op(A) * in; A operand element (i, kk) from fa(i, kk); B from accumulator tiles.
  // tri: 1 = A lower triangular, 2 = upper (the 16 x 16 tiles it leaves zero are skipped)
  auto mul = [&](auto&& fa, const V (&in)[RT][RT], V (&out)[RT][RT], T sign, int tri) {
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int step = 0; step < KS; ++step) {
        if ((tri == 1 && (step >> 2) > t) || (tri == 2 && (step >> 2) < t)) continue;
        const T av = sign * fa(16 * t + (lane & 15), frag_k<T>(step, lane >> 4));
#pragma unroll
        for (int ct = 0; ct < RT; ++ct) out[t][ct] = mfma_step(av, in[step >> 2][ct][step & 3], out[t][ct]);
      }
  };
  // out += X^T * in with X in accumulator tiles (tile-transposed A operand); X lower
  // triangular, so X^T leaves the tiles left of the row tile zero
  auto mul_tr = [&](const V (&X)[RT][RT], const V (&in)[RT][RT], V (&out)[RT][RT], T sign) {
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int step = 0; step < KS; ++step) {
        if ((step >> 2) < t) continue;
        const T av = sign * X[step >> 2][t][step & 3];
#pragma unroll
        for (int ct = 0; ct < RT; ++ct) out[t][ct] = mfma_step(av, in[step >> 2][ct][step & 3], out[t][ct]);
      }
  };

  // ---- initial state: Dc_0 (lib, row-major), Up_0 (uc), W rhs of blocks 0 and 1
  for (int o = lane; o < (2 * K + 1) * K; o += 64) slab[o] = T(0);
  wave_sync();
  slab_load(0);
  wave_sync();
  V uc[RT][RT], gc[RT][RT];
  for (int o = lane; o < K * K; o += 64) lib[(o / K) * PT + o % K] = sl(o / K, o % K - o / K);
  for_elems([&](int t, int ct, int v, int row, int col) { uc[t][ct][v] = sl(row, K + col - row); });
  zero(gc);
  wave_sync();
  if (nb > 1) slab_load(1);
  wave_sync();

  for (int b = 0; b < nb; ++b) {
    const bool last = (b == nb - 1);
    const int nr = last ? K : 2 * K;
    asm volatile("" : "+v"(lane));  // (same: no lane-derived values kept across blocks)
    T nx[NS];  // band slab of block b + 2, fetched below and stored once this block is done with the slab
    auto Li = [&](int i, int kk) -> T { return i > kk ? lib[i * PT + kk] : (i == kk ? T(1) : T(0)); };
    auto UiT = [&](int i, int kk) -> T { return kk <= i ? lib[kk * PT + i] : T(0); };
    auto L21 = [&](int i, int kk) -> T { return i <= kk ? l21b[i * PT + kk] : T(0); };
    V u12[RT][RT], dn[RT][RT];
    // ---- panel [Dc_b; Lo_{b+1}]: lane i < K takes row i of Dc_b (lib), lane K + i
    // row i of Lo_{b+1} (slab)
    {
      T pa[K], iv[K];
      {
        // one unconditional LDS read per element (no branch per column):
        // lib[lane PT + c] for the top rows, slab[(c - i) K + i] (diagonal
        // c - lane of row i = lane - K) for the bottom rows, zero outside the band
        const bool top = lane < K;
        const int i = lane - K;
#pragma unroll
        for (int c = 0; c < K; ++c) {
          const bool ok = top || (lane < nr && c >= i);
          const int off = top ? F::oLib + lane * PT + c : F::oSlab + (c - i) * K + i;
          const T v = lds[ok ? off : 0];
          pa[c] = ok ? v : T(0);
          iv[c] = T(0);
        }
      }
      if (b + 2 < nb) slab_fetch(b + 2, nx);
      T mx = T(0), dmin = T(INFINITY), dinv = T(0);
      int ln1 = lane;  // own opaque lane index (its masks are not kept for later use)
      asm volatile("" : "+v"(ln1));
      FwdElim<T, K, 0, 16>::run(pa, iv, ln1, nr, mx, dmin, dinv);
      // a zero or non-finite pivot leaves an infinite, NaN or zero reciprocal
      // in its lane: such a partition (and one that would interchange rows)
      // goes to the interchanging kernel, which latches the precise error
      const bool ok = !__any(!(mx <= T(1)) || (ln1 < K && !(isfinite(dinv) && dinv != T(0)))) && (dmin > T(0));
      if (!ok) {
        if (lane == 0) npv[j] = 1;
        return;  // refactored with row interchanges by the general kernel
      }
      if (ln1 < K && b * K + ln1 >= g.pad) diag[ln1] = fmax(diag[ln1], fabs(dinv));  // not the virtual rows
      // lib <- the 16 x 16 diagonal blocks of L11^{-1} strictly below the
      // diagonal (and, at K = 32, the block L_{21} of L11 below them, for the
      // products that follow); l21b <- L21
      if (lane < K) {
#pragma unroll
        for (int c = 0; c < K; ++c)
          if (c < lane) lib[lane * PT + c] = (c >= (lane & ~15)) ? iv[c] : pa[c];
      } else if (lane < nr) {
#pragma unroll
        for (int c = 0; c < K; ++c) l21b[(lane - K) * PT + c] = pa[c];
      }
      if constexpr (K == 32) lower_offdiag_inverse<T>(lib, PT, lane);
      wave_fence();  // L11^{-1} and L21 visible to the products issued below
      // U11^{-1} rows, then lib <- U11^{-1} on and above the diagonal (a fresh
      // opaque lane index: lane masks are not shared with the forward pass).
      // The upward pass is a chain of lane reads and vector updates; the
      // independent products U12 = L11^{-1} Up_b and Dc_{b+1} = D_{b+1} - L21 U12
      // are issued one (tile, k-step) pair per step alongside it, so the matrix
      // cores work while the chain waits.
      int ln2 = lane;
      asm volatile("" : "+v"(ln2));
#pragma unroll
      for (int c = 0; c < K; ++c) iv[c] = (c == ln2) ? T(1) : T(0);
      if (!last) zero(u12);
      constexpr int NPR = RT * KS;  // (tile, k-step) pairs of one product
      // A operand of pair S: L11^{-1} (lower triangular) for U12, -L21 (upper) for Dc
      auto opnd = [&](auto cst) -> T {
        constexpr int S = decltype(cst)::value;
        if constexpr (S < NPR) {
          constexpr int t = S / KS, step = S % KS;
          if constexpr ((step >> 2) <= t) return Li(16 * t + (lane & 15), frag_k<T>(step, lane >> 4));
        } else if constexpr (S < 2 * NPR) {
          constexpr int t = (S - NPR) / KS, step = (S - NPR) % KS;
          if constexpr ((step >> 2) >= t) return -L21(16 * t + (lane & 15), frag_k<T>(step, lane >> 4));
        }
        return T(0);
      };
      // software-pipelined: step S issues pair S with the operand read during
      // step S - 1 and reads the operand of pair S + 1
      T avn = last ? T(0) : opnd(std::integral_constant<int, 0>{});
      auto hook = [&](auto cst) {
        constexpr int S = decltype(cst)::value;
        if (last) return;
        const T av = avn;
        avn = opnd(std::integral_constant<int, S + 1>{});
        if constexpr (S == NPR - 2)  // D_{b+1} read two steps before the first Dc pair
          for_elems([&](int t2, int ct, int v, int row, int col) { dn[t2][ct][v] = sl(row, col - row); });
        if constexpr (S < NPR) {
          constexpr int t = S / KS, step = S % KS;
          if constexpr ((step >> 2) <= t) {
#pragma unroll
            for (int ct = 0; ct < RT; ++ct) u12[t][ct] = mfma_step(av, uc[step >> 2][ct][step & 3], u12[t][ct]);
          }
        } else if constexpr (S < 2 * NPR) {
          constexpr int t = (S - NPR) / KS, step = (S - NPR) % KS;
          if constexpr ((step >> 2) >= t) {
#pragma unroll
            for (int ct = 0; ct < RT; ++ct) dn[t][ct] = mfma_step(av, u12[step >> 2][ct][step & 3], dn[t][ct]);
          }
        }
      };
      static_assert(2 * NPR <= K && NPR >= 2, "the products fit the steps of the pass");
      BwdElimH<T, K, K - 1, 16>::run(pa, iv, ln2, dinv, hook);
      // lib <- the 16 x 16 diagonal blocks of U11^{-1} on and above the
      // diagonal (and, at K = 32, the block U_{12} of U11 right of them)
      if (lane < K)
#pragma unroll
        for (int c = 0; c < K; ++c)
          if (c >= lane) lib[lane * PT + c] = (c < (lane | 15) + 1) ? iv[c] : pa[c];
      if constexpr (K == 32) upper_offdiag_inverse<T>(lib, PT, lane);
      wave_sync();
    }
    // ---- G step (the columns of E_t met in this block enter the pending sum)
    {
      V gb[RT][RT];
      for_elems([&](int t, int ct, int v, int row, int col) {
        if (col == b * K + row - g.pad) gc[t][ct][v] += T(1);
      });
      zero(gb);
      mul(UiT, gc, gb, T(1), 1);
      zero(gc);
      if (!last) mul_tr(u12, gb, gc, T(-1));  // pending(b+1) = -U12^T g_b
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int step = 0; step < KS; ++step)
          gm[(size_t)b * K * K + ((t * KS + step) << 6) + lane] = gb[step >> 2][t][step & 3];
    }
    // ---- stores: LP, pivots, flags
    T* rec = fac + (size_t)b * L.rec;
    // fragment order: position 64 f + lane holds element (16 t + lane mod 16,
    // frag_k(step, lane / 16)) with f = t KS + step
    auto frag_store = [&](T* dst, auto&& val) {
#pragma unroll
      for (int f = 0; f < K * K / 64; ++f) {
        const int i = 16 * (f / KS) + (lane & 15), c = frag_k<T>(f % KS, lane >> 4);
        dst[64 * f + lane] = val(i, c);
      }
    };
    frag_store(rec, [&](int i, int c) { return (i > c) ? lib[i * PT + c] : (last ? T(0) : l21b[i * PT + c]); });
    if (lane < K) ipv[(size_t)b * K + lane] = lane;
    if (lane == 0) flg[b] = 0;
    wave_sync();
    if (!last) {
      // U12 staged row-major in l21b (L21 no longer needed), then UP = U11^{-1} | U12
      for_elems([&](int t, int ct, int v, int row, int col) { l21b[row * PT + col] = u12[t][ct][v]; });
      wave_sync();
      frag_store(rec + K * K, [&](int i, int c) { return (i <= c) ? lib[i * PT + c] : l21b[i * PT + c]; });
      if (lane < K) rec[2 * K * K + lane] = l21b[lane * PT + lane];
      wave_sync();
      // next state: Dc_{b+1} -> lib, Up_{b+1} -> uc, W window shifts, next slab
      for_elems([&](int t, int ct, int v, int row, int col) {
        lib[row * PT + col] = dn[t][ct][v];
        uc[t][ct][v] = sl(row, K + col - row);
      });
      wave_sync();
      if (b + 2 < nb) slab_put(b + 2, nx);
      wave_sync();
    } else {
      frag_store(rec + K * K, [&](int i, int c) { return (i <= c) ? lib[i * PT + c] : T(0); });
      if (lane < K) rec[2 * K * K + lane] = T(0);
    }
  }
  {
    wave_sync();
    const T pinv = wave_max(diag[lane]), am = wave_max(diag[64 + lane]);
    if ((threadIdx.x & 63) == 0) {
      int* st = wsT<int>(a.ws, L.latch);
      state_min(st, S_PIVMIN, pinv > T(0) ? 1.0 / (double)pinv : (double)INFINITY);
      state_max(st, S_AMAX, (double)am);
    }
  }
}


// Spike forward sweeps over the stored factors (partitions factored without
// interchanges; the others were fully handled by the interchanging kernel).
//   W: rhs [C_j; 0] (first K real rows):  z_b = L11^{-1} r_b, r_{b+1} -= L21 z_b,
//      W_t = sum_b G_b^T z_b, W_b = U11^{-1} z_last; z_b kept for the Gram pass (r < k)
//   V: rhs [0; B_j] lives in the last block only: z = L11^{-1} B_j there,
//      V_b = U11^{-1} z, V_t = G_last^T z.
template <typename T, int K>
__global__ __launch_bounds__(64) __attribute__((aligned(4096))) void spike_wave_kernel(FactorArgs a) {
  constexpr int MCT = K / 16;
  using W = WaveSweep<T, K, MCT>;
  using V = typename W::V;
  constexpr int NF = W::RT * W::KS;
  const Layout& L = a.L;
  const int j = blockIdx.x, k = L.k;
  int lane = threadIdx.x & 63;
  if (wsT<int>(a.ws, L.npv)[j]) return;
  const Geom g = part_geom(L, j, K);
  const T* fac = wsT<T>(a.ws, L.fac) + (size_t)j * L.nbmax * L.rec;
  const T* gm = wsT<T>(a.ws, L.gmat) + (size_t)j * L.nbmax * K * K;
  T* ym = (L.r < K) ? wsT<T>(a.ws, L.ymat) + (size_t)j * L.nbmax * 2 * K * K : nullptr;
  double* tips = wsT<double>(a.ws, L.tips) + (size_t)j * 4 * K * K;  // Vt, Vb, Wt, Wb
  auto rhs_w = [&](int R, V (&st)[W::RT][MCT]) {
#pragma unroll
    for (int t = 0; t < W::RT; ++t)
#pragma unroll
      for (int ct = 0; ct < MCT; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 16 * t + acc_row<T>(lane, v), col = 16 * ct + (lane & 15);
          const int lr = R * K + row - g.pad;
          st[t][ct][v] = (j > 0 && lr >= 0 && lr < K && lr < g.nj) ? (T)band_at(a.bands, L.n, k, g.s + lr, g.s - K + col) : T(0);
        }
  };
  auto put = [&](int which, const V (&st)[W::RT][MCT]) {
#pragma unroll
    for (int t = 0; t < W::RT; ++t)
#pragma unroll
      for (int ct = 0; ct < MCT; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 16 * t + acc_row<T>(lane, v), col = 16 * ct + (lane & 15);
          tips[(size_t)which * K * K + row * K + col] = (double)st[t][ct][v];
        }
  };
  auto put_y = [&](int b, int coff, const V (&st)[W::RT][MCT]) {
#pragma unroll
    for (int t = 0; t < W::RT; ++t)
#pragma unroll
      for (int ct = 0; ct < MCT; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 16 * t + acc_row<T>(lane, v), col = 16 * ct + (lane & 15);
          ym[(size_t)b * 2 * K * K + row * 2 * K + coff + col] = st[t][ct][v];
        }
  };
  V w0[W::RT][MCT], w1[W::RT][MCT], z[W::RT][MCT], acc[W::RT][MCT];
  zero_strip<T, K, MCT>(acc);
  rhs_w(0, w0);
  if (g.nb > 1)
    rhs_w(1, w1);
  else
    zero_strip<T, K, MCT>(w1);
  // L and G^T fragments in a prefetch ring (as in the solve sweeps): block q
  // in slot q mod NS, every prefetch unconditional, the block loop unrolled
  // over the slots; the last block, which also forms V, comes after the loop
  constexpr int PD = sweep_pd<K, MCT>(), NS = PD + 1;
  const int nb = g.nb;
  T lpq[NS][NF], gtq[NS][NF];
  auto fetch = [&](int q, T (&lp)[NF], T (&gt)[NF]) __attribute__((always_inline)) {
    const int qc = min(q, nb - 1);
    load_frags<T, K>(lp, fac + (size_t)qc * L.rec);
    load_frags<T, K>(gt, gm + (size_t)qc * K * K);
  };
  static_for<PD>([&](auto U) __attribute__((always_inline)) {
    constexpr int u = decltype(U)::value;
    fetch(u, lpq[u], gtq[u]);
  });
  // blocks 0 .. nb-2: the right-hand side [C_j; 0] lives in blocks 0 and 1 only
  auto body = [&](auto U, int b) __attribute__((always_inline)) {
    constexpr int u = decltype(U)::value, uf = (u + PD) % NS;
    fetch(b + PD, lpq[uf], gtq[uf]);
    zero_strip<T, K, MCT>(z);
    blk_mul<T, K, MCT, 0>(lpq[u], nullptr, T(1), w0, z);
    blk_mul<T, K, MCT, 1>(lpq[u], nullptr, T(-1), z, w1);
    blk_mul<T, K, MCT, 9>(gtq[u], nullptr, T(1), z, acc);
    if (ym) {
      put_y(b, 0, z);
      if (b == nb - 2) {  // V's forward result above the last block (zero here; read by the back-sweep)
        V zz[W::RT][MCT];
        zero_strip<T, K, MCT>(zz);
        put_y(b, K, zz);
      }
    }
#pragma unroll
    for (int t = 0; t < W::RT; ++t)
#pragma unroll
      for (int ct = 0; ct < MCT; ++ct) w0[t][ct] = w1[t][ct];
    zero_strip<T, K, MCT>(w1);
  };
  int b0 = 0;
  for (; b0 + NS <= nb - 1; b0 += NS)
    static_for<NS>([&](auto U) __attribute__((always_inline)) { body(U, b0 + decltype(U)::value); });
  static_for<NS>([&](auto U) __attribute__((always_inline)) {
    if (b0 + decltype(U)::value < nb - 1) body(U, b0 + decltype(U)::value);
  });
  // last block: W's bottom tip and top tip, and the V spike (its right-hand
  // side [0; B_j] lives in this block only)
  {
    const int b = nb - 1;
    T lp[NF], gt[NF], up[NF];
    load_frags<T, K>(lp, fac + (size_t)b * L.rec);
    load_frags<T, K>(gt, gm + (size_t)b * K * K);
    load_frags<T, K>(up, fac + (size_t)b * L.rec + K * K);
    zero_strip<T, K, MCT>(z);
    blk_mul<T, K, MCT, 0>(lp, nullptr, T(1), w0, z);
    blk_mul<T, K, MCT, 9>(gt, nullptr, T(1), z, acc);
    if (ym) put_y(b, 0, z);
    V wb[W::RT][MCT], bv[W::RT][MCT], zv[W::RT][MCT], vb[W::RT][MCT], vt[W::RT][MCT];
    zero_strip<T, K, MCT>(wb);
    blk_mul<T, K, MCT, 2>(up, nullptr, T(1), z, wb);
#pragma unroll
    for (int t = 0; t < W::RT; ++t)
#pragma unroll
      for (int ct = 0; ct < MCT; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 16 * t + acc_row<T>(lane, v), col = 16 * ct + (lane & 15);
          const int lr = b * K + row - g.pad;
          bv[t][ct][v] = (j < L.p - 1 && lr >= 0) ? (T)band_at(a.bands, L.n, k, g.s + lr, g.s + g.nj + col) : T(0);
        }
    zero_strip<T, K, MCT>(zv);
    blk_mul<T, K, MCT, 0>(lp, nullptr, T(1), bv, zv);
    zero_strip<T, K, MCT>(vb);
    blk_mul<T, K, MCT, 2>(up, nullptr, T(1), zv, vb);
    zero_strip<T, K, MCT>(vt);
    blk_mul<T, K, MCT, 9>(gt, nullptr, T(1), zv, vt);
    if (ym) put_y(b, K, zv);
    put(0, vt);
    put(1, vb);
    put(2, acc);
    put(3, wb);
  }
}

}  // namespace lrs
