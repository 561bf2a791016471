// Solve sweeps at K = 64 on the matrix cores: one workgroup of four waves per
// (partition, 16 right-hand-side columns), wave t owning row tile t (rows
// 16t .. 16t+15) of every 64-row block.  A 64-row block no longer fits one
// wave's registers with its prefetch (the K <= 32 sweeps keep the whole block
// in one wave), so each wave reads only its row tile's fragments of the factor
// records (one coalesced 64-lane load per fragment, as stored) and the waves
// exchange the 64 x 16 right-hand-side strips through LDS in accumulator
// layout: a product's accumulator tile is, lane for lane, the B operand of the
// next product, so wave t writes its tile and every wave reads all four.
// Partitions at K = 64 are factored without interchanges, so the sweeps are
// those of A_j = L U:
//   forward  z_b = L11^{-1} r_b,  r_{b+1} -= L21 z_b  (D-stage: y_t += G_b^T z_b,
//            y_b = U11^{-1} z_last; retrieval: z_b written for the back-sweep)
//   backward x_b = U11^{-1} (z_b - U12 x_{b+1})
// with the record blocks LP = [L11^{-1} strictly lower | L21 upper] and
// UP = [U11^{-1} upper | U12 strictly lower] + UD = diag(U12).
#pragma once
#include "common.h"
#include "layout.h"

namespace lrs {

struct Sw64 {
  static constexpr int K = 64, RT = 4, KS = 16;
  // LDS: two strips (accumulator layout: tile, lane, element) and the two
  // correction blocks of the retrieval (64 x 17 each)
  static constexpr int STRIP = RT * 64 * 4;
  static constexpr int oA = 0, oB = STRIP, oCt = 2 * STRIP, oCb = oCt + K * 17, total = oCb + K * 17;
};

using V64 = AccVec<double>::type;

// own tile -> LDS strip, barrier, all four tiles <- LDS strip
__device__ __forceinline__ void sw64_exchange(double* buf, const V64& own, int t, V64 (&all)[4]) {
  const int lane = threadIdx.x & 63;
  *reinterpret_cast<V64*>(buf + ((size_t)t * 64 + lane) * 4) = own;
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u) all[u] = *reinterpret_cast<const V64*>(buf + ((size_t)u * 64 + lane) * 4);
}

// out (+)= sign * A(row tile t) * S with A's fragments fr[step] (step = k-step
// of the 64 columns); kind: 0 L11^{-1} (strict lower + unit diagonal),
// 1 L21 (upper incl. diagonal), 2 U11^{-1} (upper incl. diagonal), 3 U12's
// strictly lower part, 9 full
template <int KIND>
__device__ __forceinline__ void sw64_mul(const double (&fr)[16], int t, const V64 (&S)[4], V64& out, double sign) {
  const int lane = threadIdx.x & 63, i = 16 * t + (lane & 15);
#pragma unroll
  for (int step = 0; step < 16; ++step) {
    const int ct = step >> 2;
    if ((KIND == 0 || KIND == 3) && ct > t) continue;  // lower: zero right of the row tile
    if ((KIND == 1 || KIND == 2) && ct < t) continue;  // upper: zero left of the row tile
    const int kk = frag_k<double>(step, lane >> 4);
    double a = fr[step];
    if (KIND == 0) a = i > kk ? a : (i == kk ? 1.0 : 0.0);
    if (KIND == 1 || KIND == 2) a = i <= kk ? a : 0.0;
    if (KIND == 3) a = i > kk ? a : 0.0;
    out = mfma_step(sign * a, S[ct][step & 3], out);
  }
}

__device__ __forceinline__ void sw64_frags(double (&fr)[16], const double* blk, int t) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int step = 0; step < 16; ++step) fr[step] = blk[(size_t)(t * 16 + step) * 64 + lane];
}

// Right-hand-side tile t of block b: rows b K + 16 t + acc_row(lane, v) - pad
// of the partition (zero on the padding rows and outside the chunk's
// columns), minus the retrieval's corrections (Ct on the first K real rows,
// Cb on the last K; pitch 17) when given.
__device__ __forceinline__ V64 sw64_rhs(const SolveArgs& a, const Geom& g, int b, int t, int c0, int mc,
                                        const double* Ct, const double* Cb) {
  const int lane = threadIdx.x & 63, col = lane & 15;
  V64 r;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int lr = b * 64 + 16 * t + acc_row<double>(lane, v) - g.pad;
    double x = 0.0;
    if (lr >= 0 && lr < g.nj && col < mc) {
      x = a.src[(g.s + lr) * (int64_t)a.ld + c0 + col];
      if (Ct && lr < 64) x -= Ct[lr * 17 + col];
      if (Cb && lr >= g.nj - 64) x -= Cb[(lr - (g.nj - 64)) * 17 + col];
    }
    r[v] = x;
  }
  return r;
}

__device__ __forceinline__ void sw64_store(const SolveArgs& a, const Geom& g, int b, int t, int c0, int mc,
                                           const V64& x) {
  const int lane = threadIdx.x & 63, col = lane & 15;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int lr = b * 64 + 16 * t + acc_row<double>(lane, v) - g.pad;
    if (lr >= 0 && lr < g.nj && col < mc) a.dst[(g.s + lr) * (int64_t)a.ld + c0 + col] = x[v];
  }
}

// Forward sweep of partition j, columns [c0, c0 + mc).
template <bool DSTAGE>
__device__ void sw64_forward(const SolveArgs& a, const Geom& g, int j, int c0, int mc, double* lds, const double* Ct,
                             const double* Cb) {
  const Layout& L = a.L;
  const int t = threadIdx.x >> 6, lane = threadIdx.x & 63, nb = g.nb;
  const double* fac = wsp<double>(a.ws, L.fac) + (size_t)j * L.nbmax * L.rec;
  const double* gm = wsp<double>(a.ws, L.gmat) + (size_t)j * L.nbmax * 64 * 64;
  double lp[16], lpn[16], gt[16], gtn[16];
  sw64_frags(lp, fac, t);
  if (DSTAGE) sw64_frags(gt, gm, t);
  V64 r = sw64_rhs(a, g, 0, t, c0, mc, Ct, Cb), acc = V64{0, 0, 0, 0}, z, S[4], Z[4];
  for (int b = 0; b < nb; ++b) {
    const bool last = b == nb - 1;
    const int bn = last ? b : b + 1;  // (clamped: the prefetch is unconditional)
    sw64_frags(lpn, fac + (size_t)bn * L.rec, t);
    if (DSTAGE) sw64_frags(gtn, gm + (size_t)bn * 64 * 64, t);
    V64 rn = sw64_rhs(a, g, bn, t, c0, mc, Ct, Cb);
    sw64_exchange(lds + Sw64::oA, r, t, S);
    z = V64{0, 0, 0, 0};
    sw64_mul<0>(lp, t, S, z, 1.0);
    sw64_exchange(lds + Sw64::oB, z, t, Z);
    if (!last) sw64_mul<1>(lp, t, Z, rn, -1.0);
    if (DSTAGE)
      sw64_mul<9>(gt, t, Z, acc, 1.0);
    else
      sw64_store(a, g, b, t, c0, mc, z);
    if (DSTAGE && last) {  // y_b = U11^{-1} z_last
      double up[16];
      sw64_frags(up, fac + (size_t)b * L.rec + 64 * 64, t);
      V64 yb = V64{0, 0, 0, 0};
      sw64_mul<2>(up, t, Z, yb, 1.0);
      double* ytip = wsp<double>(a.ws, L.ytip) + (size_t)j * 2 * 64 * L.mmax;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * t + acc_row<double>(lane, v), col = lane & 15;
        if (col < mc) {
          ytip[(size_t)row * L.mmax + c0 + col] = acc[v];
          ytip[(size_t)(64 + row) * L.mmax + c0 + col] = yb[v];
        }
      }
    }
    r = rn;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      lp[s] = lpn[s];
      if (DSTAGE) gt[s] = gtn[s];
    }
  }
}

// Backward sweep over a.dst (z in, x out), blocks from the last to the first.
__device__ void sw64_backward(const SolveArgs& a, const Geom& g, int j, int c0, int mc, double* lds) {
  const Layout& L = a.L;
  const int t = threadIdx.x >> 6, lane = threadIdx.x & 63, nb = g.nb;
  const double* fac = wsp<double>(a.ws, L.fac) + (size_t)j * L.nbmax * L.rec;
  SolveArgs ad = a;
  ad.src = a.dst;
  double up[16], upn[16];
  V64 ud, udn;
  auto load_ud = [&](int b, V64& d) {
    const double* u = fac + (size_t)b * L.rec + 2 * 64 * 64;
#pragma unroll
    for (int v = 0; v < 4; ++v) d[v] = u[16 * t + acc_row<double>(lane, v)];
  };
  sw64_frags(up, fac + (size_t)(nb - 1) * L.rec + 64 * 64, t);
  load_ud(nb - 1, ud);
  V64 zt = sw64_rhs(ad, g, nb - 1, t, c0, mc, nullptr, nullptr), X[4], Y[4];
  for (int q = 0; q < 4; ++q) X[q] = V64{0, 0, 0, 0};
  for (int b = nb - 1; b >= 0; --b) {
    const int bn = b > 0 ? b - 1 : 0;
    sw64_frags(upn, fac + (size_t)bn * L.rec + 64 * 64, t);
    load_ud(bn, udn);
    V64 ztn = sw64_rhs(ad, g, bn, t, c0, mc, nullptr, nullptr);
    if (b < nb - 1) {  // z_b - U12 x_{b+1}, U12 = strictly lower part of UP + diag(UD)
      sw64_mul<3>(up, t, X, zt, -1.0);
#pragma unroll
      for (int v = 0; v < 4; ++v) zt[v] -= ud[v] * X[t][v];
    }
    sw64_exchange(lds + Sw64::oA, zt, t, Y);
    V64 x = V64{0, 0, 0, 0};
    sw64_mul<2>(up, t, Y, x, 1.0);
    sw64_store(a, g, b, t, c0, mc, x);
    sw64_exchange(lds + Sw64::oB, x, t, X);
    zt = ztn;
    ud = udn;
#pragma unroll
    for (int s = 0; s < 16; ++s) up[s] = upn[s];
  }
}

// D-stage at K = 64: tips of A_j^{-1} f_j.  Grid (p, column chunks of 16), 256 threads.
__global__ __launch_bounds__(256) void dstage64_kernel(SolveArgs a) {
  if (gated(a.gate)) return;
  __shared__ __align__(16) double lds[Sw64::total];
  const int j = blockIdx.x, c0 = blockIdx.y * 16, mc = min(16, a.m - c0);
  const Geom g = part_geom(a.L, j, 64);
  sw64_forward<true>(a, g, j, c0, mc, lds, nullptr, nullptr);
}

// Retrieval at K = 64: x_j = A_j^{-1} (f_j - [C_j x_{j-1,b}; 0; B_j x_{j+1,t}])
// in place (block-diagonal solve with block_only).  Grid (p, column chunks of 16).
__global__ __launch_bounds__(256) void retrieve64_kernel(SolveArgs a) {
  if (gated(a.gate)) return;
  __shared__ __align__(16) double lds[Sw64::total];
  const Layout& L = a.L;
  const int j = blockIdx.x, c0 = blockIdx.y * 16, mc = min(16, a.m - c0), k = L.k;
  const Geom g = part_geom(L, j, 64);
  double* Ct = lds + Sw64::oCt;
  double* Cb = lds + Sw64::oCb;
  double* Xn = lds + Sw64::oA;  // neighbour tip staging (the strips are not in use yet)
  const bool top = j > 0 && !a.block_only, bot = j < L.p - 1 && !a.block_only;
  if (top) {
    interface_tip<double, 64>(a, j - 1, false, c0, mc, Xn);  // x_{j-1,b}, pitch 17
    __syncthreads();
    for (int o = threadIdx.x; o < 64 * mc; o += blockDim.x) {
      const int i = o / mc, c = o % mc;
      double s = 0.0;
      for (int l = 0; l < 64; ++l) s += band_at(a.bands, L.n, k, g.s + i, g.s - 64 + l) * Xn[l * 17 + c];
      Ct[i * 17 + c] = s;
    }
    __syncthreads();
  }
  if (bot) {
    interface_tip<double, 64>(a, j + 1, true, c0, mc, Xn);  // x_{j+1,t}
    __syncthreads();
    const int64_t s1 = g.s + g.nj;
    for (int o = threadIdx.x; o < 64 * mc; o += blockDim.x) {
      const int i = o / mc, c = o % mc;
      double s = 0.0;
      for (int l = 0; l < 64; ++l) s += band_at(a.bands, L.n, k, s1 - 64 + i, s1 + l) * Xn[l * 17 + c];
      Cb[i * 17 + c] = s;
    }
    __syncthreads();
  }
  sw64_forward<false>(a, g, j, c0, mc, lds, top ? Ct : nullptr, bot ? Cb : nullptr);
  __syncthreads();  // z of the whole chunk written (each wave stored its own rows)
  sw64_backward(a, g, j, c0, mc, lds);
}

// ------------------------------------------------------------------ spikes
// The spikes at K = 64 in the same layout (four waves, wave t owning row tile
// t, fragments read from the records).  Forward, grid (p, 4 groups of 16 spike
// columns, 2 spikes):
//   W (spike 0): rhs [C_j; 0], nonzero in the first K real rows only, swept
//     forward; W_t = sum_b G_b^T z_b, W_b = U11^{-1} z_last;
//   V (spike 1): rhs [0; B_j], the last block only: z = L11^{-1} B_j there,
//     V_t = G_last^T z, V_b = U11^{-1} z;
// z_b goes to the Y array (row-major, both spikes side by side) for the Gram
// back-sweeps when r < K.  Tips: V_t, V_b, W_t, W_b (K x K each, row-major).
__global__ __launch_bounds__(256) void spike64_kernel(FactorArgs a) {
  __shared__ __align__(16) double lds[2 * Sw64::STRIP];
  const Layout& L = a.L;
  const int j = blockIdx.x, c0 = blockIdx.y * 16, spike = blockIdx.z, k = L.k;
  const int t = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 15;
  const Geom g = part_geom(L, j, 64);
  const int nb = g.nb;
  const double* fac = wsp<double>(a.ws, L.fac) + (size_t)j * L.nbmax * L.rec;
  const double* gm = wsp<double>(a.ws, L.gmat) + (size_t)j * L.nbmax * 64 * 64;
  double* ym = L.r < 64 ? wsp<double>(a.ws, L.ymat) + (size_t)j * L.nbmax * 2 * 64 * 64 : nullptr;
  double* tips = wsp<double>(a.ws, L.tips) + (size_t)j * 4 * 64 * 64;
  // right-hand-side tile t of block b (the coupling blocks of the band)
  auto rhs = [&](int b) {
    V64 r = V64{0, 0, 0, 0};
    const bool nz = spike == 0 ? (j > 0 && b * 64 - g.pad < 64) : (j < L.p - 1 && b == nb - 1);
    if (nz) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int lr = b * 64 + 16 * t + acc_row<double>(lane, v) - g.pad;
        if (lr >= 0 && lr < g.nj)
          r[v] = spike == 0 ? (lr < 64 ? band_at(a.bands, L.n, k, g.s + lr, g.s - 64 + c0 + col) : 0.0)
                            : band_at(a.bands, L.n, k, g.s + lr, g.s + g.nj + c0 + col);
      }
    }
    return r;
  };
  auto store_y = [&](int b, const V64& z) {
    if (!ym) return;
#pragma unroll
    for (int v = 0; v < 4; ++v)
      ym[(size_t)b * 2 * 64 * 64 + (16 * t + acc_row<double>(lane, v)) * 128 + spike * 64 + c0 + col] = z[v];
  };
  // tips (which, which + 1) = (top, bottom); the last block's U11^{-1} z gives the bottom
  auto finish = [&](int b, const V64 (&Z)[4], const V64& top, int which) {
    double up[16];
    sw64_frags(up, fac + (size_t)b * L.rec + 64 * 64, t);
    V64 yb = V64{0, 0, 0, 0};
    sw64_mul<2>(up, t, Z, yb, 1.0);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * t + acc_row<double>(lane, v);
      tips[(size_t)which * 64 * 64 + row * 64 + c0 + col] = top[v];
      tips[(size_t)(which + 1) * 64 * 64 + row * 64 + c0 + col] = yb[v];
    }
  };
  double lp[16], gt[16];
  V64 S[4], Z[4], acc = V64{0, 0, 0, 0};
  if (spike == 1) {
    const int b = nb - 1;
    sw64_frags(lp, fac + (size_t)b * L.rec, t);
    sw64_frags(gt, gm + (size_t)b * 64 * 64, t);
    sw64_exchange(lds + Sw64::oA, rhs(b), t, S);
    V64 z = V64{0, 0, 0, 0};
    sw64_mul<0>(lp, t, S, z, 1.0);
    sw64_exchange(lds + Sw64::oB, z, t, Z);
    sw64_mul<9>(gt, t, Z, acc, 1.0);
    store_y(b, z);
    finish(b, Z, acc, 0);
    return;
  }
  double lpn[16], gtn[16];
  sw64_frags(lp, fac, t);
  sw64_frags(gt, gm, t);
  V64 r = rhs(0);
  for (int b = 0; b < nb; ++b) {
    const bool last = b == nb - 1;
    const int bn = last ? b : b + 1;  // (clamped: the prefetch is unconditional)
    sw64_frags(lpn, fac + (size_t)bn * L.rec, t);
    sw64_frags(gtn, gm + (size_t)bn * 64 * 64, t);
    V64 rn = rhs(bn);
    sw64_exchange(lds + Sw64::oA, r, t, S);
    V64 z = V64{0, 0, 0, 0};
    sw64_mul<0>(lp, t, S, z, 1.0);
    sw64_exchange(lds + Sw64::oB, z, t, Z);
    if (!last) sw64_mul<1>(lp, t, Z, rn, -1.0);
    sw64_mul<9>(gt, t, Z, acc, 1.0);
    store_y(b, z);
    if (last) finish(b, Z, acc, 2);
    r = rn;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      lp[q] = lpn[q];
      gt[q] = gtn[q];
    }
  }
}

// Gram back-sweeps at K = 64 (r < K), one workgroup per (partition, spike),
// all 64 spike columns:  z_b = U11^{-1} (Y_b - U12 z_{b+1}),  Gram += z_b^T z_b
// (V's forward result is zero above the last block).  Wave t forms row tile t
// of each product from its fragments of the records; the 64 x 64 operands
// live in LDS as 16 accumulator tiles (tile (u, c): rows 16u.., columns 16c..),
// and both the B operand of a product and the transposed A operand of the Gram
// are, lane for lane, element (step mod 4) of tile (step / 4, c).
struct P64 {
  static constexpr int TILE = 64 * 4, MAT = 16 * TILE;
  static constexpr int oT = 0, oZ = MAT, total = 2 * MAT;
};

__device__ __forceinline__ const double* p64_tile(const double* m, int u, int c) {
  return m + (size_t)(u * 4 + c) * P64::TILE;
}

// out[c] (+)= sign * A(row tile t) * M(:, column tile c) for the four column
// tiles; A's fragments fr[step] masked as in sw64_mul (kinds 2 and 3)
template <int KIND>
__device__ __forceinline__ void p64_mul(const double (&fr)[16], int t, const double* M, V64 (&out)[4], double sign) {
  const int lane = threadIdx.x & 63, i = 16 * t + (lane & 15);
#pragma unroll
  for (int step = 0; step < 16; ++step) {
    const int ct = step >> 2;
    if (KIND == 3 && ct > t) continue;
    if (KIND == 2 && ct < t) continue;
    const int kk = frag_k<double>(step, lane >> 4);
    double av = fr[step];
    if (KIND == 2) av = i <= kk ? av : 0.0;
    if (KIND == 3) av = i > kk ? av : 0.0;
    av *= sign;
#pragma unroll
    for (int c = 0; c < 4; ++c) out[c] = mfma_step(av, p64_tile(M, ct, c)[lane * 4 + (step & 3)], out[c]);
  }
}

__device__ __forceinline__ void p64_put(double* M, int t, const V64 (&x)[4]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int c = 0; c < 4; ++c) *reinterpret_cast<V64*>(M + (size_t)(t * 4 + c) * P64::TILE + lane * 4) = x[c];
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void pass2_64_kernel(FactorArgs a) {
  __shared__ __align__(16) double lds[P64::total];
  double* Tm = lds + P64::oT;
  double* Zm = lds + P64::oZ;
  const Layout& L = a.L;
  const int j = blockIdx.x, spike = blockIdx.y;
  const int t = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 15;
  const Geom g = part_geom(L, j, 64);
  const int nb = g.nb;
  const double* fac = wsp<double>(a.ws, L.fac) + (size_t)j * L.nbmax * L.rec;
  const double* ym = wsp<double>(a.ws, L.ymat) + (size_t)j * L.nbmax * 2 * 64 * 64;
  const int coff = spike == 0 ? 0 : 64;
  auto load_y = [&](int b, V64 (&y)[4]) {
    const bool nz = spike == 0 || b == nb - 1;
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        y[c][v] = nz ? ym[(size_t)b * 2 * 64 * 64 + (16 * t + acc_row<double>(lane, v)) * 128 + coff + 16 * c + col] : 0.0;
  };
  auto load_ud = [&](int b, V64& d) {
    const double* u = fac + (size_t)b * L.rec + 2 * 64 * 64;
#pragma unroll
    for (int v = 0; v < 4; ++v) d[v] = u[16 * t + acc_row<double>(lane, v)];
  };
  double up[16];
  V64 y[4], ud, zo[4], gr[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    gr[c] = V64{0, 0, 0, 0};
    zo[c] = V64{0, 0, 0, 0};
  }
  for (int b = nb - 1; b >= 0; --b) {
    // no prefetch: at two waves per SIMD (at most 256 registers, no spills)
    // the two workgroups of a CU hide each other's load latency
    sw64_frags(up, fac + (size_t)b * L.rec + 64 * 64, t);
    load_ud(b, ud);
    load_y(b, y);
    // Tm = Y_b - U12 z_{b+1}: strictly lower part of UP plus the diagonal UD
    if (b < nb - 1) {
      p64_mul<3>(up, t, Zm, y, -1.0);
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) y[c][v] -= ud[v] * zo[c][v];
    }
    p64_put(Tm, t, y);
    __syncthreads();
    // z_b = U11^{-1} Tm
#pragma unroll
    for (int c = 0; c < 4; ++c) zo[c] = V64{0, 0, 0, 0};
    p64_mul<2>(up, t, Tm, zo, 1.0);
    p64_put(Zm, t, zo);
    __syncthreads();
    // Gram row tile t += (z_b^T)(tile t) z_b
#pragma unroll
    for (int step = 0; step < 16; ++step) {
      const double av = p64_tile(Zm, step >> 2, t)[lane * 4 + (step & 3)];
#pragma unroll
      for (int c = 0; c < 4; ++c) gr[c] = mfma_step(av, p64_tile(Zm, step >> 2, c)[lane * 4 + (step & 3)], gr[c]);
    }
  }
  double* gram = wsp<double>(a.ws, L.gram) + ((size_t)j * 2 + (spike == 0 ? 1 : 0)) * 64 * 64;
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int v = 0; v < 4; ++v) gram[(16 * t + acc_row<double>(lane, v)) * 64 + 16 * c + col] = gr[c][v];
}

// ------------------------------------------------------------------ adjoint
// A_j^{-T} = L^{-T} U^{-T}: the transposed sweeps on fragments gathered
// transposed from the records (element (i, kk) of row tile t read at the
// stored position of (kk, i)).  kind 5: lower incl. diagonal of the gather
// ((U11^{-1})^T from UP, L21^T from LP), 7: strictly upper (U12^T from UP; its
// diagonal UD applies elementwise), 4: strictly upper with a unit diagonal
// ((L11^{-1})^T from LP).
__device__ __forceinline__ void sw64_tfrags(double (&fr)[16], const double* blk, int t) {
  const int lane = threadIdx.x & 63, i = 16 * t + (lane & 15);
#pragma unroll
  for (int step = 0; step < 16; ++step) fr[step] = blk[fidx<double, 64>(frag_k<double>(step, lane >> 4), i)];
}

template <int KIND>
__device__ __forceinline__ void sw64_tmul(const double (&fr)[16], int t, const V64 (&S)[4], V64& out, double sign) {
  const int lane = threadIdx.x & 63, i = 16 * t + (lane & 15);
#pragma unroll
  for (int step = 0; step < 16; ++step) {
    const int ct = step >> 2;
    if (KIND == 5 && ct > t) continue;
    if ((KIND == 7 || KIND == 4) && ct < t) continue;
    const int kk = frag_k<double>(step, lane >> 4);
    double a = fr[step];
    if (KIND == 5) a = i >= kk ? a : 0.0;
    if (KIND == 7) a = i < kk ? a : 0.0;
    if (KIND == 4) a = i < kk ? a : (i == kk ? 1.0 : 0.0);
    out = mfma_step(sign * a, S[ct][step & 3], out);
  }
}

// Transposed forward (U^T, top to bottom): W_b = U11^{-T} R_b, R_{b+1} -= U12^T W_b;
// W written to a.dst.
__device__ void sw64_tforward(const SolveArgs& a, const Geom& g, int j, int c0, int mc, double* lds,
                              const double* Ct, const double* Cb) {
  const Layout& L = a.L;
  const int t = threadIdx.x >> 6, lane = threadIdx.x & 63, nb = g.nb;
  const double* fac = wsp<double>(a.ws, L.fac) + (size_t)j * L.nbmax * L.rec;
  double up[16], upn[16];
  V64 ud, udn;
  auto load_ud = [&](int b, V64& d) {
    const double* u = fac + (size_t)b * L.rec + 2 * 64 * 64;
#pragma unroll
    for (int v = 0; v < 4; ++v) d[v] = u[16 * t + acc_row<double>(lane, v)];
  };
  sw64_tfrags(up, fac + 64 * 64, t);
  load_ud(0, ud);
  V64 r = sw64_rhs(a, g, 0, t, c0, mc, Ct, Cb), S[4], Wf[4];
  for (int b = 0; b < nb; ++b) {
    const bool last = b == nb - 1;
    const int bn = last ? b : b + 1;
    sw64_tfrags(upn, fac + (size_t)bn * L.rec + 64 * 64, t);
    load_ud(bn, udn);
    V64 rn = sw64_rhs(a, g, bn, t, c0, mc, Ct, Cb);
    sw64_exchange(lds + Sw64::oA, r, t, S);
    V64 w = V64{0, 0, 0, 0};
    sw64_tmul<5>(up, t, S, w, 1.0);
    sw64_exchange(lds + Sw64::oB, w, t, Wf);
    if (!last) {
      sw64_tmul<7>(up, t, Wf, rn, -1.0);
#pragma unroll
      for (int v = 0; v < 4; ++v) rn[v] -= ud[v] * w[v];
    }
    sw64_store(a, g, b, t, c0, mc, w);
    r = rn;
    ud = udn;
#pragma unroll
    for (int s2 = 0; s2 < 16; ++s2) up[s2] = upn[s2];
  }
}

// Transposed backward (L^T, bottom to top) over a.dst: u_b = L11^{-T}(W_b -
// L21^T u_{b+1}).  TIPS: u is not stored; its first and last K real rows go to
// the tip buffer.
template <bool TIPS>
__device__ void sw64_tbackward(const SolveArgs& a, const Geom& g, int j, int c0, int mc, double* lds) {
  const Layout& L = a.L;
  const int t = threadIdx.x >> 6, lane = threadIdx.x & 63, nb = g.nb;
  const double* fac = wsp<double>(a.ws, L.fac) + (size_t)j * L.nbmax * L.rec;
  double* yt = wsp<double>(a.ws, L.ytip) + (size_t)j * 2 * 64 * L.mmax;
  SolveArgs ad = a;
  ad.src = a.dst;
  double lp[16], lpn[16];
  sw64_tfrags(lp, fac + (size_t)(nb - 1) * L.rec, t);
  V64 zt = sw64_rhs(ad, g, nb - 1, t, c0, mc, nullptr, nullptr), U1[4], Zf[4];
  for (int q = 0; q < 4; ++q) U1[q] = V64{0, 0, 0, 0};
  for (int b = nb - 1; b >= 0; --b) {
    const int bn = b > 0 ? b - 1 : 0;
    sw64_tfrags(lpn, fac + (size_t)bn * L.rec, t);
    V64 ztn = sw64_rhs(ad, g, bn, t, c0, mc, nullptr, nullptr);
    if (b < nb - 1) sw64_tmul<5>(lp, t, U1, zt, -1.0);  // W_b - L21^T u_{b+1}
    sw64_exchange(lds + Sw64::oA, zt, t, Zf);
    V64 u = V64{0, 0, 0, 0};
    sw64_tmul<4>(lp, t, Zf, u, 1.0);
    if (TIPS) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int lr = b * 64 + 16 * t + acc_row<double>(lane, v) - g.pad, col = lane & 15;
        if (lr >= 0 && col < mc) {
          if (lr < 64) yt[(size_t)lr * L.mmax + c0 + col] = u[v];
          if (lr >= g.nj - 64) yt[(size_t)(64 + lr - (g.nj - 64)) * L.mmax + c0 + col] = u[v];
        }
      }
    } else {
      sw64_store(a, g, b, t, c0, mc, u);
    }
    sw64_exchange(lds + Sw64::oB, u, t, U1);
    zt = ztn;
#pragma unroll
    for (int s2 = 0; s2 < 16; ++s2) lp[s2] = lpn[s2];
  }
}

// Adjoint D-stage at K = 64: nu_j = A_j^{-T} g_j (W into a.dst), tips to the tip buffer.
__global__ __launch_bounds__(256) void adj_dstage64_kernel(SolveArgs a) {
  if (gated(a.gate)) return;
  __shared__ __align__(16) double lds[Sw64::total];
  const int j = blockIdx.x, c0 = blockIdx.y * 16, mc = min(16, a.m - c0);
  const Geom g = part_geom(a.L, j, 64);
  sw64_tforward(a, g, j, c0, mc, lds, nullptr, nullptr);
  __syncthreads();
  sw64_tbackward<true>(a, g, j, c0, mc, lds);
}

// Adjoint recovery at K = 64: lambda_j = A_j^{-T}(g_j - [w_{j,t}; 0; w_{j,b}]) in place,
//   w_{j,t} = B_{j-1}^T nu_{j-1,b} - Pi_{j-1} u_a(j-1)      (j >= 1)
//   w_{j,b} = C_{j+1}^T nu_{j+1,t} - Psi_{j+1} u_c(j+1)      (j <= p-2).
__global__ __launch_bounds__(256) void adj_retrieve64_kernel(SolveArgs a) {
  if (gated(a.gate)) return;
  __shared__ __align__(16) double lds[Sw64::total];
  const Layout& L = a.L;
  const int j = blockIdx.x, c0 = blockIdx.y * 16, mc = min(16, a.m - c0), k = L.k, r = L.r;
  const Geom g = part_geom(L, j, 64);
  double* Ct = lds + Sw64::oCt;
  double* Cb = lds + Sw64::oCb;
  const double* ytip = wsp<double>(a.ws, L.ytip);
  const double* proj = wsp<double>(a.ws, L.proj);
  const double* zg = wsp<double>(a.ws, L.zg);
  if (j > 0) {
    const double* nub = ytip + ((size_t)(j - 1) * 2 + 1) * 64 * L.mmax;
    const double* Pi = proj + (size_t)(j - 1) * 2 * 64 * r;
    const double* ua = zg + (size_t)(j - 1) * L.R2 * L.mmax;
    for (int o = threadIdx.x; o < 64 * mc; o += blockDim.x) {
      const int i = o / mc, c = o % mc;
      double s = 0.0;
      for (int l = 0; l < 64; ++l) s += band_at(a.bands, L.n, k, g.s - 64 + l, g.s + i) * nub[l * L.mmax + c0 + c];
      for (int q = 0; q < r; ++q) s -= Pi[i * r + q] * ua[q * L.mmax + c0 + c];
      Ct[i * 17 + c] = s;
    }
  }
  if (j < L.p - 1) {
    const double* nut = ytip + ((size_t)(j + 1) * 2 + 0) * 64 * L.mmax;
    const double* Psi = proj + ((size_t)(j + 1) * 2 + 1) * 64 * r;
    const double* uc = zg + ((size_t)j * L.R2 + r) * L.mmax;
    const int64_t s1 = g.s + g.nj;
    for (int o = threadIdx.x; o < 64 * mc; o += blockDim.x) {
      const int i = o / mc, c = o % mc;
      double s = 0.0;
      for (int l = 0; l < 64; ++l) s += band_at(a.bands, L.n, k, s1 + l, s1 - 64 + i) * nut[l * L.mmax + c0 + c];
      for (int q = 0; q < r; ++q) s -= Psi[i * r + q] * uc[q * L.mmax + c0 + c];
      Cb[i * 17 + c] = s;
    }
  }
  __syncthreads();
  sw64_tforward(a, g, j, c0, mc, lds, j > 0 ? Ct : nullptr, j < L.p - 1 ? Cb : nullptr);
  __syncthreads();
  sw64_tbackward<false>(a, g, j, c0, mc, lds);
}

}  // namespace lrs
