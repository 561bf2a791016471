// Iterative reduced solves (table solver-list):
//   LR-SPIKE-I    S~_red, the reduced system with the spikes' rank-r tips,
//   LR-SPIKE-OTF  S_red, the true reduced system (eq. spikered), multiplied
//                 on the fly (eqs. OTF-1/2): S_red x = x + the tips of
//                 A_j^{-1} [C_j x_{j-1,b}; 0; B_j x_{j+1,t}], one partition
//                 solve per product (the D-stage kernels on a right-hand side
//                 that is nonzero in the coupling rows only),
// both by BiCGStab (the recurrence of krylov.hip) right-preconditioned by
// S~~_red, the LR-SPIKE-T system: per interface i the 2 x 2 block
// [[I, V~_{i,b}], [W~_{i+1,t}, I]] inverted through its compressed form D_i
// (factored as for LR-SPIKE-T).  The vectors are interface tips in the tip
// buffer's layout: row (j * 2 + s) * K + a holds tip s (0 top, 1 bottom) of
// partition j, row stride mmax.  The solution tips then drive the recovery of
// eqs. recovery1/2 (the retrieval kernels with the compressed vector zeroed).
#pragma once
#include "common.h"
#include "layout.h"

namespace lrs {

struct IterArgs {
  const double* bands;
  char* ws;
  Layout L;
  int m;            // columns
  const int* gate;  // nonzero: the iteration has stopped, the kernel is a no-op
};

template <typename T>
__device__ inline T* itw(char* ws, size_t off) {
  return reinterpret_cast<T*>(ws + off);
}

constexpr int IT_MC = 16;  // columns per workgroup of the interface kernels

// x = S~~_red^{-1} g, in place allowed (x may equal g): interface i
// (blockIdx.x) owns the bottom tip of partition i and the top tip of
// partition i + 1:
//   [a_i; c_{i+1}] = D_i^{-1} [Pi_i^T g_{i+1,t}; Psi_{i+1}^T g_{i,b}],
//   x_{i,b} = g_{i,b} - P_{i,b} a_i,   x_{i+1,t} = g_{i+1,t} - Q_{i+1,t} c_{i+1};
// the outer tips x_{0,t}, x_{p-1,b} equal g's (copied by interface 0 and
// p - 2).  Grid (p - 1, column chunks); LDS 2 (K + 2r) IT_MC doubles.
template <int K>
__global__ __launch_bounds__(256) void iter_precond_kernel(IterArgs a, const double* g, double* x) {
  if (a.gate && *a.gate) return;
  extern __shared__ __align__(16) double ip_lds[];
  const Layout& L = a.L;
  const int i = blockIdx.x, c0 = blockIdx.y * IT_MC, mc = min(IT_MC, a.m - c0), r = L.r, R = L.R2, mm = L.mmax;
  const int tid = threadIdx.x;
  double* gb = ip_lds;           // K x IT_MC: g_{i,b}
  double* gt = gb + K * IT_MC;   // K x IT_MC: g_{i+1,t}
  double* zr = gt + K * IT_MC;   // R x IT_MC
  double* z = zr + R * IT_MC;    // R x IT_MC
  auto row = [&](int j, int s, int l) { return ((size_t)(j * 2 + s) * K + l) * mm + c0; };
  for (int o = tid; o < K * mc; o += blockDim.x) {
    const int l = o / mc, c = o % mc;
    gb[l * IT_MC + c] = g[row(i, 1, l) + c];
    gt[l * IT_MC + c] = g[row(i + 1, 0, l) + c];
  }
  // the outer tips
  if (i == 0)
    for (int o = tid; o < K * mc; o += blockDim.x) x[row(0, 0, o / mc) + o % mc] = g[row(0, 0, o / mc) + o % mc];
  if (i == L.p - 2)
    for (int o = tid; o < K * mc; o += blockDim.x)
      x[row(L.p - 1, 1, o / mc) + o % mc] = g[row(L.p - 1, 1, o / mc) + o % mc];
  __syncthreads();
  const double* proj = itw<double>(a.ws, L.proj);
  const double* Pi = proj + (size_t)i * 2 * K * r;
  const double* Psi = proj + ((size_t)(i + 1) * 2 + 1) * K * r;
  for (int o = tid; o < R * mc; o += blockDim.x) {
    const int q = o / mc, c = o % mc;
    double s = 0.0;
    if (q < r)
      for (int l = 0; l < K; ++l) s += Pi[l * r + q] * gt[l * IT_MC + c];
    else
      for (int l = 0; l < K; ++l) s += Psi[l * r + q - r] * gb[l * IT_MC + c];
    zr[q * IT_MC + c] = s;
  }
  __syncthreads();
  const double* Di = itw<double>(a.ws, L.zLU) + (size_t)i * R * R;  // D_i^{-1}, row-major
  for (int o = tid; o < R * mc; o += blockDim.x) {
    const int q = o / mc, c = o % mc;
    double s = 0.0;
    for (int u = 0; u < R; ++u) s += Di[q * R + u] * zr[u * IT_MC + c];
    z[q * IT_MC + c] = s;
  }
  __syncthreads();
  const double* ptip = itw<double>(a.ws, L.ptip);
  const double* Pb = ptip + ((size_t)i * 4 + 1) * K * r;        // P_{i,b}
  const double* Qt = ptip + ((size_t)(i + 1) * 4 + 2) * K * r;  // Q_{i+1,t}
  for (int o = tid; o < K * mc; o += blockDim.x) {
    const int l = o / mc, c = o % mc;
    double sb = gb[l * IT_MC + c], st = gt[l * IT_MC + c];
    for (int q = 0; q < r; ++q) {
      sb -= Pb[l * r + q] * z[q * IT_MC + c];
      st -= Qt[l * r + q] * z[(r + q) * IT_MC + c];
    }
    x[row(i, 1, l) + c] = sb;
    x[row(i + 1, 0, l) + c] = st;
  }
}

// y = S~_red x (LR-SPIKE-I): partition j (blockIdx.x)
//   a_j = Pi_j^T x_{j+1,t} (j < p-1),   c_j = Psi_j^T x_{j-1,b} (j > 0),
//   y_{j,t} = x_{j,t} + P_{j,t} a_j + Q_{j,t} c_j,  y_{j,b} = x_{j,b} + P_{j,b} a_j + Q_{j,b} c_j.
// Grid (p, column chunks); LDS 2 r IT_MC doubles.
template <int K>
__global__ __launch_bounds__(256) void iter_matvec_i_kernel(IterArgs a, const double* x, double* y) {
  if (a.gate && *a.gate) return;
  extern __shared__ __align__(16) double im_lds[];
  const Layout& L = a.L;
  const int j = blockIdx.x, c0 = blockIdx.y * IT_MC, mc = min(IT_MC, a.m - c0), r = L.r, mm = L.mmax;
  const int tid = threadIdx.x;
  double* av = im_lds;           // r x IT_MC
  double* cv = av + r * IT_MC;   // r x IT_MC
  auto row = [&](int jj, int s, int l) { return ((size_t)(jj * 2 + s) * K + l) * mm + c0; };
  const double* proj = itw<double>(a.ws, L.proj);
  const double* Pi = proj + (size_t)j * 2 * K * r;
  const double* Psi = proj + ((size_t)j * 2 + 1) * K * r;
  for (int o = tid; o < r * mc; o += blockDim.x) {
    const int q = o / mc, c = o % mc;
    double sa = 0.0, sc = 0.0;
    if (j < L.p - 1)
      for (int l = 0; l < K; ++l) sa += Pi[l * r + q] * x[row(j + 1, 0, l) + c];
    if (j > 0)
      for (int l = 0; l < K; ++l) sc += Psi[l * r + q] * x[row(j - 1, 1, l) + c];
    av[q * IT_MC + c] = sa;
    cv[q * IT_MC + c] = sc;
  }
  __syncthreads();
  const double* pt = itw<double>(a.ws, L.ptip) + (size_t)j * 4 * K * r;  // Pt Pb Qt Qb
  for (int o = tid; o < 2 * K * mc; o += blockDim.x) {
    const int s = o / (K * mc), e = o % (K * mc), l = e / mc, c = e % mc;
    const double* P = pt + (size_t)s * K * r;
    const double* Q = pt + (size_t)(2 + s) * K * r;
    double v = x[row(j, s, l) + c];
    for (int q = 0; q < r; ++q) v += P[l * r + q] * av[q * IT_MC + c] + Q[l * r + q] * cv[q * IT_MC + c];
    y[row(j, s, l) + c] = v;
  }
}

// LR-SPIKE-OTF product, first half: the right-hand side F (n x m, row stride
// ld) of the partition solves, zero except the first K rows of partition j,
// C_j x_{j-1,b}, and its last K rows, B_j x_{j+1,t} (K-padded couplings as in
// the retrieval).  Grid (p, row chunks of 64).
template <int K>
__global__ __launch_bounds__(256) void iter_otf_rhs_kernel(IterArgs a, const double* x, double* F, int ld) {
  if (a.gate && *a.gate) return;
  const Layout& L = a.L;
  const int j = blockIdx.x, m = a.m, k = L.k, mm = L.mmax;
  const Geom g = part_geom(L, j, K);
  auto row = [&](int jj, int s, int l) { return ((size_t)(jj * 2 + s) * K + l) * mm; };
  constexpr int ROWS = 64;
  for (int r0 = blockIdx.y * ROWS; r0 < g.nj; r0 += gridDim.y * ROWS)
    for (int o = threadIdx.x; o < ROWS * m; o += blockDim.x) {
      const int li = r0 + o / m, c = o % m;
      if (li >= g.nj) continue;
      const int64_t i = g.s + li;
      double v = 0.0;
      if (j > 0 && li < K)
        for (int l = 0; l < K; ++l) v += band_at(a.bands, L.n, k, i, g.s - K + l) * x[row(j - 1, 1, l) + c];
      if (j < L.p - 1 && li >= g.nj - K)
        for (int l = 0; l < K; ++l) v += band_at(a.bands, L.n, k, i, g.s + g.nj + l) * x[row(j + 1, 0, l) + c];
      F[i * ld + c] = v;
    }
}

// y = x + u (u null: y already holds the product) and the partial inner
// products of the BiCGStab step: mode 1: (w1, y); mode 2: (y, w1), (y, y).
// Flat over the tip vectors (ba.n rows).
__global__ __launch_bounds__(BICG_TPB) void iter_finish_kernel(BicgArgs a, const double* x, const double* u,
                                                               double* y, const double* w1, int mode) {
  if (a.gate && *a.gate) return;
  const int t = threadIdx.x, m = a.m, tp = BICG_TPB / m, c = t % m;
  int64_t r0, r1;
  bicg_rows(a, r0, r1);
  double acc[3] = {0.0, 0.0, 0.0};
  if (t < tp * m)
    for (int64_t i = r0 + t / m; i < r1; i += tp) {
      const size_t o = (size_t)i * a.ld + c;
      double yv = y[o];
      if (u) {
        yv = x[o] + u[o];
        y[o] = yv;
      }
      const double wv = w1[o];
      acc[0] = fma(wv, yv, acc[0]);
      acc[1] = fma(yv, yv, acc[1]);
    }
  bicg_partials(a, m, mode == 2 ? 2 : 1, acc);
}

// dst = src (flat over the tip vectors), or dst = b - dst when sub is set.
__global__ __launch_bounds__(BICG_TPB) void iter_copy_kernel(BicgArgs a, const double* src, double* dst, int sub) {
  if (a.gate && *a.gate) return;
  const int t = threadIdx.x, m = a.m, tp = BICG_TPB / m, c = t % m;
  if (t >= tp * m) return;
  int64_t r0, r1;
  bicg_rows(a, r0, r1);
  for (int64_t i = r0 + t / m; i < r1; i += tp) {
    const size_t o = (size_t)i * a.ld + c;
    dst[o] = sub ? src[o] - dst[o] : src[o];
  }
}

// The compressed vector set to zero, so that the retrieval's interface tips
// are the tip buffer itself.
__global__ void iter_zero_zg_kernel(double* zg, size_t count) {
  for (size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x; o < count; o += (size_t)gridDim.x * blockDim.x)
    zg[o] = 0.0;
}

}  // namespace lrs
