// BiCGStab outer iteration preconditioned by LR-SPIKE (the Krylov solver the
// paper pairs with its preconditioners; table solver-list and the BiCGStab
// experiments of section "Preconditioner Effectiveness using SuiteSparse
// Matrices").  Right preconditioning: the Krylov space is built for A M^{-1}
// and every vector update, inner product and residual is FP64, whatever the
// word size of the factors behind M^{-1}.  Each right-hand-side column runs
// its own iteration (own scalars, own convergence); a converged column is
// frozen.  One iteration:
//   rho = (rh, r);  beta = (rho / rho_old)(alpha / omega);
//   p = r + beta (p - omega v);  ph = M^{-1} p;  v = A ph;
//   alpha = rho / (rh, v);  s = r - alpha v;  sh = M^{-1} s;  t = A sh;
//   omega = (t, s) / (t, t);  x += alpha ph + omega sh;  r = s - omega t
// starting from x_0 = M^{-1} b, r_0 = rh = b - A x_0.  The scalars live on the
// device; a one-workgroup control kernel tests convergence (||r|| <= tol ||b||
// per column) and breakdown after every iteration and sets the gate that
// turns the remaining iterations into no-ops, so no host round trip is needed.
//
// Inner products are reduced deterministically: every workgroup of the vector
// kernels covers BICG_ROWS rows and writes one partial sum per (column, dot);
// bicg_reduce_kernel adds the partials of one (column, dot) in a fixed order.
#pragma once

namespace lrs {

#define BICG_TPB 256  // threads per workgroup of the vector kernels
enum BicgScalar {
  BS_RHO = 0, BS_RHO_OLD, BS_ALPHA, BS_OMEGA,  // recurrence scalars
  BS_RV, BS_TS, BS_TT, BS_RR, BS_BB, BS_RHO_NEXT,  // reduced inner products
  BS_DONE,  // 1.0 once the column converged
  BS_N = BICG_SCALARS
};

struct BicgArgs {
  int64_t n;
  int m, ld, nblk;
  double* sc;     // [mmax][BS_N]
  double* part;   // [nblk][mmax][3]
  const int* gate;
  int mmax;
};

__device__ __forceinline__ double* bsc(const BicgArgs& a, int c) { return a.sc + (size_t)c * BS_N; }
// alpha = rho / (rh, v) and omega = (t, s) / (t, t), 0 when the denominator
// vanishes (s = 0 gives t = 0: the column is then converged, not broken down)
__device__ __forceinline__ double bicg_alpha(const double* s) { return s[BS_RV] != 0.0 ? s[BS_RHO] / s[BS_RV] : 0.0; }
__device__ __forceinline__ double bicg_omega(const double* s) { return s[BS_TT] > 0.0 ? s[BS_TS] / s[BS_TT] : 0.0; }

// Thread t of the workgroup takes column t mod mc and every tp-th row of the
// workgroup's rows (tp = BICG_TPB / mc); threads t >= tp mc idle.  Partial
// sums of up to 3 inner products per column are added in LDS in a fixed order
// and written to part[blockIdx.x][c][0..2].
__device__ inline void bicg_partials(const BicgArgs& a, int mc, int ndots, const double (&v)[3]) {
  __shared__ double red[3][BICG_TPB];
  const int t = threadIdx.x, tp = BICG_TPB / mc;
  for (int q = 0; q < ndots; ++q) red[q][t] = (t < tp * mc) ? v[q] : 0.0;
  __syncthreads();
  if (t < mc) {
    for (int q = 0; q < ndots; ++q) {
      double s = 0.0;
      for (int u = 0; u < tp; ++u) s += red[q][t + u * mc];
      a.part[((size_t)blockIdx.x * a.mmax + t) * 3 + q] = s;
    }
  }
}

// rows of workgroup blockIdx.x: [r0, r1)
__device__ __forceinline__ void bicg_rows(const BicgArgs& a, int64_t& r0, int64_t& r1) {
  const int64_t per = (a.n + a.nblk - 1) / a.nblk;
  r0 = (int64_t)blockIdx.x * per;
  r1 = min(a.n, r0 + per);
}

// The vector kernels need m <= BICG_TPB columns (the plan checks it).
// Start: rh = r (r = b - A x_0 already in r), p = v = 0; partials (r, r), (b, b).
__global__ __launch_bounds__(BICG_TPB) void bicg_start_kernel(BicgArgs a, const double* b, const double* r,
                                                              double* rh, double* p, double* v) {
  if (a.gate && *a.gate) return;
  const int t = threadIdx.x, m = a.m, tp = BICG_TPB / m, c = t % m;
  int64_t r0, r1;
  bicg_rows(a, r0, r1);
  double acc[3] = {0.0, 0.0, 0.0};
  if (t < tp * m)
    for (int64_t i = r0 + t / m; i < r1; i += tp) {
      const size_t o = (size_t)i * a.ld + c;
      const double rv = r[o], bv = b[o];
      rh[o] = rv;
      p[o] = 0.0;
      v[o] = 0.0;
      acc[0] = fma(rv, rv, acc[0]);
      acc[1] = fma(bv, bv, acc[1]);
    }
  bicg_partials(a, m, 2, acc);
}

// p = r + beta (p - omega v) and ph = p (ph = 0 for converged columns).
__global__ __launch_bounds__(BICG_TPB) void bicg_p_kernel(BicgArgs a, const double* r, double* p, const double* v,
                                                          double* ph) {
  if (a.gate && *a.gate) return;
  const int t = threadIdx.x, m = a.m, tp = BICG_TPB / m, c = t % m;
  if (t >= tp * m) return;
  const double* s = bsc(a, c);
  const bool done = s[BS_DONE] != 0.0;
  const double beta = (s[BS_RHO] / s[BS_RHO_OLD]) * (s[BS_ALPHA] / s[BS_OMEGA]), om = s[BS_OMEGA];
  int64_t r0, r1;
  bicg_rows(a, r0, r1);
  for (int64_t i = r0 + t / m; i < r1; i += tp) {
    const size_t o = (size_t)i * a.ld + c;
    if (done) {
      ph[o] = 0.0;
      continue;
    }
    const double pn = fma(beta, fma(-om, v[o], p[o]), r[o]);
    p[o] = pn;
    ph[o] = pn;
  }
}

// s = r - alpha v, sh = s (0 for converged columns), alpha = rho / (rh, v).
__global__ __launch_bounds__(BICG_TPB) void bicg_s_kernel(BicgArgs a, const double* r, const double* v, double* s,
                                                          double* sh) {
  if (a.gate && *a.gate) return;
  const int t = threadIdx.x, m = a.m, tp = BICG_TPB / m, c = t % m;
  if (t >= tp * m) return;
  const double* sc = bsc(a, c);
  const bool done = sc[BS_DONE] != 0.0;
  const double alpha = bicg_alpha(sc);
  int64_t r0, r1;
  bicg_rows(a, r0, r1);
  for (int64_t i = r0 + t / m; i < r1; i += tp) {
    const size_t o = (size_t)i * a.ld + c;
    const double sv = done ? 0.0 : fma(-alpha, v[o], r[o]);
    s[o] = sv;
    sh[o] = sv;
  }
}

// x += alpha ph + omega sh, r = s - omega t; partials (rh, r), (r, r).
__global__ __launch_bounds__(BICG_TPB) void bicg_x_kernel(BicgArgs a, double* x, double* r, const double* rh,
                                                          const double* ph, const double* s, const double* sh,
                                                          const double* tv) {
  if (a.gate && *a.gate) return;
  const int t = threadIdx.x, m = a.m, tp = BICG_TPB / m, c = t % m;
  const double* sc = bsc(a, c < m ? c : 0);
  const bool done = sc[BS_DONE] != 0.0;
  const double alpha = bicg_alpha(sc), omega = bicg_omega(sc);
  int64_t r0, r1;
  bicg_rows(a, r0, r1);
  double acc[3] = {0.0, 0.0, 0.0};
  if (t < tp * m)
    for (int64_t i = r0 + t / m; i < r1; i += tp) {
      const size_t o = (size_t)i * a.ld + c;
      double rv = r[o];
      if (!done) {
        x[o] = fma(omega, sh[o], fma(alpha, ph[o], x[o]));
        rv = fma(-omega, tv[o], s[o]);
        r[o] = rv;
      }
      acc[0] = fma(rh[o], rv, acc[0]);
      acc[1] = fma(rv, rv, acc[1]);
    }
  bicg_partials(a, m, 2, acc);
}

// y = A x (or A^T x) over the workgroup's rows, with partial inner products:
// mode 1: (w1, y);  mode 2: (y, w1) and (y, y).  x is staged in LDS per tile
// of BICG_TPB rows with its k-row halo, the band entries are read once along
// each diagonal (coalesced), one thread per row.
#define BICG_MC 16
__global__ __launch_bounds__(BICG_TPB) void bicg_matvec_kernel(BicgArgs a, const double* __restrict__ bands, int k,
                                                               const double* __restrict__ x, double* __restrict__ y,
                                                               const double* __restrict__ w1, int mode, int transpose) {
  if (a.gate && *a.gate) return;
  extern __shared__ double xs[];  // (BICG_TPB + 2k) x PX
  constexpr int PX = BICG_MC + 1;
  const int t = threadIdx.x, m = a.m;
  const int64_t n = a.n;
  int64_t r0, r1;
  bicg_rows(a, r0, r1);
  // one column chunk at a time; the inner products of chunk columns go to the
  // partials of the threads that own them in the epilogue mapping
  for (int c0 = 0; c0 < m; c0 += BICG_MC) {
    const int mc = min(BICG_MC, m - c0);
    double dots[2] = {0.0, 0.0};
    for (int64_t i0 = r0; i0 < r1; i0 += BICG_TPB) {
      const int rows = BICG_TPB + 2 * k;
      __syncthreads();
      for (int o = t; o < rows * mc; o += BICG_TPB) {
        const int rr = o / mc, cc = o % mc;
        const int64_t gi = i0 - k + rr;
        xs[rr * PX + cc] = (gi >= 0 && gi < n) ? x[gi * a.ld + c0 + cc] : 0.0;
      }
      __syncthreads();
      double acc[BICG_MC];
#pragma unroll
      for (int cc = 0; cc < BICG_MC; ++cc) acc[cc] = 0.0;
      const int64_t i = i0 + t;
      if (i < r1) {
        constexpr int DG = 8;
        for (int d0 = -k; d0 <= k; d0 += DG) {
          double av[DG];
#pragma unroll
          for (int u = 0; u < DG; ++u) {
            const int d = min(d0 + u, k);
            const int64_t jj = min(max(i + d, (int64_t)0), n - 1);
            av[u] = transpose ? bands[(int64_t)(-d + k) * n + jj] : bands[(int64_t)(d + k) * n + i];
          }
#pragma unroll
          for (int u = 0; u < DG; ++u) {
            const int d = d0 + u;
            const int64_t jj = i + d;
            const double av2 = (d <= k && jj >= 0 && jj < n) ? av[u] : 0.0;
            const double* xr = xs + (t + min(d, k) + k) * PX;
#pragma unroll
            for (int cc = 0; cc < BICG_MC; ++cc) acc[cc] = fma(av2, xr[cc], acc[cc]);
          }
        }
      }
      __syncthreads();
#pragma unroll
      for (int cc = 0; cc < BICG_MC; ++cc) xs[t * PX + cc] = acc[cc];
      __syncthreads();
      // epilogue: thread t owns chunk column t mod mc (coalesced row-major stores)
      const int tpc = BICG_TPB / mc;
      if (t < tpc * mc) {
        const int cc = t % mc;
        for (int rr = t / mc; rr < BICG_TPB; rr += tpc) {
          const int64_t gi = i0 + rr;
          if (gi >= r1) break;
          const double yv = xs[rr * PX + cc];
          const size_t o = (size_t)gi * a.ld + c0 + cc;
          y[o] = yv;
          const double wv = w1[o];
          dots[0] = fma(wv, yv, dots[0]);
          if (mode == 2) dots[1] = fma(yv, yv, dots[1]);
        }
      }
    }
    // chunk partials: thread t (t < tpc mc) holds column c0 + t mod mc
    __shared__ double red[2][BICG_TPB];
    const int tpc = BICG_TPB / mc;
    __syncthreads();
    red[0][t] = (t < tpc * mc) ? dots[0] : 0.0;
    red[1][t] = (t < tpc * mc) ? dots[1] : 0.0;
    __syncthreads();
    if (t < mc) {
      for (int q = 0; q < (mode == 2 ? 2 : 1); ++q) {
        double s = 0.0;
        for (int u = 0; u < tpc; ++u) s += red[q][t + u * mc];
        a.part[((size_t)blockIdx.x * a.mmax + c0 + t) * 3 + q] = s;
      }
    }
  }
}

// sc[c][slot[q]] = sum over workgroups of part[.][c][q], q < ndots (one
// workgroup per column, fixed order).
__global__ __launch_bounds__(BICG_TPB) void bicg_reduce_kernel(BicgArgs a, int ndots, int s0, int s1, int s2) {
  if (a.gate && *a.gate) return;
  __shared__ double red[BICG_TPB];
  const int c = blockIdx.x, t = threadIdx.x;
  const int slots[3] = {s0, s1, s2};
  for (int q = 0; q < ndots; ++q) {
    double s = 0.0;
    for (int b = t; b < a.nblk; b += BICG_TPB) s += a.part[((size_t)b * a.mmax + c) * 3 + q];
    red[t] = s;
    __syncthreads();
    for (int w = BICG_TPB / 2; w > 0; w >>= 1) {
      if (t < w) red[t] += red[t + w];
      __syncthreads();
    }
    if (t == 0) bsc(a, c)[slots[q]] = red[0];
    __syncthreads();
  }
}

// After the start: rho = (r, r), rho_old = alpha = omega = 1; a column whose
// initial residual already meets the tolerance is done.
__global__ void bicg_init_kernel(BicgArgs a, int* st, double tol) {
  if (a.gate && *a.gate) return;
  const int c = threadIdx.x;
  if (c < a.m) {
    double* s = bsc(a, c);
    s[BS_RHO] = s[BS_RR];
    s[BS_RHO_OLD] = s[BS_ALPHA] = s[BS_OMEGA] = 1.0;
    s[BS_DONE] = (s[BS_RR] <= tol * tol * s[BS_BB]) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (c == 0) {
    bool all = true;
    for (int q = 0; q < a.m; ++q) all &= bsc(a, q)[BS_DONE] != 0.0;
    if (all) {
      st[S_RSTATE] = 1;
      st[S_STOP] = 1;
    }
  }
}

// End of iteration it: alpha and omega of this iteration are kept, rho moves
// to rho_old, the new (rh, r) becomes rho; a column converges when
// ||r|| <= tol ||b||.  A non-converged column whose rho, (rh, v), (t, t) or
// omega is zero has broken down (NOT_CONVERGED); a non-finite scalar latches
// NONFINITE; all columns converged stops the iteration (converged), the last
// allowed iteration without convergence latches NOT_CONVERGED.
__global__ void bicg_ctl_kernel(BicgArgs a, int* st, double tol, int it, int max_it) {
  if (st[S_STOP]) return;
  __shared__ int s_bad, s_nan, s_all;
  const int c = threadIdx.x;
  if (c == 0) {
    s_bad = 0;
    s_nan = 0;
    s_all = 1;
  }
  __syncthreads();
  if (c < a.m) {
    double* s = bsc(a, c);
    if (s[BS_DONE] == 0.0) {
      const double alpha = bicg_alpha(s), omega = bicg_omega(s);
      const double rho_new = s[BS_RHO_NEXT], rr = s[BS_RR];
      s[BS_ALPHA] = alpha;
      s[BS_OMEGA] = omega;
      s[BS_RHO_OLD] = s[BS_RHO];
      s[BS_RHO] = rho_new;
      if (!(isfinite(alpha) && isfinite(omega) && isfinite(rho_new) && isfinite(rr))) {
        atomicOr(&s_nan, 1);
      } else if (rr <= tol * tol * s[BS_BB]) {
        s[BS_DONE] = 1.0;
      } else {
        if (rho_new == 0.0 || omega == 0.0 || s[BS_RV] == 0.0) atomicOr(&s_bad, 1);
        atomicAnd(&s_all, 0);
      }
    }
  }
  __syncthreads();
  if (c != 0) return;
  st[S_ITERS] = it + 1;
  double worst = 0.0;
  for (int q = 0; q < a.m; ++q) {
    const double* s = bsc(a, q);
    worst = fmax(worst, s[BS_BB] > 0.0 ? sqrt(s[BS_RR] / s[BS_BB]) : 0.0);
  }
  *reinterpret_cast<double*>(st + S_CORR) = worst;  // largest relative residual
  int verdict = 0;
  if (s_nan) {
    verdict = 2;
    latch_error(st, 4, -1, -1);
  } else if (s_all) {
    verdict = 1;
  } else if (s_bad || it + 1 >= max_it) {
    verdict = 2;
    latch_error(st, 3, -1, -1);
  }
  if (verdict) {
    st[S_RSTATE] = verdict;
    st[S_STOP] = 1;
  }
}

}  // namespace lrs
