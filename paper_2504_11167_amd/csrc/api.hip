// C ABI of the LR-SPIKE library: argument checks, workspace layout, and the
// kernel sequences of the factorization, solve, adjoint solve and gradient.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/lrspike.h"
#include "layout.h"

namespace lrs {
struct FactorArgs;
struct SolveArgs;
struct RedArgs;
}  // namespace lrs

#include "factor.hip"
#include "reduced.hip"
#include "solve.hip"
#include "factor_wave.hip"
#include "factor_lds.hip"

using namespace lrs;

namespace {
struct BatchState;
}

struct lrspike_plan_s {
  Layout L;
  int precision;
  int max_refine;
  double refine_tol;
  hipStream_t stream;
  const double* bands;
  char* ws;
  int refine_iters;
  double last_corr;
  int last_error;
  // opt-in per-launch timing: an event pair around every kernel on the plan's stream
  int profiling;
  std::vector<std::pair<const char*, std::pair<hipEvent_t, hipEvent_t>>> prof;
  int wave = 1;                 // matrix-core wave sweeps for K >= 16 (else workgroup sweeps)
  BatchState* batch = nullptr;  // set for plans made by lrspike_factor_batched
};

// ------------------------------------------------------------------ dispatch tables
namespace {

__global__ void zero_kernel(int* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// x += d over `total` elements of an n x m row-major block, and the per-column
// squared norms of the new x and of d added into out[2c], out[2c+1].  When
// the grid stride is a multiple of m every thread stays in one column and
// accumulates in registers; otherwise each element goes to an LDS atomic.
__global__ void axpy_norms_kernel(double* x, const double* d, int64_t total, int m, double* out) {
  extern __shared__ double red[];  // 2m
  for (int c = threadIdx.x; c < 2 * m; c += blockDim.x) red[c] = 0.0;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const bool fixed = (stride % m) == 0;
  double sx = 0.0, sd = 0.0;
  int cfix = -1;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const double dv = d[e], xv = x[e] + dv;
    x[e] = xv;
    if (fixed) {
      sx = fma(xv, xv, sx);
      sd = fma(dv, dv, sd);
      cfix = (int)(e % m);
    } else {
      const int c = (int)(e % m);
      atomicAdd(&red[2 * c], xv * xv);
      atomicAdd(&red[2 * c + 1], dv * dv);
    }
  }
  if (cfix >= 0) {
    atomicAdd(&red[2 * cfix], sx);
    atomicAdd(&red[2 * cfix + 1], sd);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < 2 * m; c += blockDim.x)
    if (red[c] != 0.0) atomicAdd(out + c, red[c]);
}

__global__ void zero_d_kernel(double* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

template <typename T, int K>
size_t lds_p1() { return (size_t)P1Lds<K>::total * sizeof(T); }
template <typename T, int K>
size_t lds_p2() { return (size_t)P2Lds<K>::total * sizeof(T); }
template <typename T, int K>
size_t lds_sw() { return (size_t)SwLds<K>::total * sizeof(T); }

// Dynamic LDS above 64 KB needs the kernel attribute; each (kernel, size) is
// set once per process (so that no attribute call happens during a capture).
bool set_lds(const void* fn, size_t bytes) {
  if (bytes > 160 * 1024) return false;
  if (bytes <= 64 * 1024) return true;
  static std::vector<std::pair<const void*, size_t>> done;
  for (auto& e : done)
    if (e.first == fn && e.second >= bytes) return true;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return false;
  done.push_back({fn, bytes});
  return true;
}

#define LRS_CHECK_LAUNCH()                          \
  do {                                              \
    if (hipGetLastError() != hipSuccess) return LRSPIKE_ERR_HIP; \
  } while (0)

// Launch on the plan's stream; with profiling on, bracket it with an event pair.
template <typename... KArgs, typename... Args>
int launch(lrspike_plan P, const char* name, void (*kern)(KArgs...), dim3 grid, dim3 block, size_t lds,
           Args... args) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (P->profiling) {
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return LRSPIKE_ERR_HIP;
    if (hipEventRecord(e0, P->stream) != hipSuccess) return LRSPIKE_ERR_HIP;
  }
  hipLaunchKernelGGL(kern, grid, block, lds, P->stream, args...);
  if (hipGetLastError() != hipSuccess) return LRSPIKE_ERR_HIP;
  if (P->profiling) {
    if (hipEventRecord(e1, P->stream) != hipSuccess) return LRSPIKE_ERR_HIP;
    P->prof.push_back({name, {e0, e1}});
  }
  return 0;
}

#define LRS_LAUNCH(name, kern, grid, block, lds, ...)                     \
  do {                                                                    \
    int rc_ = launch(P, name, kern, grid, block, lds, __VA_ARGS__);       \
    if (rc_) return rc_;                                                  \
  } while (0)

template <typename T, int K>
int run_factor(lrspike_plan P) {
  const Layout& L = P->L;
  FactorArgs fa{P->bands, P->ws, L};
  size_t b1 = 0;
  if constexpr (K <= 32) {
    b1 = lds_p1<T, K>();
    if (!set_lds((const void*)factor_pass1<T, K>, b1)) return LRSPIKE_ERR_NOT_SUPPORTED;
  }
  if constexpr (K == 64) {
    // workgroup kernels with every block in LDS (no interchanges at this width)
    const size_t bf = (size_t)FLds<T, K>::total * sizeof(T), bs = (size_t)SLds<T, K>::total * sizeof(T);
    if (!set_lds((const void*)factor_lds_kernel<T, K>, bf) || !set_lds((const void*)spike_lds_kernel<T, K>, bs))
      return LRSPIKE_ERR_NOT_SUPPORTED;
    LRS_LAUNCH("factor_pass1", factor_lds_kernel<T, K>, dim3(L.p), dim3(LRS_NT), bf, fa);
    LRS_LAUNCH("spike_fwd", spike_lds_kernel<T, K>, dim3(L.p, 2, K / SLds<T, K>::MS), dim3(LRS_NT), bs, fa);
  } else if constexpr (K >= 16) {
    // one wave per partition without interchanges; partitions that need them
    // are flagged and refactored by the general kernel (a no-op elsewhere)
    LRS_LAUNCH("zero_kernel", zero_kernel, dim3((L.p + 255) / 256), dim3(256), 0,
               reinterpret_cast<int*>(P->ws + L.npv), L.p);
    const size_t bw = (size_t)FWave<T, K>::total * sizeof(T);
    if (!set_lds((const void*)factor_wave_kernel<T, K>, bw)) return LRSPIKE_ERR_NOT_SUPPORTED;
    LRS_LAUNCH("factor_pass1", factor_wave_kernel<T, K>, dim3(L.p), dim3(64), bw, fa);
    LRS_LAUNCH("spike_fwd", spike_wave_kernel<T, K>, dim3(L.p), dim3(64), 0, fa);
    fa.only_flagged = 1;
    LRS_LAUNCH("factor_pass1_pivoting", factor_pass1<T, K>, dim3(L.p), dim3(LRS_NT), b1, fa);
    fa.only_flagged = 0;
  } else {
    LRS_LAUNCH("factor_pass1", factor_pass1<T, K>, dim3(L.p), dim3(LRS_NT), b1, fa);
  }
  (void)b1;
  RedArgs ra{P->ws, L, 0, 0, 0};
  if (L.r < L.K) {
    if constexpr (K == 64) {
      const size_t b2 = (size_t)4 * K * (K + 1) * sizeof(T);
      if (!set_lds((const void*)pass2_lds_kernel<T, K>, b2)) return LRSPIKE_ERR_NOT_SUPPORTED;
      LRS_LAUNCH("factor_pass2", pass2_lds_kernel<T, K>, dim3(L.p, 2), dim3(LRS_NT), b2, fa);
    } else if constexpr (K >= 16) {
      LRS_LAUNCH("factor_pass2", pass2_wave_kernel<T, K>, dim3(L.p, 2), dim3(64), 0, fa);
    } else {
      size_t b2 = lds_p2<T, K>();
      if (!set_lds((const void*)factor_pass2<T, K>, b2)) return LRSPIKE_ERR_NOT_SUPPORTED;
      LRS_LAUNCH("factor_pass2", factor_pass2<T, K>, dim3(L.p), dim3(LRS_NT), b2, fa);
    }
    if (L.r > 0) {
      const size_t be = (size_t)2 * K * (K + 1) * 8;
      if (!set_lds((const void*)eigen_kernel<K>, be)) return LRSPIKE_ERR_NOT_SUPPORTED;
      LRS_LAUNCH("eigen_kernel", eigen_kernel<K>, dim3(L.p, 2), dim3(LRS_NT), be, ra);
      }
  } else {
    LRS_LAUNCH("identity_proj_kernel", identity_proj_kernel<K>, dim3(L.p), dim3(256), 0, ra);
  }
  if (L.r > 0) {
    LRS_LAUNCH("project_kernel", project_kernel<K>, dim3(L.p), dim3(256), 0, ra);
  }
  if (L.NI > 0 && L.r > 0) {
    LRS_LAUNCH("zassemble_kernel", zassemble_kernel<K>, dim3(L.NI), dim3(256), 0, ra);
    const int R2 = L.R2;
    const size_t bodd = (size_t)(R2 * (2 * R2 + 1) + 3 * R2) * 8, beven = (size_t)2 * R2 * (R2 + 1) * 8;
    if (!set_lds((const void*)cr_odd_kernel, bodd) || !set_lds((const void*)cr_even_kernel, beven))
      return LRSPIKE_ERR_NOT_SUPPORTED;
    for (int l = 0; l < L.levels; ++l) {
      int s = 1 << l;
      int nodd = (L.NI + s - 1) / (2 * s);  // rows (2q+1)s < NI
      ra.level = l;
      if (nodd > 0) LRS_LAUNCH("cr_odd_kernel", cr_odd_kernel, dim3(nodd), dim3(LRS_NT), bodd, ra);
      int neven = (L.NI + 2 * s - 1) / (2 * s);
      LRS_LAUNCH("cr_even_kernel", cr_even_kernel, dim3(neven), dim3(LRS_NT), beven, ra);
      }
    ra.level = L.levels;
    LRS_LAUNCH("cr_odd_kernel", cr_odd_kernel, dim3(1), dim3(LRS_NT), bodd, ra);
  }
  return 0;
}

// Reduced solve on the compressed vectors (Z or Z^T), in place in zg.
template <int K>
int run_reduced(lrspike_plan P, int m, int transpose) {
  const Layout& L = P->L;
  if (L.NI <= 0 || L.r <= 0) return 0;
  RedArgs ra{P->ws, L, 0, m, transpose};
  size_t bz = (size_t)4 * K * m * 8;
  if (!set_lds((const void*)zrhs_kernel<K>, bz)) return LRSPIKE_ERR_NOT_SUPPORTED;
  LRS_LAUNCH("zrhs_kernel", zrhs_kernel<K>, dim3(L.NI), dim3(256), bz, ra, P->bands);
  const int R2 = L.R2, mc = m < CRS_MC ? m : CRS_MC, nch = (m + CRS_MC - 1) / CRS_MC;
  const size_t bs = (size_t)(R2 * (R2 + 1) + R2 * (mc + 1) + R2 * mc) * 8;
  if (!set_lds((const void*)crs_forward_kernel, bs) || !set_lds((const void*)crs_backward_kernel, bs))
    return LRSPIKE_ERR_NOT_SUPPORTED;
  for (int l = 0; l < L.levels; ++l) {
    int s = 1 << l;
    ra.level = l;
    int neven = (L.NI + 2 * s - 1) / (2 * s);
    LRS_LAUNCH("crs_forward_kernel", crs_forward_kernel, dim3(neven, nch), dim3(LRS_NT), bs, ra);
  }
  ra.level = L.levels;
  LRS_LAUNCH("crs_backward_kernel", crs_backward_kernel, dim3(1, nch), dim3(LRS_NT), bs, ra);
  for (int l = L.levels - 1; l >= 0; --l) {
    int s = 1 << l;
    ra.level = l;
    int nodd = (L.NI + s - 1) / (2 * s);
    if (nodd > 0) LRS_LAUNCH("crs_backward_kernel", crs_backward_kernel, dim3(nodd, nch), dim3(LRS_NT), bs, ra);
  }
  return 0;
}

// One application of M_r^{-1} (transpose = 0) or M_r^{-T} (transpose = 1), in place.
template <typename T, int K>
int run_apply(lrspike_plan P, double* rhs, int m, int transpose) {
  const Layout& L = P->L;
  SolveArgs sa{P->bands, P->ws, L, rhs, rhs, m, m};
  dim3 grid(L.p, (m + mc_of<K>() - 1) / mc_of<K>());
  size_t bs = lds_sw<T, K>();
  int rc;
  if (!transpose && K >= 16 && K <= 32 && P->wave) {
    // matrix-core sweeps: one wave per partition and column chunk
    if constexpr (K >= 16 && K <= 32) {
      const bool one = m <= 16;
      dim3 gw(L.p, one ? 1 : (m + 31) / 32);
      const size_t bw = one ? (size_t)WaveSweep<T, K, 1>::total * sizeof(T) + 2 * K * sizeof(int)
                            : (size_t)WaveSweep<T, K, 2>::total * sizeof(T) + 2 * K * sizeof(int);
      if (L.p > 1) {
        if (one)
          LRS_LAUNCH("dstage_kernel", dstage_wave_kernel<T, K, 1>, gw, dim3(64), bw, sa);
        else
          LRS_LAUNCH("dstage_kernel", dstage_wave_kernel<T, K, 2>, gw, dim3(64), bw, sa);
        if ((rc = run_reduced<K>(P, m, 0))) return rc;
      }
      if (one)
        LRS_LAUNCH("retrieve_kernel", retrieve_wave_kernel<T, K, 1>, gw, dim3(64), bw, sa);
      else
        LRS_LAUNCH("retrieve_kernel", retrieve_wave_kernel<T, K, 2>, gw, dim3(64), bw, sa);
    }
  } else if (!transpose) {
    if (!set_lds((const void*)dstage_kernel<T, K>, bs) || !set_lds((const void*)retrieve_kernel<T, K>, bs))
      return LRSPIKE_ERR_NOT_SUPPORTED;
    if (L.p > 1) {
      LRS_LAUNCH("dstage_kernel", dstage_kernel<T, K>, grid, dim3(LRS_NT), bs, sa);
      if ((rc = run_reduced<K>(P, m, 0))) return rc;
    }
    LRS_LAUNCH("retrieve_kernel", retrieve_kernel<T, K>, grid, dim3(LRS_NT), bs, sa);
  } else {
    if (!set_lds((const void*)adj_dstage_kernel<T, K>, bs) || !set_lds((const void*)adj_retrieve_kernel<T, K>, bs))
      return LRSPIKE_ERR_NOT_SUPPORTED;
    if (L.p > 1) {
      SolveArgs sd = sa;
      sd.dst = reinterpret_cast<double*>(P->ws + L.scr);
      LRS_LAUNCH("adj_dstage_kernel", adj_dstage_kernel<T, K>, grid, dim3(LRS_NT), bs, sd);
        if ((rc = run_reduced<K>(P, m, 1))) return rc;
    }
    LRS_LAUNCH("adj_retrieve_kernel", adj_retrieve_kernel<T, K>, grid, dim3(LRS_NT), bs, sa);
  }
  return 0;
}

// Iterative refinement around run_apply (FP32 factors, FP64 residual/update).
template <typename T, int K>
int run_refined(lrspike_plan P, double* rhs, int m, int transpose) {
  const Layout& L = P->L;
  hipStream_t st = P->stream;
  const int64_t nm = L.n * (int64_t)m;
  double* fcopy = reinterpret_cast<double*>(P->ws + L.fcopy);
  double* scr = reinterpret_cast<double*>(P->ws + L.res);  // not the adjoint D-stage scratch
  double* norms = reinterpret_cast<double*>(P->ws + L.norms);
  if (hipMemcpyAsync(fcopy, rhs, nm * 8, hipMemcpyDeviceToDevice, st) != hipSuccess) return LRSPIKE_ERR_HIP;
  int rc = run_apply<T, K>(P, rhs, m, transpose);
  if (rc) return rc;
  std::vector<double> hn(2 * m);
  P->refine_iters = 0;
  P->last_corr = INFINITY;
  double prev = INFINITY;
  const size_t bres = (size_t)(RES_ROWS + 2 * L.k) * (RES_MC + 1) * 8;
  if (!set_lds((const void*)residual_kernel, bres)) return LRSPIKE_ERR_NOT_SUPPORTED;
  for (int it = 0; it < P->max_refine; ++it) {
    LRS_LAUNCH("residual_kernel", residual_kernel, dim3((unsigned)((L.n + RES_ROWS - 1) / RES_ROWS)), dim3(RES_ROWS),
               bres, P->bands, L.n, L.k, fcopy, rhs, scr, m, m, transpose);
    if ((rc = run_apply<T, K>(P, scr, m, transpose))) return rc;
    LRS_LAUNCH("zero_d_kernel", zero_d_kernel, dim3(1), dim3(256), 0, norms, 2 * m);
    LRS_LAUNCH("axpy_norms_kernel", axpy_norms_kernel, dim3(1024), dim3(256), (size_t)2 * m * 8, rhs, scr, nm, m,
               norms);
    if (hipMemcpyAsync(hn.data(), norms, 2 * m * 8, hipMemcpyDeviceToHost, st) != hipSuccess) return LRSPIKE_ERR_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return LRSPIKE_ERR_HIP;
    double worst = 0.0;
    for (int c = 0; c < m; ++c) {
      double rel = sqrt(hn[2 * c + 1]) / (sqrt(hn[2 * c]) > 0 ? sqrt(hn[2 * c]) : 1.0);
      if (!(rel == rel)) rel = INFINITY;
      if (rel > worst) worst = rel;
    }
    P->refine_iters = it + 1;
    P->last_corr = worst;
    if (worst <= P->refine_tol) return 0;
    if (!(worst < INFINITY)) break;
    // linear convergence: the error left after this update is about rho times
    // the correction, rho the contraction factor (ratio of successive
    // corrections; for the first one, its own relative size, i.e. the accuracy
    // of the FP32 solve), with a safety factor of 10
    const double rho = it == 0 ? worst : worst / prev;
    if (rho < 1e-2 && 10.0 * rho * worst <= P->refine_tol) return 0;
    if (it > 0 && worst > 0.5 * prev) {
      // the corrections stopped shrinking: the rounding level of an
      // ill-conditioned system when they are already small, else failure
      if (worst <= 100.0 * P->refine_tol) return 0;
      break;
    }
    prev = worst;
  }
  int* latch = reinterpret_cast<int*>(P->ws + L.latch);
  int code = LRSPIKE_ERR_NOT_CONVERGED;
  // latch from the host only if nothing is latched yet
  int cur = 0;
  if (hipMemcpy(&cur, latch, 4, hipMemcpyDeviceToHost) == hipSuccess && cur == 0) {
    int rec[2] = {code, -1};
    if (hipMemcpy(latch, rec, 8, hipMemcpyHostToDevice) != hipSuccess) return LRSPIKE_ERR_HIP;
  }
  return 0;
}

typedef int (*factor_fn)(lrspike_plan);
typedef int (*apply_fn)(lrspike_plan, double*, int, int);

template <typename T>
factor_fn pick_factor(int K) {
  switch (K) {
    case 1: return run_factor<T, 1>;
    case 2: return run_factor<T, 2>;
    case 4: return run_factor<T, 4>;
    case 8: return run_factor<T, 8>;
    case 16: return run_factor<T, 16>;
    case 32: return run_factor<T, 32>;
    case 64: return run_factor<T, 64>;
  }
  return nullptr;
}

template <typename T, bool REF>
apply_fn pick_apply(int K) {
  switch (K) {
    case 1: return REF ? run_refined<T, 1> : run_apply<T, 1>;
    case 2: return REF ? run_refined<T, 2> : run_apply<T, 2>;
    case 4: return REF ? run_refined<T, 4> : run_apply<T, 4>;
    case 8: return REF ? run_refined<T, 8> : run_apply<T, 8>;
    case 16: return REF ? run_refined<T, 16> : run_apply<T, 16>;
    case 32: return REF ? run_refined<T, 32> : run_apply<T, 32>;
    case 64: return REF ? run_refined<T, 64> : run_apply<T, 64>;
  }
  return nullptr;
}

void prof_clear(lrspike_plan P) {
  for (auto& e : P->prof) {
    (void)hipEventDestroy(e.second.first);
    (void)hipEventDestroy(e.second.second);
  }
  P->prof.clear();
}

#include "batched.hip"

bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeDevice;
}

}  // namespace

// ------------------------------------------------------------------ C ABI
extern "C" {

void lrspike_default_opts(lrspike_opts* o) {
  memset(o, 0, sizeof(*o));
  o->precision = LRSPIKE_FP64;
  o->max_refine = 30;
  o->refine_tol = 1e-13;
  o->max_nrhs = 32;
}

int lrspike_workspace_size(int64_t n, int32_t k, int32_t p, int32_t r, int32_t precision,
                           int32_t max_nrhs, size_t* bytes) {
  if (n < 1) return -1;
  if (k < 1) return -2;
  if (p < 1 || p > n) return -3;
  if (r < 0 || r > k) return -4;
  if (precision != LRSPIKE_FP64 && precision != LRSPIKE_FP32_REFINED) return -5;
  if (max_nrhs < 1) return -6;
  if (!bytes) return -7;
  Layout L;
  make_layout(L, n, k, p, r, precision == LRSPIKE_FP64 ? 8 : 4, max_nrhs);
  *bytes = L.total;
  return 0;
}

int lrspike_factor(int64_t n, int32_t k, const double* bands, int32_t p, int32_t r,
                   const lrspike_opts* opts, lrspike_plan* plan_out) {
  if (n < 1) return -1;
  if (k < 1) return -2;
  if (!is_device_ptr(bands)) return -3;
  if (p < 1 || p > n) return -4;
  if (r < 0 || r > k) return -5;
  if (!opts) return -6;
  if (!plan_out) return -7;
  const int K = kernel_K(k);
  int64_t njmin = n / p;
  if (p > 1 && njmin < 2 * (int64_t)k) return -4;
  if (njmin < K) return -4;
  if (opts->precision != LRSPIKE_FP64 && opts->precision != LRSPIKE_FP32_REFINED) return -6;
  if (opts->max_nrhs < 1) return -6;
  if (K > 64) return LRSPIKE_ERR_NOT_SUPPORTED;
  // reduced-system blocks of order 2r are inverted in one workgroup's LDS
  if (p > 1 && 2 * ((r == k) ? K : r) > 64) return LRSPIKE_ERR_NOT_SUPPORTED;
  lrspike_plan P = new lrspike_plan_s();
  make_layout(P->L, n, k, p, r, opts->precision == LRSPIKE_FP64 ? 8 : 4, opts->max_nrhs);
  if (!opts->workspace || opts->workspace_bytes < P->L.total || !is_device_ptr(opts->workspace)) {
    delete P;
    return LRSPIKE_ERR_WORKSPACE;
  }
  P->precision = opts->precision;
  P->max_refine = opts->max_refine > 0 ? opts->max_refine : 30;
  P->refine_tol = opts->refine_tol > 0 ? opts->refine_tol : 1e-13;
  P->stream = reinterpret_cast<hipStream_t>(opts->stream);
  P->bands = bands;
  P->ws = reinterpret_cast<char*>(opts->workspace);
  P->refine_iters = 0;
  P->last_corr = 0.0;
  P->profiling = opts->profile ? 1 : 0;
  LRS_LAUNCH("zero_kernel", zero_kernel, dim3(1), dim3(64), 0, reinterpret_cast<int*>(P->ws + P->L.latch), 16);
  factor_fn f = P->precision == LRSPIKE_FP64 ? pick_factor<double>(K) : pick_factor<float>(K);
  int rc = f ? f(P) : LRSPIKE_ERR_NOT_SUPPORTED;
  if (rc) {
    delete P;
    return rc;
  }
  *plan_out = P;
  return 0;
}

static int solve_common(lrspike_plan P, double* rhs, int32_t nrhs, int transpose) {
  if (!P || P->batch) return -1;
  if (!is_device_ptr(rhs)) return -2;
  if (nrhs < 1 || nrhs > P->L.mmax) return -3;
  apply_fn f;
  if (P->precision == LRSPIKE_FP64)
    f = pick_apply<double, false>(P->L.K);
  else
    f = pick_apply<float, true>(P->L.K);
  if (!f) return LRSPIKE_ERR_NOT_SUPPORTED;
  return f(P, rhs, nrhs, transpose);
}

int lrspike_solve(lrspike_plan plan, double* rhs, int32_t nrhs) { return solve_common(plan, rhs, nrhs, 0); }

int lrspike_solve_adjoint(lrspike_plan plan, double* rhs, int32_t nrhs) {
  return solve_common(plan, rhs, nrhs, 1);
}

int lrspike_band_grad(lrspike_plan P, const double* lam, const double* x, int32_t nrhs,
                      double* grad_bands) {
  if (!P || P->batch) return -1;
  if (!is_device_ptr(lam)) return -2;
  if (!is_device_ptr(x)) return -3;
  if (nrhs < 1) return -4;
  if (!is_device_ptr(grad_bands)) return -5;
  const Layout& L = P->L;
  dim3 grid((unsigned)((L.n + 255) / 256), 2 * L.k + 1);
  LRS_LAUNCH("band_grad_kernel", band_grad_kernel, grid, dim3(256), 0, L.n, L.k, lam, x, nrhs, nrhs, grad_bands);
  return hipGetLastError() == hipSuccess ? 0 : LRSPIKE_ERR_HIP;
}

int lrspike_status(lrspike_plan P, lrspike_info* info) {
  if (!P) return -1;
  if (P->batch) {
    // first latched error over the groups; partition reports the system index
    lrspike_info gi, out;
    memset(&out, 0, sizeof(out));
    out.partition = -1;
    out.row = -1;
    int first = 0;
    for (BatchGroup& G : P->batch->groups) {
      int rc = lrspike_status(G.plan, &gi);
      if (rc < 0 || rc == LRSPIKE_ERR_HIP) return rc;
      out.swapped_blocks += gi.swapped_blocks;
      out.refine_iters = std::max(out.refine_iters, gi.refine_iters);
      out.last_correction = std::max(out.last_correction, gi.last_correction);
      if (rc && !first) {
        first = rc;
        out.error = rc;
        out.partition = gi.partition >= 0 && gi.partition < (int)G.part_sys.size() ? G.part_sys[gi.partition] : -1;
        out.row = gi.row;
      }
    }
    if (info) *info = out;
    return first;
  }
  if (hipStreamSynchronize(P->stream) != hipSuccess) return LRSPIKE_ERR_HIP;
  int latch[16];
  if (hipMemcpy(latch, P->ws + P->L.latch, sizeof(latch), hipMemcpyDeviceToHost) != hipSuccess)
    return LRSPIKE_ERR_HIP;
  if (info) {
    info->error = latch[0];
    info->partition = latch[0] ? latch[1] : -1;
    int64_t row;
    memcpy(&row, latch + 2, 8);
    info->row = latch[0] ? row : -1;
    info->refine_iters = P->refine_iters;
    info->swapped_blocks = latch[8];
    info->last_correction = P->last_corr;
  }
  return latch[0];
}

int lrspike_profile(lrspike_plan P, int32_t enable) {
  if (!P || P->batch) return -1;
  P->profiling = enable ? 1 : 0;
  return 0;
}

int lrspike_profile_read(lrspike_plan P, int32_t max, char* names, double* total_ms, int32_t* launches,
                         int32_t* count) {
  if (!P || P->batch) return -1;
  if (max < 0) return -2;
  if (!count) return -6;
  if (hipStreamSynchronize(P->stream) != hipSuccess) return LRSPIKE_ERR_HIP;
  std::vector<const char*> keys;
  std::vector<double> ms;
  std::vector<int> cnt;
  for (auto& e : P->prof) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, e.second.first, e.second.second) != hipSuccess) return LRSPIKE_ERR_HIP;
    size_t i = 0;
    while (i < keys.size() && strcmp(keys[i], e.first) != 0) ++i;
    if (i == keys.size()) {
      keys.push_back(e.first);
      ms.push_back(0.0);
      cnt.push_back(0);
    }
    ms[i] += t;
    cnt[i] += 1;
  }
  prof_clear(P);
  *count = (int32_t)keys.size();
  for (int i = 0; i < (int)keys.size() && i < max; ++i) {
    if (names) {
      strncpy(names + 32 * i, keys[i], 31);
      names[32 * i + 31] = 0;
    }
    if (total_ms) total_ms[i] = ms[i];
    if (launches) launches[i] = cnt[i];
  }
  return 0;
}

int lrspike_destroy(lrspike_plan P) {
  if (P) {
    prof_clear(P);
    if (P->batch) {
      for (BatchGroup& G : P->batch->groups) free_group(G);
      if (P->batch->graph) (void)hipGraphExecDestroy(P->batch->graph);
      if (P->batch->capture) (void)hipStreamDestroy(P->batch->capture);
      delete P->batch;
    }
  }
  delete P;
  return 0;
}

int lrspike_factor_batched(int32_t count, const lrspike_batch_desc* descs, const double* bands_base,
                           const lrspike_opts* opts, lrspike_plan* plan_out) {
  if (count < 1) return -1;
  if (!descs) return -2;
  if (!is_device_ptr(bands_base)) return -3;
  if (!opts) return -4;
  if (!plan_out) return -5;
  if (opts->precision != LRSPIKE_FP64 && opts->precision != LRSPIKE_FP32_REFINED) return -4;
  for (int s = 0; s < count; ++s) {
    const lrspike_batch_desc& d = descs[s];
    if (d.n < 1 || d.k < 1 || d.r < 0 || d.r > d.k || d.nrhs < 1 || d.p < 0 || d.p > d.n || d.band_offset < 0 ||
        d.rhs_offset < 0)
      return -2;
    const int K = kernel_K(d.k);
    const int64_t minrows = std::max<int64_t>(2 * (int64_t)d.k, K);
    if ((d.p > 0 ? d.n / d.p : d.n) < minrows) return -2;
    if (K > 64 || 2 * ((d.r == d.k) ? K : d.r) > 64) return LRSPIKE_ERR_NOT_SUPPORTED;
  }
  lrspike_plan P = new lrspike_plan_s();
  P->batch = new BatchState();
  BatchState& B = *P->batch;
  B.descs.assign(descs, descs + count);
  B.bands_base = bands_base;
  B.precision = opts->precision;
  P->stream = reinterpret_cast<hipStream_t>(opts->stream);
  P->precision = opts->precision;
  // groups: equal (k, r) and padded right-hand-side count
  auto padded = [](int m) { return m <= 2 ? m : (m <= 4 ? 4 : (m + 7) / 8 * 8); };
  for (int s = 0; s < count; ++s) {
    const lrspike_batch_desc& d = descs[s];
    const int mb = padded(d.nrhs);
    size_t g = 0;
    while (g < B.groups.size() && !(B.groups[g].k == d.k && B.groups[g].r == d.r && B.groups[g].mb == mb)) ++g;
    if (g == B.groups.size()) {
      B.groups.emplace_back();
      B.groups.back().k = d.k;
      B.groups.back().r = d.r;
      B.groups.back().mb = mb;
    }
    B.groups[g].sys.push_back(s);
  }
  int rc = autotune(B, opts);
  if (!rc) rc = run_batched_eager(P, nullptr, true, false);
  if (rc) {
    lrspike_destroy(P);
    return rc;
  }
  *plan_out = P;
  return 0;
}

int lrspike_solve_batched(lrspike_plan P, double* rhs_base) {
  if (!P || !P->batch) return -1;
  if (!is_device_ptr(rhs_base)) return -2;
  return run_batched_eager(P, rhs_base, false, true);
}

int lrspike_run_batched(lrspike_plan P, double* rhs_base) {
  if (!P || !P->batch) return -1;
  if (!is_device_ptr(rhs_base)) return -2;
  BatchState& B = *P->batch;
  if (B.precision != LRSPIKE_FP64) return LRSPIKE_ERR_NOT_SUPPORTED;
  hipStream_t st = P->stream;
  if (B.graph && B.graph_rhs == rhs_base) return hipGraphLaunch(B.graph, st) == hipSuccess ? 0 : LRSPIKE_ERR_HIP;
  if (B.graph) {
    (void)hipGraphExecDestroy(B.graph);
    B.graph = nullptr;
  }
  // this call runs eagerly; the same sequence is then captured for the next calls
  int rc = run_batched_eager(P, rhs_base, true, true);
  if (rc) return rc;
  if (!B.capture && hipStreamCreateWithFlags(&B.capture, hipStreamNonBlocking) != hipSuccess) {
    B.capture = nullptr;
    return LRSPIKE_ERR_HIP;
  }
  if (hipStreamSynchronize(st) != hipSuccess) return LRSPIKE_ERR_HIP;
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(B.capture, hipStreamCaptureModeThreadLocal) != hipSuccess) return LRSPIKE_ERR_HIP;
  set_group_streams(B, B.capture);
  rc = run_batched_eager(P, rhs_base, true, true);
  set_group_streams(B, st);
  const hipError_t ce = hipStreamEndCapture(B.capture, &g);
  if (rc || ce != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return rc ? rc : LRSPIKE_ERR_HIP;
  }
  const hipError_t ie = hipGraphInstantiate(&B.graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) {
    B.graph = nullptr;
    return LRSPIKE_ERR_HIP;
  }
  B.graph_rhs = rhs_base;
  return 0;
}

int lrspike_batch_partitions(lrspike_plan P, int32_t count, int32_t* p_out) {
  if (!P || !P->batch) return -1;
  BatchState& B = *P->batch;
  if (count != (int32_t)B.descs.size()) return -2;
  if (!p_out) return -3;
  for (BatchGroup& G : B.groups)
    for (int s : G.sys) p_out[s] = sys_partitions(B.descs[s], G.target);
  return 0;
}

const char* lrspike_strerror(int code) {
  switch (code) {
    case 0: return "ok";
    case LRSPIKE_ERR_ZERO_PIVOT: return "zero pivot in a partition factorization";
    case LRSPIKE_ERR_REDUCED_SINGULAR: return "zero pivot in the reduced interface system";
    case LRSPIKE_ERR_NOT_CONVERGED: return "iterative refinement did not converge";
    case LRSPIKE_ERR_NONFINITE: return "non-finite value in the input or result";
    case LRSPIKE_ERR_HIP: return "HIP runtime error";
    case LRSPIKE_ERR_NOT_SUPPORTED: return "parameter combination not supported by this build";
    case LRSPIKE_ERR_WORKSPACE: return "workspace missing or too small";
  }
  if (code < 0) return "invalid argument";
  return "unknown error";
}

}  // extern "C"
