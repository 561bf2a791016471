// C ABI of the LR-SPIKE library: argument checks, workspace layout, and the
// kernel sequences of the factorization, solve, adjoint solve and gradient.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
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
#include "sweep64.hip"
#include "factor_wave.hip"
#include "factor_lds.hip"
#include "krylov.hip"
#include "rsvd.hip"
#include "iter.hip"

using namespace lrs;

namespace {
struct BatchState;
}

// Device scratch of the allocation-free entry point lrspike_solve_noalloc: a
// file-scope array, one copy per GPU, held until the process ends.  Host code
// never uses the name itself as an address: the address of the current
// device's copy comes from hipGetSymbolAddress (scratch_address below).
#define LRS_SCRATCH_BYTES ((size_t)64 << 20)
static __device__ __align__(256) char scratch[LRS_SCRATCH_BYTES];

struct lrspike_plan_s {
  Layout L;
  int precision;
  int max_refine;
  double refine_tol;
  hipStream_t stream;
  const double* bands;
  char* ws;
  int variant = 0;                // LRSPIKE_VARIANT_*
  int* hstate = nullptr;          // pinned host slots: refinement state copied back per correction
  hipEvent_t hev[2] = {nullptr, nullptr};
  // opt-in per-launch timing: an event pair around every kernel on the plan's stream
  int profiling;
  std::vector<std::pair<const char*, std::pair<hipEvent_t, hipEvent_t>>> prof;
  int wave = 1;                 // matrix-core wave sweeps for K >= 16 (else workgroup sweeps)
  const double* rsvd_omega = nullptr;  // randomized spike SVD: Gaussian test matrices (device, borrowed)
  int rsvd_power = 0;                  // its power steps
  BatchState* batch = nullptr;  // set for plans made by lrspike_factor_batched
};

// ------------------------------------------------------------------ dispatch tables
namespace {

__global__ void zero_kernel(int* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// State block at factor time: everything 0, the running minima +inf.
__global__ void state_init_kernel(int* st) {
  const int i = threadIdx.x;
  if (i < STATE_INTS) st[i] = 0;
  __syncthreads();
  if (i == 0) {
    const unsigned long long inf = 0x7FF0000000000000ull;
    *reinterpret_cast<unsigned long long*>(st + S_PIVMIN) = inf;
    *reinterpret_cast<unsigned long long*>(st + S_GAPMIN) = inf;
  }
}

// Start of a refined solve: control slots cleared, norms zeroed.
__global__ void refine_reset_kernel(int* st, double* norms, int nslots) {
  const int i = threadIdx.x;
  if (i == 0) {
    st[S_STOP] = 0;
    st[S_ITERS] = 0;
    st[S_RSTATE] = 0;
    *reinterpret_cast<double*>(st + S_CORR) = 0.0;
    *reinterpret_cast<double*>(st + S_CPREV) = 0.0;
  }
  for (int o = i; o < 2 * nslots; o += blockDim.x) norms[o] = 0.0;
}

// x += d on the rows of one partition (blockIdx.x) and chunk of REF_ROWS rows
// (blockIdx.y), and the squared norms of the new x and of d per (system slot
// of the partition, column) added into norms[(slot mmax + c) 2 + {0, 1}].
// When the block size is a multiple of m every thread stays in one column
// and accumulates in registers; otherwise each element goes to an LDS atomic.
#define REF_ROWS 2048
__global__ __launch_bounds__(256) void refine_update_kernel(double* x, const double* d, Layout L, int m,
                                                            double* norms, const int* gate) {
  if (gate && *gate) return;
  extern __shared__ double red[];  // 2m
  const int j = blockIdx.x;
  int64_t s0, nj;
  if (L.offs) {
    s0 = L.offs[j];
    nj = L.offs[j + 1] - s0;
  } else {
    const int64_t base = L.n / L.p, extra = L.n % L.p;
    nj = base + (j < extra ? 1 : 0);
    s0 = (int64_t)j * base + (j < extra ? j : extra);
  }
  const int64_t r0 = (int64_t)blockIdx.y * REF_ROWS;
  if (r0 >= nj) return;
  const int64_t rows = min((int64_t)REF_ROWS, nj - r0);
  for (int c = threadIdx.x; c < 2 * m; c += blockDim.x) red[c] = 0.0;
  __syncthreads();
  const bool fixed = (blockDim.x % m) == 0;
  const int64_t e0 = (s0 + r0) * m, total = rows * m;
  double sx = 0.0, sd = 0.0;
  for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
    const double dv = d[e0 + e], xv = x[e0 + e] + dv;
    x[e0 + e] = xv;
    if (fixed) {
      sx = fma(xv, xv, sx);
      sd = fma(dv, dv, sd);
    } else {
      const int c = (int)(e % m);
      atomicAdd(&red[2 * c], xv * xv);
      atomicAdd(&red[2 * c + 1], dv * dv);
    }
  }
  if (fixed && threadIdx.x < total) {
    const int c = (int)(threadIdx.x % m);
    atomicAdd(&red[2 * c], sx);
    atomicAdd(&red[2 * c + 1], sd);
  }
  __syncthreads();
  const int slot = L.psys ? L.psys[j] : 0;
  for (int c = threadIdx.x; c < 2 * m; c += blockDim.x)
    if (red[c] != 0.0) atomicAdd(norms + (size_t)slot * 2 * L.mmax + c, red[c]);
}

// Stopping rule of the refinement, on the device (no host round trip per
// correction).  With c_i = max over (system, column) of ||d|| / ||x|| for
// correction i: stop converged when c_i <= tol, or when the error left after
// the update, estimated by linear convergence as 10 rho c_i, is <= tol
// (rho = c_i / c_{i-1}, or c_0 itself for the first correction, trusted only
// below 1e-2); a correction that shrinks by less than half stops the
// iteration, converged if c_i <= 100 tol (the rounding level of an
// ill-conditioned system), else NOT_CONVERGED; a non-finite correction
// latches NONFINITE; the last allowed correction without convergence latches
// NOT_CONVERGED.  A stop sets the gate that turns the later corrections into
// no-ops.  The norms are cleared for the next correction.
__global__ void refine_ctl_kernel(int* st, double* norms, int nsys, int m, int mmax, double tol, int it,
                                  int max_it) {
  if (st[S_STOP]) return;
  const int lane = threadIdx.x;  // one wave
  double worst = 0.0;
  bool bad = false;
  for (int o = lane; o < nsys * m; o += 64) {
    const int sy = o / m, c = o % m;
    const double nx = sqrt(norms[((size_t)sy * mmax + c) * 2]), nd = sqrt(norms[((size_t)sy * mmax + c) * 2 + 1]);
    double rel = nd == 0.0 ? 0.0 : nd / (nx > 0.0 ? nx : 1.0);
    bad |= !(rel <= 1.7976931348623157e308);
    worst = fmax(worst, rel);
  }
  worst = wave_max(worst);
  bad = __any(bad);
  __syncthreads();
  for (int o = lane; o < 2 * nsys * mmax; o += 64) norms[o] = 0.0;
  if (lane != 0) return;
  double* corr = reinterpret_cast<double*>(st + S_CORR);
  double* cprev = reinterpret_cast<double*>(st + S_CPREV);
  const double prev = *corr;
  *cprev = prev;
  *corr = bad ? INFINITY : worst;
  st[S_ITERS] = it + 1;
  int verdict = 0;  // 1 converged, 2 failed
  if (bad) {
    verdict = 2;
    latch_error(st, 4, -1, -1);
  } else if (worst <= tol) {
    verdict = 1;
  } else {
    const double rho = it == 0 ? worst : worst / prev;
    if (rho < 1e-2 && 10.0 * rho * worst <= tol)
      verdict = 1;
    else if (it > 0 && worst > 0.5 * prev)
      verdict = worst <= 100.0 * tol ? 1 : 2;
    else if (it + 1 >= max_it)
      verdict = 2;
    if (verdict == 2) latch_error(st, 3, -1, -1);
  }
  if (verdict) {
    st[S_RSTATE] = verdict;
    st[S_STOP] = 1;
  }
}

template <typename T, int K>
size_t lds_p1() { return (size_t)P1Lds<K>::total * sizeof(T); }
template <typename T, int K>
size_t lds_p2() { return (size_t)P2Lds<K>::total * sizeof(T); }
template <typename T, int K>
size_t lds_sw() { return (size_t)SwLds<K>::total * sizeof(T); }

// Dynamic LDS above 64 KB needs the kernel attribute; each (kernel, size) is
// set once per process (so that no attribute call happens during a capture).
// (A fixed table, so that no call path allocates host memory for it.)
bool set_lds(const void* fn, size_t bytes) {
  if (bytes > 160 * 1024) return false;
  if (bytes <= 64 * 1024) return true;
  struct Done {
    const void* fn;
    size_t bytes;
  };
  static Done done[512];
  static int ndone = 0;
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  for (int i = 0; i < ndone; ++i)
    if (done[i].fn == fn && done[i].bytes >= bytes) return true;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return false;
  if (ndone < 512) done[ndone++] = {fn, bytes};
  return true;
}

#define LRS_CHECK_LAUNCH()                          \
  do {                                              \
    if (hipGetLastError() != hipSuccess) return LRSPIKE_ERR_HIP; \
  } while (0)

// Timing events are recycled through a process-wide pool, so that a profiled
// launch only records two events (no event creation inside a timed region).
std::vector<hipEvent_t>& event_pool() {
  static std::vector<hipEvent_t> pool;
  return pool;
}
hipEvent_t event_get() {
  auto& pool = event_pool();
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}
void event_put(hipEvent_t e) { event_pool().push_back(e); }

// Launch on the plan's stream; with profiling on, bracket it with an event pair.
template <typename... KArgs, typename... Args>
int launch(lrspike_plan P, const char* name, void (*kern)(KArgs...), dim3 grid, dim3 block, size_t lds,
           Args... args) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (P->profiling) {
    if (!(e0 = event_get()) || !(e1 = event_get())) return LRSPIKE_ERR_HIP;
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

// Randomized spike SVD (kernels in rsvd.hip): q + 1 sketch passes, each a
// block-diagonal solve of the sketch right-hand side followed by an adjoint
// solve of which only the tips are kept; the last pass also forms the sketch
// Gram.  The sweeps are the plan's own solve kernels (matrix-core waves for
// K = 16, 32, with the workgroup kernels for partitions factored with
// interchanges; workgroup kernels otherwise), run on the n x 2 ell sketch.
template <typename T, int K>
int run_rsvd(lrspike_plan P) {
  const Layout& L = P->L;
  const int w = 2 * L.ell;
  RsvdArgs ra{P->bands, P->ws, L, P->rsvd_omega};
  double* Y = reinterpret_cast<double*>(P->ws + L.ysk);
  double* scr = reinterpret_cast<double*>(P->ws + L.scr);
  SolveArgs sa{P->bands, P->ws, L, Y, Y, w, w, nullptr};
  sa.block_only = 1;
  const size_t bs = lds_sw<T, K>();
  if (!set_lds((const void*)retrieve_kernel<T, K>, bs) || !set_lds((const void*)adj_dstage_kernel<T, K>, bs))
    return LRSPIKE_ERR_NOT_SUPPORTED;
  const bool rows31 = (int64_t)L.nbmax * L.K * w * 8 < ((int64_t)1 << 31);
  const bool wv = K >= 16 && K <= 32 && P->wave && rows31;
  const dim3 grid(L.p, (w + mc_of<K>() - 1) / mc_of<K>()), gw(L.p, (w + 15) / 16);
  const dim3 grhs(L.p, (unsigned)std::min<int64_t>(64, ((int64_t)L.nbmax * K + 63) / 64));
  for (int it = 0; it <= P->rsvd_power; ++it) {
    LRS_LAUNCH("rsvd_rhs_kernel", rsvd_rhs_kernel, grhs, dim3(256), 0, ra);
    // Y = A_j^{-1} (sketch right-hand side), in place
    if (wv) {
      if constexpr (K >= 16 && K <= 32) {
        const size_t bw = (size_t)WaveSweep<T, K, 1>::total * sizeof(T) + 2 * K * sizeof(int);
        LRS_LAUNCH("rsvd_solve", retrieve_wave_kernel<T, K, 1>, gw, dim3(64), bw, sa);
      }
    } else if (K == 64 && std::is_same<T, double>::value && P->wave) {
      LRS_LAUNCH("rsvd_solve", retrieve64_kernel, dim3(L.p, (w + 15) / 16), dim3(256), 0, sa);
    } else {
      LRS_LAUNCH("rsvd_solve", retrieve_kernel<T, K>, grid, dim3(LRS_NT), bs, sa);
    }
    if (it == P->rsvd_power) LRS_LAUNCH("rsvd_gram_kernel", rsvd_gram_kernel, dim3(L.p, 2), dim3(256), 0, ra);
    // tips of A_j^{-T} Y (the full result goes to the scratch)
    SolveArgs sd = sa, sdf = sa;
    sd.dst = sdf.dst = scr;
    sd.block_only = sdf.block_only = 0;
    sdf.only_flagged = 1;
    if (wv) {
      if constexpr (K >= 16 && K <= 32) {
        LRS_LAUNCH("rsvd_adjoint", adj_dstage_wave_kernel<T, K>, gw, dim3(64), 0, sd);
        LRS_LAUNCH("rsvd_adjoint_pivoting", adj_dstage_kernel<T, K>, grid, dim3(LRS_NT), bs, sdf);
      }
    } else if (K == 64 && std::is_same<T, double>::value && P->wave) {
      LRS_LAUNCH("rsvd_adjoint", adj_dstage64_kernel, dim3(L.p, (w + 15) / 16), dim3(256), 0, sd);
    } else {
      LRS_LAUNCH("rsvd_adjoint", adj_dstage_kernel<T, K>, grid, dim3(LRS_NT), bs, sd);
    }
    LRS_LAUNCH("rsvd_vty_kernel", rsvd_vty_kernel, dim3(L.p, 2), dim3(256), 0, ra);
    ra.om = reinterpret_cast<const double*>(P->ws + L.rmv);  // a power step sketches with V^T Y
  }
  const size_t bsm = rsvd_small_lds(L.ell, L.k);
  if (!set_lds((const void*)rsvd_small_kernel, bsm)) return LRSPIKE_ERR_NOT_SUPPORTED;
  LRS_LAUNCH("rsvd_small_kernel", rsvd_small_kernel, dim3(L.p, 2), dim3(256), bsm, ra);
  return 0;
}

// The randomized truncation's small eigenproblem: R_h R_h^T of order KE (a
// power of two <= 64) per (partition, spike), eigenvectors written at re.L.proj.
template <int KE>
static int eigen_small_t(lrspike_plan P, const RedArgs& re) {
  const size_t be = (size_t)2 * KE * (KE + 1) * 8;
  if (!set_lds((const void*)eigen_kernel<KE>, be)) return LRSPIKE_ERR_NOT_SUPPORTED;
  LRS_LAUNCH("eigen_kernel", eigen_kernel<KE>, dim3(P->L.p, 2), dim3(LRS_NT), be, re);
  return 0;
}
static int eigen_small(lrspike_plan P, int KE, const RedArgs& re) {
  switch (KE) {
    case 1: return eigen_small_t<1>(P, re);
    case 2: return eigen_small_t<2>(P, re);
    case 4: return eigen_small_t<4>(P, re);
    case 8: return eigen_small_t<8>(P, re);
    case 16: return eigen_small_t<16>(P, re);
    case 32: return eigen_small_t<32>(P, re);
    case 64: return eigen_small_t<64>(P, re);
    default: return LRSPIKE_ERR_NOT_SUPPORTED;
  }
}

template <typename T, int K>
int run_factor(lrspike_plan P) {
  const Layout& L = P->L;
  FactorArgs fa{P->bands, P->ws, L};
  const bool rsvd = L.ell > 0 && L.r < L.K && L.p > 1;
  int rc;
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
    if (!rsvd) {
      if constexpr (std::is_same<T, double>::value)
        LRS_LAUNCH("spike_fwd", spike64_kernel, dim3(L.p, 4, 2), dim3(256), 0, fa);
      else
        LRS_LAUNCH("spike_fwd", spike_lds_kernel<T, K>, dim3(L.p, 2, K / SLds<T, K>::MS), dim3(LRS_NT), bs, fa);
    }
  } else if constexpr (K >= 16) {
    // one wave per partition without interchanges; partitions that need them
    // are flagged and refactored by the general kernel (a no-op elsewhere)
    LRS_LAUNCH("zero_kernel", zero_kernel, dim3((L.p + 255) / 256), dim3(256), 0,
               reinterpret_cast<int*>(P->ws + L.npv), L.p);
    const size_t bw = (size_t)FWave<T, K>::total * sizeof(T);
    if (!set_lds((const void*)factor_wave_kernel<T, K>, bw)) return LRSPIKE_ERR_NOT_SUPPORTED;
    LRS_LAUNCH("factor_pass1", factor_wave_kernel<T, K>, dim3(L.p), dim3(64), bw, fa);
    if (!rsvd) LRS_LAUNCH("spike_fwd", spike_wave_kernel<T, K>, dim3(L.p), dim3(64), 0, fa);
    fa.only_flagged = 1;
    LRS_LAUNCH("factor_pass1_pivoting", factor_pass1<T, K>, dim3(L.p), dim3(LRS_NT), b1, fa);
    fa.only_flagged = 0;
  } else {
    LRS_LAUNCH("factor_pass1", factor_pass1<T, K>, dim3(L.p), dim3(LRS_NT), b1, fa);
  }
  (void)b1;
  RedArgs ra{P->ws, L, 0, 0, 0};
  if (L.r < L.K && rsvd) {
    // randomized SVD: Grams and tips of the sketched spikes Q Q^T V
    if ((rc = run_rsvd<T, K>(P))) return rc;
  } else if (L.r < L.K) {
    if constexpr (K == 64 && std::is_same<T, double>::value) {
      LRS_LAUNCH("factor_pass2", pass2_64_kernel, dim3(L.p, 2), dim3(256), 0, fa);
    } else if constexpr (K == 64) {
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
  }
  if (L.r < L.K) {
    if (L.r > 0 && rsvd) {
      // eigenvectors W of R_h R_h^T over the sketch (no longer needed), then Pi = Q_b W
      RedArgs re = ra;
      re.L.proj = L.ysk;
      if ((rc = eigen_small(P, rsvd_ke(L.ell), re))) return rc;
      RsvdArgs rl{P->bands, P->ws, L, nullptr};
      LRS_LAUNCH("rsvd_lift_kernel", rsvd_lift_kernel, dim3(L.p, 2), dim3(256), 0, rl,
                 reinterpret_cast<const double*>(P->ws + L.ysk));
    } else if (L.r > 0) {
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
    if (L.variant) {
      // LR-SPIKE-T: the interface blocks are independent, each inverted on its own
      ra.level = -1;
      LRS_LAUNCH("cr_odd_kernel", cr_odd_kernel, dim3(L.NI), dim3(LRS_NT), bodd, ra);
      return 0;
    }
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
int run_reduced(lrspike_plan P, int m, int transpose, const int* gate) {
  const Layout& L = P->L;
  if (L.NI <= 0 || L.r <= 0) return 0;
  RedArgs ra{P->ws, L, 0, m, transpose, gate};
  size_t bz = (size_t)4 * K * m * 8;
  if (!set_lds((const void*)zrhs_kernel<K>, bz)) return LRSPIKE_ERR_NOT_SUPPORTED;
  LRS_LAUNCH("zrhs_kernel", zrhs_kernel<K>, dim3(L.NI), dim3(256), bz, ra, P->bands);
  const int R2 = L.R2, mc = m < CRS_MC ? m : CRS_MC, nch = (m + CRS_MC - 1) / CRS_MC;
  const size_t bs = (size_t)(R2 * (R2 + 1) + R2 * (mc + 1) + R2 * mc) * 8;
  if (!set_lds((const void*)crs_forward_kernel, bs) || !set_lds((const void*)crs_backward_kernel, bs))
    return LRSPIKE_ERR_NOT_SUPPORTED;
  if (L.variant) {  // LR-SPIKE-T: z_i = D_i^{-1} g_i (or D_i^{-T} g_i) for every interface at once
    ra.level = -1;
    LRS_LAUNCH("crs_backward_kernel", crs_backward_kernel, dim3(L.NI, nch), dim3(LRS_NT), bs, ra);
    return 0;
  }
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
// gate: refinement gate (null outside refinement), see refine_ctl_kernel.
template <typename T, int K>
int run_apply(lrspike_plan P, double* rhs, int m, int transpose, const int* gate = nullptr) {
  const Layout& L = P->L;
  SolveArgs sa{P->bands, P->ws, L, rhs, rhs, m, m, gate};
  dim3 grid(L.p, (m + mc_of<K>() - 1) / mc_of<K>());
  size_t bs = lds_sw<T, K>();
  int rc;
  // (the matrix-core sweeps address a partition's rows with 32-bit byte offsets)
  const bool rows31 = (int64_t)L.nbmax * L.K * m * 8 < ((int64_t)1 << 31);
  if (!transpose && K >= 16 && K <= 32 && P->wave && rows31) {
    // matrix-core sweeps: one wave per partition and chunk of 16 columns (one
    // accumulator tile wide, which leaves the registers for the prefetch ring)
    if constexpr (K >= 16 && K <= 32) {
      dim3 gw(L.p, (m + 15) / 16);
      const size_t bw = (size_t)WaveSweep<T, K, 1>::total * sizeof(T) + 2 * K * sizeof(int);
      if (L.p > 1) {
        LRS_LAUNCH("dstage_kernel", dstage_wave_kernel<T, K, 1>, gw, dim3(64), bw, sa);
        if ((rc = run_reduced<K>(P, m, 0, gate))) return rc;
      }
      LRS_LAUNCH("retrieve_kernel", retrieve_wave_kernel<T, K, 1>, gw, dim3(64), bw, sa);
    }
  } else if (!transpose && K == 64 && std::is_same<T, double>::value && P->wave) {
    // K = 64 on the matrix cores: four waves per (partition, 16 columns)
    const dim3 g64(L.p, (m + 15) / 16);
    if (L.p > 1) {
      LRS_LAUNCH("dstage_kernel", dstage64_kernel, g64, dim3(256), 0, sa);
      if ((rc = run_reduced<K>(P, m, 0, gate))) return rc;
    }
    LRS_LAUNCH("retrieve_kernel", retrieve64_kernel, g64, dim3(256), 0, sa);
  } else if (!transpose) {
    if (!set_lds((const void*)dstage_kernel<T, K>, bs) || !set_lds((const void*)retrieve_kernel<T, K>, bs))
      return LRSPIKE_ERR_NOT_SUPPORTED;
    if (L.p > 1) {
      LRS_LAUNCH("dstage_kernel", dstage_kernel<T, K>, grid, dim3(LRS_NT), bs, sa);
      if ((rc = run_reduced<K>(P, m, 0, gate))) return rc;
    }
    LRS_LAUNCH("retrieve_kernel", retrieve_kernel<T, K>, grid, dim3(LRS_NT), bs, sa);
  } else if (K >= 16 && K <= 32 && P->wave && rows31) {
    // adjoint on the matrix cores for the partitions factored without
    // interchanges; the workgroup kernels take the others
    if constexpr (K >= 16 && K <= 32) {
      if (!set_lds((const void*)adj_dstage_kernel<T, K>, bs) || !set_lds((const void*)adj_retrieve_kernel<T, K>, bs))
        return LRSPIKE_ERR_NOT_SUPPORTED;
      dim3 gw(L.p, (m + 15) / 16);
      const size_t bw = (size_t)WaveSweep<T, K, 1>::total * sizeof(T);
      SolveArgs sf = sa;
      sf.only_flagged = 1;
      if (L.p > 1) {
        SolveArgs sd = sa, sdf = sf;
        sd.dst = sdf.dst = reinterpret_cast<double*>(P->ws + L.scr);
        LRS_LAUNCH("adj_dstage_kernel", adj_dstage_wave_kernel<T, K>, gw, dim3(64), 0, sd);
        LRS_LAUNCH("adj_dstage_pivoting", adj_dstage_kernel<T, K>, grid, dim3(LRS_NT), bs, sdf);
        if ((rc = run_reduced<K>(P, m, 1, gate))) return rc;
      }
      LRS_LAUNCH("adj_retrieve_kernel", adj_retrieve_wave_kernel<T, K>, gw, dim3(64), bw, sa);
      LRS_LAUNCH("adj_retrieve_pivoting", adj_retrieve_kernel<T, K>, grid, dim3(LRS_NT), bs, sf);
    }
  } else if (K == 64 && std::is_same<T, double>::value && P->wave) {
    // K = 64 adjoint on the matrix cores
    const dim3 g64(L.p, (m + 15) / 16);
    if (L.p > 1) {
      SolveArgs sd = sa;
      sd.dst = reinterpret_cast<double*>(P->ws + L.scr);
      LRS_LAUNCH("adj_dstage_kernel", adj_dstage64_kernel, g64, dim3(256), 0, sd);
      if ((rc = run_reduced<K>(P, m, 1, gate))) return rc;
    }
    LRS_LAUNCH("adj_retrieve_kernel", adj_retrieve64_kernel, g64, dim3(256), 0, sa);
  } else {
    if (!set_lds((const void*)adj_dstage_kernel<T, K>, bs) || !set_lds((const void*)adj_retrieve_kernel<T, K>, bs))
      return LRSPIKE_ERR_NOT_SUPPORTED;
    if (L.p > 1) {
      SolveArgs sd = sa;
      sd.dst = reinterpret_cast<double*>(P->ws + L.scr);
      LRS_LAUNCH("adj_dstage_kernel", adj_dstage_kernel<T, K>, grid, dim3(LRS_NT), bs, sd);
        if ((rc = run_reduced<K>(P, m, 1, gate))) return rc;
    }
    LRS_LAUNCH("adj_retrieve_kernel", adj_retrieve_kernel<T, K>, grid, dim3(LRS_NT), bs, sa);
  }
  return 0;
}

// Iterative refinement around run_apply: x_0 = M^{-1} f, then corrections
// x += M^{-1}(f - A x) with the residual, the update and the norms in FP64
// (M from FP32 factors in FP32_REFINED plans, from FP64 factors in
// FP64_REFINED ones).  Every correction is a fixed kernel sequence gated by
// the device stopping rule (refine_ctl_kernel), so the whole solve can be
// captured into a graph: under capture all max_refine corrections are
// enqueued (the ones after the stop are no-ops).  Run eagerly, the host
// enqueues one correction ahead and stops enqueueing once the state copied
// back from the previous one shows the stop, so the GPU never waits for it.
template <typename T, int K>
int run_refined(lrspike_plan P, double* rhs, int m, int transpose) {
  const Layout& L = P->L;
  hipStream_t st = P->stream;
  const int64_t nm = L.n * (int64_t)m;
  double* fcopy = reinterpret_cast<double*>(P->ws + L.fcopy);
  double* scr = reinterpret_cast<double*>(P->ws + L.res);  // not the adjoint D-stage scratch
  double* norms = reinterpret_cast<double*>(P->ws + L.norms);
  int* state = reinterpret_cast<int*>(P->ws + L.latch);
  const int* gate = state + S_STOP;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cap) != hipSuccess) return LRSPIKE_ERR_HIP;
  const bool capturing = cap != hipStreamCaptureStatusNone;
  if (hipMemcpyAsync(fcopy, rhs, nm * 8, hipMemcpyDeviceToDevice, st) != hipSuccess) return LRSPIKE_ERR_HIP;
  LRS_LAUNCH("refine_reset_kernel", refine_reset_kernel, dim3(1), dim3(256), 0, state, norms, L.nsys * L.mmax);
  int rc = run_apply<T, K>(P, rhs, m, transpose);
  if (rc) return rc;
  const size_t bres = (size_t)(RES_ROWS + 2 * L.k) * (RES_MC + 1) * 8;
  if (!set_lds((const void*)residual_kernel, bres)) return LRSPIKE_ERR_NOT_SUPPORTED;
  const dim3 gu(L.p, (unsigned)((L.nbmax * (int64_t)L.K + REF_ROWS - 1) / REF_ROWS));
  for (int it = 0; it < P->max_refine; ++it) {
    LRS_LAUNCH("residual_kernel", residual_kernel, dim3((unsigned)((L.n + RES_ROWS - 1) / RES_ROWS)), dim3(RES_ROWS),
               bres, P->bands, L.n, L.k, fcopy, rhs, scr, m, m, transpose, gate);
    if ((rc = run_apply<T, K>(P, scr, m, transpose, gate))) return rc;
    LRS_LAUNCH("refine_update_kernel", refine_update_kernel, gu, dim3(256), (size_t)2 * m * 8, rhs, scr, L, m,
               norms, gate);
    LRS_LAUNCH("refine_ctl_kernel", refine_ctl_kernel, dim3(1), dim3(64), 0, state, norms, L.nsys, m, L.mmax,
               P->refine_tol, it, P->max_refine);
    if (capturing) continue;
    int* slot = P->hstate + 4 * (it & 1);
    if (hipMemcpyAsync(slot, state + S_STOP, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipEventRecord(P->hev[it & 1], st) != hipSuccess)
      return LRSPIKE_ERR_HIP;
    if (it >= 1) {
      if (hipEventSynchronize(P->hev[(it - 1) & 1]) != hipSuccess) return LRSPIKE_ERR_HIP;
      if (P->hstate[4 * ((it - 1) & 1)] != 0) break;  // stopped: this correction was a no-op
    }
  }
  return 0;
}

// BiCGStab preconditioned by the plan's M_r^{-1} (M_r^{-T} for the adjoint,
// which then runs on A^T): x_0 = M^{-1} b, then the iteration of krylov.hip,
// every kernel gated by the device stopping rule; like run_refined, eager
// solves enqueue one iteration ahead of the stop flag they read back, and a
// captured solve records all max_refine iterations.
template <typename T, int K>
int run_bicgstab(lrspike_plan P, double* rhs, int m, int transpose) {
  const Layout& L = P->L;
  hipStream_t st = P->stream;
  const int64_t nm = L.n * (int64_t)m;
  double* b = reinterpret_cast<double*>(P->ws + L.fcopy);
  double* r = reinterpret_cast<double*>(P->ws + L.res);
  double* vec = reinterpret_cast<double*>(P->ws + L.bvec);
  double *rh = vec, *pv = vec + nm, *vv = vec + 2 * nm, *ph = vec + 3 * nm, *sv = vec + 4 * nm, *sh = vec + 5 * nm,
         *tv = vec + 6 * nm;
  int* state = reinterpret_cast<int*>(P->ws + L.latch);
  const int* gate = state + S_STOP;
  BicgArgs ba{L.n, m, m, L.bblk, reinterpret_cast<double*>(P->ws + L.bsc), reinterpret_cast<double*>(P->ws + L.bpart),
              gate, L.mmax};
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cap) != hipSuccess) return LRSPIKE_ERR_HIP;
  const bool capturing = cap != hipStreamCaptureStatusNone;
  if (hipMemcpyAsync(b, rhs, nm * 8, hipMemcpyDeviceToDevice, st) != hipSuccess) return LRSPIKE_ERR_HIP;
  LRS_LAUNCH("refine_reset_kernel", refine_reset_kernel, dim3(1), dim3(256), 0, state,
             reinterpret_cast<double*>(P->ws + L.norms), L.nsys * L.mmax);
  int rc = run_apply<T, K>(P, rhs, m, transpose);
  if (rc) return rc;
  const size_t bres = (size_t)(RES_ROWS + 2 * L.k) * (RES_MC + 1) * 8;
  if (!set_lds((const void*)residual_kernel, bres)) return LRSPIKE_ERR_NOT_SUPPORTED;
  const size_t bmv = (size_t)(BICG_TPB + 2 * L.k) * (BICG_MC + 1) * 8;
  if (!set_lds((const void*)bicg_matvec_kernel, bmv)) return LRSPIKE_ERR_NOT_SUPPORTED;
  LRS_LAUNCH("residual_kernel", residual_kernel, dim3((unsigned)((L.n + RES_ROWS - 1) / RES_ROWS)), dim3(RES_ROWS),
             bres, P->bands, L.n, L.k, (const double*)b, (const double*)rhs, r, m, m, transpose, gate);
  const dim3 gv(L.bblk), tb(BICG_TPB), gc(m);
  LRS_LAUNCH("bicg_start_kernel", bicg_start_kernel, gv, tb, 0, ba, (const double*)b, (const double*)r, rh, pv, vv);
  LRS_LAUNCH("bicg_reduce_kernel", bicg_reduce_kernel, gc, tb, 0, ba, 2, (int)BS_RR, (int)BS_BB, 0);
  LRS_LAUNCH("bicg_init_kernel", bicg_init_kernel, dim3(1), dim3(BICG_TPB), 0, ba, state, P->refine_tol);
  for (int it = 0; it < P->max_refine; ++it) {
    LRS_LAUNCH("bicg_p_kernel", bicg_p_kernel, gv, tb, 0, ba, (const double*)r, pv, (const double*)vv, ph);
    if ((rc = run_apply<T, K>(P, ph, m, transpose, gate))) return rc;
    LRS_LAUNCH("bicg_matvec_kernel", bicg_matvec_kernel, gv, tb, bmv, ba, P->bands, L.k, (const double*)ph, vv,
               (const double*)rh, 1, transpose);
    LRS_LAUNCH("bicg_reduce_kernel", bicg_reduce_kernel, gc, tb, 0, ba, 1, (int)BS_RV, 0, 0);
    LRS_LAUNCH("bicg_s_kernel", bicg_s_kernel, gv, tb, 0, ba, (const double*)r, (const double*)vv, sv, sh);
    if ((rc = run_apply<T, K>(P, sh, m, transpose, gate))) return rc;
    LRS_LAUNCH("bicg_matvec_kernel", bicg_matvec_kernel, gv, tb, bmv, ba, P->bands, L.k, (const double*)sh, tv,
               (const double*)sv, 2, transpose);
    LRS_LAUNCH("bicg_reduce_kernel", bicg_reduce_kernel, gc, tb, 0, ba, 2, (int)BS_TS, (int)BS_TT, 0);
    LRS_LAUNCH("bicg_x_kernel", bicg_x_kernel, gv, tb, 0, ba, rhs, r, (const double*)rh, (const double*)ph,
               (const double*)sv, (const double*)sh, (const double*)tv);
    LRS_LAUNCH("bicg_reduce_kernel", bicg_reduce_kernel, gc, tb, 0, ba, 2, (int)BS_RHO_NEXT, (int)BS_RR, 0);
    LRS_LAUNCH("bicg_ctl_kernel", bicg_ctl_kernel, dim3(1), dim3(BICG_TPB), 0, ba, state, P->refine_tol, it,
               P->max_refine);
    if (capturing) continue;
    int* slot = P->hstate + 4 * (it & 1);
    if (hipMemcpyAsync(slot, state + S_STOP, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipEventRecord(P->hev[it & 1], st) != hipSuccess)
      return LRSPIKE_ERR_HIP;
    if (it >= 1) {
      if (hipEventSynchronize(P->hev[(it - 1) & 1]) != hipSuccess) return LRSPIKE_ERR_HIP;
      if (P->hstate[4 * ((it - 1) & 1)] != 0) break;  // stopped: this iteration was a no-op
    }
  }
  return 0;
}

// LR-SPIKE-I / LR-SPIKE-OTF solve (kernels in iter.hip): the D-stage gives
// the reduced right-hand side y (interface tips), BiCGStab solves S x = y
// (S = S~_red or S_red) right-preconditioned by S~~_red from x_0 = S~~_red^{-1} y,
// with the device-side stopping rule of run_bicgstab (tolerance refine_tol on
// ||y - S x|| / ||y|| per column, at most max_refine iterations), and the
// retrieval recovers x_j from the solution tips.  Forward solves only.
template <typename T, int K>
int run_iter(lrspike_plan P, double* rhs, int m) {
  const Layout& L = P->L;
  hipStream_t st = P->stream;
  const bool otf = L.variant == LRSPIKE_VARIANT_OTF;
  int* state = reinterpret_cast<int*>(P->ws + L.latch);
  const int* gate = state + S_STOP;
  const int64_t NT = (int64_t)2 * K * L.p, vs = NT * L.mmax;
  double* vec = reinterpret_cast<double*>(P->ws + L.itv);
  double *b = vec, *x = vec + vs, *r = vec + 2 * vs, *rh = vec + 3 * vs, *pv = vec + 4 * vs, *vv = vec + 5 * vs,
         *ph = vec + 6 * vs, *sv = vec + 7 * vs, *sh = vec + 8 * vs, *tv = vec + 9 * vs;
  double* ytip = reinterpret_cast<double*>(P->ws + L.ytip);
  double* F = reinterpret_cast<double*>(P->ws + L.scr);  // OTF: right-hand sides of the partition solves
  BicgArgs ba{NT, m, L.mmax, L.iblk, reinterpret_cast<double*>(P->ws + L.isc),
              reinterpret_cast<double*>(P->ws + L.ipart), gate, L.mmax};
  IterArgs ia{P->bands, P->ws, L, m, gate};
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cap) != hipSuccess) return LRSPIKE_ERR_HIP;
  const bool capturing = cap != hipStreamCaptureStatusNone;
  const dim3 gv(L.iblk), tb(BICG_TPB), gc(m), gi(L.NI, (m + IT_MC - 1) / IT_MC), gp(L.p, (m + IT_MC - 1) / IT_MC);
  const size_t bpre = (size_t)2 * (K + L.R2) * IT_MC * 8, bmv = (size_t)2 * (L.r > 0 ? L.r : 1) * IT_MC * 8;
  if (!set_lds((const void*)iter_precond_kernel<K>, bpre)) return LRSPIKE_ERR_NOT_SUPPORTED;
  const dim3 gf(L.p, (unsigned)std::min<int64_t>(64, ((int64_t)L.nbmax * K + 63) / 64));
  const bool rows31 = (int64_t)L.nbmax * L.K * m * 8 < ((int64_t)1 << 31);
  const bool wv = K >= 16 && K <= 32 && P->wave && rows31;
  const size_t bs = lds_sw<T, K>();
  if (!set_lds((const void*)dstage_kernel<T, K>, bs) || !set_lds((const void*)retrieve_kernel<T, K>, bs))
    return LRSPIKE_ERR_NOT_SUPPORTED;
  // tips of A_j^{-1} src into the tip buffer (the D-stage kernels), gated
  auto dstage = [&](double* src, int ld, const int* g) -> int {
    SolveArgs sa{P->bands, P->ws, L, src, src, ld, m, g};
    if (wv) {
      if constexpr (K >= 16 && K <= 32) {
        const size_t bw = (size_t)WaveSweep<T, K, 1>::total * sizeof(T) + 2 * K * sizeof(int);
        LRS_LAUNCH("dstage_kernel", dstage_wave_kernel<T, K, 1>, dim3(L.p, (m + 15) / 16), dim3(64), bw, sa);
      }
    } else if (K == 64 && std::is_same<T, double>::value && P->wave) {
      LRS_LAUNCH("dstage_kernel", dstage64_kernel, dim3(L.p, (m + 15) / 16), dim3(256), 0, sa);
    } else {
      LRS_LAUNCH("dstage_kernel", dstage_kernel<T, K>, dim3(L.p, (m + mc_of<K>() - 1) / mc_of<K>()), dim3(LRS_NT),
                 bs, sa);
    }
    return 0;
  };
  // y = S src, with the partial inner products of the step (mode 1 or 2 against w1)
  auto matvec = [&](const double* src, double* y, const double* w1, int mode) -> int {
    if (otf) {
      LRS_LAUNCH("iter_otf_rhs_kernel", iter_otf_rhs_kernel<K>, gf, dim3(256), 0, ia, src, F, m);
      int rc2 = dstage(F, m, gate);
      if (rc2) return rc2;
      LRS_LAUNCH("iter_finish_kernel", iter_finish_kernel, gv, tb, 0, ba, src, (const double*)ytip, y, w1, mode);
    } else {
      LRS_LAUNCH("iter_matvec_i_kernel", iter_matvec_i_kernel<K>, gp, dim3(256), bmv, ia, src, y);
      LRS_LAUNCH("iter_finish_kernel", iter_finish_kernel, gv, tb, 0, ba, src, (const double*)nullptr, y, w1, mode);
    }
    return 0;
  };
  LRS_LAUNCH("refine_reset_kernel", refine_reset_kernel, dim3(1), dim3(256), 0, state,
             reinterpret_cast<double*>(P->ws + L.norms), L.nsys * L.mmax);
  // y_red = tips of D^{-1} f
  int rc = dstage(rhs, m, nullptr);
  if (rc) return rc;
  LRS_LAUNCH("iter_copy_kernel", iter_copy_kernel, gv, tb, 0, ba, (const double*)ytip, b, 0);
  // x_0 = S~~^{-1} b, r = b - S x_0
  LRS_LAUNCH("iter_precond_kernel", iter_precond_kernel<K>, gi, dim3(256), bpre, ia, (const double*)b, x);
  if ((rc = matvec(x, r, b, 1))) return rc;
  LRS_LAUNCH("iter_copy_kernel", iter_copy_kernel, gv, tb, 0, ba, (const double*)b, r, 1);
  LRS_LAUNCH("bicg_start_kernel", bicg_start_kernel, gv, tb, 0, ba, (const double*)b, (const double*)r, rh, pv, vv);
  LRS_LAUNCH("bicg_reduce_kernel", bicg_reduce_kernel, gc, tb, 0, ba, 2, (int)BS_RR, (int)BS_BB, 0);
  LRS_LAUNCH("bicg_init_kernel", bicg_init_kernel, dim3(1), dim3(BICG_TPB), 0, ba, state, P->refine_tol);
  for (int it = 0; it < P->max_refine; ++it) {
    LRS_LAUNCH("bicg_p_kernel", bicg_p_kernel, gv, tb, 0, ba, (const double*)r, pv, (const double*)vv, ph);
    LRS_LAUNCH("iter_precond_kernel", iter_precond_kernel<K>, gi, dim3(256), bpre, ia, (const double*)ph, ph);
    if ((rc = matvec(ph, vv, rh, 1))) return rc;
    LRS_LAUNCH("bicg_reduce_kernel", bicg_reduce_kernel, gc, tb, 0, ba, 1, (int)BS_RV, 0, 0);
    LRS_LAUNCH("bicg_s_kernel", bicg_s_kernel, gv, tb, 0, ba, (const double*)r, (const double*)vv, sv, sh);
    LRS_LAUNCH("iter_precond_kernel", iter_precond_kernel<K>, gi, dim3(256), bpre, ia, (const double*)sh, sh);
    if ((rc = matvec(sh, tv, sv, 2))) return rc;
    LRS_LAUNCH("bicg_reduce_kernel", bicg_reduce_kernel, gc, tb, 0, ba, 2, (int)BS_TS, (int)BS_TT, 0);
    LRS_LAUNCH("bicg_x_kernel", bicg_x_kernel, gv, tb, 0, ba, x, r, (const double*)rh, (const double*)ph,
               (const double*)sv, (const double*)sh, (const double*)tv);
    LRS_LAUNCH("bicg_reduce_kernel", bicg_reduce_kernel, gc, tb, 0, ba, 2, (int)BS_RHO_NEXT, (int)BS_RR, 0);
    LRS_LAUNCH("bicg_ctl_kernel", bicg_ctl_kernel, dim3(1), dim3(BICG_TPB), 0, ba, state, P->refine_tol, it,
               P->max_refine);
    if (capturing) continue;
    int* slot = P->hstate + 4 * (it & 1);
    if (hipMemcpyAsync(slot, state + S_STOP, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipEventRecord(P->hev[it & 1], st) != hipSuccess)
      return LRSPIKE_ERR_HIP;
    if (it >= 1) {
      if (hipEventSynchronize(P->hev[(it - 1) & 1]) != hipSuccess) return LRSPIKE_ERR_HIP;
      if (P->hstate[4 * ((it - 1) & 1)] != 0) break;  // stopped: this iteration was a no-op
    }
  }
  // recovery from the solution tips: tip buffer = x, compressed vector = 0
  BicgArgs bu = ba;
  bu.gate = nullptr;
  LRS_LAUNCH("iter_copy_kernel", iter_copy_kernel, gv, tb, 0, bu, (const double*)x, ytip, 0);
  if (L.NI > 0 && L.r > 0)
    LRS_LAUNCH("iter_zero_zg_kernel", iter_zero_zg_kernel, dim3(64), dim3(256), 0,
               reinterpret_cast<double*>(P->ws + L.zg), (size_t)L.NI * L.R2 * L.mmax);
  SolveArgs sa{P->bands, P->ws, L, rhs, rhs, m, m, nullptr};
  if (wv) {
    if constexpr (K >= 16 && K <= 32) {
      const size_t bw = (size_t)WaveSweep<T, K, 1>::total * sizeof(T) + 2 * K * sizeof(int);
      LRS_LAUNCH("retrieve_kernel", retrieve_wave_kernel<T, K, 1>, dim3(L.p, (m + 15) / 16), dim3(64), bw, sa);
    }
  } else if (K == 64 && std::is_same<T, double>::value && P->wave) {
    LRS_LAUNCH("retrieve_kernel", retrieve64_kernel, dim3(L.p, (m + 15) / 16), dim3(256), 0, sa);
  } else {
    LRS_LAUNCH("retrieve_kernel", retrieve_kernel<T, K>, dim3(L.p, (m + mc_of<K>() - 1) / mc_of<K>()), dim3(LRS_NT),
               bs, sa);
  }
  return 0;
}

typedef int (*factor_fn)(lrspike_plan);
typedef int (*apply_fn)(lrspike_plan, double*, int, int);

// one ungated application of M_r^{-1} (or M_r^{-T})
template <typename T, int K>
int run_plain(lrspike_plan P, double* rhs, int m, int transpose) {
  return run_apply<T, K>(P, rhs, m, transpose, nullptr);
}

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

// OUTER: 0 one application, 1 iterative refinement, 2 BiCGStab
template <typename T, int OUTER>
apply_fn pick_apply(int K) {
#define LRS_APPLY(KK) \
  case KK: return OUTER == 0 ? run_plain<T, KK> : (OUTER == 1 ? run_refined<T, KK> : run_bicgstab<T, KK>);
  switch (K) {
    LRS_APPLY(1)
    LRS_APPLY(2)
    LRS_APPLY(4)
    LRS_APPLY(8)
    LRS_APPLY(16)
    LRS_APPLY(32)
    LRS_APPLY(64)
  }
#undef LRS_APPLY
  return nullptr;
}

bool prec_valid(int prec) { return prec >= LRSPIKE_FP64 && prec <= LRSPIKE_FP32_BICGSTAB; }
// Sketch columns of the randomized spike SVD for these options: 0 for the
// exact truncation (also at r = k or r = 0, where nothing is truncated), -1
// for invalid settings (an unknown svd code; at 0 < r < k, rsvd_ell outside
// [r, k] or power steps outside [0, 4]).
int svd_ell(const lrspike_opts* o, int k, int r) {
  if (o->svd == LRSPIKE_SVD_EXACT) return 0;
  if (o->svd != LRSPIKE_SVD_RANDOMIZED) return -1;
  if (r == 0 || r >= k) return 0;
  if (o->rsvd_ell < r || o->rsvd_ell > k || o->rsvd_power < 0 || o->rsvd_power > 4) return -1;
  return o->rsvd_ell;
}

int prec_tsize(int prec) { return (prec == LRSPIKE_FP32_REFINED || prec == LRSPIKE_FP32_BICGSTAB) ? 4 : 8; }
// 0 one application of M, 1 iterative refinement, 2 BiCGStab
int prec_refined(int prec) {
  if (prec == LRSPIKE_FP64) return 0;
  return (prec == LRSPIKE_FP64_BICGSTAB || prec == LRSPIKE_FP32_BICGSTAB) ? 2 : 1;
}
factor_fn factor_for(int prec, int K) { return prec_tsize(prec) == 8 ? pick_factor<double>(K) : pick_factor<float>(K); }
apply_fn apply_for(int prec, int K) {
  const int outer = prec_refined(prec);
  if (prec_tsize(prec) == 8)
    return outer == 0 ? pick_apply<double, 0>(K) : (outer == 1 ? pick_apply<double, 1>(K) : pick_apply<double, 2>(K));
  return outer == 1 ? pick_apply<float, 1>(K) : pick_apply<float, 2>(K);
}

// Pinned host slots and events of the eager refinement loop (refined plans).
int alloc_refine_host(lrspike_plan P) {
  if (hipHostMalloc((void**)&P->hstate, 8 * sizeof(int), hipHostMallocDefault) != hipSuccess) {
    P->hstate = nullptr;
    return LRSPIKE_ERR_HIP;
  }
  for (int i = 0; i < 2; ++i)
    if (hipEventCreateWithFlags(&P->hev[i], hipEventDisableTiming) != hipSuccess) {
      P->hev[i] = nullptr;
      return LRSPIKE_ERR_HIP;
    }
  return 0;
}
void free_refine_host(lrspike_plan P) {
  if (P->hstate) (void)hipHostFree(P->hstate);
  for (int i = 0; i < 2; ++i)
    if (P->hev[i]) (void)hipEventDestroy(P->hev[i]);
  P->hstate = nullptr;
  P->hev[0] = P->hev[1] = nullptr;
}

void prof_clear(lrspike_plan P) {
  for (auto& e : P->prof) {
    event_put(e.second.first);
    event_put(e.second.second);
  }
  P->prof.clear();
}

#include "batched.hip"

// Per-device address of `scratch`, looked up once per device (with that
// device current) and kept.
constexpr int kMaxDevices = 64;
void* scratch_dev[kMaxDevices];
std::mutex scratch_mu;
int scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return LRSPIKE_ERR_HIP;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return LRSPIKE_ERR_HIP;
    scratch_dev[dev] = ptr;
  }
  *out = scratch_dev[dev];
  return 0;
}

// status_out[0] = the latched error code of the state block at st.
__global__ void copy_status_kernel(const int* st, int* status_out) {
  if (threadIdx.x == 0) status_out[0] = st[S_CODE];
}

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
  if (!prec_valid(precision)) return -5;
  if (max_nrhs < 1) return -6;
  if (!bytes) return -7;
  Layout L;
  make_layout(L, n, k, p, r, prec_tsize(precision), max_nrhs, prec_refined(precision));
  *bytes = L.total;
  return 0;
}

int lrspike_workspace_size_opts(int64_t n, int32_t k, int32_t p, int32_t r, const lrspike_opts* opts,
                                size_t* bytes) {
  if (n < 1) return -1;
  if (k < 1) return -2;
  if (p < 1 || p > n) return -3;
  if (r < 0 || r > k) return -4;
  if (!opts || !prec_valid(opts->precision) || opts->max_nrhs < 1) return -5;
  const int ell = svd_ell(opts, k, r);
  if (ell < 0) return -5;
  if (!bytes) return -6;
  Layout L;
  make_layout(L, n, k, p, r, prec_tsize(opts->precision), opts->max_nrhs, prec_refined(opts->precision),
              opts->variant, nullptr, nullptr, 1, nullptr, ell);
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
  if (!prec_valid(opts->precision)) return -6;
  if (opts->variant < LRSPIKE_VARIANT_FULL || opts->variant > LRSPIKE_VARIANT_OTF) return -6;
  // the iterative reduced solves: FP64 plans with at least one interface
  if (opts->variant >= LRSPIKE_VARIANT_I && (opts->precision != LRSPIKE_FP64 || p < 2)) return -6;
  if (opts->max_nrhs < 1) return -6;
  const int ell = svd_ell(opts, k, r);
  if (ell < 0) return -6;
  if (ell > 0 && !is_device_ptr(opts->rsvd_omega)) return -6;
  if (prec_refined(opts->precision) == 2 && opts->max_nrhs > BICG_TPB) return -6;  // one thread per column
  if (K > 64) return LRSPIKE_ERR_NOT_SUPPORTED;
  // reduced-system blocks of order 2r are inverted in one workgroup's LDS
  if (p > 1 && 2 * ((r == k) ? K : r) > 64) return LRSPIKE_ERR_NOT_SUPPORTED;
  lrspike_plan P = new lrspike_plan_s();
  make_layout(P->L, n, k, p, r, prec_tsize(opts->precision), opts->max_nrhs, prec_refined(opts->precision),
              opts->variant, nullptr, nullptr, 1, nullptr, ell);
  if (!opts->workspace || opts->workspace_bytes < P->L.total || !is_device_ptr(opts->workspace)) {
    delete P;
    return LRSPIKE_ERR_WORKSPACE;
  }
  P->precision = opts->precision;
  P->variant = opts->variant;
  P->max_refine = opts->max_refine > 0 ? opts->max_refine : 30;
  P->refine_tol = opts->refine_tol > 0 ? opts->refine_tol : 1e-13;
  P->stream = reinterpret_cast<hipStream_t>(opts->stream);
  P->bands = bands;
  P->ws = reinterpret_cast<char*>(opts->workspace);
  P->profiling = opts->profile ? 1 : 0;
  P->rsvd_omega = ell > 0 ? opts->rsvd_omega : nullptr;
  P->rsvd_power = ell > 0 ? opts->rsvd_power : 0;
  int rc = (prec_refined(P->precision) || P->variant >= LRSPIKE_VARIANT_I) ? alloc_refine_host(P) : 0;
  if (!rc) rc = launch(P, "state_init_kernel", state_init_kernel, dim3(1), dim3(64), 0,
                       reinterpret_cast<int*>(P->ws + P->L.latch));
  factor_fn f = factor_for(P->precision, K);
  if (!rc) rc = f ? f(P) : LRSPIKE_ERR_NOT_SUPPORTED;
  if (rc) {
    lrspike_destroy(P);
    return rc;
  }
  *plan_out = P;
  return 0;
}

static int solve_common(lrspike_plan P, double* rhs, int32_t nrhs, int transpose) {
  if (!P || P->batch) return -1;
  if (!is_device_ptr(rhs)) return -2;
  if (nrhs < 1 || nrhs > P->L.mmax) return -3;
  if (P->variant >= LRSPIKE_VARIANT_I) {  // LR-SPIKE-I / -OTF: forward solves (FP64 plans)
    if (transpose) return LRSPIKE_ERR_NOT_SUPPORTED;
    if (nrhs > BICG_TPB) return -3;
    switch (P->L.K) {
      case 1: return run_iter<double, 1>(P, rhs, nrhs);
      case 2: return run_iter<double, 2>(P, rhs, nrhs);
      case 4: return run_iter<double, 4>(P, rhs, nrhs);
      case 8: return run_iter<double, 8>(P, rhs, nrhs);
      case 16: return run_iter<double, 16>(P, rhs, nrhs);
      case 32: return run_iter<double, 32>(P, rhs, nrhs);
      case 64: return run_iter<double, 64>(P, rhs, nrhs);
    }
    return LRSPIKE_ERR_NOT_SUPPORTED;
  }
  apply_fn f = apply_for(P->precision, P->L.K);
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
    // first latched error over the groups (partition = that system's index);
    // counters summed, diagnostics combined (min of minima, max of maxima)
    lrspike_info gi, out;
    memset(&out, 0, sizeof(out));
    out.partition = -1;
    out.row = -1;
    out.min_pivot = INFINITY;
    out.min_sigma_gap = INFINITY;
    int first = 0;
    for (BatchGroup& G : P->batch->groups) {
      int rc = lrspike_status(G.plan, &gi);
      if (rc < 0 || rc == LRSPIKE_ERR_HIP) return rc;
      out.swapped_blocks += gi.swapped_blocks;
      out.refine_iters = std::max(out.refine_iters, gi.refine_iters);
      out.last_correction = std::max(out.last_correction, gi.last_correction);
      out.min_pivot = std::min(out.min_pivot, gi.min_pivot);
      out.max_abs_entry = std::max(out.max_abs_entry, gi.max_abs_entry);
      out.min_sigma_gap = std::min(out.min_sigma_gap, gi.min_sigma_gap);
      out.reduced_growth = std::max(out.reduced_growth, gi.reduced_growth);
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
  int st[STATE_INTS];
  if (hipMemcpy(st, P->ws + P->L.latch, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess) return LRSPIKE_ERR_HIP;
  auto dbl = [&](int slot) {
    double v;
    memcpy(&v, st + slot, 8);
    return v;
  };
  if (info) {
    info->error = st[S_CODE];
    info->partition = st[S_CODE] ? st[S_PART] : -1;
    int64_t row;
    memcpy(&row, st + S_ROW, 8);
    info->row = st[S_CODE] ? row : -1;
    info->refine_iters = st[S_ITERS];
    info->swapped_blocks = st[S_SWAPPED];
    info->last_correction = dbl(S_CORR);
    info->min_pivot = dbl(S_PIVMIN);
    info->max_abs_entry = dbl(S_AMAX);
    info->min_sigma_gap = dbl(S_GAPMIN);
    const double zmax = dbl(S_ZMAX), zgrow = dbl(S_ZGROW);
    info->reduced_growth = zmax > 0.0 ? zgrow / zmax : 0.0;
  }
  return st[S_CODE];
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
    free_refine_host(P);
    if (P->batch) {
      for (BatchGroup& G : P->batch->groups) free_group(G);
      if (P->batch->graph) (void)hipGraphExecDestroy(P->batch->graph);
      if (P->batch->capture) (void)hipStreamDestroy(P->batch->capture);
      for (hipStream_t s : P->batch->gstreams) (void)hipStreamDestroy(s);
      for (hipEvent_t e : P->batch->joins) (void)hipEventDestroy(e);
      if (P->batch->fork) (void)hipEventDestroy(P->batch->fork);
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
  if (!prec_valid(opts->precision) || prec_refined(opts->precision) == 2) return -4;  // no BiCGStab for batches
  if (opts->svd != LRSPIKE_SVD_EXACT) return -4;  // nor the randomized spike SVD
  if (opts->variant >= LRSPIKE_VARIANT_I) return -4;  // nor the iterative reduced solves
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
  rc = run_batched_on(P, B.capture, rhs_base, true, true);
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

int lrspike_solve_noalloc(int64_t n, int32_t k, const double* bands, int32_t p, int32_t r, double* rhs,
                          int32_t nrhs, void* stream, int32_t* status_out) {
  if (n < 1) return -1;
  if (k < 1) return -2;
  if (p < 1 || p > n) return -4;
  if (r < 0 || r > k) return -5;
  if (nrhs < 1) return -7;
  const int K = kernel_K(k);
  const int64_t njmin = n / p;
  if ((p > 1 && njmin < 2 * (int64_t)k) || njmin < K) return -4;
  if (K > 64 || (p > 1 && 2 * ((r == k) ? K : r) > 64)) return LRSPIKE_ERR_NOT_SUPPORTED;
  // the plan lives on the stack; its workspace is the static scratch
  lrspike_plan_s P;
  make_layout(P.L, n, k, p, r, 8, nrhs);
  if (P.L.total > LRS_SCRATCH_BYTES) return LRSPIKE_ERR_WORKSPACE;
  if (!is_device_ptr(bands)) return -3;
  if (!is_device_ptr(rhs)) return -6;
  if (status_out && !is_device_ptr(status_out)) return -9;
  void* ws = nullptr;
  int rc = scratch_address(&ws);
  if (rc) return rc;
  P.precision = LRSPIKE_FP64;
  P.variant = LRSPIKE_VARIANT_FULL;
  P.max_refine = 0;
  P.refine_tol = 0.0;
  P.stream = reinterpret_cast<hipStream_t>(stream);
  P.bands = bands;
  P.ws = reinterpret_cast<char*>(ws);
  P.profiling = 0;
  int* state = reinterpret_cast<int*>(P.ws + P.L.latch);
  rc = launch(&P, "state_init_kernel", state_init_kernel, dim3(1), dim3(64), 0, state);
  factor_fn f = factor_for(LRSPIKE_FP64, K);
  apply_fn a = apply_for(LRSPIKE_FP64, K);
  if (!rc) rc = (f && a) ? f(&P) : LRSPIKE_ERR_NOT_SUPPORTED;
  if (!rc) rc = a(&P, rhs, nrhs, 0);
  if (!rc && status_out)
    rc = launch(&P, "copy_status_kernel", copy_status_kernel, dim3(1), dim3(64), 0, (const int*)state,
                (int*)status_out);
  return rc;
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
