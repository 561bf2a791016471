/*
 * lrspike.h -- C ABI of the MI355X (gfx950) LR-SPIKE banded solver.
 *
 * Method: Spring, Polizzi and Sameh, "Low-Rank SPIKE Framework for Solving
 * Large Sparse Linear Systems with Applications", arXiv 2504.11167.
 *   Problem statement A x = f, A n x n banded with half-bandwidth k, f holding
 *   n_rhs columns                                  (section "SPIKE partitioning")
 *   p diagonal blocks A_j and couplings B_j, C_j    (same section)
 *   spikes V_j = A_j^{-1}[0; B_j], W_j = A_j^{-1}[C_j; 0]   (eq. Veqn)
 *   rank-r truncated SVD of the whole spikes (n_svd = r)    (section "SVD
 *                                                  representation of the spikes")
 *   reduced system on the spike tips                 (eq. spikered)
 *   recovery x_j = A_j^{-1}(f_j - [C_j x_{j-1,b}; 0; B_j x_{j+1,t}])
 *                                                    (eqs. recovery1, recovery2)
 * The factorization is computed once and reused for many solves.
 *
 * Conventions (every call):
 *   - Every array argument is a DEVICE pointer (hipMalloc'd or a torch CUDA
 *     tensor's data) unless stated otherwise.  Host pointers are rejected.
 *   - bands: band-major (2k+1) x n doubles, bands[(d + k) * n + i] = A[i, i+d]
 *     for d in [-k, k].  Entries with i + d outside [0, n) are ignored but must
 *     be finite.
 *   - rhs / x: row-major n x nrhs doubles (a contiguous torch (n, nrhs) tensor).
 *   - Work is enqueued on opts->stream (0 = the null stream) and is
 *     asynchronous: no call below synchronizes except lrspike_status.
 *   - Return values: 0 ok; -i means argument i is invalid (LAPACK INFO < 0
 *     convention, 1-based); positive values are the LRSPIKE_ERR_* codes.
 *     Argument errors are detected on the host before anything is enqueued.
 *     Numerical errors (zero pivot, singular reduced system, non-finite data,
 *     refinement not converged) are latched on the device and reported by
 *     lrspike_status, so that factor and solve stay free of host syncs.
 *   - A plan must not be used concurrently from two streams.
 */
#ifndef LRSPIKE_H
#define LRSPIKE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lrspike_plan_s *lrspike_plan; /* opaque host object */

enum {
  LRSPIKE_FP64 = 0,         /* factors, spikes and sweeps in FP64; one application of M_r^{-1} */
  LRSPIKE_FP32_REFINED = 1, /* FP32 factors/spikes/sweeps; FP64 reduced system,
                               residual and update in iterative refinement */
  LRSPIKE_FP64_REFINED = 2, /* FP64 factors; M_r^{-1} as the preconditioner of an iterative
                               refinement with FP64 residual: x = A^{-1} rhs to refine_tol for
                               any r (and A^{-T} for the adjoint) */
  LRSPIKE_FP64_BICGSTAB = 3, /* FP64 factors; M_r^{-1} as the right preconditioner of BiCGStab
                               (the outer Krylov solver of table solver-list), FP64 vectors and
                               inner products, per-column iterations: x = A^{-1} rhs until
                               ||rhs - A x||_2 <= refine_tol ||rhs||_2 for every column, for
                               systems where refinement does not contract (non-dominant A,
                               small r); the adjoint runs the same iteration on A^T with M_r^{-T}.
                               max_refine caps the iterations.  Not for batched plans */
  LRSPIKE_FP32_BICGSTAB = 4  /* the same with FP32 factors behind M_r^{-1} */
};

/* Reduced interface system (the variant table of section "Selected LR-SPIKE
 * Algorithms"). */
enum {
  LRSPIKE_VARIANT_FULL = 0, /* the whole truncated reduced system S~_red, solved directly */
  LRSPIKE_VARIANT_T = 1,    /* LR-SPIKE-T: the truncated-SPIKE form of it, S~~_red (eqs.
                               truncated_redsys, red_sys_prec_mid_1/2): only the 2 x 2 interface
                               blocks [[I, V~_{j,b}], [W~_{j+1,t}, I]] are kept, solved
                               independently per interface (eqs. red_sys_1, red_sys_mid,
                               red_sys_3); the tips V~_{j,t}, W~_{j,b} are dropped */
  LRSPIKE_VARIANT_I = 2,    /* LR-SPIKE-I: S~_red solved by BiCGStab right-preconditioned by
                               S~~_red; at convergence the result equals LR-SPIKE's */
  LRSPIKE_VARIANT_OTF = 3   /* LR-SPIKE-OTF: the true reduced system S_red (eq. spikered) solved
                               by BiCGStab right-preconditioned by S~~_red, each product formed on
                               the fly by partition solves (eqs. OTF-1/2), then the exact recovery
                               of eqs. recovery1/2: x = A^{-1} rhs to the tolerance for any r.
                               Variants I and OTF: FP64 plans with p >= 2, forward solves only
                               (lrspike_solve_adjoint returns NOT_SUPPORTED), refine_tol and
                               max_refine are the inner iteration's relative tolerance on the
                               reduced residual and its iteration cap, non-convergence latches
                               NOT_CONVERGED; not for batched plans */
};

enum {
  LRSPIKE_OK = 0,
  LRSPIKE_ERR_ZERO_PIVOT = 1,       /* a partition LU met an exactly zero pivot */
  LRSPIKE_ERR_REDUCED_SINGULAR = 2, /* zero pivot in the reduced system */
  LRSPIKE_ERR_NOT_CONVERGED = 3,    /* refinement did not reach refine_tol */
  LRSPIKE_ERR_NONFINITE = 4,        /* Inf/NaN met in a pivot of a partition LU (partition, row),
                                       in the reduced system (interface, -1), or in a correction
                                       of a refined solve (-1, -1) */
  LRSPIKE_ERR_HIP = 5,              /* a HIP runtime call failed */
  LRSPIKE_ERR_NOT_SUPPORTED = 6,    /* parameter combination not built (k > 64, 2r > 64), or a
                                       partition at k > 32 that needs row interchanges */
  LRSPIKE_ERR_WORKSPACE = 7         /* workspace missing or too small */
};

/* How a spike is truncated to rank r (section "SVD representation of the
 * spikes"). */
enum {
  LRSPIKE_SVD_EXACT = 0,     /* rank-r truncation of the whole spike (its Gram's leading eigenvectors) */
  LRSPIKE_SVD_RANDOMIZED = 1 /* the randomized SVD the paper uses (the proto-algorithm of Halko,
                                Martinsson and Tropp): the spike is sketched with ell = rsvd_ell
                                columns, Y = (V V^T)^q V Omega, by q + 1 block solves with 2 ell
                                right-hand sides and as many adjoint ones; V is replaced by its
                                projection Q Q^T V onto range(Y), which is then truncated like
                                the whole spike.  Omega: Gaussian test matrices supplied by the
                                caller.  Only at 0 < r < k; not for batched plans */
};

typedef struct {
  int32_t precision;     /* LRSPIKE_FP64 (default), LRSPIKE_FP32_REFINED or LRSPIKE_FP64_REFINED */
  int32_t max_refine;    /* refined precisions: max corrections (default 30).  The stopping rule
                            runs on the device; under stream capture all max_refine corrections
                            are recorded (those after the stop do nothing), so keep it small there */
  double refine_tol;     /* refined precisions: relative accuracy to reach (default 1e-13).  With
                            c_i = max over (system, column) of ||d_c||_2 / ||x_c||_2 for correction i, the
                            iteration stops when c_i <= tol, or when the error left after the update,
                            estimated as 10 rho c_i, is <= tol, where the contraction rho is
                            c_i / c_{i-1} (c_0 itself for the first correction, the accuracy of the
                            FP32 solve) and is trusted only below 1e-2.  A correction that shrinks
                            by less than half ends the iteration: converged if it is already
                            <= 100 tol (the rounding level of an ill-conditioned system), else
                            NOT_CONVERGED is latched (also after max_refine corrections); a
                            non-finite correction latches NONFINITE */
  void *stream;          /* hipStream_t to enqueue on; NULL = null stream */
  void *workspace;       /* device memory of >= lrspike_workspace_size bytes, caller-owned,
                            must outlive the plan */
  size_t workspace_bytes;
  int32_t max_nrhs;      /* largest nrhs a solve will be called with (default 32);
                            sizes the per-solve vectors inside the workspace */
  int32_t profile;       /* nonzero: time every kernel launch of this plan with a HIP
                            event pair on the plan's stream (see lrspike_profile_read) */
  int32_t variant;       /* LRSPIKE_VARIANT_FULL (default), _T, _I or _OTF */
  int32_t svd;           /* LRSPIKE_SVD_EXACT (default) or LRSPIKE_SVD_RANDOMIZED */
  int32_t rsvd_ell;      /* randomized SVD: sketch columns ell, r <= ell <= k (the paper oversamples
                            by r/2 to r: ell = 1.5 r .. 2 r) */
  int32_t rsvd_power;    /* randomized SVD: power steps q, 0..4 (2 + 2q passes over each spike) */
  const double *rsvd_omega; /* randomized SVD: device array p x 2 x k x ell, row-major: the
                            Gaussian test matrix (k x ell) of V_j, then that of W_j, for every
                            partition j (those of V_{p-1} and W_0 are not read).  Borrowed:
                            read by the factorization's kernels on the plan's stream, so it
                            must stay valid until that work has completed */
} lrspike_opts;

/* Fill *opts with the defaults above (no workspace, null stream). */
void lrspike_default_opts(lrspike_opts *opts);

/*
 * Bytes of device workspace a plan for (n, k, p, r, precision, max_nrhs)
 * needs.  Pure host computation.  Returns 0 or a negative argument code.
 */
int lrspike_workspace_size(int64_t n, int32_t k, int32_t p, int32_t r,
                           int32_t precision, int32_t max_nrhs, size_t *bytes);

/*
 * The same for a full option set (precision, max_nrhs, variant and the spike
 * truncation; the randomized SVD adds the n x 2 ell sketch and needs at least
 * 2 ell solve columns).  lrspike_workspace_size equals this with the other
 * options at their defaults.  Pure host computation.  Returns 0 or a negative
 * argument code (-5: invalid options).
 */
int lrspike_workspace_size_opts(int64_t n, int32_t k, int32_t p, int32_t r, const lrspike_opts *opts,
                                size_t *bytes);

/*
 * Factorization stage (section "SPIKE partitioning", the DS factorization,
 * the spikes of eq. Veqn and their rank-r truncated SVD).  Splits A into p
 * partitions of floor(n/p) + [j < n mod p] rows, factors every A_j (partial
 * pivoting inside the band), forms both spikes of every partition, keeps
 * their tips in rank-r form (r = k keeps them whole and the method is exact),
 * and factors the reduced interface system.
 *   n      matrix order, n >= 1
 *   k      half-bandwidth, 1 <= k <= 64.  Blocks are K x K with K the next power
 *          of two >= k; for K = 64 the partitions are factored without row
 *          interchanges, and one that would need an interchange (a multiplier
 *          above 1 in magnitude) latches NOT_SUPPORTED for that partition
 *   bands  device pointer, (2k+1) x n band-major doubles; borrowed: it must
 *          stay valid (unchanged) for the plan's lifetime when precision is
 *          refined (the residual reads it), for LRSPIKE_VARIANT_T and the
 *          retrieval (the coupling blocks are read from it) and for lrspike_band_grad
 *   p      number of partitions, 1 <= p <= n; each partition needs >= 2k rows
 *          when p > 1
 *   r      retained singular values per spike (the paper's n_svd), 0 <= r <= k;
 *          with p > 1 the interface blocks need 2r <= 64 (2K <= 64 when r = k)
 *   opts   options; workspace required (see lrspike_workspace_size, or
 *          lrspike_workspace_size_opts with the randomized spike SVD)
 *   plan_out  receives a new plan (host object) on success
 */
int lrspike_factor(int64_t n, int32_t k, const double *bands, int32_t p, int32_t r,
                   const lrspike_opts *opts, lrspike_plan *plan_out);

/*
 * Solve stage (D-stage, reduced system, recovery; the summary of the SPIKE
 * solve).  In place: rhs (n x nrhs, row-major) is overwritten by
 * x = M_r^{-1} rhs, which is A^{-1} rhs at r = k.  With a refined precision the
 * solve iterates x += M_r^{-1}(rhs - A x) with the residual in FP64 until the
 * tolerance (then x is A^{-1} rhs to that tolerance for any r).
 *   nrhs   1 <= nrhs <= opts.max_nrhs of the factor call
 */
int lrspike_solve(lrspike_plan plan, double *rhs, int32_t nrhs);

/*
 * Adjoint solve: rhs is overwritten by M_r^{-T} rhs, the exact transpose of
 * the operator lrspike_solve applies (A^{-T} rhs at r = k; with a refined precision
 * refined against A^T to the same tolerance).
 */
int lrspike_solve_adjoint(lrspike_plan plan, double *rhs, int32_t nrhs);

/*
 * grad_bands[(d+k) n + i] = - sum_c lam[i, c] x[i+d, c] for d in [-k, k]
 * (zero where i + d is outside the matrix): the gradient of a loss with
 * respect to the band entries, given lam = A^{-T} dL/dx and the solution x.
 * lam, x: n x nrhs row-major; grad_bands: (2k+1) x n, overwritten.
 */
int lrspike_band_grad(lrspike_plan plan, const double *lam, const double *x,
                      int32_t nrhs, double *grad_bands);

typedef struct {
  int32_t error;          /* first latched LRSPIKE_ERR_* code, 0 if none */
  int32_t partition;      /* partition (or interface) of the first error, -1 if none */
  int64_t row;            /* partition-local row of the first error, -1 if none */
  int32_t refine_iters;   /* corrections applied by the last refined solve */
  int32_t swapped_blocks; /* k-row blocks whose LU needed a row interchange */
  double last_correction; /* max over (system, column) of ||d_c|| / ||x_c|| of the last correction */
  /* diagnostics of the factorization (the failure flags of the paper's
     experiments made quantitative): */
  double min_pivot;       /* min |pivot| over all partition LUs */
  double max_abs_entry;   /* max |a_ij| over the band: min_pivot / max_abs_entry small = near-singular A_j */
  double min_sigma_gap;   /* min over the truncated spikes of (sigma_r - sigma_{r+1}) / sigma_1; the
                             rank-r truncation is well defined (unique) only when it is >> 1e-16;
                             +inf when nothing is truncated (r = k or p = 1) */
  double reduced_growth;  /* max |entry| of the reduced-system blocks inverted during its
                             elimination / max |entry| of the reduced system (0 without one) */
} lrspike_info;

/* Synchronizes the plan's stream and returns (and reports) the latched state. */
int lrspike_status(lrspike_plan plan, lrspike_info *info);

/*
 * Per-kernel timing (instrumentation, not part of the method).  While enabled,
 * every kernel the plan enqueues is bracketed by a HIP event pair on the
 * plan's stream.  lrspike_profile_read synchronizes the stream, sums the
 * elapsed times per kernel name over all launches recorded since the last
 * read, and clears the record.
 *   names     max x 32 chars (NUL-terminated names), may be NULL
 *   total_ms  max doubles, may be NULL;  launches  max ints, may be NULL
 *   count     receives the number of distinct kernels (may exceed max)
 */
int lrspike_profile(lrspike_plan plan, int32_t enable);
int lrspike_profile_read(lrspike_plan plan, int32_t max, char *names, double *total_ms,
                         int32_t *launches, int32_t *count);

/* Frees the host object (the workspace belongs to the caller; a batched
 * plan also frees the device memory it allocated). */
int lrspike_destroy(lrspike_plan plan);

/*
 * Batched independent systems: many banded systems of different orders,
 * bandwidths and right-hand-side counts factored and solved together (the
 * partitioned solve of section "SPIKE partitioning" applied to every system).
 * Systems with equal (k, r) are solved as one LR-SPIKE problem over their
 * concatenated band with a partition boundary at every system boundary: the
 * coupling blocks across a system boundary are zero, so the reduced system
 * splits into independent per-system blocks and every result equals that of
 * the system's own plan with the same p.
 */
typedef struct {
  int64_t n;            /* order, >= 1 */
  int32_t k;            /* half-bandwidth, 1 <= k <= 64 */
  int32_t p;            /* partitions (n / p >= max(2k, K), K = next power of two >= k);
                           0 = chosen by the autotuner */
  int32_t r;            /* retained rank, 0 <= r <= k (2r <= 64) */
  int32_t nrhs;         /* right-hand-side columns, >= 1 */
  int64_t band_offset;  /* element offset of the system's (2k+1) x n band-major band in bands_base */
  int64_t rhs_offset;   /* element offset of its n x nrhs row-major right-hand sides in rhs_base */
} lrspike_batch_desc;

/*
 * Factor every system.  descs: HOST array of count descriptors.  bands_base:
 * device pointer, borrowed for the plan's lifetime (lrspike_run_batched
 * re-reads it).  opts: precision and stream are used; the plan allocates its
 * own device memory (the concatenated bands, right-hand sides and
 * workspaces), so opts.workspace is ignored.  Systems with p = 0 get their
 * partition count from the autotuner, which times candidate partition sizes
 * (and, for K >= 16, matrix-core against workgroup sweeps) on the systems
 * themselves and keeps the fastest; this synchronizes the stream.
 * Returns -2 for an invalid descriptor, NOT_SUPPORTED for k > 64 or 2r > 64.
 */
int lrspike_factor_batched(int32_t count, const lrspike_batch_desc *descs, const double *bands_base,
                           const lrspike_opts *opts, lrspike_plan *plan_out);

/* In place: every system's right-hand sides at rhs_base + rhs_offset are
 * overwritten by its solution.  rhs_base: device pointer. */
int lrspike_solve_batched(lrspike_plan plan, double *rhs_base);

/*
 * Factor (from the current contents of bands_base) and solve every system, as
 * one HIP graph: the first call with a given rhs_base runs eagerly and
 * captures the sequence; later calls with the same rhs_base replay the graph
 * (a new rhs_base captures again).  Refined plans record max_refine gated
 * corrections per group (the device stopping rule makes the surplus no-ops).
 */
int lrspike_run_batched(lrspike_plan plan, double *rhs_base);

/* p_out[s] = the partition count used for system s (count = the descriptor count). */
int lrspike_batch_partitions(lrspike_plan plan, int32_t count, int32_t *p_out);

/* For a batched plan, lrspike_status reports the first latched error of any
 * system (info.partition = that system's index) and sums swapped_blocks;
 * lrspike_solve, lrspike_solve_adjoint, lrspike_band_grad and the profiling
 * calls return -1 for it. */

/*
 * Allocation-free factor + solve, for callers that cannot allocate (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  The same kernels as lrspike_factor followed by lrspike_solve
 * in FP64 (LRSPIKE_FP64, LRSPIKE_VARIANT_FULL), but the factors and every
 * other intermediate live in a device scratch array of 64 MiB that the
 * library holds per GPU for the life of the process; no host or device
 * memory is allocated and no plan is returned.
 *   n, k, bands, p, r   as for lrspike_factor
 *   rhs        device pointer, n x nrhs row-major, overwritten by x = M_r^{-1} rhs
 *   nrhs       >= 1
 *   stream     hipStream_t to enqueue on (NULL = null stream); nothing synchronizes
 *   status_out device pointer to one int32 that receives the latched error code
 *              (0 or an LRSPIKE_ERR_* value) when the work completes, or NULL
 * Returns 0, a negative argument code, LRSPIKE_ERR_NOT_SUPPORTED, or
 * LRSPIKE_ERR_WORKSPACE when the problem's workspace (lrspike_workspace_size
 * with precision FP64 and max_nrhs = nrhs) exceeds the 64 MiB scratch.
 * Every call on a GPU shares that GPU's scratch: calls that overlap in time
 * on one GPU (two streams, two host threads) race and must be serialized by
 * the caller.  The scratch keeps the last call's contents; everything a call
 * reads is written by that call first.
 */
int lrspike_solve_noalloc(int64_t n, int32_t k, const double *bands, int32_t p, int32_t r,
                          double *rhs, int32_t nrhs, void *stream, int32_t *status_out);

const char *lrspike_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif
