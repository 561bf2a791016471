// Device building blocks shared by the LR-SPIKE kernels (gfx950, wave64).
//
// Block view of a partition.  Partition j (rows s_j .. s_j + n_j - 1 of A,
// n_j = floor(n/p) + [j < n mod p]) is treated as a block-tridiagonal matrix
// of K x K blocks, K >= k (K = k, or the next size the library is built for,
// with the extra diagonals zero).  Blocks are aligned to the BOTTOM of the
// partition: the first block holds K0 = n_j - (nb - 1) K real rows preceded by
// K - K0 virtual rows that carry an identity (so ragged partitions need no
// special case: the padded system is block-diagonal in the virtual rows).
// "Padded" row q in [0, nb K) is partition row q - pad, pad = K - K0.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <limits>

#include "layout.h"

#define LRS_NT 256  // threads per workgroup (4 wave64)

namespace lrs {

struct Geom {
  int64_t s;  // first global row of the partition
  int nj;     // rows
  int nb;     // K-row blocks
  int pad;    // virtual identity rows before the first real row
};

__device__ __host__ inline Geom part_geom(int64_t n, int p, int j, int K) {
  int64_t base = n / p, extra = n % p;
  Geom g;
  g.nj = (int)(base + (j < extra ? 1 : 0));
  g.s = (int64_t)j * base + (j < extra ? j : extra);
  g.nb = (g.nj + K - 1) / K;
  g.pad = g.nb * K - g.nj;
  return g;
}

// geometry of partition j of a plan (explicit offsets or the uniform rule)
__device__ inline Geom part_geom(const Layout& L, int j, int K) {
  if (!L.offs) return part_geom(L.n, L.p, j, K);
  Geom g;
  g.s = L.offs[j];
  g.nj = (int)(L.offs[j + 1] - L.offs[j]);
  g.nb = (g.nj + K - 1) / K;
  g.pad = g.nb * K - g.nj;
  return g;
}

// A[gi, gc] from the band-major input (true half-bandwidth k), zero outside.
__device__ inline double band_at(const double* __restrict__ bands, int64_t n, int k,
                                 int64_t gi, int64_t gc) {
  int64_t d = gc - gi;
  if (gi < 0 || gc < 0 || gi >= n || gc >= n || d < -k || d > k) return 0.0;
  return bands[(d + k) * n + gi];
}

// Entry (q, c) of the padded partition matrix (padded coordinates).
__device__ inline double part_at(const double* __restrict__ bands, int64_t n, int k,
                                 const Geom& g, int q, int c) {
  if (q < g.pad || c < g.pad) return (q == c) ? 1.0 : 0.0;
  if (q >= g.pad + g.nj || c >= g.pad + g.nj) return 0.0;
  return band_at(bands, n, k, g.s + q - g.pad, g.s + c - g.pad);
}

// ------------------------------------------------------------------------
// Storage order of the K x K factor blocks.  For K >= 16 a block is stored in
// the A-operand fragment order of the 16x16x4 matrix-core instructions, so
// that one fragment (16 rows x 4 k-columns) is one contiguous 64-element run
// and a wave loads it with one fully coalesced access.  Within each 16-wide
// k chunk the k index is permuted so that the f64 (f32) accumulator layout of
// a product can be fed back as the B operand without moving data between
// lanes: f64 accumulator element v of lane group g holds row g + 4v, f32 holds
// row 4g + v.  For K < 16 blocks are row-major.
template <typename T, int K>
__host__ __device__ constexpr int fidx(int i, int c) {
  if constexpr (K >= 16) {
    const int t = i >> 4, r = i & 15, cc = c >> 4, w = c & 15;
    const int s = (sizeof(T) == 8) ? (w >> 2) : (w & 3);
    const int gq = (sizeof(T) == 8) ? (w & 3) : (w >> 2);
    return ((t * (K / 4) + cc * 4 + s) << 6) + r + 16 * gq;
  } else {
    return i * K + c;
  }
}
// (row, column) of the element stored at position o of a K x K block
template <typename T, int K>
__host__ __device__ inline void fidx_inv(int o, int& i, int& c) {
  if constexpr (K >= 16) {
    const int lane = o & 63, frag = o >> 6;
    const int t = frag / (K / 4), step = frag % (K / 4), gq = lane >> 4;
    i = 16 * t + (lane & 15);
    c = 16 * (step >> 2) + ((sizeof(T) == 8) ? 4 * (step & 3) + gq : 4 * gq + (step & 3));
  } else {
    i = o / K;
    c = o % K;
  }
}
// k index (within the K columns) of lane group gq at k-step `step`
template <typename T>
__host__ __device__ constexpr int frag_k(int step, int gq) {
  return 16 * (step >> 2) + ((sizeof(T) == 8) ? 4 * (step & 3) + gq : 4 * gq + (step & 3));
}

// ------------------------------------------------------------------------
// Device error latch: the first error wins (code, partition, row).
// Layout: int32 [0] = code, [1] = partition, int64 at [2..3] = row.
// ------------------------------------------------------------------------
__device__ inline void latch_error(int* latch, int code, int part, int64_t row) {
  if (atomicCAS(latch, 0, code) == 0) {
    latch[1] = part;
    reinterpret_cast<int64_t*>(latch + 2)[0] = row;
  }
}

// Running min / max of non-negative doubles in the state block: the IEEE bit
// patterns of non-negative doubles are ordered like their values, so 64-bit
// integer atomics on the patterns keep the extreme (+inf is the min's start).
// The stored extreme is read first and the atomic issued only when v would
// change it, so that thousands of workgroups do not serialise on one address.
__device__ inline void state_min(int* st, int slot, double v) {
  unsigned long long* a = reinterpret_cast<unsigned long long*>(st + slot);
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  if (b < __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMin(a, b);
}
__device__ inline void state_max(int* st, int slot, double v) {
  unsigned long long* a = reinterpret_cast<unsigned long long*>(st + slot);
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  if (b > __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(a, b);
}

// Wave-wide min / max (all 64 lanes; every lane gets the result).
template <typename T>
__device__ inline T wave_min(T v) {
  for (int off = 32; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off));
  return v;
}
template <typename T>
__device__ inline T wave_max(T v) {
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}

// ------------------------------------------------------------------------
// LDS block GEMM, whole workgroup:  C[M x N] = beta * C + alpha * op(A) B
//   op(A)(i, l) = TA ? A[l * lda + i] : A[i * lda + l]      (M x KD)
//   B(l, j) = B[l * ldb + j]                                  (KD x N)
// C must not alias A or B.  No barrier inside; the caller synchronizes.
// ------------------------------------------------------------------------
template <typename T, bool TA>
__device__ inline void gemm_valu(int M, int N, int KD, T alpha, const T* A, int lda,
                                 const T* B, int ldb, T beta, T* C, int ldc) {
  for (int o = threadIdx.x; o < M * N; o += blockDim.x) {
    int i = o / N, j = o - (o / N) * N;
    T acc = 0;
    for (int l = 0; l < KD; ++l) acc += (TA ? A[l * lda + i] : A[i * lda + l]) * B[l * ldb + j];
    C[i * ldc + j] = (beta == T(0) ? T(0) : beta * C[i * ldc + j]) + alpha * acc;
  }
}

// Matrix-core tile product for 16 x 16 output tiles (M, N multiples of 16,
// KD a multiple of 4).  Lane layouts of the 16x16x4 instructions (checked on
// gfx950): A fragment lane l = A(l%16, l/16), B fragment = B(l/16, l%16);
// the f64 accumulator holds D(l/16 + 4v, l%16), the f32 one D(4(l/16) + v, l%16).
// Output columns >= nvalid are computed but not stored (B may hold garbage there).
typedef double lrs_d4 __attribute__((ext_vector_type(4)));
typedef float lrs_f4 __attribute__((ext_vector_type(4)));

template <typename T, bool TA>
__device__ inline void gemm_mfma(int M, int N, int KD, T alpha, const T* A, int lda, const T* B,
                                 int ldb, T beta, T* C, int ldc, int nvalid) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int tm = M >> 4, tn = N >> 4;
  const int li = lane & 15, lk = lane >> 4;
  for (int t = wave; t < tm * tn; t += nw) {
    const int i0 = (t / tn) << 4, j0 = (t % tn) << 4;
    if constexpr (sizeof(T) == 8) {
      lrs_d4 acc;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int i = i0 + lk + 4 * v, j = j0 + li;
        acc[v] = (beta == T(0) || j >= nvalid) ? 0.0 : (double)(beta * C[i * ldc + j]);
      }
      for (int k0 = 0; k0 < KD; k0 += 4) {
        int kk = k0 + lk;
        double av = alpha * (TA ? A[kk * lda + i0 + li] : A[(i0 + li) * lda + kk]);
        double bv = B[kk * ldb + j0 + li];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int i = i0 + lk + 4 * v, j = j0 + li;
        if (j < nvalid) C[i * ldc + j] = (T)acc[v];
      }
    } else {
      lrs_f4 acc;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int i = i0 + 4 * lk + v, j = j0 + li;
        acc[v] = (beta == T(0) || j >= nvalid) ? 0.0f : (float)(beta * C[i * ldc + j]);
      }
      for (int k0 = 0; k0 < KD; k0 += 4) {
        int kk = k0 + lk;
        float av = alpha * (TA ? A[kk * lda + i0 + li] : A[(i0 + li) * lda + kk]);
        float bv = B[kk * ldb + j0 + li];
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int i = i0 + 4 * lk + v, j = j0 + li;
        if (j < nvalid) C[i * ldc + j] = (T)acc[v];
      }
    }
  }
}

// One 16x16x4 matrix-core step on a register accumulator tile, and the row
// of accumulator element v held by a lane (column = lane % 16).
template <typename T>
struct AccVec;
template <>
struct AccVec<double> {
  typedef lrs_d4 type;
};
template <>
struct AccVec<float> {
  typedef lrs_f4 type;
};
__device__ __forceinline__ lrs_d4 mfma_step(double a, double b, lrs_d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ lrs_f4 mfma_step(float a, float b, lrs_f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename T>
__device__ __forceinline__ int acc_row(int lane, int v) {
  return sizeof(T) == 8 ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v;
}

// C[M x N] = beta C + alpha op(A) B on LDS tiles.  Uses the matrix cores when
// M and KD allow it; N is padded up to a multiple of 16 (the caller's tiles
// must have room for the padded columns, whose values are ignored).
template <typename T, bool TA>
__device__ inline void gemm(int M, int N, int KD, T alpha, const T* A, int lda,
                            const T* B, int ldb, T beta, T* C, int ldc) {
  if ((M & 15) == 0 && (KD & 3) == 0 && N >= 8)
    gemm_mfma<T, TA>(M, (N + 15) & ~15, KD, alpha, A, lda, B, ldb, beta, C, ldc, N);
  else
    gemm_valu<T, TA>(M, N, KD, alpha, A, lda, B, ldb, beta, C, ldc);
}

// Broadcast lane `l`'s value of v to the whole wave (uniform result).
__device__ __forceinline__ double bcast(double v, int l) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float bcast(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// One column step of the register-resident panel LU; C is a compile-time
// column index so that every register of a[] is addressed statically.
template <typename T, int K, int C>
struct PanelCol {
  static __device__ __forceinline__ void run(T (&a)[K], int lane, bool act, T* P, int ld, int ncols,
                                             T* X, int ldx, int ncx, int* ipiv, int* latch, int part,
                                             int64_t row0, bool& any_swap, T& pmin) {
    if constexpr (C < K) {
      T d = bcast(a[C], C);
      const bool beats = act && lane > C && fabs(a[C]) > fabs(d);
      int piv = C;
      if (__any(beats)) {
        // full argmax (first maximum) over rows C .. nr-1
        T bv = (act && lane >= C) ? fabs(a[C]) : T(-1);
        int bi = lane;
        for (int off = 32; off >= 1; off >>= 1) {
          T ov = __shfl_xor(bv, off);
          int oi = __shfl_xor(bi, off);
          if (ov > bv || (ov == bv && oi < bi)) {
            bv = ov;
            bi = oi;
          }
        }
        piv = __builtin_amdgcn_readfirstlane(bi);
      }
      if (lane == 0) ipiv[C] = piv;
      if (piv != C) {
        any_swap = true;
#pragma unroll
        for (int jj = 0; jj < K; ++jj) {
          T vc = bcast(a[jj], C), vp = bcast(a[jj], piv);
          if (lane == C) a[jj] = vp;
          if (lane == piv) a[jj] = vc;
        }
        for (int col = K + lane; col < ncols; col += 64) {
          T t = P[C * ld + col];
          P[C * ld + col] = P[piv * ld + col];
          P[piv * ld + col] = t;
        }
        for (int col = lane; col < ncx; col += 64) {
          T t = X[C * ldx + col];
          X[C * ldx + col] = X[piv * ldx + col];
          X[piv * ldx + col] = t;
        }
        d = bcast(a[C], C);
      }
      // an exactly zero pivot, or a non-finite one (Inf/NaN in the band reach
      // some pivot of the elimination), is latched with its row
      if (lane == 0) {
        if (d == T(0))
          latch_error(latch, 1, part, row0 + C);
        else if (!isfinite(d))
          latch_error(latch, 4, part, row0 + C);
      }
      if (row0 + C >= 0) pmin = fmin(pmin, fabs(d));  // not the unit pivots of virtual rows
      const bool below = act && lane > C;
      const T inv = T(1) / d;
      const T l = a[C] * inv;
      if (below) a[C] = l;
#pragma unroll
      for (int jj = C + 1; jj < K; ++jj) {
        const T pj = bcast(a[jj], C);
        if (below) a[jj] -= l * pj;
      }
      PanelCol<T, K, C + 1>::run(a, lane, act, P, ld, ncols, X, ldx, ncx, ipiv, latch, part, row0, any_swap, pmin);
    }
  }
};

// Register-resident partial-pivoting LU of an nr x K panel (nr <= 64) by ONE
// wave (call from all lanes of a single wave; no workgroup barrier inside).
// Lane q holds panel row q.  The pivot of column c is the first row of
// largest magnitude among rows c .. nr-1; the common case (no row beats the
// diagonal) is detected with one vote and costs no reduction.  Interchanges
// move the panel registers and, in LDS, columns K..ncols-1 of P and the first
// ncx columns of X.  On exit the panel (unit L strictly below the diagonal,
// U on and above) is written back to P.  Multipliers are formed as a * (1/d).
// Branch-free elimination step without interchanges (compile-time column C);
// records the largest multiplier magnitude of the lane in mx.
template <typename T, int K, int C>
struct PanelColNoPiv {
  static __device__ __forceinline__ void run(T (&a)[K], int lane, bool act, T& mx, T& dmin, int64_t row0) {
    if constexpr (C < K) {
      const T d = bcast(a[C], C);
      const T inv = T(1) / d;
      const bool below = act && lane > C;
      const T l = below ? a[C] * inv : T(0);
      // sticky on NaN (an Inf pivot counts as NaN): a non-finite panel fails
      // the no-interchange test and goes to the pivoting pass, which latches it
      const T al = fabs(l), ad = fabs(d), adc = ad <= std::numeric_limits<T>::max() ? ad : T(NAN);
      mx = (mx != mx || mx >= al) ? mx : al;
      if (row0 + C >= 0) dmin = (dmin != dmin || dmin <= adc) ? dmin : adc;
      if (below) a[C] = l;
#pragma unroll
      for (int jj = C + 1; jj < K; ++jj) a[jj] -= l * bcast(a[jj], C);
      PanelColNoPiv<T, K, C + 1>::run(a, lane, act, mx, dmin, row0);
    }
  }
};

template <typename T, int K>
// pmin: running min |pivot| (updated, uniform over the wave).
__device__ inline bool panel_lu_wave(T* P, int ld, int nr, int ncols, T* X, int ldx, int ncx,
                                     int* ipiv, int* latch, int part, int64_t row0, T& pmin) {
  const int lane = threadIdx.x & 63;
  const bool act = lane < nr;
  T a[K];
#pragma unroll
  for (int c = 0; c < K; ++c) a[c] = act ? P[lane * ld + c] : T(0);
  // Optimistic pass: elimination without interchanges.  Partial pivoting
  // interchanges at column c exactly when some row below has |a_rc| > |a_cc|,
  // i.e. when a multiplier exceeds 1 in magnitude; if none does, this IS the
  // partial-pivoting factorization (same operations, same order).
  T mx = T(0), dmin = T(INFINITY);
  PanelColNoPiv<T, K, 0>::run(a, lane, act, mx, dmin, row0);
  const bool ok = !__any(!(mx <= T(1))) && __all(dmin > T(0));
  if (ok) {
    if (lane < K) ipiv[lane] = lane;
    pmin = fmin(pmin, dmin);
#pragma unroll
    for (int c = 0; c < K; ++c)
      if (act) P[lane * ld + c] = a[c];
    return false;
  }
#pragma unroll
  for (int c = 0; c < K; ++c) a[c] = act ? P[lane * ld + c] : T(0);
  bool any_swap = false;
  PanelCol<T, K, 0>::run(a, lane, act, P, ld, ncols, X, ldx, ncx, ipiv, latch, part, row0, any_swap, pmin);
#pragma unroll
  for (int c = 0; c < K; ++c)
    if (act) P[lane * ld + c] = a[c];
  return any_swap;
}

// Register-resident triangular inverses by single waves: lane j computes
// column j, column-oriented (each step's updates are independent):
//   lower:  x = e_j;  for l: x_i -= L[i][l] x_l  (i > l)            -> (unit L)^{-1} e_j
//   upper:  x = e_j;  for l desc: x_l /= U[l][l]; x_i -= U[i][l] x_l (i < l) -> U^{-1} e_j
template <typename T, int K, int Lc>
struct InvLowerCol {
  static __device__ __forceinline__ void run(const T* L, int ldl, T (&x)[K]) {
    if constexpr (Lc < K) {
#pragma unroll
      for (int i = Lc + 1; i < K; ++i) x[i] -= L[i * ldl + Lc] * x[Lc];
      InvLowerCol<T, K, Lc + 1>::run(L, ldl, x);
    }
  }
};
template <typename T, int K, int Lc>
struct InvUpperCol {  // Lc counts down
  static __device__ __forceinline__ void run(const T* U, int ldu, T (&x)[K], const T* dinv) {
    if constexpr (Lc >= 0) {
      x[Lc] *= dinv[Lc];
#pragma unroll
      for (int i = 0; i < Lc; ++i) x[i] -= U[i * ldu + Lc] * x[Lc];
      InvUpperCol<T, K, Lc - 1>::run(U, ldu, x, dinv);
    }
  }
};

template <typename T, int K>
__device__ inline void tri_inv_lower_wave(const T* L, int ldl, T* Li, int ldli) {
  const int j = threadIdx.x & 63;
  T x[K];
#pragma unroll
  for (int i = 0; i < K; ++i) x[i] = (i == j) ? T(1) : T(0);
  InvLowerCol<T, K, 0>::run(L, ldl, x);
  if (j < K)
#pragma unroll
    for (int i = 0; i < K; ++i) Li[i * ldli + j] = x[i];
}

// dinv: K reciprocals of the diagonal of U (LDS or registers visible to the wave)
template <typename T, int K>
__device__ inline void tri_inv_upper_wave(const T* U, int ldu, T* Ui, int ldui, T* dinv) {
  const int j = threadIdx.x & 63;
  if (j < K) dinv[j] = T(1) / U[j * ldu + j];
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  T x[K];
#pragma unroll
  for (int i = 0; i < K; ++i) x[i] = (i == j) ? T(1) : T(0);
  InvUpperCol<T, K, K - 1>::run(U, ldu, x, dinv);
  if (j < K)
#pragma unroll
    for (int i = 0; i < K; ++i) Ui[i * ldui + j] = x[i];
}

// Inverse of the unit lower triangle of L (K x K, pitch ldl) into Li (strictly
// lower part; upper part and diagonal set to 0 / 1), and inverse of the upper
// triangle of U (pitch ldu) into Ui (lower part 0).  Column j of each inverse
// is one forward / backward substitution; 2K threads work at once.
template <typename T, int K>
__device__ inline void tri_inverses(const T* L, int ldl, const T* U, int ldu, T* Li, int ldli,
                                    T* Ui, int ldui) {
  const int tid = threadIdx.x;
  if (tid < K) {
    const int j = tid;  // column j of L^{-1}: x_i = -sum_{j<=l<i} L[i][l] x_l, x_j = 1
    for (int i = 0; i < K; ++i) {
      T x;
      if (i < j)
        x = 0;
      else if (i == j)
        x = 1;
      else {
        T acc = 0;
        for (int l = j; l < i; ++l) acc += L[i * ldl + l] * Li[l * ldli + j];
        x = -acc;
      }
      Li[i * ldli + j] = x;
    }
  } else if (tid < 2 * K) {
    const int j = tid - K;  // column j of U^{-1}
    for (int i = K - 1; i >= 0; --i) {
      T x;
      if (i > j)
        x = 0;
      else {
        T acc = (i == j) ? T(1) : T(0);
        for (int l = i + 1; l <= j; ++l) acc -= U[i * ldu + l] * Ui[l * ldui + j];
        x = acc / U[i * ldu + i];
      }
      Ui[i * ldui + j] = x;
    }
  }
}

// Compose the interchanges ipiv[0..K) of a 2K (or K) row window into a gather
// permutation: row q of the permuted window is row perm[q] of the original.
__device__ inline void compose_perm(const int* ipiv, int K, int nr, int* perm) {
  for (int q = 0; q < nr; ++q) perm[q] = q;
  for (int c = 0; c < K; ++c) {
    int t = perm[c];
    perm[c] = perm[ipiv[c]];
    perm[ipiv[c]] = t;
  }
}

}  // namespace lrs
