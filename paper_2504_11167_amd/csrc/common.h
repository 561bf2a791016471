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
// Device error latch: the first error wins (code, partition, row).
// Layout: int32 [0] = code, [1] = partition, int64 at [2..3] = row.
// ------------------------------------------------------------------------
__device__ inline void latch_error(int* latch, int code, int part, int64_t row) {
  if (atomicCAS(latch, 0, code) == 0) {
    latch[1] = part;
    reinterpret_cast<int64_t*>(latch + 2)[0] = row;
  }
}

// ------------------------------------------------------------------------
// LDS block GEMM, whole workgroup:  C[M x N] = beta * C + alpha * op(A) B
//   op(A)(i, l) = TA ? A[l * lda + i] : A[i * lda + l]      (M x KD)
//   B(l, j) = B[l * ldb + j]                                  (KD x N)
// C must not alias A or B.  No barrier inside; the caller synchronizes.
// ------------------------------------------------------------------------
template <typename T, bool TA>
__device__ inline void gemm(int M, int N, int KD, T alpha, const T* A, int lda,
                            const T* B, int ldb, T beta, T* C, int ldc) {
  for (int o = threadIdx.x; o < M * N; o += blockDim.x) {
    int i = o / N, j = o - (o / N) * N;
    T acc = 0;
    for (int l = 0; l < KD; ++l) acc += (TA ? A[l * lda + i] : A[i * lda + l]) * B[l * ldb + j];
    C[i * ldc + j] = (beta == T(0) ? T(0) : beta * C[i * ldc + j]) + alpha * acc;
  }
}

// ------------------------------------------------------------------------
// Partial-pivoting LU of an nr x K panel held in LDS (row pitch ld), nr in
// {K, 2K}, nr <= 64: the pivot of column c is the first row of largest
// magnitude among rows c .. nr-1 (first-max tie-break).  Interchanges move
// whole rows: the first ncols columns of P (the panel and the block columns
// to its right) and the first ncx columns of X (right-hand sides riding
// along), so on exit the panel holds L (unit, strictly below the diagonal, in
// final row order) and U.  ipiv[c] = row swapped with c.
// Returns (uniformly) whether any interchange happened.  A zero pivot is
// latched with the partition-local row `row0 + c` and the factorization
// continues (the result is then non-finite).
// ------------------------------------------------------------------------
template <typename T, int K>
__device__ inline bool panel_lu(T* P, int ld, int nr, int ncols, T* X, int ldx, int ncx,
                                int* ipiv, int* latch, int part, int64_t row0, int* s_flag) {
  const int tid = threadIdx.x;
  if (tid == 0) *s_flag = 0;
  __syncthreads();
  for (int c = 0; c < K; ++c) {
    if (tid < 64) {
      // wave 0: argmax over candidate rows (value, index), first max wins ties
      T v = (tid >= c && tid < nr) ? fabs(P[tid * ld + c]) : T(-1);
      int idx = tid;
      for (int off = 32; off >= 1; off >>= 1) {
        T ov = __shfl_xor(v, off);
        int oi = __shfl_xor(idx, off);
        if (ov > v || (ov == v && oi < idx)) {
          v = ov;
          idx = oi;
        }
      }
      if (tid == 0) {
        ipiv[c] = idx;
        if (idx != c) *s_flag = 1;
      }
    }
    __syncthreads();
    const int piv = ipiv[c];
    if (piv != c) {
      for (int col = tid; col < ncols; col += blockDim.x) {
        T t = P[c * ld + col];
        P[c * ld + col] = P[piv * ld + col];
        P[piv * ld + col] = t;
      }
      for (int col = tid; col < ncx; col += blockDim.x) {
        T t = X[c * ldx + col];
        X[c * ldx + col] = X[piv * ldx + col];
        X[piv * ldx + col] = t;
      }
      __syncthreads();
    }
    const T d = P[c * ld + c];
    if (d == T(0)) {
      if (tid == 0) latch_error(latch, 1, part, row0 + c);
    }
    // multipliers
    for (int r = c + 1 + tid; r < nr; r += blockDim.x) P[r * ld + c] = P[r * ld + c] / d;
    __syncthreads();
    const int w = K - c - 1;
    for (int o = tid; o < (nr - c - 1) * w; o += blockDim.x) {
      int r = c + 1 + o / w, col = c + 1 + o % w;
      P[r * ld + col] -= P[r * ld + c] * P[c * ld + col];
    }
    __syncthreads();
  }
  return *s_flag != 0;
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
