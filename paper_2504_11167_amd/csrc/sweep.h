// Block sweeps over the packed partition factors (one workgroup per partition
// and per chunk of at most MC right-hand-side columns).
//
// Forward (L^{-1} P^T, top -> bottom), per block b, on the 2K-row window
// [r_b; r_{b+1}]:  interchange rows as the factorization did, z_b = L11^{-1} r_b,
// r_{b+1} -= L21 z_b.
// Backward (U^{-1}, bottom -> top): x_b = U11^{-1} (z_b - U12 x_{b+1} - U13 x_{b+2}).
// Transposed forward (U^{-T}, top -> bottom) and transposed backward
// (P L^{-T}, bottom -> top) apply the exact transposes of those block steps
// in reverse order.
#pragma once
#include "common.h"
#include "layout.h"

namespace lrs {

constexpr int MC = 32;  // right-hand-side columns per workgroup (K <= 32)
// columns per workgroup of the generic sweeps: 16 at K = 64, so that the
// three K x K factor blocks and the strips fit in LDS (157 KB in FP64) and a
// strip is one matrix-core tile wide
template <int K>
constexpr int mc_of() { return K <= 32 ? MC : 16; }

template <typename T>
__device__ inline T* wsp(char* ws, size_t off) {
  return reinterpret_cast<T*>(ws + off);
}

// Load the K x K forward factors of block b: Li (unit lower L11^{-1}) and L21.
// Block flags: bit 0 = the block interchanged rows (full L21 and U13 in the
// side slots), bit 1 = U12 is full (side slot) because of fill from an
// interchange in this or the previous block.
template <typename T, int K>
__device__ inline void load_lfac(const T* rec, const T* sx, int fl, bool last, T* Li, T* L21) {
  const bool sw = (fl & 1) != 0;
  constexpr int LDK = K + 1;
  for (int o = threadIdx.x; o < K * K; o += blockDim.x) {
    int i = o / K, c = o % K;
    const int fo = fidx<T, K>(i, c);
    T lp = rec[fo];
    Li[i * LDK + c] = (i > c) ? lp : (i == c ? T(1) : T(0));
    T l21;
    if (last)
      l21 = T(0);
    else if (sw)
      l21 = sx[fo];
    else
      l21 = (i <= c) ? lp : T(0);
    L21[i * LDK + c] = l21;
  }
}

// Load the backward factors of block b: Ui (U11^{-1}), U12, U13.
template <typename T, int K>
__device__ inline void load_ufac(const T* rec, const T* sx, int fl, bool last, T* Ui, T* U12,
                                 T* U13) {
  constexpr int LDK = K + 1;
  for (int o = threadIdx.x; o < K * K; o += blockDim.x) {
    int i = o / K, c = o % K;
    const int fo = fidx<T, K>(i, c);
    T up = rec[K * K + fo];
    Ui[i * LDK + c] = (i <= c) ? up : T(0);
    T u12 = T(0), u13 = T(0);
    if (!last) {
      if (fl & 2)
        u12 = sx[K * K + fo];
      else
        u12 = (i > c) ? up : (i == c ? rec[2 * K * K + i] : T(0));
      if (fl & 1) u13 = sx[2 * K * K + fo];
    }
    U12[i * LDK + c] = u12;
    U13[i * LDK + c] = u13;
  }
}

// Apply the interchanges of block b (ipiv, K entries) to the first nr rows of
// the window W (pitch ldw, mc columns) in place, using tmp (nr x ldw) and perm.
template <typename T, int K>
__device__ inline void permute_rows(T* W, int ldw, int nr, int mc, const int* ipiv_g, int* s_perm,
                                    T* tmp) {
  if (threadIdx.x == 0) {
    for (int q = 0; q < nr; ++q) s_perm[q] = q;
    for (int c = 0; c < K; ++c) {
      int pv = ipiv_g[c];
      int t = s_perm[c];
      s_perm[c] = s_perm[pv];
      s_perm[pv] = t;
    }
  }
  __syncthreads();
  for (int o = threadIdx.x; o < nr * mc; o += blockDim.x) {
    int q = o / mc, c = o % mc;
    tmp[q * ldw + c] = W[s_perm[q] * ldw + c];
  }
  __syncthreads();
  for (int o = threadIdx.x; o < nr * mc; o += blockDim.x) {
    int q = o / mc, c = o % mc;
    W[q * ldw + c] = tmp[q * ldw + c];
  }
  __syncthreads();
}

// Transposed interchanges: the swaps of block b applied in reverse order.
template <typename T, int K>
__device__ inline void permute_rows_t(T* W, int ldw, int nr, int mc, const int* ipiv_g, int* s_perm,
                                      T* tmp) {
  if (threadIdx.x == 0) {
    // gather form of the inverse permutation
    int fw[2 * K];
    for (int q = 0; q < nr; ++q) fw[q] = q;
    for (int c = 0; c < K; ++c) {
      int pv = ipiv_g[c];
      int t = fw[c];
      fw[c] = fw[pv];
      fw[pv] = t;
    }
    for (int q = 0; q < nr; ++q) s_perm[fw[q]] = q;
  }
  __syncthreads();
  for (int o = threadIdx.x; o < nr * mc; o += blockDim.x) {
    int q = o / mc, c = o % mc;
    tmp[q * ldw + c] = W[s_perm[q] * ldw + c];
  }
  __syncthreads();
  for (int o = threadIdx.x; o < nr * mc; o += blockDim.x) {
    int q = o / mc, c = o % mc;
    W[q * ldw + c] = tmp[q * ldw + c];
  }
  __syncthreads();
}

}  // namespace lrs
