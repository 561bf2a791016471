// Workspace layout of a plan (host and device).  All offsets are bytes from
// the workspace base, 256-byte aligned.  T is the factor element type (double
// for FP64 plans, float for FP32_REFINED plans); the tips, the reduced system
// and all solve vectors are double.
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace lrs {

struct Layout {
  int64_t n;
  // partition j covers rows [offs[j], offs[j+1]) when offs (device, p + 1
  // entries) is set; otherwise the uniform rule floor(n/p) + [j < n mod p]
  const int64_t* offs;
  int k, K, p, r, R2, nbmax, mmax, tsize;  // r: compressed rank (K when the user's r = k)
  int refined;  // iterative refinement around the solve (residual, correction and norm buffers)
  int variant;  // reduced system: 0 = the whole block-tridiagonal Z, 1 = its diagonal blocks only (LR-SPIKE-T),
                // 2 = LR-SPIKE-I and 3 = LR-SPIKE-OTF (iterative, preconditioned by the variant-1 system)
  int ell;      // randomized spike SVD: sketch columns per spike (0 = exact truncation of the whole spike)
  // systems a plan holds (1, or the systems of a batched group) and, per
  // partition, the system slot it belongs to (device; null = all in slot 0):
  // refinement norms are kept per (system, column)
  int nsys;
  const int* psys;
  int NI;       // interfaces p - 1
  int levels;   // cyclic-reduction levels (ceil(log2(NI)))
  int lvl_off[32];  // first slot of each level in the F/E arrays
  int nfe;      // total slots
  // per block records (T): LP (K*K) | UP (K*K) | UD (K)  ->  rec elements
  int64_t rec;
  size_t fac, swx, gmat, ymat, ipiv, flag;
  // per partition (double): tips Vt,Vb,Wt,Wb (4 K*K), Grams GV,GW (2 K*K),
  // projectors Pi,Psi (2 K*r) and projected tips Pt,Pb,Qt,Qb (4 K*r)
  size_t tips, gram, proj, ptip;
  // reduced system (double): current D [NI][R2][R2], LU [NI][R2][R2], pivots int [NI][R2],
  // F/E per (level, active row) [nfe][2][R2][R2], scratch X [NI][2][R2][R2]
  size_t zD, zLU, zpiv, zFE, zX;
  // solve vectors (double): y tips [p][2][K][mmax], compressed rhs [NI][R2][mmax],
  // scratch n x mmax (adjoint D-stage), refinement copy of f and residual n x mmax,
  // norms [nsys][mmax][2]
  size_t ytip, zg, scr, fcopy, res, norms;
  // BiCGStab (refined == 2): vectors rh, p, v, ph, s, sh, t (n x mmax each),
  // per-column scalars [mmax][BICG_SCALARS] and per-workgroup partial inner
  // products [bblk][mmax][3] (bblk workgroups cover the rows)
  size_t bvec, bsc, bpart;
  int bblk;
  // randomized spike SVD (ell > 0): sketch Y (n x 2 ell, the V_j sketch in
  // columns [0, ell), W_j's in [ell, 2 ell)), its Grams Y^T Y [p][2][ell][ell]
  // and the products V^T Y, W^T Y [p][2][k][ell]
  size_t ysk, rgy, rmv;
  // iterative reduced solves (variant >= 2): ten tip vectors [p][2][K][mmax]
  // (b, x, r, rh, p, v, ph, s, sh, t), per-column scalars [mmax][BICG_SCALARS]
  // and partial inner products [iblk][mmax][3]
  size_t itv, isc, ipart;
  int iblk;
  size_t npv;    // int32[p]: partition needs the interchanging factorization
  size_t latch;  // device state block (STATE_BYTES): error latch, diagnostics, refinement control
  size_t total;
};

// Device state block at L.latch, int32 slots (doubles at even int indices):
//   error latch: code, partition, partition-local row (int64)
//   counters and refinement control
//   diagnostics kept by atomic min / max on the bit patterns of non-negative
//   doubles (ordered like the values), initialised to +inf (min) or 0 (max)
constexpr int STATE_INTS = 64;
constexpr int BICG_SCALARS = 12;  // per-column scalars of the BiCGStab iteration
constexpr size_t STATE_BYTES = STATE_INTS * 4;
enum StateSlot {
  S_CODE = 0, S_PART = 1, S_ROW = 2,  // S_ROW: int64 over slots 2, 3
  S_SWAPPED = 8,                      // k-row blocks that interchanged rows
  S_STOP = 9,                         // refinement: nonzero = no further correction runs
  S_ITERS = 10,                       // refinement: corrections applied
  S_RSTATE = 11,                      // refinement: 0 running, 1 converged, 2 failed
  S_PIVMIN = 16,                      // double: min |pivot| of the partition LUs
  S_AMAX = 18,                        // double: max |a_ij| over the band entries read
  S_GAPMIN = 20,                      // double: min (sigma_r - sigma_{r+1}) / sigma_1 over the truncated spikes
  S_ZMAX = 22,                        // double: max |entry| of the reduced system Z
  S_ZGROW = 24,                       // double: max |entry| of its eliminated blocks (cyclic reduction)
  S_CORR = 26,                        // double: last correction  max_c ||d_c|| / ||x_c||
  S_CPREV = 28                        // double: the correction before it
};

inline size_t lrs_align(size_t x) { return (x + 255) & ~(size_t)255; }

inline int kernel_K(int k) {
  int K = 1;
  while (K < k) K <<= 1;
  return K;
}

// offs_host / offs_dev: explicit partition offsets (p + 1 entries, host and
// device copies) or null for the uniform partition rule
// refined: the plan iterates the solve: 1 = iterative refinement (residual and
// correction buffers), 2 = BiCGStab (also its vectors, scalars and partials);
// variant: 0 = LR-SPIKE with the whole reduced system, 1 = its truncated form;
// nsys / psys: systems held and the partition -> system slot map (batches);
// ell: sketch columns of the randomized spike SVD (0: exact truncation), which
// also needs 2 ell solve columns (the sketch passes run as solves)
inline void make_layout(Layout& L, int64_t n, int k, int p, int r, int tsize, int mmax, int refined = 0,
                        int variant = 0, const int64_t* offs_host = nullptr, const int64_t* offs_dev = nullptr,
                        int nsys = 1, const int* psys = nullptr, int ell = 0) {
  if (ell > 0 && mmax < 2 * ell) mmax = 2 * ell;
  L.ell = ell;
  L.n = n;
  L.offs = offs_dev;
  L.refined = refined;
  L.variant = variant;
  L.nsys = nsys;
  L.psys = psys;
  L.k = k;
  L.K = kernel_K(k);
  L.p = p;
  // r = k keeps the spikes whole: with K > k the padded spikes have K - k zero
  // columns (the last ones for V, the first ones for W), so exactness needs the
  // full K-wide identity projector rather than the first k columns.
  L.r = (r == k) ? kernel_K(k) : r;
  L.R2 = 2 * L.r;
  L.tsize = tsize;
  L.mmax = mmax;
  const int K = L.K;
  int64_t njmax = (n + p - 1) / p;
  if (offs_host) {
    njmax = 0;
    for (int j = 0; j < p; ++j)
      if (offs_host[j + 1] - offs_host[j] > njmax) njmax = offs_host[j + 1] - offs_host[j];
  }
  L.nbmax = (int)((njmax + K - 1) / K);
  L.NI = p - 1;
  L.levels = 0;
  while ((1 << L.levels) < L.NI) ++L.levels;
  int off = 0;
  for (int l = 0; l <= L.levels; ++l) {
    L.lvl_off[l] = off;
    int s = 1 << l;
    off += (L.NI + s - 1) / s;
  }
  L.nfe = off;
  L.rec = 2 * (int64_t)K * K + K;
  size_t o = 0;
  const size_t nblk = (size_t)p * L.nbmax;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = lrs_align(o + bytes);
    return at;
  };
  L.fac = take(nblk * L.rec * tsize);
  L.swx = take(nblk * 3 * (size_t)K * K * tsize);
  L.gmat = take(nblk * (size_t)K * K * tsize);
  // (kept with the randomized SVD too: the interchanging factorization kernel
  // still forms the spikes of the partitions it refactors)
  L.ymat = take(L.r < K ? nblk * 2 * (size_t)K * K * tsize : 0);
  L.ipiv = take(nblk * (size_t)K * 4);
  L.flag = take(nblk * 4);
  L.tips = take((size_t)p * 4 * K * K * 8);
  L.gram = take((size_t)p * 2 * K * K * 8);
  L.proj = take((size_t)p * 2 * K * L.r * 8);
  L.ptip = take((size_t)p * 4 * K * L.r * 8);
  const size_t R2 = L.R2, NI = L.NI > 0 ? L.NI : 0;
  L.zD = take(NI * R2 * R2 * 8);
  L.zLU = take(NI * R2 * R2 * 8);
  L.zpiv = take(NI * R2 * 4);
  L.zFE = take((size_t)L.nfe * 2 * R2 * R2 * 8);
  L.zX = take(NI * 2 * R2 * R2 * 8);
  L.ytip = take((size_t)p * 2 * K * mmax * 8);
  L.zg = take(NI * R2 * mmax * 8);
  L.scr = take((size_t)n * mmax * 8);
  L.fcopy = take(refined ? (size_t)n * mmax * 8 : 0);
  L.res = take(refined ? (size_t)n * mmax * 8 : 0);  // residual / correction (refinement)
  L.norms = take((size_t)2 * nsys * mmax * 8 + 64);
  {
    const int64_t blocks = (n + 2047) / 2048;
    L.bblk = (int)(blocks < 4096 ? blocks : 4096);
  }
  L.bvec = take(refined == 2 ? (size_t)7 * n * mmax * 8 : 0);
  L.bsc = take(refined == 2 ? (size_t)mmax * BICG_SCALARS * 8 : 0);
  L.bpart = take(refined == 2 ? (size_t)L.bblk * mmax * 3 * 8 : 0);
  L.ysk = take(ell > 0 ? (size_t)n * 2 * ell * 8 : 0);
  L.rgy = take(ell > 0 ? (size_t)p * 2 * ell * ell * 8 : 0);
  L.rmv = take(ell > 0 ? (size_t)p * 2 * k * ell * 8 : 0);
  {
    const int64_t rows = (int64_t)2 * K * p, blocks = (rows + 2047) / 2048;
    L.iblk = (int)(blocks < 4096 ? blocks : 4096);
    const bool it = variant >= 2;
    L.itv = take(it ? (size_t)10 * rows * mmax * 8 : 0);
    L.isc = take(it ? (size_t)mmax * BICG_SCALARS * 8 : 0);
    L.ipart = take(it ? (size_t)L.iblk * mmax * 3 * 8 : 0);
  }
  L.npv = take((size_t)p * 4);
  L.latch = take(STATE_BYTES);
  L.total = o;
}

}  // namespace lrs
