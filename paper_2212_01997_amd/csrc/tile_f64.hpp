// The FP64 tile product shared by the response and the purification kernels:
// one TMxTM block of A^T diag(h) B for column-major n x n operands on the
// four-block 4x4x4 FP64 MFMA of gfx950.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace gq {

// v_mfma_f64_4x4x4f64 on gfx950 (four blocks per instruction): lane l supplies
// A_b(l%4, l/16) and B_b(l/16, l%4) of block b = (l/4)%4 and receives
// D_b(l/16, l%4).  With the four blocks side by side along the columns, one
// instruction yields a 4x16 strip: A (4 rows x 4 deep) is shared by the four
// blocks, B is the 4 x 16 slice, and lane l holds row l/16, column l%16.
__device__ __forceinline__ double mfma4b(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

// The TMxTM block X(k0.., l0..) of one subgraph (columns k >= kend or l >= lend
// read as zero) on the four-block 4x4x4 FP64 MFMA.  Wave w owns rows [w TM/4, (w+1) TM/4) and
// all TM columns: TM/16 x TM/16 independent accumulators, lane l holding row
// w TM/4 + 4 r + l/16 (xy_row(r, w) + l/16), column 16 c + l%16 in acc[r][c].  The K dimension is
// staged through LDS in chunks of kXK rows, stored [m][column] with a row
// stride of TM + 1 doubles: each group of 16 lanes then touches 16 distinct
// 8-byte bank pairs in the staging writes (16 consecutive m) and in the B reads
// (16 consecutive columns), and 4 broadcast addresses in the A reads.  h(m) is
// applied to the B side while staging.
//
// In general the block is sum_m A(m, k) h(m) B(m, l) with A and B column-major
// n x n: A = B = Q for a diagonal perturbation (H = true), or without h for
// the general kind, where W = h1_s Q is formed as G^T Q (G = h1_s, symmetric)
// and X as Q^T W.
//
// DIAG: a block on the diagonal (k0 = l0) of which only the lower triangle
// (k >= l) is wanted.  The TM rows are cut into strips of 4; strip s needs the
// 16-column blocks c <= s/4.  Wave w takes the strips 8 (r/2) + (r odd ?
// 7 - w : w) for r = 0 .. TM/16 - 1, which need exactly the blocks c <= r, so
// every wave runs (R4 (R4 + 1) / 2) of the R4^2 products (10 of 16 for
// TM = 64) and the waves stay balanced.  Each element is still the same sum
// in the same order, so its bits do not depend on DIAG.  xy_row gives the
// first row of sub-strip r in either mode.
template <int TM, bool DIAG>
__device__ __forceinline__ int xy_row(int r, int w) {
  if constexpr (DIAG) return 4 * (8 * (r >> 1) + ((r & 1) ? 7 - w : w));
  else return w * (TM / 4) + 4 * r;
}

template <int TM, bool H, bool DIAG = false>
__device__ __forceinline__ void xy_block_4b(const double* __restrict__ Am,
                                            const double* __restrict__ Bm,
                                            const double* __restrict__ hl, int n, int k0, int l0,
                                            int kend, int lend, double (&acc)[TM / 16][TM / 16]) {
  constexpr int kXK = 16;  // FP64 K chunk: 16 rows keep four workgroups per CU
  constexpr int kNT = 256, LD = TM + 1, R4 = TM / 16, C16 = TM / 16;
  constexpr int kPer = kXK * TM / kNT;
  __shared__ double As[kXK][LD];
  __shared__ double Bs[kXK][LD];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lq = lane & 3, lr = lane >> 4, l15 = lane & 15;
  const int mm_t = tid & (kXK - 1), c_t = tid / kXK;
  double pa[kPer], pb[kPer];
  // out-of-range elements load a clamped (valid) address; the zeroing and the
  // h factor are applied when the registers are written to LDS, after the
  // MFMAs of the current chunk, so the loads stay in flight across them
  double ph = 0.0;
  auto fetch = [&](int m0) {
    const int mc = min(m0 + mm_t, n - 1);
    if constexpr (H) ph = hl[mc];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int c = c_t + u * (kNT / kXK);
      pa[u] = Am[mc + (size_t)n * min(k0 + c, n - 1)];
      pb[u] = Bm[mc + (size_t)n * min(l0 + c, n - 1)];
    }
  };
#pragma unroll
  for (int r = 0; r < R4; ++r)
#pragma unroll
    for (int c = 0; c < C16; ++c) acc[r][c] = 0.0;
  fetch(0);
  for (int m0 = 0; m0 < n; m0 += kXK) {
    __syncthreads();
    const bool okm = m0 + mm_t < n;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int c = c_t + u * (kNT / kXK);
      As[mm_t][c] = (okm && k0 + c < kend) ? pa[u] : 0.0;
      if constexpr (H) Bs[mm_t][c] = (okm && l0 + c < lend) ? ph * pb[u] : 0.0;
      else Bs[mm_t][c] = (okm && l0 + c < lend) ? pb[u] : 0.0;
    }
    __syncthreads();
    if (m0 + kXK < n) fetch(m0 + kXK);
#pragma unroll
    for (int ks = 0; ks < kXK / 4; ++ks) {
      const int mm = 4 * ks + lr;
      double a[R4], bb[C16];
#pragma unroll
      for (int r = 0; r < R4; ++r) a[r] = As[mm][xy_row<TM, DIAG>(r, w) + lq];
#pragma unroll
      for (int c = 0; c < C16; ++c) bb[c] = Bs[mm][16 * c + l15];
#pragma unroll
      for (int r = 0; r < R4; ++r)
#pragma unroll
        for (int c = 0; c < C16; ++c)
          if (!DIAG || c <= r) acc[r][c] = mfma4b(a[r], bb[c], acc[r][c]);
    }
  }
}

}  // namespace gq
