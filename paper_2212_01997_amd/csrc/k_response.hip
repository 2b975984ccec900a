// Canonical first-order response in the eigenbasis and the collect step.
//
// Sec. IV.A: for a perturbation H1 the fixed-mu response of each subgraph is
// the Frechet derivative of the Fermi function, which in the eigenbasis reads
//   d1lambda = Q [(Q^T h1 Q) o dF] Q^T,
// the mu response is beta d0 (I - d0) (Eq. (dddmu)), and Eq. (dmu_1) fixes
//   mu1 = -sum_i Tr_c d1lambda_i / sum_i Tr_c d1mu_i,
// so that the collected rho1 = 2 (d1lambda + mu1 d1mu) core rows has zero trace
// (Eq. (D1)).  Every kernel takes all K perturbations of a call in one launch
// (grid dimension q):
//   k_xy       lower-triangular tiles of X = Q^T diag(h1) Q, times dF, into Y
//              (each symmetric pair stored once).  Subgraphs are binned by
//              size; per bin the tile shape (64x64 or 32x32, four waves each)
//              and the grid (one workgroup per tile or a persistent grid) are
//              chosen by gq_autotune.  Tiles of one subgraph stay on
//              one XCD, whose L2 then serves their shared columns of Q.
//              FP64 on the four-block 4x4x4 MFMA, or in the split-FP32
//              variant the FP32 leading part of Q on FP32 MFMA (FP32 sums
//              within 32-deep chunks, FP64 across them); k_xy_kq takes two
//              perturbations per workgroup, sharing the staged columns of Q,
//              when K > 1.  The split variant is followed by
//   k_win      one FP64 correction of the thermal-window block, where dF
//              amplifies rounding most
//   k_t_mfma   T = Q_c Y;  k_p_mfma  P = 2 T Q^T (c x n core rows) and diag(P)
//   k_mu1      fixed-order traces -> mu1_q
//   k_combine  P += mu1_q M
// Eq. (sub_f) / (dCollect): k_assemble scatters block rows into CSR values.
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <mutex>

#include "gq_internal.hpp"
#include "tile_f64.hpp"

namespace gq {

namespace {

constexpr int kThreads = 256;
constexpr int kTile = 64;  // the storage rule of Y is defined on 64x64 tiles

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// ---------------------------------------------------------------- FP64 MFMA
// v_mfma_f64_16x16x4f64 on gfx950: lane l supplies A(l%16, l/16) and
// B(l/16, l%16); D(i, j) is returned in lane j + 16*(i%4), register i/4.
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// v_mfma_f32_16x16x4f32 on gfx950: same operand lanes; D(i, j) is returned in
// lane j + 16*(i/4), register i%4.
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4f mfma16f(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

constexpr int kXK = 32;  // K chunk of the FP32 X tiles
constexpr int kXyKq = 3;  // perturbations per workgroup when K > 1 (two workgroups per CU)

// FP32 tiles: four waves in a 2x2 arrangement; each wave owns a (TM/2)x(TM/2)
// quarter of the tile, made of WB x WB 16x16 MFMA blocks.
template <int TM>
struct XyShape {
  static constexpr int kNT = 256;
  static constexpr int kWB = TM / 32;
  static constexpr int kPer = kXK * TM / kNT;  // operand values per thread per chunk
};

// The same TMxTM block for nq <= KQ perturbations at once: the Q columns are
// staged once, and each perturbation's h(m) multiplies the B operand in
// registers (the same double product h(m) Q(m, l) as in xy_block_4b, so each
// perturbation's block is bit for bit what xy_block_4b gives).
template <int TM, int KQ, bool DIAG = false>
__device__ __forceinline__ void xy_block_4b_kq(const double* __restrict__ Q,
                                               const double* __restrict__ hl, int64_t hstride,
                                               int nq, int n, int k0, int l0,
                                               double (&acc)[KQ][TM / 16][TM / 16]) {
  constexpr int kXK = 16;
  constexpr int kNT = 256, LD = TM + 1, R4 = TM / 16, C16 = TM / 16;
  constexpr int kPer = kXK * TM / kNT;
  __shared__ double As[kXK][LD];
  __shared__ double Bs[kXK][LD];
  __shared__ double hs[KQ][kXK];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lq = lane & 3, lr = lane >> 4, l15 = lane & 15;
  const int mm_t = tid & (kXK - 1), c_t = tid / kXK;
  const int hq_t = min(c_t, nq - 1);  // perturbation whose h this thread stages (c_t < KQ)
  double pa[kPer], pb[kPer], ph = 0.0;
  auto fetch = [&](int m0) {
    const int mc = min(m0 + mm_t, n - 1);
    ph = hl[(int64_t)hq_t * hstride + mc];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int c = c_t + u * (kNT / kXK);
      pa[u] = Q[mc + (size_t)n * min(k0 + c, n - 1)];
      pb[u] = Q[mc + (size_t)n * min(l0 + c, n - 1)];
    }
  };
#pragma unroll
  for (int q = 0; q < KQ; ++q)
#pragma unroll
    for (int r = 0; r < R4; ++r)
#pragma unroll
      for (int c = 0; c < C16; ++c) acc[q][r][c] = 0.0;
  fetch(0);
  for (int m0 = 0; m0 < n; m0 += kXK) {
    __syncthreads();
    const bool okm = m0 + mm_t < n;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int c = c_t + u * (kNT / kXK);
      As[mm_t][c] = (okm && k0 + c < n) ? pa[u] : 0.0;
      Bs[mm_t][c] = (okm && l0 + c < n) ? pb[u] : 0.0;
    }
    if (c_t < KQ) hs[c_t][mm_t] = ph;
    __syncthreads();
    if (m0 + kXK < n) fetch(m0 + kXK);
#pragma unroll
    for (int ks = 0; ks < kXK / 4; ++ks) {
      const int mm = 4 * ks + lr;
      double a[R4], braw[C16];
#pragma unroll
      for (int r = 0; r < R4; ++r) a[r] = As[mm][xy_row<TM, DIAG>(r, w) + lq];
#pragma unroll
      for (int c = 0; c < C16; ++c) braw[c] = Bs[mm][16 * c + l15];
#pragma unroll
      for (int q = 0; q < KQ; ++q) {
        const double h = hs[q][mm];
        double bb[C16];
#pragma unroll
        for (int c = 0; c < C16; ++c) bb[c] = h * braw[c];
#pragma unroll
        for (int r = 0; r < R4; ++r)
#pragma unroll
          for (int c = 0; c < C16; ++c)
            if (!DIAG || c <= r) acc[q][r][c] = mfma4b(a[r], bb[c], acc[q][r][c]);
      }
    }
  }
}

// The same block from the FP32 leading parts: each kXK-deep chunk is summed by
// FP32 MFMA in FP32 and the chunk sums are added in FP64.  acc[x][y][r] holds
// row 4*(lane/16) + r of the 16x16 block (x, y).
// The B side is the FP32 part of Q scaled by h (diagonal kind, TB = float)
// or W = h1_s Q rounded to FP32 as it is staged (general kind, TB = double,
// no h).
template <int TM, typename TB, bool H>
__device__ __forceinline__ void xy_block_f32(
    const float* __restrict__ Q, const TB* __restrict__ Bm, const double* __restrict__ hl, int n,
    int k0, int l0, double (&acc)[XyShape<TM>::kWB][XyShape<TM>::kWB][4]) {
  using S = XyShape<TM>;
  constexpr int WB = S::kWB;
  __shared__ float As[kXK][TM + 1];
  __shared__ float Bs[kXK][TM + 1];
  __shared__ float hs[kXK];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr = (w >> 1) * (TM / 2), wc = (w & 1) * (TM / 2);
  float pa[S::kPer], pb[S::kPer], ph = 0.f;
  // clamped (valid) addresses; zeroing is applied at the LDS write, after the
  // current chunk's MFMAs, so the loads stay in flight across them
  auto fetch = [&](int m0) {
#pragma unroll
    for (int u = 0; u < S::kPer; ++u) {
      const int idx = tid + u * S::kNT;
      const int mm = idx % kXK, kk = idx / kXK;
      const int mc = min(m0 + mm, n - 1);
      pa[u] = Q[mc + (size_t)n * min(k0 + kk, n - 1)];
      pb[u] = (float)Bm[mc + (size_t)n * min(l0 + kk, n - 1)];
    }
    if constexpr (H) ph = (float)hl[min(m0 + (tid & (kXK - 1)), n - 1)];
  };
#pragma unroll
  for (int x = 0; x < WB; ++x)
#pragma unroll
    for (int y = 0; y < WB; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[x][y][r] = 0.0;
  fetch(0);
  for (int m0 = 0; m0 < n; m0 += kXK) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < S::kPer; ++u) {
      const int idx = tid + u * S::kNT;
      const int mm = idx % kXK, kk = idx / kXK;
      const bool okm = m0 + mm < n;
      As[mm][kk] = (okm && k0 + kk < n) ? pa[u] : 0.f;
      Bs[mm][kk] = (okm && l0 + kk < n) ? pb[u] : 0.f;
    }
    if constexpr (H) {
      if (tid < kXK) hs[tid] = (m0 + tid < n) ? ph : 0.f;
    }
    __syncthreads();
    if (m0 + kXK < n) fetch(m0 + kXK);
    v4f c[WB][WB];
#pragma unroll
    for (int x = 0; x < WB; ++x)
#pragma unroll
      for (int y = 0; y < WB; ++y) c[x][y] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < kXK / 4; ++ks) {
      const int row = 4 * ks + lk;
      float a[WB], bb[WB];
#pragma unroll
      for (int x = 0; x < WB; ++x) {
        a[x] = As[row][wr + 16 * x + li];
        if constexpr (H) bb[x] = hs[row] * Bs[row][wc + 16 * x + li];
        else bb[x] = Bs[row][wc + 16 * x + li];
      }
#pragma unroll
      for (int x = 0; x < WB; ++x)
#pragma unroll
        for (int y = 0; y < WB; ++y) c[x][y] = mfma16f(a[x], bb[y], c[x][y]);
    }
#pragma unroll
    for (int x = 0; x < WB; ++x)
#pragma unroll
      for (int y = 0; y < WB; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[x][y][r] += (double)c[x][y][r];
  }
}

// The FP32 block for nq <= KQ perturbations at once: the FP32 columns of Q are
// staged once and each perturbation's h(m) multiplies the B operand in FP32
// registers, as xy_block_f32 does for one (same products, same sums).
template <int TM, int KQ>
__device__ __forceinline__ void xy_block_f32_kq(
    const float* __restrict__ Q, const double* __restrict__ hl, int64_t hstride, int nq, int n,
    int k0, int l0, double (&acc)[KQ][XyShape<TM>::kWB][XyShape<TM>::kWB][4]) {
  using S = XyShape<TM>;
  constexpr int WB = S::kWB;
  __shared__ float As[kXK][TM + 1];
  __shared__ float Bs[kXK][TM + 1];
  __shared__ float hs[KQ][kXK];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr = (w >> 1) * (TM / 2), wc = (w & 1) * (TM / 2);
  const int hq_t = min(tid / kXK, nq - 1);  // perturbation whose h this thread stages
  float pa[S::kPer], pb[S::kPer], ph = 0.f;
  auto fetch = [&](int m0) {
#pragma unroll
    for (int u = 0; u < S::kPer; ++u) {
      const int idx = tid + u * S::kNT;
      const int mm = idx % kXK, kk = idx / kXK;
      const int mc = min(m0 + mm, n - 1);
      pa[u] = Q[mc + (size_t)n * min(k0 + kk, n - 1)];
      pb[u] = Q[mc + (size_t)n * min(l0 + kk, n - 1)];
    }
    ph = (float)hl[(int64_t)hq_t * hstride + min(m0 + (tid & (kXK - 1)), n - 1)];
  };
#pragma unroll
  for (int q = 0; q < KQ; ++q)
#pragma unroll
    for (int x = 0; x < WB; ++x)
#pragma unroll
      for (int y = 0; y < WB; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[q][x][y][r] = 0.0;
  fetch(0);
  for (int m0 = 0; m0 < n; m0 += kXK) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < S::kPer; ++u) {
      const int idx = tid + u * S::kNT;
      const int mm = idx % kXK, kk = idx / kXK;
      const bool okm = m0 + mm < n;
      As[mm][kk] = (okm && k0 + kk < n) ? pa[u] : 0.f;
      Bs[mm][kk] = (okm && l0 + kk < n) ? pb[u] : 0.f;
    }
    if (tid < KQ * kXK) hs[tid / kXK][tid & (kXK - 1)] = (m0 + (tid & (kXK - 1)) < n) ? ph : 0.f;
    __syncthreads();
    if (m0 + kXK < n) fetch(m0 + kXK);
    v4f c[KQ][WB][WB];
#pragma unroll
    for (int q = 0; q < KQ; ++q)
#pragma unroll
      for (int x = 0; x < WB; ++x)
#pragma unroll
        for (int y = 0; y < WB; ++y) c[q][x][y] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < kXK / 4; ++ks) {
      const int row = 4 * ks + lk;
      float a[WB], braw[WB];
#pragma unroll
      for (int x = 0; x < WB; ++x) {
        a[x] = As[row][wr + 16 * x + li];
        braw[x] = Bs[row][wc + 16 * x + li];
      }
#pragma unroll
      for (int q = 0; q < KQ; ++q) {
        const float hr = hs[q][row];
        float bb[WB];
#pragma unroll
        for (int x = 0; x < WB; ++x) bb[x] = hr * braw[x];
#pragma unroll
        for (int x = 0; x < WB; ++x)
#pragma unroll
          for (int y = 0; y < WB; ++y) c[q][x][y] = mfma16f(a[x], bb[y], c[q][x][y]);
      }
    }
#pragma unroll
    for (int q = 0; q < KQ; ++q)
#pragma unroll
      for (int x = 0; x < WB; ++x)
#pragma unroll
        for (int y = 0; y < WB; ++y)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[q][x][y][r] += (double)c[q][x][y][r];
  }
}

// Y = X o dF on the tiles of one size bin.  A computed value y(k, l) is stored
// at Y[l + n k] (row l, column k): the tile lists hold only tiles whose 64x64
// parent is on or below the diagonal, so every value of the symmetric Y sits at
// the position whose row tile is not above its column tile, written coalesced.
// Workgroup b serves XCD b % 8 and walks that XCD's range of the list with
// stride gridDim.x / 8 (one tile per workgroup, or persistent).  GEN: the
// general kind, X = Q^T W with W = h1_s Q of perturbation q in wbuf.
// Stores of an FP64 X tile times dF into Y (element (k, l) at l + n k).
// mirror: the tile lies in a diagonal 64x64 tile, whose upper triangle is
// written from its lower one: elements with k < l are dropped and those with
// k > l are also stored at (l, k), with dF(l, k).  DIAG: acc was formed in the
// diagonal mode of xy_block_4b (rows by xy_row; blocks c > r not formed).
// The dF values (and, with mirror, their mirrors) are loaded first, once per
// tile, from clamped addresses.
template <int TM, bool DIAG>
struct XyDf {
  double v[TM / 16][TM / 16], m[TM / 16][TM / 16];
  __device__ __forceinline__ void load(const double* __restrict__ dF, int n, int k0, int l0,
                                       int w, int lane, bool mirror) {
#pragma unroll
    for (int r = 0; r < TM / 16; ++r)
#pragma unroll
      for (int c = 0; c < TM / 16; ++c) {
        const int k = min(k0 + xy_row<TM, DIAG>(r, w) + (lane >> 4), n - 1);
        const int l = min(l0 + 16 * c + (lane & 15), n - 1);
        v[r][c] = dF[(size_t)l + (size_t)n * k];
        m[r][c] = mirror ? dF[(size_t)k + (size_t)n * l] : 0.0;
      }
  }
  __device__ __forceinline__ void store(const double (&acc)[TM / 16][TM / 16],
                                        double* __restrict__ Y, int n, int k0, int l0, int w,
                                        int lane, bool mirror) const {
#pragma unroll
    for (int r = 0; r < TM / 16; ++r)
#pragma unroll
      for (int c = 0; c < TM / 16; ++c) {
        if (DIAG && c > r) continue;
        const int k = k0 + xy_row<TM, DIAG>(r, w) + (lane >> 4);
        const int l = l0 + 16 * c + (lane & 15);
        if (k >= n || l >= n) continue;
        if (!mirror) {
          Y[(size_t)l + (size_t)n * k] = acc[r][c] * v[r][c];
        } else if (k >= l) {
          Y[(size_t)l + (size_t)n * k] = acc[r][c] * v[r][c];
          if (k > l) Y[(size_t)k + (size_t)n * l] = acc[r][c] * m[r][c];
        }
      }
  }
};

template <int TM, bool SPLIT, bool GEN>
__global__ __launch_bounds__(256, 4) void k_xy(
    const double* __restrict__ qbuf, const float* __restrict__ q32,
    const double* __restrict__ dfbuf, double* __restrict__ ybuf, const double* __restrict__ hloc,
    const double* __restrict__ wbuf, const int32_t* __restrict__ tiles, XcdSplit split,
    const int64_t* __restrict__ off2, const int32_t* __restrict__ sub_orb_ptr, int64_t sum_n2,
    int64_t sum_n, const int32_t* __restrict__ wflag, int mode) {
  constexpr int WB = XyShape<TM>::kWB;
  const int q = blockIdx.y;
  const int xcd = blockIdx.x & 7, stride = gridDim.x >> 3;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr = (w >> 1) * (TM / 2), wc = (w & 1) * (TM / 2);
  for (int t = split.off[xcd] + (int)(blockIdx.x >> 3); t < split.off[xcd + 1]; t += stride) {
    const int s = tiles[3 * t], ti = tiles[3 * t + 1], tj = tiles[3 * t + 2];
    // mode 1: subgraphs refined by window only; mode 2: the others (FP64 X)
    if (mode != 0 && (wflag[s] != 0) != (mode == 2)) continue;
    const int b = sub_orb_ptr[s];
    const int n = sub_orb_ptr[s + 1] - b;
    const int k0 = ti * TM, l0 = tj * TM;
    const double* hl = hloc + (size_t)q * sum_n + b;
    const double* W = GEN ? wbuf + (size_t)q * sum_n2 + off2[s] : nullptr;
    const double* dF = dfbuf + off2[s];
    double* Y = ybuf + (size_t)q * sum_n2 + off2[s];
    if constexpr (SPLIT) {
      double acc[WB][WB][4];
      if constexpr (GEN) xy_block_f32<TM, double, false>(q32 + off2[s], W, hl, n, k0, l0, acc);
      else xy_block_f32<TM, float, true>(q32 + off2[s], q32 + off2[s], hl, n, k0, l0, acc);
      // all dF loads first (clamped addresses), then the stores
      double dfv[WB][WB][4];
#pragma unroll
      for (int x = 0; x < WB; ++x)
#pragma unroll
        for (int y = 0; y < WB; ++y)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int k = min(k0 + wr + 16 * x + 4 * lk + r, n - 1);
            const int l = min(l0 + wc + 16 * y + li, n - 1);
            dfv[x][y][r] = dF[(size_t)l + (size_t)n * k];
          }
#pragma unroll
      for (int x = 0; x < WB; ++x)
#pragma unroll
        for (int y = 0; y < WB; ++y)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int k = k0 + wr + 16 * x + 4 * lk + r;
            const int l = l0 + wc + 16 * y + li;
            if (k < n && l < n) Y[(size_t)l + (size_t)n * k] = acc[x][y][r] * dfv[x][y][r];
          }
    } else {
      // FP64: inside a diagonal 64x64 tile only the lower triangle is formed
      // and each element is also stored at its mirror (X is symmetric); the
      // upper 32x32 tile of a diagonal 64x64 tile is therefore skipped
      const bool mirror = k0 / kTile == l0 / kTile;
      if (mirror && ti < tj) continue;
      double acc[TM / 16][TM / 16];
      if (ti == tj) {
        if constexpr (GEN) xy_block_4b<TM, false, true>(qbuf + off2[s], W, hl, n, k0, l0, n, n, acc);
        else xy_block_4b<TM, true, true>(qbuf + off2[s], qbuf + off2[s], hl, n, k0, l0, n, n, acc);
        XyDf<TM, true> df;
        df.load(dF, n, k0, l0, w, lane, true);
        df.store(acc, Y, n, k0, l0, w, lane, true);
      } else {
        if constexpr (GEN) xy_block_4b<TM, false>(qbuf + off2[s], W, hl, n, k0, l0, n, n, acc);
        else xy_block_4b<TM, true>(qbuf + off2[s], qbuf + off2[s], hl, n, k0, l0, n, n, acc);
        XyDf<TM, false> df;
        df.load(dF, n, k0, l0, w, lane, mirror);
        df.store(acc, Y, n, k0, l0, w, lane, mirror);
      }
    }
  }
}

// W = h1_s Q for the general kind, perturbation q = blockIdx.y: the gathered
// h1_s (symmetric, so its column r is its row r) is the A side and Q the B
// side.  The 64x64 tile list holds (ti, tj) with tj <= ti; a workgroup forms
// the W tiles (ti, tj) and, off the diagonal, (tj, ti), so every tile of the
// full n x n W is written once, column-major like Q.
__global__ __launch_bounds__(256, 4) void k_wq(
    const double* __restrict__ gbuf, const double* __restrict__ qbuf, double* __restrict__ wbuf,
    const int32_t* __restrict__ tiles, XcdSplit split, const int64_t* __restrict__ off2,
    const int32_t* __restrict__ sub_orb_ptr, int64_t sum_n2) {
  constexpr int TM = kTile;
  const int q = blockIdx.y;
  const int xcd = blockIdx.x & 7, stride = gridDim.x >> 3;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int t = split.off[xcd] + (int)(blockIdx.x >> 3); t < split.off[xcd + 1]; t += stride) {
    const int s = tiles[3 * t], ti = tiles[3 * t + 1], tj = tiles[3 * t + 2];
    const int n = sub_orb_ptr[s + 1] - sub_orb_ptr[s];
    const double* Gs = gbuf + (size_t)q * sum_n2 + off2[s];
    const double* Q = qbuf + off2[s];
    double* W = wbuf + (size_t)q * sum_n2 + off2[s];
    for (int side = 0; side < (ti == tj ? 1 : 2); ++side) {
      const int r0 = (side == 0 ? ti : tj) * TM, c0 = (side == 0 ? tj : ti) * TM;
      double acc[TM / 16][TM / 16];
      xy_block_4b<TM, false>(Gs, Q, nullptr, n, r0, c0, n, n, acc);
#pragma unroll
      for (int r = 0; r < TM / 16; ++r)
#pragma unroll
        for (int c = 0; c < TM / 16; ++c) {
          const int row = r0 + w * (TM / 4) + 4 * r + (lane >> 4);
          const int col = c0 + 16 * c + (lane & 15);
          if (row < n && col < n) W[(size_t)row + (size_t)n * col] = acc[r][c];
        }
    }
  }
}

// Y tiles for KQ perturbations per workgroup (grid.y = ceil(K / KQ)), FP64 or
// split-FP32.
template <int TM, int KQ, bool SPLIT>
__global__ __launch_bounds__(256, 2) void k_xy_kq(
    const double* __restrict__ qbuf, const float* __restrict__ q32,
    const double* __restrict__ dfbuf, double* __restrict__ ybuf, const double* __restrict__ hloc,
    const int32_t* __restrict__ tiles, XcdSplit split, const int64_t* __restrict__ off2,
    const int32_t* __restrict__ sub_orb_ptr, int64_t sum_n2, int64_t sum_n, int K,
    const int32_t* __restrict__ wflag, int mode) {
  const int q0 = blockIdx.y * KQ, nq = min(KQ, K - q0);
  const int xcd = blockIdx.x & 7, stride = gridDim.x >> 3;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int t = split.off[xcd] + (int)(blockIdx.x >> 3); t < split.off[xcd + 1]; t += stride) {
    const int s = tiles[3 * t], ti = tiles[3 * t + 1], tj = tiles[3 * t + 2];
    if (mode != 0 && (wflag[s] != 0) != (mode == 2)) continue;
    const int b = sub_orb_ptr[s];
    const int n = sub_orb_ptr[s + 1] - b;
    const int k0 = ti * TM, l0 = tj * TM;
    const double* dF = dfbuf + off2[s];
    const double* hl = hloc + (size_t)q0 * sum_n + b;
    if constexpr (SPLIT) {
      constexpr int WB = XyShape<TM>::kWB;
      const int li = lane & 15, lk = lane >> 4;
      const int wr = (w >> 1) * (TM / 2), wc = (w & 1) * (TM / 2);
      double acc[KQ][WB][WB][4];
      xy_block_f32_kq<TM, KQ>(q32 + off2[s], hl, sum_n, nq, n, k0, l0, acc);
      double dfv[WB][WB][4];
#pragma unroll
      for (int x = 0; x < WB; ++x)
#pragma unroll
        for (int y = 0; y < WB; ++y)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int k = min(k0 + wr + 16 * x + 4 * lk + r, n - 1);
            const int l = min(l0 + wc + 16 * y + li, n - 1);
            dfv[x][y][r] = dF[(size_t)l + (size_t)n * k];
          }
#pragma unroll
      for (int q = 0; q < KQ; ++q) {
        if (q >= nq) break;
        double* Y = ybuf + (size_t)(q0 + q) * sum_n2 + off2[s];
#pragma unroll
        for (int x = 0; x < WB; ++x)
#pragma unroll
          for (int y = 0; y < WB; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int k = k0 + wr + 16 * x + 4 * lk + r;
              const int l = l0 + wc + 16 * y + li;
              if (k < n && l < n) Y[(size_t)l + (size_t)n * k] = acc[q][x][y][r] * dfv[x][y][r];
            }
      }
    } else {
      // FP64: diagonal 64x64 tiles formed on their lower triangle and stored
      // with the mirror, as in k_xy
      const bool mirror = k0 / kTile == l0 / kTile;
      if (mirror && ti < tj) continue;
      double acc[KQ][TM / 16][TM / 16];
      if (ti == tj) {
        xy_block_4b_kq<TM, KQ, true>(qbuf + off2[s], hl, sum_n, nq, n, k0, l0, acc);
        XyDf<TM, true> df;
        df.load(dF, n, k0, l0, w, lane, true);
#pragma unroll
        for (int q = 0; q < KQ; ++q) {
          if (q >= nq) break;
          df.store(acc[q], ybuf + (size_t)(q0 + q) * sum_n2 + off2[s], n, k0, l0, w, lane, true);
        }
      } else {
        xy_block_4b_kq<TM, KQ, false>(qbuf + off2[s], hl, sum_n, nq, n, k0, l0, acc);
        XyDf<TM, false> df;
        df.load(dF, n, k0, l0, w, lane, mirror);
#pragma unroll
        for (int q = 0; q < KQ; ++q) {
          if (q >= nq) break;
          df.store(acc[q], ybuf + (size_t)(q0 + q) * sum_n2 + off2[s], n, k0, l0, w, lane, mirror);
        }
      }
    }
  }
}

// Leading FP32 part of every eigenvector matrix (once per eigenbasis).
__global__ __launch_bounds__(kThreads) void k_split32(const double* __restrict__ q,
                                                      float* __restrict__ q32, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * kThreads)
    q32[i] = (float)q[i];
}

// The FP64 refinement window.  X o dF amplifies the FP32 rounding of X by dF,
// which for a pair of states at the same energy eps is f'(eps) =
// (beta/4) sech^2(beta (eps - mu)/2): pairs in a dense or degenerate level
// next to mu carry up to beta/4.  Every state with f'(eps) > tau_F (tau_F per
// context, gq_ctx_set_split_window) is in the window, i.e.
// |eps - mu| <= w kT with w = 2 acosh(sqrt(beta / (4 tau_F))), and none when
// beta/4 <= tau_F; all pairs of window states are recomputed in FP64.  A
// subgraph whose window holds more than `cap` states gets its whole X in FP64
// instead (refining a larger window would cost about as much as X itself).
__device__ __forceinline__ double win_half_width(double kT, double tau_F) {
  const double r = 1.0 / (4.0 * kT * tau_F);
  return r > 1.0 ? 2.0 * acosh(sqrt(r)) * kT : -1.0;  // negative: no window
}
constexpr int kWinGroups = 4;  // workgroups per (subgraph, perturbation)

// first index i in [0, n) with v[i] >= x (n if none)
__device__ __forceinline__ int lower_index(const double* v, int n, double x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (v[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// window [lo, hi) of a subgraph's ascending eigenvalues e[0..n)
__device__ __forceinline__ void win_range(const double* e, int n, double mu, double half, int& lo,
                                          int& hi) {
  lo = lower_index(e, n, mu - half);
  hi = lower_index(e, n, mu + half);
  while (hi < n && e[hi] <= mu + half) ++hi;
}

// wflag[s] = 1 when subgraph s's window exceeds win_cap states (its X is then
// formed in FP64), else 0.
__global__ __launch_bounds__(kThreads) void k_win_size(const double* __restrict__ eps,
                                                       const double* __restrict__ mu_state,
                                                       const int32_t* __restrict__ sub_orb_ptr,
                                                       int n_sub, double win_dF, int win_cap,
                                                       int32_t* __restrict__ wflag) {
  const int s = blockIdx.x * kThreads + threadIdx.x;
  if (s >= n_sub) return;
  const int b = sub_orb_ptr[s];
  int lo = 0, hi = 0;
  const double half = win_half_width(mu_state[3], win_dF);
  if (half >= 0.0) win_range(eps + b, sub_orb_ptr[s + 1] - b, mu_state[2], half, lo, hi);
  wflag[s] = hi - lo > win_cap ? 1 : 0;
}

// FP64 refinement of the thermal window: the dF weights are largest, up to
// beta/4, between states within a few kT of mu, and there the FP32 rounding of
// X would be amplified most.  The window block X[lo..hi, lo..hi] is covered by
// 64x64 sub-blocks (bi, bj) of rows lo + 64 bi.., columns lo + 64 bj..; only
// those with bi >= bj - 1 hold positions of the stored half of Y (row tile not
// above column tile).  Workgroup (subgraph, perturbation, z) recomputes the
// sub-blocks z, z + kWinGroups, ... of that list on FP64 MFMA and overwrites
// those entries of Y.
template <bool GEN>
__global__ __launch_bounds__(kThreads) void k_win(
    const double* __restrict__ qbuf, const double* __restrict__ dfbuf, double* __restrict__ ybuf,
    const double* __restrict__ hloc, const double* __restrict__ wbuf,
    const double* __restrict__ eps, const double* __restrict__ mu_state,
    const int64_t* __restrict__ off2, const int32_t* __restrict__ sub_orb_ptr, int64_t sum_n2,
    int64_t sum_n, double win_dF, int win_cap) {
  const int s = blockIdx.x, q = blockIdx.y;
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  const double half = win_half_width(mu_state[3], win_dF);
  if (half < 0.0) return;
  int lo, hi;
  win_range(eps + b, n, mu_state[2], half, lo, hi);
  // empty window, or X of this subgraph already in FP64
  if (hi <= lo || hi - lo > win_cap) return;
  const int nb = (hi - lo + kTile - 1) / kTile;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double* dF = dfbuf + off2[s];
  double* Y = ybuf + (size_t)q * sum_n2 + off2[s];
  for (int z = blockIdx.z; z < nb * nb; z += kWinGroups) {
    const int bi = z / nb, bj = z % nb;
    if (bi < bj - 1) continue;  // no stored position (uniform over the workgroup)
    const int k0 = lo + kTile * bi, l0 = lo + kTile * bj;
    double acc[kTile / 16][kTile / 16];
    if constexpr (GEN)
      xy_block_4b<kTile, false>(qbuf + off2[s], wbuf + (size_t)q * sum_n2 + off2[s], nullptr, n,
                                k0, l0, hi, hi, acc);
    else
      xy_block_4b<kTile, true>(qbuf + off2[s], qbuf + off2[s], hloc + (size_t)q * sum_n + b, n,
                               k0, l0, hi, hi, acc);
#pragma unroll
    for (int r = 0; r < kTile / 16; ++r)
#pragma unroll
      for (int c = 0; c < kTile / 16; ++c) {
        const int k = k0 + w * (kTile / 4) + 4 * r + (lane >> 4);
        const int l = l0 + 16 * c + (lane & 15);
        // each stored position is written by the one (k, l) that owns it
        if (k < hi && l < hi && k / kTile >= l / kTile) {
          const size_t at = (size_t)l + (size_t)n * k;
          Y[at] = acc[r][c] * dF[at];
        }
      }
  }
}

// h1 restricted to every subgraph, in subgraph order, for K perturbations:
// hloc[q][b + m] = h1[q][orbs[b + m]]
__global__ __launch_bounds__(kThreads) void k_h1_gather(const double* __restrict__ h1, int N,
                                                        const int32_t* __restrict__ sub_orbs,
                                                        int64_t sum_n, double* __restrict__ hloc) {
  const int q = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < sum_n;
       i += (int64_t)gridDim.x * kThreads)
    hloc[(size_t)q * sum_n + i] = h1[(size_t)q * N + sub_orbs[i]];
}


// T = Q_c Y for 128 columns of one subgraph and the 32 core rows J0 .. J0 + 31
// (one launch per block of 32 core rows; subgraphs whose core ends before J0
// return); T stored as tbuf[(b + l) * 32 + (j - J0)].
// K (the rows of Y) is staged through LDS 32 rows at a time, each half of the
// 128 columns read along its stored direction (a 32-row stage lies inside one
// 64-row tile of Y); the next stage is prefetched into registers meanwhile.
// Each wave owns 32 columns and the (at most 32) core rows.
constexpr int kTC = 128;  // columns per workgroup of the row products
constexpr int kTK = 32;

__global__ __launch_bounds__(kThreads) void k_t_mfma(
    const double* __restrict__ qbuf, const double* __restrict__ ybuf, double* __restrict__ tbuf,
    const int64_t* __restrict__ off2, const int32_t* __restrict__ sub_orb_ptr,
    const int32_t* __restrict__ n_core, const int32_t* __restrict__ order, int64_t sum_n2,
    int64_t sum_n, int J0) {
  __shared__ double As[kTK][33];
  __shared__ double Bs[kTK][kTC + 1];
  const int s = order[blockIdx.x];
  const int q = blockIdx.z;
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  const int c = n_core[s];
  const int L0 = blockIdx.y * kTC;
  if (L0 >= n || J0 >= c) return;
  const double* Q = qbuf + off2[s];
  const double* Y = ybuf + (size_t)q * sum_n2 + off2[s];
  double* Tq = tbuf + (size_t)q * sum_n * 32;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  constexpr int kPa = kTK * 32 / kThreads, kPh = kTK * kTile / kThreads;
  double pa[kPa], pb[2][kPh];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < kPa; ++u) {
      const int idx = tid + u * kThreads;
      const int j = idx % 32, kk = idx / 32;
      pa[u] = (J0 + j < c && k0 + kk < n) ? Q[J0 + j + (size_t)n * (k0 + kk)] : 0.0;
    }
#pragma unroll
    for (int hlf = 0; hlf < 2; ++hlf) {
      const int C0 = L0 + hlf * kTile;
      const bool lower = (k0 / kTile) >= (C0 / kTile);
#pragma unroll
      for (int u = 0; u < kPh; ++u) {
        const int idx = tid + u * kThreads;
        int kk, ll;
        if (lower) {
          ll = idx % kTile;
          kk = idx / kTile;
        } else {
          kk = idx % kTK;
          ll = idx / kTK;
        }
        const int k = k0 + kk, l = C0 + ll;
        pb[hlf][u] = (k < n && l < n)
                         ? (lower ? Y[(size_t)l + (size_t)n * k] : Y[(size_t)k + (size_t)n * l])
                         : 0.0;
      }
    }
  };
  v4d acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = v4d{0.0, 0.0, 0.0, 0.0};
  fetch(0);
  for (int k0 = 0; k0 < n; k0 += kTK) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPa; ++u) {
      const int idx = tid + u * kThreads;
      As[idx / 32][idx % 32] = pa[u];
    }
#pragma unroll
    for (int hlf = 0; hlf < 2; ++hlf) {
      const bool lower = (k0 / kTile) >= ((L0 + hlf * kTile) / kTile);
#pragma unroll
      for (int u = 0; u < kPh; ++u) {
        const int idx = tid + u * kThreads;
        if (lower) Bs[idx / kTile][hlf * kTile + idx % kTile] = pb[hlf][u];
        else Bs[idx % kTK][hlf * kTile + idx / kTK] = pb[hlf][u];
      }
    }
    __syncthreads();
    if (k0 + kTK < n) fetch(k0 + kTK);
#pragma unroll
    for (int ks = 0; ks < kTK / 4; ++ks) {
      const int row = 4 * ks + lk;
      const double a0 = As[row][li], a1 = As[row][16 + li];
      const double b0 = Bs[row][32 * w + li], b1 = Bs[row][32 * w + 16 + li];
      acc[0][0] = mfma16(a0, b0, acc[0][0]);
      acc[1][0] = mfma16(a1, b0, acc[1][0]);
      acc[0][1] = mfma16(a0, b1, acc[0][1]);
      acc[1][1] = mfma16(a1, b1, acc[1][1]);
    }
  }
#pragma unroll
  for (int y = 0; y < 2; ++y) {
    const int l = L0 + 32 * w + 16 * y + li;
    if (l < n) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        Tq[(size_t)(b + l) * 32 + lk + 4 * r] = acc[0][y][r];
        Tq[(size_t)(b + l) * 32 + 16 + lk + 4 * r] = acc[1][y][r];
      }
    }
  }
}

// P = 2 T Q^T (c x n core rows, block layout) and its diagonal for the core
// rows J0 .. J0 + 31 that T holds, 128 columns per workgroup.  Each wave owns 32 columns; T and Q are read straight from memory
// along their stored directions, kPU steps of 4 rows loaded ahead of their MFMAs.
constexpr int kPU = 8;

__global__ __launch_bounds__(kThreads) void k_p_mfma(
    const double* __restrict__ tbuf, const double* __restrict__ qbuf, double* __restrict__ out,
    double* __restrict__ pdiag, const int64_t* __restrict__ off2, const int64_t* __restrict__ offc,
    const int32_t* __restrict__ offcd, const int32_t* __restrict__ sub_orb_ptr,
    const int32_t* __restrict__ n_core, const int32_t* __restrict__ order, int64_t sum_n,
    int64_t nnz, int sum_c, int n_sub, int ncb, int K, int J0) {
  // group g = (subgraph in order, column block) holds the K perturbations that
  // read the same 128 rows of Q.  Groups go round-robin to the XCDs (workgroup
  // b runs on XCD b mod 8), and on each XCD a group's K workgroups are
  // consecutive, so they run together and share those rows through its L2.
  const int x = blockIdx.x & 7, j = blockIdx.x >> 3;
  const int g = (j / K) * 8 + x;
  const int q = j % K;
  if (g >= n_sub * ncb) return;
  const int s = order[g / ncb];
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  const int c = n_core[s];
  const int L0 = (g % ncb) * kTC;
  if (L0 >= n || J0 >= c) return;
  const double* Q = qbuf + off2[s];
  const double* Tq = tbuf + (size_t)q * sum_n * 32;
  double* outq = out + (size_t)q * nnz;
  double* pdq = pdiag + (size_t)q * sum_c;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  int lcol[2];
  bool colok[2];
#pragma unroll
  for (int y = 0; y < 2; ++y) {
    lcol[y] = L0 + 32 * w + 16 * y + li;
    colok[y] = lcol[y] < n;
  }
  v4d acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int m0 = 0; m0 < n; m0 += 4 * kPU) {
    double a0[kPU], a1[kPU], bv[2][kPU];
#pragma unroll
    for (int u = 0; u < kPU; ++u) {
      const int m = m0 + 4 * u + lk;
      const bool ok = m < n;
      a0[u] = ok ? Tq[(size_t)(b + m) * 32 + li] : 0.0;
      a1[u] = ok ? Tq[(size_t)(b + m) * 32 + 16 + li] : 0.0;
#pragma unroll
      for (int y = 0; y < 2; ++y) bv[y][u] = (ok && colok[y]) ? Q[lcol[y] + (size_t)n * m] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kPU; ++u)
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        acc[0][y] = mfma16(a0[u], bv[y][u], acc[0][y]);
        acc[1][y] = mfma16(a1[u], bv[y][u], acc[1][y]);
      }
  }
  const size_t base = offc[s];
#pragma unroll
  for (int y = 0; y < 2; ++y) {
    if (!colok[y]) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j0 = J0 + lk + 4 * r, j1 = J0 + 16 + lk + 4 * r;
      if (j0 < c) {
        const double v = 2.0 * acc[0][y][r];
        outq[base + (size_t)j0 * n + lcol[y]] = v;
        if (lcol[y] == j0) pdq[offcd[s] + j0] = v;
      }
      if (j1 < c) {
        const double v = 2.0 * acc[1][y][r];
        outq[base + (size_t)j1 * n + lcol[y]] = v;
        if (lcol[y] == j1) pdq[offcd[s] + j1] = v;
      }
    }
  }
}

// Diagonal of P = 2 T Q^T only (the core charges of the response need no
// more): P_jj = 2 sum_l T[j, l] Q[j, l] for the core rows J0 .. J0 + 31 that T
// holds; workgroup (subgraph, q), each thread sums its columns l in order,
// then a fixed-order reduction.
__global__ __launch_bounds__(kThreads) void k_pdiag(
    const double* __restrict__ tbuf, const double* __restrict__ qbuf, double* __restrict__ pdiag,
    const int64_t* __restrict__ off2, const int32_t* __restrict__ offcd,
    const int32_t* __restrict__ sub_orb_ptr, const int32_t* __restrict__ n_core, int64_t sum_n,
    int sum_c, int J0) {
  __shared__ double red[kThreads / 64][32];
  const int s = blockIdx.x, q = blockIdx.y;
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  const int c = n_core[s] - J0;  // core rows of this block: J0 .. J0 + min(c, 32) - 1
  if (c <= 0) return;
  const double* Q = qbuf + off2[s] + J0;
  const double* Tq = tbuf + (size_t)q * sum_n * 32;
  double acc[32];
#pragma unroll
  for (int j = 0; j < 32; ++j) acc[j] = 0.0;
  for (int l = threadIdx.x; l < n; l += kThreads) {
#pragma unroll
    for (int j = 0; j < 32; ++j)
      if (j < c) acc[j] += Tq[(size_t)(b + l) * 32 + j] * Q[j + (size_t)n * l];
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    const double t = wave_sum(acc[j]);
    if (lane == 0) red[w][j] = t;
  }
  __syncthreads();
  if (threadIdx.x < min(c, 32)) {
    double t = 0.0;
    for (int x = 0; x < kThreads / 64; ++x) t += red[x][threadIdx.x];
    pdiag[(size_t)q * sum_c + offcd[s] + J0 + threadIdx.x] = 2.0 * t;
  }
}

// mu1_q = -sum_i sum_{j<c_i} P_i[j,j] / sum_i tmu_i, fixed order; one block per q
__global__ __launch_bounds__(kThreads) void k_mu1(const double* __restrict__ pdiag, int sum_c,
                                                  const double* __restrict__ tmu, int n_sub,
                                                  double* __restrict__ mu1) {
  __shared__ double red[8];
  const int q = blockIdx.x;
  double a = 0.0, t = 0.0;
  for (int i = threadIdx.x; i < sum_c; i += kThreads) a += pdiag[(size_t)q * sum_c + i];
  for (int i = threadIdx.x; i < n_sub; i += kThreads) t += tmu[i];
  a = wave_sum(a);
  t = wave_sum(t);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    red[w] = a;
    red[4 + w] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double A = red[0] + red[1] + red[2] + red[3];
    const double Tm = red[4] + red[5] + red[6] + red[7];
    mu1[q] = -A / Tm;
  }
}

__global__ __launch_bounds__(kThreads) void k_combine(double* __restrict__ p,
                                                      const double* __restrict__ m,
                                                      const double* __restrict__ mu1,
                                                      int64_t nnz) {
  const int q = blockIdx.y;
  const double f = mu1[q];
  double* pq = p + (size_t)q * nnz;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < nnz;
       i += (int64_t)gridDim.x * kThreads)
    pq[i] += f * m[i];
}

__global__ __launch_bounds__(kThreads) void k_assemble(
    const double* __restrict__ blocks, double* __restrict__ vals, int64_t nnz,
    const int64_t* __restrict__ offc, const int32_t* __restrict__ sub_orb_ptr,
    const int32_t* __restrict__ sub_orbs, const int32_t* __restrict__ n_core,
    const int32_t* __restrict__ slot, const int32_t* __restrict__ rho_row_ptr) {
  const int s = blockIdx.x;
  const int q = blockIdx.z;
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  const int c = n_core[s];
  const size_t total = (size_t)c * n;
  const double* src = blocks + (size_t)q * nnz + offc[s];
  double* dst = vals + (size_t)q * nnz;
  for (size_t idx = (size_t)blockIdx.y * kThreads + threadIdx.x; idx < total;
       idx += (size_t)gridDim.y * kThreads) {
    const int j = (int)(idx / n), l = (int)(idx % n);
    const int a = sub_orbs[b + j];
    dst[rho_row_ptr[a] + slot[b + l]] = src[idx];
  }
}

// ------------------------------------------------------------ xy launches
using XyKernel = void (*)(const double*, const float*, const double*, double*, const double*,
                          const double*, const int32_t*, XcdSplit, const int64_t*,
                          const int32_t*, int64_t, int64_t, const int32_t*, int);
using XyKqKernel = void (*)(const double*, const float*, const double*, double*, const double*,
                            const int32_t*, XcdSplit, const int64_t*, const int32_t*, int64_t,
                            int64_t, int, const int32_t*, int);

template <bool GEN>
XyKernel xy_kernel_t(int shape, bool split) {
  if (shape == 0) return split ? k_xy<64, true, GEN> : k_xy<64, false, GEN>;
  return split ? k_xy<32, true, GEN> : k_xy<32, false, GEN>;
}

XyKernel xy_kernel(int shape, bool split, bool gen) {
  return gen ? xy_kernel_t<true>(shape, split) : xy_kernel_t<false>(shape, split);
}

XyKqKernel xy_kq_kernel(int shape, bool split) {
  if (shape == 0) return split ? k_xy_kq<64, kXyKq, true> : k_xy_kq<64, kXyKq, false>;
  return split ? k_xy_kq<32, kXyKq, true> : k_xy_kq<32, kXyKq, false>;
}

int xy_threads(int shape) { return shape == 0 ? XyShape<64>::kNT : XyShape<32>::kNT; }

// Workgroups of one variant (0: FP64, 1: split, 2 / 3: FP64 / split with kXyKq
// perturbations per workgroup) resident on one XCD (32 CUs) at a time.
int xy_resident_per_xcd(int shape, int variant) {
  static std::atomic<int> cache[2][4];
  std::atomic<int>& c = cache[shape][variant];
  int v = c.load(std::memory_order_relaxed);
  if (v == 0) {
    const void* fn = variant >= 2 ? (const void*)xy_kq_kernel(shape, variant == 3)
                                  : (const void*)xy_kernel(shape, variant == 1, false);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, xy_threads(shape), 0) !=
            hipSuccess ||
        per_cu < 1) {
      (void)hipGetLastError();
      per_cu = 1;
    }
    v = per_cu * 32;
    c.store(v, std::memory_order_relaxed);
  }
  return v;
}

// Launch of one bin with variant `choice` (bit 0: 32x32 tiles, bit 1: persistent).
// Diagonal launches with K > 1 take kXyKq perturbations per workgroup; the
// general kind (gen) takes one perturbation per workgroup, X = Q^T W with W in
// rb.Y, written to rb.G.
void launch_xy_bin(gq_ctx* ctx, const gq_graph* g, gq_eigs* e, const RespBufs& rb, int bin,
                   int choice, bool split, bool gen, int K, int mode = 0,
                   const double* qx = nullptr) {
  if (!qx) qx = e->Q;
  const int shape = choice & 1;
  const bool persistent = (choice & 2) != 0;
  const bool kq = K > 1 && !gen;
  const XcdSplit& sp = g->xy_split[shape][bin];
  int longest = 0;
  for (int x = 0; x < 8; ++x) longest = std::max(longest, sp.off[x + 1] - sp.off[x]);
  if (longest == 0) return;
  int per_xcd = longest;
  if (persistent)
    per_xcd = std::min(longest, xy_resident_per_xcd(shape, (kq ? 2 : 0) + (split ? 1 : 0)));
  const gq_graph_dev& dv = g->dev;
  if (kq) {
    hipLaunchKernelGGL(xy_kq_kernel(shape, split), dim3(8 * per_xcd, (K + kXyKq - 1) / kXyKq),
                       dim3(xy_threads(shape)), 0, ctx->stream, qx, e->Q32, e->A, rb.Y,
                       rb.hloc, dv.xy_tiles[shape], sp, dv.off2, dv.sub_orb_ptr, g->info.sum_n2,
                       g->info.sum_n, K, e->wflag, mode);
    return;
  }
  hipLaunchKernelGGL(xy_kernel(shape, split, gen), dim3(8 * per_xcd, K), dim3(xy_threads(shape)),
                     0, ctx->stream, qx, e->Q32, e->A, gen ? rb.G : rb.Y, rb.hloc,
                     gen ? rb.Y : nullptr, dv.xy_tiles[shape], sp, dv.off2, dv.sub_orb_ptr,
                     g->info.sum_n2, g->info.sum_n, e->wflag, mode);
}

void launch_split32(gq_ctx* ctx, const gq_graph* g, gq_eigs* e) {
  prof_begin(ctx, "k_split32");
  const int64_t cnt = g->info.sum_n2;
  hipLaunchKernelGGL(k_split32,
                     dim3((unsigned)std::min<int64_t>(8192, (cnt + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, ctx->stream, e->Q, e->Q32, cnt);
  prof_end(ctx);
}

}  // namespace

void build_xy_tiles(gq_graph* g) {
  // bins by subgraph size; tiles of a subgraph contiguous, subgraphs in the
  // order of decreasing size; per bin and shape the list is cut into 8
  // contiguous XCD ranges of about equal tile count at subgraph boundaries
  for (int shape = 0; shape < 2; ++shape) {
    const int tm = shape == 0 ? 64 : 32;
    std::vector<int32_t>& tl = g->xy_tiles[shape];
    tl.clear();
    {
      // an upper bound of the list's length: every tile of every subgraph
      size_t cap = 0;
      for (int32_t s = 0; s < g->n_sub; ++s) {
        const size_t nt = (g->sub_orb_ptr[s + 1] - g->sub_orb_ptr[s] + tm - 1) / tm;
        cap += 3 * nt * nt;
      }
      tl.resize(cap);
    }
    size_t at = 0;  // ints written so far
    for (int bin = 0; bin < kXyBins; ++bin) {
      const int lo = bin == 0 ? 0 : kXyBinMax[bin - 1];
      const int hi = kXyBinMax[bin];
      const int32_t start = (int32_t)(at / 3);
      std::vector<int32_t> sub_start;  // first tile of each subgraph of the bin
      for (int32_t s : g->order) {
        const int32_t n = g->sub_orb_ptr[s + 1] - g->sub_orb_ptr[s];
        if (n <= lo || n > hi) continue;
        sub_start.push_back((int32_t)(at / 3));
        const int32_t nt = (n + tm - 1) / tm;
        int32_t* t = tl.data();
        for (int32_t ti = 0; ti < nt; ++ti)
          for (int32_t tj = 0; tj < nt; ++tj) {
            // parent 64x64 tile on or below the diagonal
            if ((ti * tm) / 64 < (tj * tm) / 64) continue;
            if (tm == 64 && tj > ti) continue;
            t[at++] = s;
            t[at++] = ti;
            t[at++] = tj;
          }
      }
      const int32_t end = (int32_t)(at / 3);
      XcdSplit& sp = g->xy_split[shape][bin];
      const int64_t total = end - start;
      size_t next = 0;
      sp.off[0] = start;
      for (int x = 1; x < 8; ++x) {
        const int64_t target = start + (total * x + 7) / 8;
        while (next < sub_start.size() && sub_start[next] < target) ++next;
        sp.off[x] = next < sub_start.size() ? sub_start[next] : end;
        sp.off[x] = std::max(sp.off[x], sp.off[x - 1]);
      }
      sp.off[8] = end;
    }
    tl.resize(at);
  }
  for (int p = 0; p < 2; ++p)
    for (int bin = 0; bin < kXyBins; ++bin) g->xy_choice[p][bin] = 0;
  // every lower-triangular 64x64 tile (ti >= tj) of every subgraph, subgraphs
  // in decreasing size, the tiles of a subgraph together on one XCD
  std::vector<int32_t>& ft = g->tri_tiles;
  ft.clear();
  std::vector<int32_t> sub_start;
  sub_start.reserve(g->n_sub);
  {
    size_t cap = 0;
    for (int32_t s = 0; s < g->n_sub; ++s) {
      const size_t nt = (g->sub_orb_ptr[s + 1] - g->sub_orb_ptr[s] + 63) / 64;
      cap += 3 * nt * (nt + 1) / 2;
    }
    ft.reserve(cap);
  }
  for (int32_t s : g->order) {
    const int32_t n = g->sub_orb_ptr[s + 1] - g->sub_orb_ptr[s];
    const int32_t nt = (n + 63) / 64;
    sub_start.push_back((int32_t)(ft.size() / 3));
    for (int32_t ti = 0; ti < nt; ++ti)
      for (int32_t tj = 0; tj <= ti; ++tj) {
        ft.push_back(s);
        ft.push_back(ti);
        ft.push_back(tj);
      }
  }
  const int64_t total = (int64_t)(ft.size() / 3);
  size_t next = 0;
  g->tri_split.off[0] = 0;
  for (int x = 1; x < 8; ++x) {
    const int64_t target = (total * x + 7) / 8;
    while (next < sub_start.size() && sub_start[next] < target) ++next;
    g->tri_split.off[x] = next < sub_start.size() ? sub_start[next] : (int32_t)total;
    g->tri_split.off[x] = std::max(g->tri_split.off[x], g->tri_split.off[x - 1]);
  }
  g->tri_split.off[8] = (int32_t)total;
}

// ----------------------------------------------------- static scratch
// Response scratch of gq_response_static, for callers that cannot allocate
// device memory: 2^25 doubles (256 MiB) per device, held from the library's
// first context on that device until the process ends.  Host code never uses
// this name as an address: scratch_init takes the device address once per
// device with hipGetSymbolAddress, and everything else uses that pointer.
constexpr int64_t kScratchDoubles = int64_t(1) << 25;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

gq_status scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("static scratch: device %d beyond %d", device, kMaxDevices);
    return GQ_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return GQ_OK;
  // the caller has made `device` current
  void* ptr = nullptr;
  const hipError_t rc = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (rc != hipSuccess || !ptr) {
    set_error("static scratch: hipGetSymbolAddress failed on device %d: %s", device,
              hipGetErrorString(rc));
    return GQ_EDEVICE;
  }
  g_scratch_ptr[device] = static_cast<double*>(ptr);
  return GQ_OK;
}

double* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

int64_t scratch_doubles() { return kScratchDoubles; }

int64_t resp_doubles_per_k(const gq_graph* g, uint32_t kind) {
  // hloc, Y, G (general kind), T, pdiag, mu1, each rounded up to 32 doubles
  auto up = [](int64_t x) { return (x + 31) & ~int64_t(31); };
  const int64_t sum_c = g->offcd[g->n_sub];
  return up(g->info.sum_n) + up(g->info.sum_n2) * (kind == GQ_H1_CSR ? 2 : 1) +
         up(g->info.sum_n * 32) + up(std::max<int64_t>(sum_c, 1)) + up(1);
}

void launch_response(gq_ctx* ctx, const gq_graph* g, gq_eigs* e, const RespBufs& rb,
                     const H1Spec& h1, int32_t K, uint32_t precision, double* p_blocks,
                     RespOpts opt) {
  hipStream_t st = ctx->stream;
  const gq_graph_dev& dv = g->dev;
  const int64_t nnz = g->info.nnz;
  const int64_t sum_n = g->info.sum_n, sum_n2 = g->info.sum_n2;
  const int sum_c = g->offcd[g->n_sub];
  const bool split = precision == GQ_PREC_SPLIT32;
  const bool gen = !opt.local_h1 && h1.kind == GQ_H1_CSR;
  // non-orthogonal basis: X = C^T h1 C with C = z Q (h1 in the atomic-orbital
  // basis); split precision is not offered there
  const bool ao = e->overlap_solved;
  const double* qx = ao ? e->C : e->Q;
  // a captured sequence must not depend on the host-side validity flag
  if (split && (!e->q32_valid || ctx->capturing)) {
    launch_split32(ctx, g, e);
    e->q32_valid = true;
  }
  if (gen) {
    // h1_s of every subgraph and perturbation into G, then W = h1_s Q into Y
    for (int q = 0; q < K; ++q)
      launch_gather(ctx, g, &h1.csr[q], rb.G + (size_t)q * sum_n2, nullptr, "k_h1_gather");
    prof_begin(ctx, "k_wq");
    const XcdSplit* sp = g->xy_split[0];
    for (int bin = 0; bin < kXyBins; ++bin) {
      int longest = 0;
      for (int x = 0; x < 8; ++x) longest = std::max(longest, sp[bin].off[x + 1] - sp[bin].off[x]);
      if (longest == 0) continue;
      hipLaunchKernelGGL(k_wq, dim3(8 * longest, K), dim3(kThreads), 0, st, rb.G, qx, rb.Y,
                         dv.xy_tiles[0], sp[bin], dv.off2, dv.sub_orb_ptr, sum_n2);
    }
    prof_end(ctx);
  }
  prof_begin(ctx, split ? "k_xy32" : "k_xy");
  if (!gen && !opt.local_h1)
    hipLaunchKernelGGL(k_h1_gather,
                       dim3((unsigned)std::min<int64_t>(1024, (sum_n + kThreads - 1) / kThreads), K),
                       dim3(kThreads), 0, st, h1.diag, g->N, dv.sub_orbs, sum_n, rb.hloc);
  if (split) {
    // subgraphs whose window is too wide for the refinement get FP64 X
    hipLaunchKernelGGL(k_win_size, dim3((g->n_sub + kThreads - 1) / kThreads), dim3(kThreads), 0,
                       st, e->eps, e->mu_state, dv.sub_orb_ptr, g->n_sub, ctx->win_dF,
                       ctx->win_cap, e->wflag);
    for (int bin = 0; bin < kXyBins; ++bin)
      launch_xy_bin(ctx, g, e, rb, bin, g->xy_choice[1][bin], true, gen, K, 1);
    // the FP64 pass serves the few subgraphs with wide windows: a persistent
    // grid walks the tile list and skips the others cheaply
    for (int bin = 0; bin < kXyBins; ++bin)
      launch_xy_bin(ctx, g, e, rb, bin, (g->xy_choice[0][bin] & 1) | 2, false, gen, K, 2);
  } else {
    for (int bin = 0; bin < kXyBins; ++bin)
      launch_xy_bin(ctx, g, e, rb, bin, g->xy_choice[0][bin], false, gen, K, 0, qx);
  }
  prof_end(ctx);
  // X o dF of perturbation q is in ybuf: Y for the diagonal kind, G for the general
  double* ybuf = gen ? rb.G : rb.Y;
  if (split) {
    prof_begin(ctx, "k_win");
    hipLaunchKernelGGL(gen ? k_win<true> : k_win<false>, dim3(g->n_sub, K, kWinGroups),
                       dim3(kThreads), 0,
                       st, e->Q, e->A, ybuf, rb.hloc, rb.Y, e->eps, e->mu_state, dv.off2,
                       dv.sub_orb_ptr, sum_n2, sum_n, ctx->win_dF, ctx->win_cap);
    prof_end(ctx);
  }
  // the core rows in blocks of 32 (T holds one block at a time)
  prof_begin(ctx, "k_rows");
  dim3 grid_cols(g->n_sub, (g->info.max_n + kTC - 1) / kTC, K);
  const int ncb = (g->info.max_n + kTC - 1) / kTC;
  const int groups_per_xcd = (g->n_sub * ncb + 7) / 8;
  const int n_jb = (g->info.max_c + 31) / 32;
  if (opt.charge_only || ao) {
    // the orthogonalized core traces (the diagonal of P only) fix mu1
    for (int jb = 0; jb < n_jb; ++jb) {
      hipLaunchKernelGGL(k_t_mfma, grid_cols, dim3(kThreads), 0, st, e->Q, ybuf, rb.T, dv.off2,
                         dv.sub_orb_ptr, dv.n_core, dv.order, sum_n2, sum_n, 32 * jb);
      hipLaunchKernelGGL(k_pdiag, dim3(g->n_sub, K), dim3(kThreads), 0, st, rb.T, e->Q,
                         rb.pdiag, dv.off2, dv.offcd, dv.sub_orb_ptr, dv.n_core, sum_n, sum_c,
                         32 * jb);
    }
    prof_end(ctx);
    prof_begin(ctx, "k_mu1_combine");
    hipLaunchKernelGGL(k_mu1, dim3(K), dim3(kThreads), 0, st, rb.pdiag, sum_c, e->tmu, g->n_sub,
                       rb.mu1);
    prof_end(ctx);
    if (opt.charge_only) return;
    // the atomic-orbital rows 2 C_c Y C^T (their diagonal overwrites pdiag,
    // which k_mu1 has consumed)
    prof_begin(ctx, "k_rows");
  }
  for (int jb = 0; jb < n_jb; ++jb) {
    hipLaunchKernelGGL(k_t_mfma, grid_cols, dim3(kThreads), 0, st, qx, ybuf, rb.T, dv.off2,
                       dv.sub_orb_ptr, dv.n_core, dv.order, sum_n2, sum_n, 32 * jb);
    hipLaunchKernelGGL(k_p_mfma, dim3(8 * groups_per_xcd * K), dim3(kThreads), 0, st, rb.T, qx,
                       p_blocks, rb.pdiag, dv.off2, dv.offc, dv.offcd, dv.sub_orb_ptr, dv.n_core,
                       dv.order, sum_n, nnz, sum_c, g->n_sub, ncb, K, 32 * jb);
  }
  prof_end(ctx);
  prof_begin(ctx, "k_mu1_combine");
  if (!ao)
    hipLaunchKernelGGL(k_mu1, dim3(K), dim3(kThreads), 0, st, rb.pdiag, sum_c, e->tmu, g->n_sub,
                       rb.mu1);
  const int blocks = (int)std::min<int64_t>(4096, (nnz + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(k_combine, dim3(blocks, K), dim3(kThreads), 0, st, p_blocks, e->M, rb.mu1,
                     nnz);
  prof_end(ctx);
}

gq_status autotune_xy(gq_ctx* ctx, const gq_graph* g, gq_eigs* e, uint32_t precision,
                      std::string* report) {
  const bool split = precision == GQ_PREC_SPLIT32;
  if (split && !e->q32_valid) {
    launch_split32(ctx, g, e);
    e->q32_valid = true;
  }
  hipStream_t st = ctx->stream;
  const RespBufs rb{e->hloc, e->Y, e->G, e->T, e->pdiag, e->mu1};
  // the tuning launches read whatever h1 the workspace holds; only their time matters
  GQ_HIP(hipMemsetAsync(e->hloc, 0, g->info.sum_n * sizeof(double), st));
  hipEvent_t t0, t1;
  GQ_HIP(hipEventCreate(&t0));
  GQ_HIP(hipEventCreate(&t1));
  char line[256];
  static const char* names[4] = {"64x64 tiles, one workgroup per tile",
                                 "32x32 tiles, one workgroup per tile",
                                 "64x64 tiles, persistent", "32x32 tiles, persistent"};
  gq_status rc = GQ_OK;
  for (int bin = 0; bin < kXyBins && rc == GQ_OK; ++bin) {
    const XcdSplit& sp = g->xy_split[0][bin];
    if (sp.off[8] == sp.off[0]) continue;
    float best = 1e30f;
    int best_c = 0;
    for (int choice = 0; choice < 4; ++choice) {
      launch_xy_bin(ctx, g, e, rb, bin, choice, split, false, 1);  // warm-up
      float ms_min = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        if (hipEventRecord(t0, st) != hipSuccess) rc = GQ_EDEVICE;
        launch_xy_bin(ctx, g, e, rb, bin, choice, split, false, 1);
        if (hipEventRecord(t1, st) != hipSuccess || hipEventSynchronize(t1) != hipSuccess)
          rc = GQ_EDEVICE;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, t0, t1) != hipSuccess) rc = GQ_EDEVICE;
        ms_min = std::min(ms_min, ms);
      }
      if (rc != GQ_OK) break;
      std::snprintf(line, sizeof line, "bin n<=%d (%d 64-tiles) %s: %.4f ms\n", kXyBinMax[bin],
                    sp.off[8] - sp.off[0], names[choice], ms_min);
      *report += line;
      if (ms_min < best) {
        best = ms_min;
        best_c = choice;
      }
    }
    g->xy_choice[split ? 1 : 0][bin] = (int8_t)best_c;
    std::snprintf(line, sizeof line, "bin n<=%d -> %s\n", kXyBinMax[bin], names[best_c]);
    *report += line;
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (rc != GQ_OK) set_error("gq_autotune: timing failed: %s", hipGetErrorString(hipGetLastError()));
  return rc;
}

void launch_assemble(gq_ctx* ctx, const gq_graph* g, const double* blocks, int32_t K,
                     double* vals) {
  const gq_graph_dev& dv = g->dev;
  hipStream_t st = ctx->stream;
  prof_begin(ctx, "k_assemble");
  const int64_t maxcn = (int64_t)g->info.max_c * g->info.max_n;
  dim3 grid(g->n_sub, (unsigned)std::max<int64_t>(1, (maxcn + kThreads * 8 - 1) / (kThreads * 8)), K);
  hipLaunchKernelGGL(k_assemble, grid, dim3(kThreads), 0, st, blocks, vals, g->info.nnz, dv.offc,
                     dv.sub_orb_ptr, dv.sub_orbs, dv.n_core, dv.slot, dv.rho_row_ptr);
  prof_end(ctx);
}

}  // namespace gq
