// Canonical first-order response in the eigenbasis and the collect step.
//
// Sec. IV.A: for a perturbation H1 the fixed-mu response of each subgraph is
// the Frechet derivative of the Fermi function, which in the eigenbasis reads
//   d1lambda = Q [(Q^T h1 Q) o dF] Q^T,
// the mu response is beta d0 (I - d0) (Eq. (dddmu)), and Eq. (dmu_1) fixes
//   mu1 = -sum_i Tr_c d1lambda_i / sum_i Tr_c d1mu_i,
// so that the collected rho1 = 2 (d1lambda + mu1 d1mu) core rows has zero trace
// (Eq. (D1)).  Kernels per perturbation q:
//   k_xy_mfma  lower-triangular 64x64 tiles of X = Q^T diag(h1) Q on FP64
//              MFMA, times dF, into Y (each symmetric pair stored once)
//   k_xy32_mfma, k_win_mfma  the split-FP32 variant of the same: X from the
//              FP32 leading part of Q on FP32 MFMA (FP32 sums within 32-deep
//              chunks, FP64 across them), then one FP64 correction of the
//              thermal-window block, where dF amplifies rounding most
//   k_t_mfma   T = Q_c Y;  k_p_mfma  P = 2 T Q^T (c x n core rows) and diag(P)
//   k_mu1      fixed-order traces -> mu1_q
//   k_combine  P += mu1_q M
// Eq. (sub_f) / (dCollect): k_assemble scatters block rows into CSR values.
#include <algorithm>

#include "gq_internal.hpp"

namespace gq {

namespace {

constexpr int kThreads = 256;
constexpr int kTile = 64;

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

constexpr int kXK = 32;  // K chunk of the X tiles

// Accumulates the 64x64 block X(k0.., l0..) = sum_m Q(m, k) h(m) Q(m, l) of one
// subgraph on FP64 MFMA (columns k >= kend or l >= lend read as zero).  Waves
// own 32x32 quarters; the K dimension is staged through LDS in chunks of kXK
// rows, the next chunk prefetched into registers while the current one is used.
__device__ __forceinline__ void xy_block_f64(const double* __restrict__ Q,
                                             const double* __restrict__ hl, int n, int k0,
                                             int l0, int kend, int lend, v4d (&acc)[2][2]) {
  __shared__ double As[kXK][kTile + 1];
  __shared__ double Bs[kXK][kTile + 1];
  __shared__ double hs[kXK];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  constexpr int kPer = kXK * kTile / kThreads;  // values of As (and of Bs) per thread
  double pa[kPer], pb[kPer], ph = 0.0;
  auto fetch = [&](int m0) {
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int idx = tid + u * kThreads;
      const int mm = idx % kXK, kk = idx / kXK;
      const int m = m0 + mm;
      const bool okm = m < n;
      pa[u] = (okm && k0 + kk < kend) ? Q[m + (size_t)n * (k0 + kk)] : 0.0;
      pb[u] = (okm && l0 + kk < lend) ? Q[m + (size_t)n * (l0 + kk)] : 0.0;
    }
    if (tid < kXK) ph = (m0 + tid < n) ? hl[m0 + tid] : 0.0;
  };
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = v4d{0.0, 0.0, 0.0, 0.0};
  fetch(0);
  for (int m0 = 0; m0 < n; m0 += kXK) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int idx = tid + u * kThreads;
      As[idx % kXK][idx / kXK] = pa[u];
      Bs[idx % kXK][idx / kXK] = pb[u];
    }
    if (tid < kXK) hs[tid] = ph;
    __syncthreads();
    if (m0 + kXK < n) fetch(m0 + kXK);
#pragma unroll
    for (int ks = 0; ks < kXK / 4; ++ks) {
      const int row = 4 * ks + lk;
      const double hr = hs[row];
      const double a0 = As[row][wr + li], a1 = As[row][wr + 16 + li];
      const double b0 = hr * Bs[row][wc + li], b1 = hr * Bs[row][wc + 16 + li];
      acc[0][0] = mfma16(a0, b0, acc[0][0]);
      acc[0][1] = mfma16(a0, b1, acc[0][1]);
      acc[1][0] = mfma16(a1, b0, acc[1][0]);
      acc[1][1] = mfma16(a1, b1, acc[1][1]);
    }
  }
}

// Y = (Q^T diag(h1) Q) o dF on the lower 64x64 tiles (ti >= tj).  A tile's
// value y(k, l), k in tile ti, l in tile tj, is stored at Y[l + n k]
// (row l, column k): every value of the symmetric Y sits at the position
// whose row tile is not above its column tile, written coalesced.
__global__ __launch_bounds__(kThreads) void k_xy_mfma(
    const double* __restrict__ qbuf, const double* __restrict__ dfbuf, double* __restrict__ ybuf,
    const double* __restrict__ hloc, const int32_t* __restrict__ tiles,
    const int64_t* __restrict__ off2, const int32_t* __restrict__ sub_orb_ptr) {
  const int s = tiles[3 * blockIdx.x], ti = tiles[3 * blockIdx.x + 1], tj = tiles[3 * blockIdx.x + 2];
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  const int k0 = ti * kTile, l0 = tj * kTile;
  v4d acc[2][2];
  xy_block_f64(qbuf + off2[s], hloc + b, n, k0, l0, n, n, acc);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  const double* dF = dfbuf + off2[s];
  double* Y = ybuf + off2[s];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k = k0 + wr + 16 * x + lk + 4 * r;
        const int l = l0 + wc + 16 * y + li;
        if (k < n && l < n) {
          const size_t at = (size_t)l + (size_t)n * k;
          Y[at] = acc[x][y][r] * dF[at];
        }
      }
}

// ------------------------------------------------- split-FP32 congruence
// v_mfma_f32_16x16x4f32 on gfx950: lane l supplies A(l%16, l/16) and
// B(l/16, l%16); D(i, j) is returned in lane j + 16*(i/4), register i%4.
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4f mfma16f(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Leading FP32 part of every eigenvector matrix (once per eigenbasis).
__global__ __launch_bounds__(kThreads) void k_split32(const double* __restrict__ q,
                                                      float* __restrict__ q32, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * kThreads)
    q32[i] = (float)q[i];
}

// As k_xy_mfma from the FP32 leading parts: each kXK-deep chunk of the sum is
// accumulated by FP32 MFMA in FP32, and the chunk sums are added in FP64.
__global__ __launch_bounds__(kThreads) void k_xy32_mfma(
    const float* __restrict__ q32, const double* __restrict__ dfbuf, double* __restrict__ ybuf,
    const double* __restrict__ hloc, const int32_t* __restrict__ tiles,
    const int64_t* __restrict__ off2, const int32_t* __restrict__ sub_orb_ptr) {
  __shared__ float As[kXK][kTile + 1];
  __shared__ float Bs[kXK][kTile + 1];
  __shared__ float hs[kXK];
  const int s = tiles[3 * blockIdx.x], ti = tiles[3 * blockIdx.x + 1], tj = tiles[3 * blockIdx.x + 2];
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  const float* Q = q32 + off2[s];
  const double* hl = hloc + b;
  const int k0 = ti * kTile, l0 = tj * kTile;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  constexpr int kPer = kXK * kTile / kThreads;
  float pa[kPer], pb[kPer], ph = 0.f;
  auto fetch = [&](int m0) {
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int idx = tid + u * kThreads;
      const int mm = idx % kXK, kk = idx / kXK;
      const int m = m0 + mm;
      const bool okm = m < n;
      pa[u] = (okm && k0 + kk < n) ? Q[m + (size_t)n * (k0 + kk)] : 0.f;
      pb[u] = (okm && l0 + kk < n) ? Q[m + (size_t)n * (l0 + kk)] : 0.f;
    }
    if (tid < kXK) ph = (m0 + tid < n) ? (float)hl[m0 + tid] : 0.f;
  };
  double acc[2][2][4];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[x][y][r] = 0.0;
  fetch(0);
  for (int m0 = 0; m0 < n; m0 += kXK) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int idx = tid + u * kThreads;
      As[idx % kXK][idx / kXK] = pa[u];
      Bs[idx % kXK][idx / kXK] = pb[u];
    }
    if (tid < kXK) hs[tid] = ph;
    __syncthreads();
    if (m0 + kXK < n) fetch(m0 + kXK);
    v4f c[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) c[x][y] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < kXK / 4; ++ks) {
      const int row = 4 * ks + lk;
      const float hr = hs[row];
      const float a0 = As[row][wr + li], a1 = As[row][wr + 16 + li];
      const float b0 = hr * Bs[row][wc + li], b1 = hr * Bs[row][wc + 16 + li];
      c[0][0] = mfma16f(a0, b0, c[0][0]);
      c[0][1] = mfma16f(a0, b1, c[0][1]);
      c[1][0] = mfma16f(a1, b0, c[1][0]);
      c[1][1] = mfma16f(a1, b1, c[1][1]);
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[x][y][r] += (double)c[x][y][r];
  }
  const double* dF = dfbuf + off2[s];
  double* Y = ybuf + off2[s];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k = k0 + wr + 16 * x + 4 * lk + r;
        const int l = l0 + wc + 16 * y + li;
        if (k < n && l < n) {
          const size_t at = (size_t)l + (size_t)n * k;
          Y[at] = acc[x][y][r] * dF[at];
        }
      }
}

// Window half-width, in units of kT, of the FP64 refinement.
constexpr double kWinKT = 8.0;

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

// FP64 refinement of the thermal window: the dF weights are largest, up to
// beta/4, between states within a few kT of mu, and there the FP32 rounding of
// X would be amplified most.  One workgroup per subgraph recomputes the block of
// X over the states with |eps - mu| <= kWinKT kT (at most 64, the ones nearest
// mu) on FP64 MFMA and overwrites those entries of Y.
__global__ __launch_bounds__(kThreads) void k_win_mfma(
    const double* __restrict__ qbuf, const double* __restrict__ dfbuf, double* __restrict__ ybuf,
    const double* __restrict__ hloc, const double* __restrict__ eps,
    const double* __restrict__ mu_state, const int64_t* __restrict__ off2,
    const int32_t* __restrict__ sub_orb_ptr) {
  const int s = blockIdx.x;
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  const double mu = mu_state[2], half = kWinKT * mu_state[3];
  const double* e = eps + b;  // ascending
  int lo = lower_index(e, n, mu - half);
  int hi = lower_index(e, n, mu + half);
  while (hi < n && e[hi] <= mu + half) ++hi;
  if (hi - lo > kTile) {
    const int mid = lower_index(e, n, mu);
    lo = max(lo, min(mid - kTile / 2, hi - kTile));
    hi = lo + kTile;
  }
  if (hi <= lo) return;
  v4d acc[2][2];
  xy_block_f64(qbuf + off2[s], hloc + b, n, lo, lo, hi, hi, acc);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  const double* dF = dfbuf + off2[s];
  double* Y = ybuf + off2[s];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k = lo + wr + 16 * x + lk + 4 * r;
        const int l = lo + wc + 16 * y + li;
        // each stored position is written by the one (k, l) that owns it
        if (k < hi && l < hi && k / kTile >= l / kTile) {
          const size_t at = (size_t)l + (size_t)n * k;
          Y[at] = acc[x][y][r] * dF[at];
        }
      }
}

// h1 restricted to every subgraph, in subgraph order: hloc[b + m] = h1[orbs[b + m]]
__global__ __launch_bounds__(kThreads) void k_h1_gather(const double* __restrict__ h1,
                                                        const int32_t* __restrict__ sub_orbs,
                                                        int64_t sum_n, double* __restrict__ hloc) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < sum_n;
       i += (int64_t)gridDim.x * kThreads)
    hloc[i] = h1[sub_orbs[i]];
}

// Y(k, l) under the storage rule of k_xy_mfma
__device__ __forceinline__ size_t ypos(int k, int l, int n) {
  return (k / kTile >= l / kTile) ? (size_t)l + (size_t)n * k : (size_t)k + (size_t)n * l;
}

// T = Q_c Y for 64 columns of one subgraph; T stored as tbuf[(b + l) * 32 + j].
__global__ __launch_bounds__(kThreads) void k_t_mfma(
    const double* __restrict__ qbuf, const double* __restrict__ ybuf, double* __restrict__ tbuf,
    const int64_t* __restrict__ off2, const int32_t* __restrict__ sub_orb_ptr,
    const int32_t* __restrict__ n_core, const int32_t* __restrict__ order) {
  __shared__ double As[16][33];
  __shared__ double Bs[16][kTile + 1];
  const int s = order[blockIdx.x];
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  const int c = n_core[s];
  const int L0 = blockIdx.y * kTile;
  if (L0 >= n) return;
  const double* Q = qbuf + off2[s];
  const double* Y = ybuf + off2[s];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  v4d acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < n; k0 += 16) {
    __syncthreads();
    for (int idx = tid; idx < 16 * 32; idx += kThreads) {
      const int j = idx % 32, kk = idx / 32;
      As[kk][j] = (j < c && k0 + kk < n) ? Q[j + (size_t)n * (k0 + kk)] : 0.0;
    }
    // Y rows k0..k0+15, columns L0..L0+63; coalesced along the stored direction
    const bool lower = (k0 / kTile) >= (L0 / kTile);
    for (int idx = tid; idx < 16 * kTile; idx += kThreads) {
      int kk, ll;
      if (lower) {
        ll = idx % kTile;
        kk = idx / kTile;
      } else {
        kk = idx % 16;
        ll = idx / 16;
      }
      const int k = k0 + kk, l = L0 + ll;
      Bs[kk][ll] = (k < n && l < n) ? Y[ypos(k, l, n)] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int row = 4 * ks + lk;
      const double bv = Bs[row][16 * w + li];
      acc0 = mfma16(As[row][li], bv, acc0);
      acc1 = mfma16(As[row][16 + li], bv, acc1);
    }
  }
  const int l = L0 + 16 * w + li;
  if (l < n) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      tbuf[(size_t)(b + l) * 32 + lk + 4 * r] = acc0[r];
      tbuf[(size_t)(b + l) * 32 + 16 + lk + 4 * r] = acc1[r];
    }
  }
}

// P = 2 T Q^T (c x n core rows, block layout) and its diagonal.
__global__ __launch_bounds__(kThreads) void k_p_mfma(
    const double* __restrict__ tbuf, const double* __restrict__ qbuf, double* __restrict__ out,
    double* __restrict__ pdiag, const int64_t* __restrict__ off2, const int64_t* __restrict__ offc,
    const int32_t* __restrict__ offcd, const int32_t* __restrict__ sub_orb_ptr,
    const int32_t* __restrict__ n_core, const int32_t* __restrict__ order) {
  const int s = order[blockIdx.x];
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  const int c = n_core[s];
  const int L0 = blockIdx.y * kTile;
  if (L0 >= n) return;
  const double* Q = qbuf + off2[s];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int lcol = L0 + 16 * w + li;
  v4d acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
  for (int q0 = 0; q0 < n; q0 += 4) {
    const int q = q0 + lk;
    const bool ok = q < n;
    const double a0 = ok ? tbuf[(size_t)(b + q) * 32 + li] : 0.0;
    const double a1 = ok ? tbuf[(size_t)(b + q) * 32 + 16 + li] : 0.0;
    const double bv = (ok && lcol < n) ? Q[lcol + (size_t)n * q] : 0.0;
    acc0 = mfma16(a0, bv, acc0);
    acc1 = mfma16(a1, bv, acc1);
  }
  if (lcol < n) {
    const size_t base = offc[s];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j0 = lk + 4 * r, j1 = 16 + lk + 4 * r;
      if (j0 < c) {
        const double v = 2.0 * acc0[r];
        out[base + (size_t)j0 * n + lcol] = v;
        if (lcol == j0) pdiag[offcd[s] + j0] = v;
      }
      if (j1 < c) {
        const double v = 2.0 * acc1[r];
        out[base + (size_t)j1 * n + lcol] = v;
        if (lcol == j1) pdiag[offcd[s] + j1] = v;
      }
    }
  }
}

// mu1_q = -sum_i sum_{j<c_i} P_i[j,j] / sum_i tmu_i, fixed order
__global__ __launch_bounds__(kThreads) void k_mu1(const double* __restrict__ pdiag, int sum_c,
                                                  const double* __restrict__ tmu, int n_sub,
                                                  double* __restrict__ mu1, int q) {
  __shared__ double red[8];
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
                                                      const double* __restrict__ mu1, int q,
                                                      int64_t nnz) {
  const double f = mu1[q];
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < nnz;
       i += (int64_t)gridDim.x * kThreads)
    p[i] += f * m[i];
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

}  // namespace

void launch_response(gq_ctx* ctx, const gq_graph* g, gq_eigs* e, const double* h1, int32_t K,
                     uint32_t precision, double* p_blocks) {
  hipStream_t st = ctx->stream;
  const gq_graph_dev& dv = g->dev;
  const int64_t nnz = g->info.nnz;
  const int sum_c = g->offcd[g->n_sub];
  const bool split = precision == GQ_PREC_SPLIT32;
  dim3 grid_cols(g->n_sub, (g->info.max_n + kTile - 1) / kTile);
  if (split && !e->q32_valid) {
    prof_begin(ctx, "k_split32");
    const int64_t cnt = g->info.sum_n2;
    hipLaunchKernelGGL(k_split32, dim3((unsigned)std::min<int64_t>(8192, (cnt + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, st, e->Q, e->Q32, cnt);
    prof_end(ctx);
    e->q32_valid = true;
  }
  for (int q = 0; q < K; ++q) {
    prof_begin(ctx, split ? "k_xy32" : "k_xy");
    const int64_t sum_n = g->info.sum_n;
    hipLaunchKernelGGL(k_h1_gather, dim3((unsigned)std::min<int64_t>(1024, (sum_n + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, st, h1 + (size_t)q * g->N, dv.sub_orbs, sum_n, e->hloc);
    if (split) {
      hipLaunchKernelGGL(k_xy32_mfma, dim3(dv.n_tiles), dim3(kThreads), 0, st, e->Q32, e->A, e->Y,
                         e->hloc, dv.tiles, dv.off2, dv.sub_orb_ptr);
      prof_end(ctx);
      prof_begin(ctx, "k_win");
      hipLaunchKernelGGL(k_win_mfma, dim3(g->n_sub), dim3(kThreads), 0, st, e->Q, e->A, e->Y,
                         e->hloc, e->eps, e->mu_state, dv.off2, dv.sub_orb_ptr);
    } else {
      hipLaunchKernelGGL(k_xy_mfma, dim3(dv.n_tiles), dim3(kThreads), 0, st, e->Q, e->A, e->Y,
                         e->hloc, dv.tiles, dv.off2, dv.sub_orb_ptr);
    }
    prof_end(ctx);
    prof_begin(ctx, "k_rows");
    hipLaunchKernelGGL(k_t_mfma, grid_cols, dim3(kThreads), 0, st, e->Q, e->Y, e->T, dv.off2,
                       dv.sub_orb_ptr, dv.n_core, dv.order);
    hipLaunchKernelGGL(k_p_mfma, grid_cols, dim3(kThreads), 0, st, e->T, e->Q,
                       p_blocks + (size_t)q * nnz, e->pdiag + (size_t)q * sum_c, dv.off2, dv.offc,
                       dv.offcd, dv.sub_orb_ptr, dv.n_core, dv.order);
    prof_end(ctx);
  }
  prof_begin(ctx, "k_mu1_combine");
  for (int q = 0; q < K; ++q) {
    hipLaunchKernelGGL(k_mu1, dim3(1), dim3(kThreads), 0, st, e->pdiag, sum_c, e->tmu, g->n_sub,
                       e->mu1, q);
    const int blocks = (int)std::min<int64_t>(4096, (nnz + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_combine, dim3(blocks), dim3(kThreads), 0, st, p_blocks + (size_t)q * nnz,
                       e->M, e->mu1, q, nnz);
  }
  prof_end(ctx);
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
