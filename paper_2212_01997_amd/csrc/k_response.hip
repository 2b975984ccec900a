// Canonical first-order response in the eigenbasis and the collect step.
//
// Sec. IV.A: for a perturbation H1 the fixed-mu response of each subgraph is
// the Frechet derivative of the Fermi function, which in the eigenbasis reads
//   d1lambda = Q [(Q^T h1 Q) o dF] Q^T,
// the mu response is beta d0 (I - d0) (Eq. (dddmu)), and Eq. (dmu_1) fixes
//   mu1 = -sum_i Tr_c d1lambda_i / sum_i Tr_c d1mu_i,
// so that the collected rho1 = 2 (d1lambda + mu1 d1mu) core rows has zero trace
// (Eq. (D1)).  Kernels per perturbation q:
//   k_xy       lower-triangular 64x64 tiles of X = Q^T diag(h1) Q, times dF,
//              written with their mirror into Y (symmetric)
//   k_rows     T = Q_c Y, then P = 2 T Q^T (c x n core rows), P's diagonal
//   k_mu1      fixed-order traces -> mu1_q
//   k_combine  P += mu1_q M
// Eq. (sub_f) / (dCollect): k_assemble scatters block rows into CSR values.
#include <algorithm>

#include "gq_internal.hpp"

namespace gq {

namespace {

constexpr int kThreads = 256;
constexpr int kTile = 64;
constexpr int kKc = 16;

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

__global__ __launch_bounds__(kThreads) void k_xy(
    const double* __restrict__ qbuf, const double* __restrict__ dfbuf, double* __restrict__ ybuf,
    const double* __restrict__ h1, int N, const int32_t* __restrict__ tiles,
    const int64_t* __restrict__ off2, const int32_t* __restrict__ sub_orb_ptr,
    const int32_t* __restrict__ sub_orbs) {
  __shared__ double As[kKc][kTile + 1];
  __shared__ double Bs[kKc][kTile + 1];
  __shared__ double hs[kKc];
  const int s = tiles[3 * blockIdx.x], ti = tiles[3 * blockIdx.x + 1], tj = tiles[3 * blockIdx.x + 2];
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  const double* Q = qbuf + off2[s];
  const int k0 = ti * kTile, l0 = tj * kTile;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int m0 = 0; m0 < n; m0 += kKc) {
    __syncthreads();
    if (threadIdx.x < kKc) {
      const int m = m0 + threadIdx.x;
      hs[threadIdx.x] = m < n ? h1[sub_orbs[b + m]] : 0.0;
    }
    for (int idx = threadIdx.x; idx < kKc * kTile; idx += kThreads) {
      const int mm = idx % kKc, kk = idx / kKc;
      const int m = m0 + mm;
      As[mm][kk] = (m < n && k0 + kk < n) ? Q[m + (size_t)n * (k0 + kk)] : 0.0;
      Bs[mm][kk] = (m < n && l0 + kk < n) ? Q[m + (size_t)n * (l0 + kk)] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int mm = 0; mm < kKc; ++mm) {
      const double h = hs[mm];
      double a[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[mm][tx + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = h * Bs[mm][ty + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * bv[j];
    }
  }
  const double* dF = dfbuf + off2[s];
  double* Y = ybuf + off2[s];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int k = k0 + tx + 16 * i;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int l = l0 + ty + 16 * j;
      if (k < n && l < n) {
        const double y = acc[i][j] * dF[k + (size_t)n * l];
        Y[k + (size_t)n * l] = y;
        if (ti != tj) Y[l + (size_t)n * k] = y;
      }
    }
  }
}

// out[j, l] = alpha * sum_k L[j, k] R[l + n k] for kRowChunk core rows and
// kThreads columns.  mode 0: L = Q_c (rows of Q), R = Y.  mode 1: L = T
// (row-major c x n), R = Q; also writes out's diagonal for the core trace.
template <int MODE>
__global__ __launch_bounds__(kThreads) void k_rows(
    const double* __restrict__ lsrc, const double* __restrict__ rbuf, double* __restrict__ out,
    double* __restrict__ pdiag, double alpha, const int64_t* __restrict__ off2,
    const int64_t* __restrict__ offc, const int32_t* __restrict__ offcd,
    const int32_t* __restrict__ sub_orb_ptr, const int32_t* __restrict__ n_core,
    const int32_t* __restrict__ order) {
  __shared__ double L[kRowChunk][64 + 1];
  const int s = order[blockIdx.x];
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  const int c = n_core[s];
  const int l = blockIdx.y * kThreads + threadIdx.x;
  const int j0 = blockIdx.z * kRowChunk;
  if (blockIdx.y * kThreads >= n || j0 >= c) return;
  const double* R = rbuf + off2[s];
  double acc[kRowChunk];
#pragma unroll
  for (int jj = 0; jj < kRowChunk; ++jj) acc[jj] = 0.0;
  for (int k0 = 0; k0 < n; k0 += 64) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < kRowChunk * 64; idx += kThreads) {
      int jj, kk;
      double v = 0.0;
      if (MODE == 0) {
        jj = idx % kRowChunk;
        kk = idx / kRowChunk;
        if (j0 + jj < c && k0 + kk < n) v = lsrc[off2[s] + (j0 + jj) + (size_t)n * (k0 + kk)];
      } else {
        kk = idx % 64;
        jj = idx / 64;
        if (j0 + jj < c && k0 + kk < n) v = lsrc[offc[s] + (size_t)(j0 + jj) * n + (k0 + kk)];
      }
      L[jj][kk] = v;
    }
    __syncthreads();
    if (l < n) {
      const int kend = min(64, n - k0);
      for (int kk = 0; kk < kend; ++kk) {
        const double r = R[l + (size_t)n * (k0 + kk)];
#pragma unroll
        for (int jj = 0; jj < kRowChunk; ++jj) acc[jj] += L[jj][kk] * r;
      }
    }
  }
  if (l < n) {
#pragma unroll
    for (int jj = 0; jj < kRowChunk; ++jj) {
      const int j = j0 + jj;
      if (j < c) {
        const double v = alpha * acc[jj];
        out[offc[s] + (size_t)j * n + l] = v;
        if (MODE == 1 && l == j) pdiag[offcd[s] + j] = v;
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
  (void)precision;
  hipStream_t st = ctx->stream;
  const gq_graph_dev& dv = g->dev;
  const int64_t nnz = g->info.nnz;
  const int sum_c = g->offcd[g->n_sub];
  dim3 grid_rows(g->n_sub, (g->info.max_n + kThreads - 1) / kThreads,
                 (g->info.max_c + kRowChunk - 1) / kRowChunk);
  for (int q = 0; q < K; ++q) {
    prof_begin(ctx, "k_xy");
    hipLaunchKernelGGL(k_xy, dim3(dv.n_tiles), dim3(kThreads), 0, st, e->Q, e->A, e->Y,
                       h1 + (size_t)q * g->N, g->N, dv.tiles, dv.off2, dv.sub_orb_ptr,
                       dv.sub_orbs);
    prof_end(ctx);
    prof_begin(ctx, "k_rows");
    hipLaunchKernelGGL(k_rows<0>, grid_rows, dim3(kThreads), 0, st, e->Q, e->Y, e->T,
                       (double*)nullptr, 1.0, dv.off2, dv.offc, dv.offcd, dv.sub_orb_ptr, dv.n_core,
                       dv.order);
    hipLaunchKernelGGL(k_rows<1>, grid_rows, dim3(kThreads), 0, st, e->T, e->Q,
                       p_blocks + (size_t)q * nnz, e->pdiag + (size_t)q * sum_c, 2.0, dv.off2,
                       dv.offc, dv.offcd, dv.sub_orb_ptr, dv.n_core, dv.order);
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
