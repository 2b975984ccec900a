// Principal submatrices and their FP64 eigendecomposition on gfx950.
//
// Fig. 1: each subgraph selects the principal submatrix h = H[orbs, orbs].
// Eq. (SmallKS): h = Q diag(eps) Q^T.  One workgroup (4 waves) per subgraph:
//   k_gather    CSR rows of H -> dense column-major h (binary search of each
//               column index in the subgraph's sorted orbital list, in LDS)
//   k_tridiag   Householder reduction to tridiagonal form, reflectors kept in
//               the lower triangle (symv + rank-2 update streamed from L2)
//   then the tridiagonal eigenproblem by divide and conquer and the
//   back-transformation (k_dc.hip).
#include <cfloat>
#include <utility>

#include "gq_internal.hpp"

namespace gq {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Sum over the workgroup in a fixed order; every thread gets the total.
__device__ double block_sum(double x, double* red) {
  x = wave_sum(x);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = x;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) t += red[i];
  return t;
}

__global__ __launch_bounds__(kThreads) void k_gather(
    const int32_t* __restrict__ h_rp, const int32_t* __restrict__ h_col,
    const double* __restrict__ h_val, double* __restrict__ abuf,
    const int64_t* __restrict__ off2, const int32_t* __restrict__ sub_orb_ptr,
    const int32_t* __restrict__ sub_orbs, const int32_t* __restrict__ sorted_orbs,
    const int32_t* __restrict__ sorted_local, const int32_t* __restrict__ order,
    int32_t* __restrict__ status) {
  extern __shared__ int32_t si[];
  const int s = order[blockIdx.x];
  if (threadIdx.x == 0) status[s] = 0;
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  int32_t* so = si;
  int32_t* sl = si + n;
  double* A = abuf + off2[s];
  for (int i = threadIdx.x; i < n; i += kThreads) {
    so[i] = sorted_orbs[b + i];
    sl[i] = sorted_local[b + i];
  }
  const size_t nn = (size_t)n * n;
  for (size_t i = threadIdx.x; i < nn; i += kThreads) A[i] = 0.0;
  __syncthreads();
  for (int r = threadIdx.x; r < n; r += kThreads) {
    const int a = sub_orbs[b + r];
    for (int p = h_rp[a]; p < h_rp[a + 1]; ++p) {
      const int c = h_col[p];
      int lo = 0, hi = n;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (so[mid] < c) lo = mid + 1;
        else hi = mid;
      }
      if (lo < n && so[lo] == c) A[r + (size_t)n * sl[lo]] = h_val[p];
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_tridiag(
    double* __restrict__ abuf, const int64_t* __restrict__ off2,
    const int32_t* __restrict__ sub_orb_ptr, const int32_t* __restrict__ order,
    double* __restrict__ D, double* __restrict__ E, double* __restrict__ TAU) {
  extern __shared__ double sm[];
  const int s = order[blockIdx.x];
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  double* A = abuf + off2[s];
  double* v = sm;
  double* w = sm + n;
  double* red = sm + 2 * n;
  const int tid = threadIdx.x;
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    double* x = A + (k + 1) + (size_t)n * k;
    double part = 0.0;
    for (int i = 1 + tid; i < m; i += kThreads) part += x[i] * x[i];
    const double sigma = block_sum(part, red);
    const double alpha = x[0];
    if (tid == 0) D[b + k] = A[k + (size_t)n * k];
    if (sigma == 0.0) {
      if (tid == 0) {
        TAU[b + k] = 0.0;
        E[b + k] = alpha;
      }
      __syncthreads();
      continue;
    }
    const double nrm = sqrt(alpha * alpha + sigma);
    const double beta = alpha >= 0.0 ? -nrm : nrm;
    const double t = (beta - alpha) / beta;
    const double scale = 1.0 / (alpha - beta);
    for (int i = tid; i < m; i += kThreads) v[i] = (i == 0) ? 1.0 : x[i] * scale;
    __syncthreads();
    double* A22 = A + (k + 1) + (size_t)n * (k + 1);
    for (int i = tid; i < m; i += kThreads) {
      double acc = 0.0;
      for (int j = 0; j < m; ++j) acc += A22[i + (size_t)n * j] * v[j];
      w[i] = t * acc;
    }
    __syncthreads();
    double pv = 0.0;
    for (int i = tid; i < m; i += kThreads) pv += w[i] * v[i];
    const double K = 0.5 * t * block_sum(pv, red);
    for (int i = tid; i < m; i += kThreads) w[i] -= K * v[i];
    __syncthreads();
    for (int j = 0; j < m; ++j) {
      const double vj = v[j], wj = w[j];
      for (int i = tid; i < m; i += kThreads) A22[i + (size_t)n * j] -= v[i] * wj + w[i] * vj;
    }
    for (int i = 1 + tid; i < m; i += kThreads) x[i] = v[i];
    if (tid == 0) {
      TAU[b + k] = t;
      E[b + k] = beta;
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (n >= 2) {
      D[b + n - 2] = A[(n - 2) + (size_t)n * (n - 2)];
      E[b + n - 2] = A[(n - 1) + (size_t)n * (n - 2)];
    }
    D[b + n - 1] = A[(size_t)(n - 1) * (n + 1)];
    E[b + n - 1] = 0.0;
  }
}

}  // namespace

void eig_set_attributes() {}

void launch_gather(gq_ctx* ctx, const gq_graph* g, const gq_csr* H, double* A, int32_t* status) {
  const gq_graph_dev& dv = g->dev;
  const int maxn = g->info.max_n;
  hipStream_t st = ctx->stream;
  prof_begin(ctx, "k_gather");
  hipLaunchKernelGGL(k_gather, dim3(g->n_sub), dim3(kThreads), 2 * maxn * sizeof(int32_t), st,
                     H->row_ptr, H->col, H->val, A, dv.off2, dv.sub_orb_ptr, dv.sub_orbs,
                     dv.sorted_orbs, dv.sorted_local, dv.order, status);
  prof_end(ctx);
}

void launch_eigensolve(gq_ctx* ctx, const gq_graph* g, gq_eigs* e) {
  const gq_graph_dev& dv = g->dev;
  const int maxn = g->info.max_n;
  hipStream_t st = ctx->stream;
  prof_begin(ctx, "k_tridiag");
  hipLaunchKernelGGL(k_tridiag, dim3(g->n_sub), dim3(kThreads), (2 * maxn + 8) * sizeof(double),
                     st, e->A, dv.off2, dv.sub_orb_ptr, dv.order, e->dd, e->ee, e->tau);
  prof_end(ctx);
  launch_dc(ctx, g, e);
  // the eigenvectors were formed in e->Y; from here on they are e->Q
  std::swap(e->Q, e->Y);
}

}  // namespace gq
