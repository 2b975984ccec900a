// Principal submatrices and their FP64 eigendecomposition on gfx950.
//
// Fig. 1: each subgraph selects the principal submatrix h = H[orbs, orbs].
// Eq. (SmallKS): h = Q diag(eps) Q^T.  One workgroup (4 waves) per subgraph:
//   k_gather    CSR rows of H -> dense column-major h (binary search of each
//               column index in the subgraph's sorted orbital list, in LDS)
//   k_tridiag   Householder reduction to tridiagonal form, reflectors kept in
//               the lower triangle (symv + rank-2 update streamed from L2)
//   k_formq     explicit Q_H = H_0 H_1 ... H_{n-3}, backward accumulation
//   k_ql        implicit QL with Wilkinson shift on the tridiagonal; every
//               wave runs the scalar rotation recurrence redundantly on its
//               own LDS copy, so rotations need no barrier, and applies them
//               to its quarter of the rows of Q_H (column-major, coalesced,
//               8 columns in flight); then eigenvalues are ranked ascending,
//               the columns permuted into place and the core weights formed.
#include <cfloat>

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

__global__ __launch_bounds__(kThreads) void k_formq(
    const double* __restrict__ abuf, double* __restrict__ qbuf, const int64_t* __restrict__ off2,
    const int32_t* __restrict__ sub_orb_ptr, const int32_t* __restrict__ order,
    const double* __restrict__ TAU) {
  extern __shared__ double v[];
  const int s = order[blockIdx.x];
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  const double* A = abuf + off2[s];
  double* Q = qbuf + off2[s];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const size_t nn = (size_t)n * n;
  for (size_t i = tid; i < nn; i += kThreads) Q[i] = (i % (size_t)(n + 1) == 0) ? 1.0 : 0.0;
  __syncthreads();
  for (int k = n - 3; k >= 0; --k) {
    const double t = TAU[b + k];
    if (t == 0.0) continue;
    const int m = n - k - 1;
    for (int i = tid; i < m; i += kThreads) v[i] = (i == 0) ? 1.0 : A[(k + 1 + i) + (size_t)n * k];
    __syncthreads();
    for (int j = k + 1 + wv; j < n; j += kWaves) {
      double* q = Q + (k + 1) + (size_t)n * j;
      double acc = 0.0;
      for (int i = lane; i < m; i += 64) acc += v[i] * q[i];
      acc = wave_sum(acc) * t;
      for (int i = lane; i < m; i += 64) q[i] -= acc * v[i];
    }
    __syncthreads();
  }
}

// Rotations i = hi, hi-1, ..., lo act on columns (i, i+1) of the rows owned by
// this thread: z_{i+1} <- s z_i + c z_{i+1},  z_i <- c z_i - s z_{i+1}.
__device__ __forceinline__ void apply_sweep(double* __restrict__ Q, int n, int row,
                                            const double* __restrict__ cs, int lo, int hi) {
  double carry = Q[row + (size_t)n * (hi + 1)];
  int i = hi;
  while (i >= lo) {
    const int cnt = min(8, i - lo + 1);
    double z[8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (u < cnt) z[u] = Q[row + (size_t)n * (i - u)];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (u < cnt) {
        const double c = cs[2 * (i - u)], sn = cs[2 * (i - u) + 1];
        Q[row + (size_t)n * (i - u + 1)] = sn * z[u] + c * carry;
        carry = c * z[u] - sn * carry;
      }
    }
    i -= cnt;
  }
  Q[row + (size_t)n * lo] = carry;
}

__global__ __launch_bounds__(kThreads) void k_ql(
    double* __restrict__ zbuf, double* __restrict__ qbuf, const int64_t* __restrict__ off2,
    const int32_t* __restrict__ sub_orb_ptr, const int32_t* __restrict__ n_core,
    const int32_t* __restrict__ order, const double* __restrict__ D,
    const double* __restrict__ E, double* __restrict__ eps, double* __restrict__ wts,
    int32_t* __restrict__ status) {
  extern __shared__ double sm[];
  const int s = order[blockIdx.x];
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double* d = sm + (size_t)wv * 4 * n;
  double* e = d + n;
  double* cs = e + n;
  int32_t* rank = reinterpret_cast<int32_t*>(sm + (size_t)kWaves * 4 * n);
  double* Z = zbuf + off2[s];
  for (int i = lane; i < n; i += 64) {
    d[i] = D[b + i];
    e[i] = (i + 1 < n) ? E[b + i] : 0.0;
  }
  __syncthreads();

  int failed = 0;
  for (int l = 0; l < n && !failed; ++l) {
    int iter = 0;
    for (;;) {
      int m = l;
      while (m < n - 1) {
        const double dd = fabs(d[m]) + fabs(d[m + 1]);
        if (fabs(e[m]) <= DBL_EPSILON * dd) break;
        ++m;
      }
      if (m == l) break;
      if (++iter > 60) {
        failed = 1;
        break;
      }
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + copysign(r, g));
      double sn = 1.0, c = 1.0, p = 0.0;
      int i = m - 1;
      bool early = false;
      for (; i >= l; --i) {
        const double f = sn * e[i];
        const double bb = c * e[i];
        r = hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= p;
          e[m] = 0.0;
          early = true;
          break;
        }
        sn = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * sn + 2.0 * c * bb;
        p = sn * r;
        d[i + 1] = g + p;
        g = c * r - bb;
        cs[2 * i] = c;
        cs[2 * i + 1] = sn;
      }
      const int lo = early ? i + 1 : l;
      if (lo <= m - 1)
        for (int row = tid; row < n; row += kThreads) apply_sweep(Z, n, row, cs, lo, m - 1);
      if (early) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  __syncthreads();
  if (failed && tid == 0) status[s] = 1;
  // ascending order (ties by index), taken from wave 0's copy
  const double* d0 = sm;
  for (int k = tid; k < n; k += kThreads) {
    const double x = d0[k];
    int rk = 0;
    for (int j = 0; j < n; ++j) rk += (d0[j] < x) || (d0[j] == x && j < k);
    rank[k] = rk;
    eps[b + rk] = x;
  }
  __syncthreads();
  double* Q = qbuf + off2[s];
  for (int k = 0; k < n; ++k) {
    const size_t dst = (size_t)n * rank[k], src = (size_t)n * k;
    for (int row = tid; row < n; row += kThreads) Q[row + dst] = Z[row + src];
  }
  __syncthreads();
  const int c = n_core[s];
  for (int k = tid; k < n; k += kThreads) {
    double acc = 0.0;
    for (int j = 0; j < c; ++j) {
      const double q = Q[j + (size_t)n * k];
      acc += q * q;
    }
    wts[b + k] = acc;
  }
}

}  // namespace

void eig_set_attributes() {
  const size_t lds = (size_t)kWaves * 4 * kMaxN * sizeof(double) + kMaxN * sizeof(int32_t);
  (void)hipFuncSetAttribute((const void*)k_ql, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

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
  prof_begin(ctx, "k_formq");
  hipLaunchKernelGGL(k_formq, dim3(g->n_sub), dim3(kThreads), maxn * sizeof(double), st, e->A,
                     e->Y, dv.off2, dv.sub_orb_ptr, dv.order, e->tau);
  prof_end(ctx);
  const size_t lds = (size_t)kWaves * 4 * maxn * sizeof(double) + maxn * sizeof(int32_t);
  prof_begin(ctx, "k_ql");
  hipLaunchKernelGGL(k_ql, dim3(g->n_sub), dim3(kThreads), lds, st, e->Y, e->Q, dv.off2,
                     dv.sub_orb_ptr, dv.n_core, dv.order, e->dd, e->ee, e->eps, e->wts, e->status);
  prof_end(ctx);
}

}  // namespace gq
