// Principal submatrices and their FP64 eigendecomposition on gfx950.
//
// Fig. 1: each subgraph selects the principal submatrix h = H[orbs, orbs].
// Eq. (SmallKS): h = Q diag(eps) Q^T.  One workgroup (4 waves) per subgraph:
//   k_gather    CSR rows of H -> dense column-major h (binary search of each
//               column index in the subgraph's sorted orbital list, in LDS)
//   k_tridiag   blocked Householder reduction to tridiagonal form, reflectors
//               kept in the lower triangle
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

// Blocked Householder tridiagonalisation, one 1024-thread workgroup per
// subgraph.  Rows are owned by threads (H = 1024/next_pow2(n) threads share a
// row and split its columns).  A panel of kPanel reflectors is formed before
// the trailing matrix is touched: inside the panel the current column and the
// symmetric product use the stale trailing matrix plus the panel corrections
//   A_cur = A - sum_q (v_q w_q^T + w_q v_q^T);
// v_q is kept in A's column k0+q (v[0] = 1 stored at row k0+q+1) and w_q in a
// global panel scratch, so the symmetric product keeps its registers for 16
// loads in flight.  At the end of the panel one pass applies the rank-2*kPanel
// update.  d, e and tau go to D, E, TAU.
constexpr int kTdThreads = 1024;
constexpr int kPanel = 16;
constexpr int kStage = 128;
constexpr int kUnroll = 8;

__device__ double tsum(double x, double* red) {
  x = wave_sum(x);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = x;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < kTdThreads / 64; ++i) t += red[i];
  return t;
}

__global__ __launch_bounds__(kTdThreads) void k_tridiag(
    double* __restrict__ abuf, double* __restrict__ wsc, const int64_t* __restrict__ off2,
    const int32_t* __restrict__ sub_orb_ptr, const int32_t* __restrict__ order,
    double* __restrict__ D, double* __restrict__ E, double* __restrict__ TAU) {
  __shared__ double vl[kMaxN], part[kTdThreads];
  __shared__ double red[kTdThreads / 64];
  __shared__ double ysh[2 * kPanel][kTdThreads / 64];
  __shared__ double yfin[2 * kPanel];
  __shared__ double rowc[2 * kPanel];
  __shared__ double stage[kStage][kPanel + 1];
  __shared__ double alpha_sh;
  const int s = order[blockIdx.x];
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  double* A = abuf + off2[s];
  double* W = wsc + (size_t)b * kPanel;  // W[q * n + r]
  const int tid = threadIdx.x;
  const int H = n <= 128 ? 8 : n <= 256 ? 4 : n <= 512 ? 2 : 1;
  const int P = kTdThreads / H;
  const int r = tid % P, h = tid / P;
  const bool own = (h == 0) && (r < n);
  const int lane = tid & 63, wv = tid >> 6;

  for (int k0 = 0; k0 + 2 < n; k0 += kPanel) {
    const int nb = min(kPanel, n - 2 - k0);
    for (int j = 0; j < nb; ++j) {
      const int c = k0 + j;
      if (own && r == c) {
        for (int q = 0; q < j; ++q) {
          rowc[q] = A[r + (size_t)n * (k0 + q)];
          rowc[kPanel + q] = W[q * n + r];
        }
      }
      __syncthreads();
      double a = 0.0;
      if (own && r >= c) {
        a = A[r + (size_t)n * c];
        for (int q = 0; q < j; ++q)
          a -= A[r + (size_t)n * (k0 + q)] * rowc[kPanel + q] + W[q * n + r] * rowc[q];
        if (r == c) D[b + c] = a;
        if (r == c + 1) alpha_sh = a;
      }
      const double sigma = tsum(own && r >= c + 2 ? a * a : 0.0, red);
      const double alpha = alpha_sh;
      double tau = 0.0, beta = alpha, scale = 0.0;
      if (sigma != 0.0) {
        const double nrm = sqrt(alpha * alpha + sigma);
        beta = alpha >= 0.0 ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      if (own) {
        const double v = r == c + 1 ? 1.0 : (r >= c + 2 ? a * scale : 0.0);
        vl[r] = v;
        if (r >= c + 1) A[r + (size_t)n * c] = v;
        if (r == c) {
          TAU[b + c] = tau;
          E[b + c] = beta;
        }
      }
      __syncthreads();
      if (tau == 0.0) {
        // H = I (column already reduced): it adds no correction to the panel
        if (own) W[j * n + r] = 0.0;
        if (own && r >= c + 1) A[r + (size_t)n * c] = 0.0;
        continue;
      }
      const double vr = r < n ? vl[r] : 0.0;
      // p = A22 v over the stale trailing matrix (row r, columns = h mod H)
      double acc = 0.0;
      if (r >= c + 1 && r < n) {
        const double* row = A + r;
        int col = c + 1 + h;
        double ac[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) ac[u] = 0.0;
        for (; col + (kUnroll - 1) * H < n; col += kUnroll * H) {
          double x[kUnroll];
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) x[u] = row[(size_t)n * (col + u * H)];
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) ac[u] += x[u] * vl[col + u * H];
        }
        for (; col < n; col += H) ac[0] += row[(size_t)n * col] * vl[col];
#pragma unroll
        for (int u = 1; u < kUnroll; ++u) ac[0] += ac[u];
        acc = ac[0];
      }
      part[tid] = acc;
      // y1 = W^T v, y2 = V^T v over the panel so far (rows > c; V, W vanish above)
      for (int q = 0; q < j; ++q) {
        double t1 = 0.0, t2 = 0.0;
        if (own && r > c) {
          t1 = W[q * n + r] * vr;
          t2 = A[r + (size_t)n * (k0 + q)] * vr;
        }
        t1 = wave_sum(t1);
        t2 = wave_sum(t2);
        if (lane == 0) {
          ysh[q][wv] = t1;
          ysh[kPanel + q][wv] = t2;
        }
      }
      __syncthreads();
      if (tid < 2 * kPanel && (tid % kPanel) < j) {
        double t = 0.0;
        for (int w = 0; w < kTdThreads / 64; ++w) t += ysh[tid][w];
        yfin[tid] = t;
      }
      __syncthreads();
      double p = 0.0;
      if (own && r >= c + 1) {
        for (int hh = 0; hh < H; ++hh) p += part[hh * P + r];
        for (int q = 0; q < j; ++q)
          p -= A[r + (size_t)n * (k0 + q)] * yfin[q] + W[q * n + r] * yfin[kPanel + q];
        p *= tau;
      }
      const double K = 0.5 * tau * tsum(own && r >= c + 1 ? p * vr : 0.0, red);
      if (own) W[j * n + r] = r >= c + 1 ? p - K * vr : 0.0;
    }
    __syncthreads();
    // trailing update of rows/cols >= k0 + nb, in two halves of the panel so
    // that a thread's row factors fit in registers
    const int t0 = k0 + nb;
#pragma unroll 1
    for (int qh = 0; qh < kPanel; qh += kPanel / 2) {
      double Vr[kPanel / 2], Wr[kPanel / 2];
#pragma unroll
      for (int q = 0; q < kPanel / 2; ++q) {
        const bool ok = qh + q < nb && r >= t0 && r < n;
        Vr[q] = ok ? A[r + (size_t)n * (k0 + qh + q)] : 0.0;
        Wr[q] = ok ? W[(qh + q) * n + r] : 0.0;
      }
      for (int cc0 = t0; cc0 < n; cc0 += kStage) {
        __syncthreads();
        if (own && r >= cc0 && r < cc0 + kStage) {
#pragma unroll
          for (int q = 0; q < kPanel / 2; ++q) {
            stage[r - cc0][q] = Vr[q];
            stage[r - cc0][kPanel / 2 + q] = Wr[q];
          }
        }
        __syncthreads();
        if (r >= t0 && r < n) {
          const int cend = min(n, cc0 + kStage);
          for (int col = cc0 + h; col < cend; col += H) {
            double* ap = A + r + (size_t)n * col;
            double a = *ap;
            const double* sv = stage[col - cc0];
#pragma unroll
            for (int q = 0; q < kPanel / 2; ++q) a -= Vr[q] * sv[kPanel / 2 + q] + Wr[q] * sv[q];
            *ap = a;
          }
        }
      }
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
  (void)maxn;
  hipLaunchKernelGGL(k_tridiag, dim3(g->n_sub), dim3(kTdThreads), 0, st, e->A, e->wsc, dv.off2,
                     dv.sub_orb_ptr, dv.order, e->dd, e->ee, e->tau);
  prof_end(ctx);
  launch_dc(ctx, g, e);
}

}  // namespace gq
