// Recursive Fermi-operator expansion on the subgraphs (Sec. II.D): the
// zero-temperature density of every principal submatrix by purification,
// with matrix products on FP64 MFMA only, as an alternative to the eigensolve.
//
// Eqs. (Step), (Recur): d = Theta(mu I - h) = lim g_n(... g_0(h)).  Here g_0
// maps the spectrum of h into [0, 1] with mu at 1/2,
//   X_0 = I/2 - (h - mu I) / (2 R),  R >= max |eig(h) - mu| (Gershgorin),
// and g(X) = 3 X^2 - 2 X^3 (McWeeny) drives every eigenvalue above 1/2 to 1
// and below to 0, so X_k -> Theta(mu - h); Eq. (dCollect) keeps the core rows.
// Every X_k is a polynomial in h, so it is symmetric and commutes with X_k^2.
//
//   k_bgemm         C = alpha A^T B + beta D + gamma I on every subgraph:
//                   the four-block 4x4x4 FP64 MFMA tile product of the
//                   response kernels over 64x64 tiles, the tiles of one
//                   subgraph on one XCD; for a symmetric result only the
//                   lower tiles, mirrored
//   k_purify_init   Gershgorin radius and X_0 in place of the gathered h
//   k_purify_check  convergence flags from max |X_{k+1} - X_k| per subgraph
//   k_purify_rows   2 X[0:c, :] into the core-row blocks
#include <algorithm>
#include <type_traits>

#include "gq_internal.hpp"
#include "tile_f64.hpp"

namespace gq {

namespace {

constexpr int kNT = 256;
constexpr int kTM = 64;

// C = alpha A^T B + beta D + gamma I per subgraph, all n x n column-major at
// off2[s], over the lower tiles (ti >= tj) of every subgraph.
//   SYM: A^T B is symmetric (here: A symmetric and commuting with B, or
//        A = B).  Each lower tile writes its block and the mirrored one (a
//        diagonal tile its lower triangle and the mirror), so C is exactly
//        symmetric and every element is written once.
//   else: a general product; the workgroup of tile (ti, tj) also computes
//        block (tj, ti).
// conv (when given): subgraphs with conv[s] >= skip_level are skipped, and
// with copy_b their B is copied to C.  errbits (SYM, when given): the largest
// |C - B| of each subgraph, as the bits of a non-negative double (an atomic
// max, so the result does not depend on the order of the tiles).
template <bool SYM>
__global__ __launch_bounds__(kNT, 4) void k_bgemm(
    const double* __restrict__ A, const double* __restrict__ B, const double* __restrict__ D,
    double* __restrict__ C, double alpha, double beta, double gamma,
    const int32_t* __restrict__ tiles, XcdSplit split, const int64_t* __restrict__ off2,
    const int32_t* __restrict__ sub_orb_ptr, const int32_t* __restrict__ conv, int skip_level,
    int copy_b, unsigned long long* __restrict__ errbits) {
  const int xcd = blockIdx.x & 7, stride = gridDim.x >> 3;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int t = split.off[xcd] + (int)(blockIdx.x >> 3); t < split.off[xcd + 1]; t += stride) {
    const int s = tiles[3 * t], ti = tiles[3 * t + 1], tj = tiles[3 * t + 2];
    const int n = sub_orb_ptr[s + 1] - sub_orb_ptr[s];
    const size_t o = off2[s];
    if (conv && conv[s] >= skip_level) {
      if (copy_b)
        for (int i = threadIdx.x; i < kTM * kTM; i += kNT) {
          const int k = ti * kTM + (i & 63), l = tj * kTM + (i >> 6);
          if (k < n && l < n) {
            C[o + k + (size_t)n * l] = B[o + k + (size_t)n * l];
            if (ti != tj) C[o + l + (size_t)n * k] = B[o + l + (size_t)n * k];
          }
        }
      continue;
    }
    // one block: C(k, l) = alpha acc + beta D + gamma delta_kl for the rows of
    // the product's mode (DG: the diagonal mode, blocks c > r not formed)
    auto put = [&](auto dg, const double (&acc)[4][4], int k0, int l0) {
      constexpr bool DG = decltype(dg)::value;
      double emax = 0.0;
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if (DG && c > r) continue;
          const int k = k0 + xy_row<kTM, DG>(r, w) + (lane >> 4);
          const int l = l0 + 16 * c + (lane & 15);
          if (k < n && l < n && (!SYM || ti != tj || k >= l)) {
            const size_t at = o + k + (size_t)n * l;
            double v = alpha * acc[r][c];
            if (beta != 0.0) v += beta * D[at];
            if (k == l) v += gamma;
            C[at] = v;
            if constexpr (SYM) {
              if (k != l) C[o + l + (size_t)n * k] = v;
              if (errbits) emax = fmax(emax, fabs(v - B[at]));
            }
          }
        }
      if (SYM && errbits) {
#pragma unroll
        for (int o2 = 32; o2 > 0; o2 >>= 1) emax = fmax(emax, __shfl_xor(emax, o2, 64));
        if (lane == 0) atomicMax(errbits + s, (unsigned long long)__double_as_longlong(emax));
      }
    };
    if (SYM && ti == tj) {
      // a diagonal tile of a symmetric result: its lower triangle only
      double acc[4][4];
      xy_block_4b<kTM, false, true>(A + o, B + o, nullptr, n, ti * kTM, tj * kTM, n, n, acc);
      put(std::true_type{}, acc, ti * kTM, tj * kTM);
      continue;
    }
    const int passes = (!SYM && ti != tj) ? 2 : 1;
    for (int pass = 0; pass < passes; ++pass) {
      const int k0 = (pass ? tj : ti) * kTM, l0 = (pass ? ti : tj) * kTM;
      double acc[4][4];
      xy_block_4b<kTM, false>(A + o, B + o, nullptr, n, k0, l0, n, n, acc);
      put(std::false_type{}, acc, k0, l0);
    }
  }
}

// Gershgorin radius of h - mu I and X_0 = I/2 - (h - mu I)/(2R) in place,
// from the lower triangle of h (so X_0 is exactly symmetric); one workgroup
// per subgraph.  Clears the convergence state.
__global__ __launch_bounds__(kNT) void k_purify_init(double* __restrict__ X,
                                                     const int64_t* __restrict__ off2,
                                                     const int32_t* __restrict__ sub_orb_ptr,
                                                     double mu, int32_t* __restrict__ conv,
                                                     unsigned long long* __restrict__ errbits) {
  __shared__ double red[kNT / 64];
  const int s = blockIdx.x;
  const int n = sub_orb_ptr[s + 1] - sub_orb_ptr[s];
  double* h = X + off2[s];
  auto at = [&](int k, int l) { return k >= l ? h[k + (size_t)n * l] : h[l + (size_t)n * k]; };
  double rmax = 0.0;
  for (int k = threadIdx.x; k < n; k += kNT) {
    double acc = 0.0;
    for (int l = 0; l < n; ++l) acc += l == k ? fabs(at(k, l) - mu) : fabs(at(k, l));
    rmax = fmax(rmax, acc);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) rmax = fmax(rmax, __shfl_xor(rmax, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = rmax;
  __syncthreads();
  double R = red[0];
  for (int i = 1; i < kNT / 64; ++i) R = fmax(R, red[i]);
  R = R > 0.0 ? R : 1.0;
  const double sc = -0.5 / R;
  // every thread reads the full lower triangle before any element changes
  __syncthreads();
  for (size_t i = threadIdx.x; i < (size_t)n * n; i += kNT) {
    const int k = (int)(i % n), l = (int)(i / n);
    if (k < l) continue;
    const double v = k == l ? 0.5 + sc * (h[i] - mu) : sc * h[i];
    h[i] = v;
    h[l + (size_t)n * k] = v;
  }
  if (threadIdx.x == 0) {
    conv[s] = 0;
    errbits[s] = 0ull;
  }
}

// After X^2: conv 0 -> 1 once max |X^2 - X| <= tol (the last step runs), and
// 1 -> 2 (done; later steps copy).  Counts the subgraphs still at 0 into *open.
__global__ __launch_bounds__(kNT) void k_purify_check(int n_sub, double tol,
                                                      int32_t* __restrict__ conv,
                                                      unsigned long long* __restrict__ errbits,
                                                      int32_t* __restrict__ open) {
  const int s = blockIdx.x * kNT + threadIdx.x;
  if (s >= n_sub) return;
  if (conv[s] == 1) conv[s] = 2;
  else if (conv[s] == 0) {
    const double e = __longlong_as_double((long long)errbits[s]);
    if (e <= tol) conv[s] = 1;
    else atomicAdd(open, 1);
  }
  errbits[s] = 0ull;
}

__global__ void k_zero_int(int32_t* p) { *p = 0; }

__global__ __launch_bounds__(kNT) void k_purify_rows(const double* __restrict__ X,
                                                     const int64_t* __restrict__ off2,
                                                     const int64_t* __restrict__ offc,
                                                     const int32_t* __restrict__ sub_orb_ptr,
                                                     const int32_t* __restrict__ n_core,
                                                     double* __restrict__ rho) {
  const int s = blockIdx.x;
  const int n = sub_orb_ptr[s + 1] - sub_orb_ptr[s], c = n_core[s];
  const double* x = X + off2[s];
  for (int i = threadIdx.x; i < c * n; i += kNT) {
    const int j = i / n, l = i % n;
    rho[offc[s] + i] = 2.0 * x[j + (size_t)n * l];
  }
}

}  // namespace

// One batched product over every subgraph (lower tiles; see k_bgemm).
template <bool SYM>
void launch_bgemm(gq_ctx* ctx, const gq_graph* g, const double* A, const double* B,
                  const double* D, double* C, double alpha, double beta, double gamma,
                  const int32_t* conv, int skip_level, int copy_b, unsigned long long* errbits) {
  const XcdSplit& sp = g->tri_split;
  int longest = 0;
  for (int x = 0; x < 8; ++x) longest = std::max(longest, sp.off[x + 1] - sp.off[x]);
  if (longest == 0) return;
  hipLaunchKernelGGL((k_bgemm<SYM>), dim3(8 * longest), dim3(kNT), 0, ctx->stream, A, B, D, C,
                     alpha, beta, gamma, g->dev.tri_tiles, sp, g->dev.off2, g->dev.sub_orb_ptr,
                     conv, skip_level, copy_b, errbits);
}
template void launch_bgemm<true>(gq_ctx*, const gq_graph*, const double*, const double*,
                                 const double*, double*, double, double, double, const int32_t*,
                                 int, int, unsigned long long*);
template void launch_bgemm<false>(gq_ctx*, const gq_graph*, const double*, const double*,
                                  const double*, double*, double, double, double, const int32_t*,
                                  int, int, unsigned long long*);

}  // namespace gq

using namespace gq;

extern "C" gq_status gq_purify(gq_ctx* ctx, const gq_graph* g, const gq_csr* H_dev, gq_eigs* e,
                               double mu, int32_t max_iter, double tol, double* rho_blocks_dev,
                               int32_t* iterations) {
  if (!ctx || !g || !H_dev || !e || e->g != g || !rho_blocks_dev) {
    set_error("gq_purify: bad argument (workspace must belong to this graph)");
    return GQ_EINVAL;
  }
  if (H_dev->n_rows != g->N || max_iter < 1 || !(tol > 0.0) || !std::isfinite(mu)) {
    set_error("gq_purify: H rows %d (N = %d), max_iter %d, tol %g or mu %g not valid",
              H_dev->n_rows, g->N, max_iter, tol, mu);
    return GQ_EINVAL;
  }
  if (ctx->capturing) {
    set_error("gq_purify: not available while capturing (it checks convergence on the host)");
    return GQ_EINVAL;
  }
  GQ_HIP(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  const gq_graph_dev& dv = g->dev;
  // buffers: X ping-pongs between A and Q, X^2 in Y; flags in the workspace
  // status and merge arrays (the eigenbasis is overwritten)
  double* X[2] = {e->A, e->Q};
  double* X2 = e->Y;
  int32_t* conv = e->md_cols;                                     // [n_sub] <= sum_n
  unsigned long long* err = reinterpret_cast<unsigned long long*>(e->md_delta);  // [n_sub]
  int32_t* open = e->md_org;                                      // [1]
  e->have_density = false;
  e->q32_valid = false;
  e->overlap_solved = false;
  launch_gather(ctx, g, H_dev, X[0], e->status, "k_gather");
  prof_begin(ctx, "k_purify");
  hipLaunchKernelGGL(k_purify_init, dim3(g->n_sub), dim3(kNT), 0, st, X[0], dv.off2,
                     dv.sub_orb_ptr, mu, conv, err);
  prof_end(ctx);
  int cur = 0, it = 0, left = g->n_sub;
  while (it < max_iter && left > 0) {
    prof_begin(ctx, "k_bgemm");
    // X^2, and max |X^2 - X| per subgraph (idempotency)
    launch_bgemm<true>(ctx, g, X[cur], X[cur], nullptr, X2, 1.0, 0.0, 0.0, conv, 1, 0, err);
    prof_end(ctx);
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, st, open);
    hipLaunchKernelGGL(k_purify_check, dim3((g->n_sub + kNT - 1) / kNT), dim3(kNT), 0, st,
                       g->n_sub, tol, conv, err, open);
    // X' = 3 X^2 - 2 X^2 X (one more step after convergence), done ones copy X
    prof_begin(ctx, "k_bgemm");
    launch_bgemm<true>(ctx, g, X2, X[cur], X2, X[1 - cur], -2.0, 3.0, 0.0, conv, 2, 1, nullptr);
    prof_end(ctx);
    cur = 1 - cur;
    ++it;
    GQ_HIP(hipMemcpyAsync(&left, open, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    GQ_HIP(hipStreamSynchronize(st));
  }
  prof_begin(ctx, "k_purify_rows");
  hipLaunchKernelGGL(k_purify_rows, dim3(g->n_sub), dim3(kNT), 0, st, X[cur], dv.off2, dv.offc,
                     dv.sub_orb_ptr, dv.n_core, rho_blocks_dev);
  prof_end(ctx);
  GQ_HIP(hipGetLastError());
  if (iterations) *iterations = it;
  if (left > 0) {
    set_error("gq_purify: %d subgraphs not converged after %d iterations (an eigenvalue at mu?)",
              left, it);
    return GQ_ENOCONV;
  }
  return GQ_OK;
}
