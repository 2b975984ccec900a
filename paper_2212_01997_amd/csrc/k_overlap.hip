// Non-orthogonal basis (Sec. II.D, Eqs. (SmallKS), (ksSmall) and the
// atomic-orbital congruence after them): per subgraph the Lowdin inverse
// factor z = s^(-1/2) of the overlap submatrix, the orthogonalized
// Hamiltonian h = z h_ao z and the atomic-orbital eigenvectors C = z Q, all
// products on the batched FP64 MFMA kernel.
//
//   k_ov_min            smallest eigenvalue of every s_i (positive definiteness)
//   k_transpose_scale   W^T with W = U diag(sigma^(-1/4)), U the eigenvectors of
//                       s_i, through 64x65 LDS tiles (coalesced both ways)
//   then                z = (W^T)^T W^T = U diag(sigma^(-1/2)) U^T   (symmetric)
//                       h = z (h_ao z)                            (symmetric)
//                       C = z Q                                   (general)
#include <algorithm>

#include "gq_internal.hpp"

namespace gq {

namespace {

constexpr int kNT = 256;
constexpr int kTM = 64;

__global__ __launch_bounds__(kNT) void k_ov_min(const double* __restrict__ eps,
                                                const int32_t* __restrict__ sub_orb_ptr,
                                                int n_sub, double* __restrict__ out) {
  const int s = blockIdx.x * kNT + threadIdx.x;
  if (s >= n_sub) return;
  double m = eps[sub_orb_ptr[s]];
  for (int k = sub_orb_ptr[s] + 1; k < sub_orb_ptr[s + 1]; ++k) m = fmin(m, eps[k]);
  out[s] = m;
}

// Wt(m, k) = sigma_m^(-1/4) U(k, m) for the tile pair (ti, tj) / (tj, ti) of
// every lower tile of the list: read along columns of U, written along
// columns of Wt.
__global__ __launch_bounds__(kNT) void k_transpose_scale(const double* __restrict__ U,
                                                         const double* __restrict__ sigma,
                                                         double* __restrict__ Wt,
                                                         const int32_t* __restrict__ tiles,
                                                         XcdSplit split,
                                                         const int64_t* __restrict__ off2,
                                                         const int32_t* __restrict__ sub_orb_ptr) {
  __shared__ double tile[kTM][kTM + 1];
  const int xcd = blockIdx.x & 7, stride = gridDim.x >> 3;
  for (int t = split.off[xcd] + (int)(blockIdx.x >> 3); t < split.off[xcd + 1]; t += stride) {
    const int s = tiles[3 * t], ti = tiles[3 * t + 1], tj = tiles[3 * t + 2];
    const int b = sub_orb_ptr[s], n = sub_orb_ptr[s + 1] - b;
    const double* u = U + off2[s];
    double* w = Wt + off2[s];
    for (int pass = 0; pass < (ti != tj ? 2 : 1); ++pass) {
      // input block: rows k0.. of U, columns m0..; output rows m0.., columns k0..
      const int k0 = (pass ? tj : ti) * kTM, m0 = (pass ? ti : tj) * kTM;
      __syncthreads();
      for (int i = threadIdx.x; i < kTM * kTM; i += kNT) {
        const int r = i & (kTM - 1), c = i >> 6;  // r along k, c along m
        const int k = k0 + r, m = m0 + c;
        if (k < n && m < n) tile[c][r] = u[k + (size_t)n * m] / sqrt(sqrt(sigma[b + m]));
      }
      __syncthreads();
      for (int i = threadIdx.x; i < kTM * kTM; i += kNT) {
        const int r = i & (kTM - 1), c = i >> 6;  // r along m, c along k
        const int m = m0 + r, k = k0 + c;
        if (k < n && m < n) w[m + (size_t)n * k] = tile[r][c];
      }
    }
  }
}

}  // namespace

void launch_overlap_min(gq_ctx* ctx, const gq_graph* g, gq_eigs* e, double* out) {
  hipLaunchKernelGGL(k_ov_min, dim3((g->n_sub + kNT - 1) / kNT), dim3(kNT), 0, ctx->stream,
                     e->eps, g->dev.sub_orb_ptr, g->n_sub, out);
}

// z_i = U diag(sigma^(-1/2)) U^T from the eigenpairs of s_i in (Q, eps), into
// Z (Y serves as the W^T scratch).
void launch_overlap_factor(gq_ctx* ctx, const gq_graph* g, gq_eigs* e) {
  const XcdSplit& sp = g->tri_split;
  int longest = 0;
  for (int x = 0; x < 8; ++x) longest = std::max(longest, sp.off[x + 1] - sp.off[x]);
  if (longest == 0) return;
  prof_begin(ctx, "k_transpose_scale");
  hipLaunchKernelGGL(k_transpose_scale, dim3(8 * longest), dim3(kNT), 0, ctx->stream, e->Q, e->eps,
                     e->Y, g->dev.tri_tiles, sp, g->dev.off2, g->dev.sub_orb_ptr);
  prof_end(ctx);
  prof_begin(ctx, "k_bgemm");
  launch_bgemm<true>(ctx, g, e->Y, e->Y, nullptr, e->Z, 1.0, 0.0, 0.0, nullptr, 0, 0, nullptr);
  prof_end(ctx);
}

// h = z h_ao z with h_ao gathered in A: W = h_ao z into Y, then A = z W.
void launch_overlap_congruence(gq_ctx* ctx, const gq_graph* g, gq_eigs* e) {
  prof_begin(ctx, "k_bgemm");
  launch_bgemm<false>(ctx, g, e->A, e->Z, nullptr, e->Y, 1.0, 0.0, 0.0, nullptr, 0, 0, nullptr);
  launch_bgemm<true>(ctx, g, e->Z, e->Y, nullptr, e->A, 1.0, 0.0, 0.0, nullptr, 0, 0, nullptr);
  prof_end(ctx);
}

// C = z Q.
void launch_overlap_vectors(gq_ctx* ctx, const gq_graph* g, gq_eigs* e) {
  prof_begin(ctx, "k_bgemm");
  launch_bgemm<false>(ctx, g, e->Z, e->Q, nullptr, e->C, 1.0, 0.0, 0.0, nullptr, 0, 0, nullptr);
  prof_end(ctx);
}

}  // namespace gq
