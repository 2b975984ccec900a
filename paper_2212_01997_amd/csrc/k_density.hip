// Shared chemical potential, density core rows, mu-response rows and the
// divided-difference matrix of the Fermi function (gfx950, FP64).
//
// Sec. II.G: one mu for all subgraphs solves 2 sum_{i,k} w_ik f(eps_ik; mu) =
// N_e with w_ik the squared core part of eigenvector k.  Found here by
// multisection: every pass evaluates the occupation at kMuPoints chemical
// potentials inside the current bracket (block partial sums, then one
// fixed-order reduction), keeping the bracket on the device.
// Eq. (DD): core rows 2 Q_c diag(f) Q^T.  Eq. (dddmu): 2 beta Q_c diag(f(1-f)) Q^T.
// Divided differences dF_kl = (f_k - f_l)/(e_k - e_l) use the exact form
//   -(beta/4) sinhc(x) / (cosh(y_k) cosh(y_l)),  y = beta (e - mu)/2,  x = y_k - y_l,
// with each cosh written as e^{|y|}(1 + e^{-2|y|})/2, so that nothing overflows
// and equal eigenvalues give f'(e) without a special case.
#include <cfloat>

#include "gq_internal.hpp"

namespace gq {

namespace {

constexpr int kThreads = 256;
constexpr int kMuChunk = 256;  // (eps, w) pairs per block of the occupation pass

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

__device__ double block_sum(double x, double* red) {
  x = wave_sum(x);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = x;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < kThreads / 64; ++i) t += red[i];
  return t;
}

// Fermi occupation and f(1-f) from t = exp(-|x|), x = (e - mu)/kT
__device__ __forceinline__ void fermi2(double e, double mu, double beta, double& f, double& f1f) {
  const double x = (e - mu) * beta;
  const double t = exp(-fabs(x));
  const double inv = 1.0 / (1.0 + t);
  f = x > 0.0 ? t * inv : inv;
  f1f = t * inv * inv;
}

// state: [0] lo, [1] hi, [2] mu, [3] kT, [4] n_elec, [5] warm-start guess,
// [6] 1 while the next pass is the warm-start pass, else 0.  Eigenvalues are
// ascending within each subgraph, so the extremes are the first and last of
// each.  The bracket starts at the eigenvalue span widened by 50 kT, where the
// occupation sum is below and above N_e.
__global__ __launch_bounds__(kThreads) void k_mu_init(const double* __restrict__ eps,
                                                      const int32_t* __restrict__ sub_orb_ptr,
                                                      int n_sub, double* __restrict__ state,
                                                      double kT, double n_elec, double guess) {
  __shared__ double rmin[kThreads], rmax[kThreads];
  double lo = DBL_MAX, hi = -DBL_MAX;
  for (int s = threadIdx.x; s < n_sub; s += kThreads) {
    lo = fmin(lo, eps[sub_orb_ptr[s]]);
    hi = fmax(hi, eps[sub_orb_ptr[s + 1] - 1]);
  }
  rmin[threadIdx.x] = lo;
  rmax[threadIdx.x] = hi;
  __syncthreads();
  for (int o = kThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      rmin[threadIdx.x] = fmin(rmin[threadIdx.x], rmin[threadIdx.x + o]);
      rmax[threadIdx.x] = fmax(rmax[threadIdx.x], rmax[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    state[0] = rmin[0] - 50.0 * kT;
    state[1] = rmax[0] + 50.0 * kT;
    state[2] = 0.5 * (state[0] + state[1]);
    state[3] = kT;
    state[4] = n_elec;
    const bool warm = guess == guess;  // not NaN
    state[5] = warm ? guess : 0.0;
    state[6] = warm ? 1.0 : 0.0;
  }
}

// Point j of a pass over the bracket [lo, hi]: evenly spaced, or in the
// warm-start pass guess -+ kT 4^k (k = 7 .. -8 below the guess, -8 .. 7 above),
// clipped to the bracket; ascending in j either way.
__device__ __forceinline__ double mu_point(const double* state, double lo, double hi, int j) {
  if (state[6] != 0.0) {
    const double g = state[5], kT = state[3];
    const double off = j < kMuPoints / 2 ? -kT * ldexp(1.0, 2 * (7 - j))
                                         : kT * ldexp(1.0, 2 * (j - kMuPoints / 2 - 8));
    return fmin(hi, fmax(lo, g + off));
  }
  return lo + (hi - lo) * ((double)(j + 1) / (double)(kMuPoints + 1));
}

// true once the bracket holds no double strictly inside: later passes would
// not change it
__device__ __forceinline__ bool mu_done(double lo, double hi) { return !(nextafter(lo, hi) < hi); }

__global__ __launch_bounds__(kThreads) void k_mu_eval(const double* __restrict__ eps,
                                                      const double* __restrict__ wts, int64_t count,
                                                      const double* __restrict__ state,
                                                      double* __restrict__ part) {
  constexpr int kH = kThreads / kMuPoints;  // threads per point
  __shared__ double se[kMuChunk], sw[kMuChunk];
  __shared__ double hp[kH][kMuPoints];
  const double lo = state[0], hi = state[1], beta = 1.0 / state[3];
  if (mu_done(lo, hi)) return;
  const int64_t base = (int64_t)blockIdx.x * kMuChunk;
  const int cnt = (int)min<int64_t>(kMuChunk, count - base);
  for (int i = threadIdx.x; i < cnt; i += kThreads) {
    se[i] = eps[base + i];
    sw[i] = wts[base + i];
  }
  __syncthreads();
  const int j = threadIdx.x % kMuPoints;
  const int h = threadIdx.x / kMuPoints;
  const double mu = mu_point(state, lo, hi, j);
  double acc = 0.0;
  for (int p = h; p < cnt; p += kH) {
    double f, f1f;
    fermi2(se[p], mu, beta, f, f1f);
    acc += sw[p] * f;
  }
  hp[h][j] = acc;
  __syncthreads();
  if (h == 0) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kH; ++q) t += hp[q][j];
    part[(size_t)blockIdx.x * kMuPoints + j] = t;
  }
}

// Fixed-order reduction of the block partials: group g of kMuGroups sums the
// blocks g, g + kMuGroups, ... in order, then the groups are added in order.
constexpr int kMuGroups = 8;

__global__ __launch_bounds__(kMuPoints * kMuGroups) void k_mu_update(
    const double* __restrict__ part, int nblk, double* __restrict__ state) {
  __shared__ double G[kMuGroups][kMuPoints];
  __shared__ double F[kMuPoints];
  const int j = threadIdx.x % kMuPoints, g = threadIdx.x / kMuPoints;
  if (mu_done(state[0], state[1])) return;
  double acc = 0.0;
  // unrolled so that the loads are in flight together; the adds keep their order
#pragma unroll 8
  for (int b = g; b < nblk; b += kMuGroups) acc += part[(size_t)b * kMuPoints + j];
  G[g][j] = acc;
  __syncthreads();
  if (g == 0) {
    double t = 0.0;
    for (int q = 0; q < kMuGroups; ++q) t += G[q][j];
    F[j] = 2.0 * t - state[4];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double lo = state[0], hi = state[1];
    int first = kMuPoints;
    for (int q = 0; q < kMuPoints; ++q)
      if (F[q] >= 0.0) {
        first = q;
        break;
      }
    const double nlo = first == 0 ? lo : mu_point(state, lo, hi, first - 1);
    const double nhi = first == kMuPoints ? hi : mu_point(state, lo, hi, first);
    state[0] = nlo;
    state[1] = nhi;
    state[2] = 0.5 * (nlo + nhi);
    state[6] = 0.0;
  }
}

// v_mfma_f64_16x16x4f64 on gfx950: lane l supplies A(l%16, l/16) and
// B(l/16, l%16); D(i, j) is returned in lane j + 16*(i%4), register i/4.
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kDC = 128;  // columns per workgroup of the core-row products
constexpr int kDU = 4;    // K steps of operands loaded ahead

// Core rows of both products for kDC columns l of one subgraph:
//   rho[j, l] = sum_m Q[j, m] 2 f_m Q[l, m],
//   M[j, l]   = sum_m Q[j, m] 2 beta f_m (1 - f_m) Q[l, m],   j < c,
// 32 core rows J0 .. J0 + 31 per workgroup (J0 = 32 blockIdx.y; blocks past
// the core return).  Wave w owns columns L0 + 32 w .. + 31 (two 16-column
// tiles) and both 16-row tiles of the block's core rows; the K steps run over
// m, the A operand Q[j, m] g(m) is formed in registers and one load of
// Q[l, m] feeds both products.  The workgroup of the first column and row
// block also forms tmu = 2 beta sum f(1-f) w.
__global__ __launch_bounds__(kThreads) void k_density_rows(
    const double* __restrict__ qbuf, const double* __restrict__ eps,
    const double* __restrict__ wts, const int64_t* __restrict__ off2,
    const int64_t* __restrict__ offc, const int32_t* __restrict__ sub_orb_ptr,
    const int32_t* __restrict__ n_core, const int32_t* __restrict__ order,
    const double* __restrict__ state, double* __restrict__ rho, double* __restrict__ mrows,
    double* __restrict__ tmu, int ncb) {
  __shared__ double red[kThreads / 64];
  const int s = order[blockIdx.x / ncb];
  const int L0 = (blockIdx.x % ncb) * kDC;
  const int J0 = 32 * blockIdx.y;
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  if (L0 >= n) return;
  const int c = n_core[s];
  if (J0 >= c) return;
  const double mu = state[2], beta = 1.0 / state[3];
  const double* Q = qbuf + off2[s];
  const double* e = eps + b;

  if (L0 == 0 && J0 == 0) {
    double acc = 0.0;
    for (int k = threadIdx.x; k < n; k += kThreads) {
      double f, f1f;
      fermi2(e[k], mu, beta, f, f1f);
      acc += f1f * wts[b + k];
    }
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0) tmu[s] = 2.0 * beta * t;
  }

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  int lcol[2];
  bool colok[2];
#pragma unroll
  for (int y = 0; y < 2; ++y) {
    lcol[y] = L0 + 32 * w + 16 * y + li;
    colok[y] = lcol[y] < n;
  }
  // rows J0 + li and J0 + 16 + li of Q, clamped to valid rows (zeroed below
  // when not core)
  const int r0 = min(J0 + li, n - 1), r1 = min(J0 + 16 + li, n - 1);
  const bool ok0 = J0 + li < c, ok1 = J0 + 16 + li < c;
  v4d ar[2][2], am[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) ar[x][y] = am[x][y] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int m0 = 0; m0 < n; m0 += 4 * kDU) {
    double q0[kDU], q1[kDU], bv[2][kDU], em[kDU];
#pragma unroll
    for (int u = 0; u < kDU; ++u) {
      const int mc = min(m0 + 4 * u + lk, n - 1);
      q0[u] = Q[r0 + (size_t)n * mc];
      q1[u] = Q[r1 + (size_t)n * mc];
#pragma unroll
      for (int y = 0; y < 2; ++y) bv[y][u] = Q[min(lcol[y], n - 1) + (size_t)n * mc];
      em[u] = e[mc];
    }
#pragma unroll
    for (int u = 0; u < kDU; ++u) {
      const bool ok = m0 + 4 * u + lk < n;
      double f, f1f;
      fermi2(em[u], mu, beta, f, f1f);
      const double gf = ok ? 2.0 * f : 0.0, gm = ok ? 2.0 * beta * f1f : 0.0;
      const double a0 = ok0 ? q0[u] : 0.0, a1 = ok1 ? q1[u] : 0.0;
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        ar[0][y] = mfma16(a0 * gf, bv[y][u], ar[0][y]);
        ar[1][y] = mfma16(a1 * gf, bv[y][u], ar[1][y]);
        am[0][y] = mfma16(a0 * gm, bv[y][u], am[0][y]);
        am[1][y] = mfma16(a1 * gm, bv[y][u], am[1][y]);
      }
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
        if (rho) rho[base + (size_t)j0 * n + lcol[y]] = ar[0][y][r];
        mrows[base + (size_t)j0 * n + lcol[y]] = am[0][y][r];
      }
      if (j1 < c) {
        if (rho) rho[base + (size_t)j1 * n + lcol[y]] = ar[1][y][r];
        mrows[base + (size_t)j1 * n + lcol[y]] = am[1][y][r];
      }
    }
  }
}

constexpr int kDdCols = 32;  // columns of dF per workgroup

// sinh(x)/x for |x| < 0.5 by its Taylor series sum_k x^2k / (2k+1)! up to
// x^16 (the first omitted term is below 1e-19)
__device__ __forceinline__ double sinhc_small(double x) {
  const double u = x * x;
  double p = 1.0 / 355687428096000.0;
  p = fma(p, u, 1.0 / 1307674368000.0);
  p = fma(p, u, 1.0 / 6227020800.0);
  p = fma(p, u, 1.0 / 39916800.0);
  p = fma(p, u, 1.0 / 362880.0);
  p = fma(p, u, 1.0 / 5040.0);
  p = fma(p, u, 1.0 / 120.0);
  p = fma(p, u, 1.0 / 6.0);
  return fma(p, u, 1.0);
}

// dF for kDdCols columns l of one subgraph, all rows k.  The per-orbital
// factors |y_k|, e^{-|y_k|} and 1 + e^{-2|y_k|} are formed once in LDS; an
// element then needs no exponential for x < 0.5 and two otherwise.
__global__ __launch_bounds__(kThreads) void k_divided_differences(
    const double* __restrict__ eps, const int64_t* __restrict__ off2,
    const int32_t* __restrict__ sub_orb_ptr, const int32_t* __restrict__ order,
    const double* __restrict__ state, double* __restrict__ dfbuf, int ldn) {
  extern __shared__ double dd_lds[];  // four arrays of ldn (the largest n) doubles
  double* se = dd_lds;
  double* sa = se + ldn;
  double* sx = sa + ldn;
  double* sd = sx + ldn;
  const int s = order[blockIdx.x];
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  const int l0 = blockIdx.y * kDdCols;
  if (l0 >= n) return;
  const double mu = state[2], beta = 1.0 / state[3];
  for (int k = threadIdx.x; k < n; k += kThreads) {
    const double ek = eps[b + k];
    const double ak = fabs(0.5 * beta * (ek - mu));
    const double xk = exp(-ak);
    se[k] = ek;
    sa[k] = ak;
    sx[k] = xk;
    sd[k] = 1.0 + xk * xk;
  }
  __syncthreads();
  double* dF = dfbuf + off2[s];
  const int l1 = min(n, l0 + kDdCols);
  for (int l = l0; l < l1; ++l) {
    const double el = se[l], al = sa[l], xl = sx[l], dl = sd[l];
    for (int k = threadIdx.x; k < n; k += kThreads) {
      const double den = sd[k] * dl;
      const double x = fabs(0.5 * beta * (se[k] - el));
      double val;
      if (x < 0.5) {
        val = -beta * sinhc_small(x) * (sx[k] * xl) / den;
      } else {
        const double g = exp(x - sa[k] - al), t = exp(-2.0 * x);
        val = -beta * g * (1.0 - t) / (2.0 * x * den);
      }
      dF[k + (size_t)n * l] = val;
    }
  }
}

}  // namespace

void launch_mu(gq_ctx* ctx, const gq_graph* g, gq_eigs* e, double guess) {
  const int64_t count = g->info.sum_n;
  hipStream_t st = ctx->stream;
  prof_begin(ctx, "k_mu");
  hipLaunchKernelGGL(k_mu_init, dim3(1), dim3(kThreads), 0, st, e->eps, g->dev.sub_orb_ptr,
                     g->n_sub, e->mu_state, e->kT, e->n_elec, guess);
  const int nblk = (int)((count + kMuChunk - 1) / kMuChunk);
  // the warm pass narrows the bracket to the two points around the root, at
  // worst the whole span: one pass more keeps the cold-start resolution
  const int passes = kMuPasses + (guess == guess ? 1 : 0);
  for (int pass = 0; pass < passes; ++pass) {
    hipLaunchKernelGGL(k_mu_eval, dim3(nblk), dim3(kThreads), 0, st, e->eps, e->wts, count,
                       e->mu_state, e->mu_part);
    hipLaunchKernelGGL(k_mu_update, dim3(1), dim3(kMuPoints * kMuGroups), 0, st, e->mu_part, nblk,
                       e->mu_state);
  }
  prof_end(ctx);
}

int mu_blocks_for(int64_t count) { return (int)((count + kMuChunk - 1) / kMuChunk); }

void launch_density(gq_ctx* ctx, const gq_graph* g, gq_eigs* e, double* rho_blocks) {
  const gq_graph_dev& dv = g->dev;
  hipStream_t st = ctx->stream;
  prof_begin(ctx, "k_density_rows");
  const int ncb = (g->info.max_n + kDC - 1) / kDC;
  // in a non-orthogonal basis the rows are the atomic-orbital ones, from
  // C = z Q; mu and tmu stay on the orthogonalized weights
  const double* qrows = e->overlap_solved ? e->C : e->Q;
  hipLaunchKernelGGL(k_density_rows, dim3(g->n_sub * ncb, (g->info.max_c + 31) / 32),
                     dim3(kThreads), 0, st, qrows, e->eps,
                     e->wts, dv.off2, dv.offc, dv.sub_orb_ptr, dv.n_core, dv.order, e->mu_state,
                     rho_blocks, e->M, e->tmu, ncb);
  prof_end(ctx);
}

void launch_divided_differences(gq_ctx* ctx, const gq_graph* g, gq_eigs* e, hipStream_t st) {
  const gq_graph_dev& dv = g->dev;
  prof_begin_on(ctx, "k_divided_differences", st);
  dim3 grid(g->n_sub, (g->info.max_n + kDdCols - 1) / kDdCols);
  // 4 kMaxN doubles (64 KiB) at most: within the default LDS limit
  const int ldn = g->info.max_n;
  hipLaunchKernelGGL(k_divided_differences, grid, dim3(kThreads), 4 * ldn * sizeof(double), st,
                     e->eps, dv.off2, dv.sub_orb_ptr, dv.order, e->mu_state, e->A, ldn);
  prof_end(ctx);
}

}  // namespace gq
