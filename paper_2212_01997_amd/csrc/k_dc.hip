// Divide-and-conquer eigensolver of the symmetric tridiagonal matrices and
// the back-transformation by the Householder reflectors (gfx950, FP64).
//
// Each subgraph's tridiagonal T (from k_tridiag) is split recursively in
// halves down to leaves of at most kLeaf rows: T = diag(T1, T2) + rho v v^T
// with rho = |e| of the cut and v = e_last + sign(e) e_first (both adjacent
// diagonals lowered by rho).  Leaves are solved by implicit QL in one wave.
// A merge of two solved halves diagonalises D + rho z z^T (Cuppen):
//   k_dc_prep   one workgroup per merge: z from the halves' boundary rows,
//               merge-sort of the eigenvalues, deflation of small z_i and of
//               close pairs by plane rotations, the secular roots (two-pole
//               rational iteration with a bisection safeguard, roots kept as
//               offsets from the nearer pole), Gu-Eisenstat recomputed z for
//               orthogonal vectors, column norms and the output order;
//   k_dc_gemm   tiles of Z_new[:, pos] = Z[:, cols] U with U_ij = zh_i n_j /
//               (d_i - lambda_j) formed on the fly, plus the deflated columns;
//   k_dc_copy   the merged block back into place.
// k_backtransform applies H_0 ... H_{n-3} to the eigenvectors of T in blocks
// of 16 reflectors (compact WY, I - V T V^T) on 16-column panels held in LDS,
// and forms the core weights of each eigenvector.
#include <algorithm>
#include <cfloat>

#include "gq_internal.hpp"

namespace gq {

namespace {

constexpr int kThreads = 256;
constexpr int kTile = 64;
constexpr int kKc = 16;
constexpr int kNb = 16;   // reflectors per compact-WY block
constexpr int kCb = 16;   // eigenvector columns per back-transform workgroup

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

__device__ double block_max(double x, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = x;
  __syncthreads();
  double t = red[0];
#pragma unroll
  for (int i = 1; i < kThreads / 64; ++i) t = fmax(t, red[i]);
  return t;
}

// ------------------------------------------------------------------ leaves
// One wave per leaf [lo, lo+m) of subgraph s; every lane runs the scalar QL
// recurrence on a wave-private copy of (d, e) and applies each rotation to its
// own row of Z, kept in LDS.
__global__ __launch_bounds__(64) void k_dc_leaves(
    const int32_t* __restrict__ leaves, const int32_t* __restrict__ sub_orb_ptr,
    const int64_t* __restrict__ off2, const double* __restrict__ D, const double* __restrict__ E,
    double* __restrict__ zbuf, double* __restrict__ lam, int32_t* __restrict__ status) {
  __shared__ double zl[kLeaf][kLeaf + 1];
  __shared__ double d[kLeaf], e[kLeaf], cs[2 * kLeaf];
  __shared__ int rank[kLeaf];
  const int s = leaves[3 * blockIdx.x], lo = leaves[3 * blockIdx.x + 1], m = leaves[3 * blockIdx.x + 2];
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  const int lane = threadIdx.x;
  if (lane < m) {
    double dv = D[b + lo + lane];
    if (lane == 0 && lo > 0) dv -= fabs(E[b + lo - 1]);
    if (lane == m - 1 && lo + m < n) dv -= fabs(E[b + lo + m - 1]);
    d[lane] = dv;
    e[lane] = (lane + 1 < m) ? E[b + lo + lane] : 0.0;
    for (int c = 0; c < m; ++c) zl[lane][c] = (c == lane) ? 1.0 : 0.0;
  }
  __syncthreads();
  int failed = 0;
  for (int l = 0; l < m && !failed; ++l) {
    int iter = 0;
    for (;;) {
      int mm = l;
      while (mm < m - 1) {
        const double dd = fabs(d[mm]) + fabs(d[mm + 1]);
        if (fabs(e[mm]) <= DBL_EPSILON * dd) break;
        ++mm;
      }
      if (mm == l) break;
      if (++iter > 60) {
        failed = 1;
        break;
      }
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = hypot(g, 1.0);
      g = d[mm] - d[l] + e[l] / (g + copysign(r, g));
      double sn = 1.0, c = 1.0, p = 0.0;
      int i = mm - 1;
      bool early = false;
      for (; i >= l; --i) {
        const double f = sn * e[i];
        const double bb = c * e[i];
        r = hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= p;
          e[mm] = 0.0;
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
      const int ilo = early ? i + 1 : l;
      if (lane < m) {
        for (int q = mm - 1; q >= ilo; --q) {
          const double cc = cs[2 * q], ss = cs[2 * q + 1];
          const double zi = zl[lane][q], zj = zl[lane][q + 1];
          zl[lane][q + 1] = ss * zi + cc * zj;
          zl[lane][q] = cc * zi - ss * zj;
        }
      }
      if (early) continue;
      d[l] -= p;
      e[l] = g;
      e[mm] = 0.0;
    }
  }
  __syncthreads();
  if (failed && lane == 0) status[s] = 1;
  if (lane < m) {
    const double x = d[lane];
    int rk = 0;
    for (int j = 0; j < m; ++j) rk += (d[j] < x) || (d[j] == x && j < lane);
    rank[lane] = rk;
    lam[b + lo + rk] = x;
  }
  __syncthreads();
  double* Z = zbuf + off2[s];
  if (lane < m)
    for (int c = 0; c < m; ++c) Z[(lo + lane) + (size_t)n * (lo + rank[c])] = zl[lane][c];
}

// ------------------------------------------------------------- merge prep

struct PrepLds {
  double *D, *z, *dS, *zS, *rc, *rs, *delta, *zeta, *tau, *zhat, *inv, *vals;
  int *perm, *defl, *nd, *rp, *ri, *org, *pos;
};

__device__ PrepLds carve(void* base, int m) {
  PrepLds L;
  double* dp = reinterpret_cast<double*>(base);
  L.D = dp; dp += m;
  L.z = dp; dp += m;
  L.dS = dp; dp += m;
  L.zS = dp; dp += m;
  L.rc = dp; dp += m;
  L.rs = dp; dp += m;
  L.delta = dp; dp += m;
  L.zeta = dp; dp += m;
  L.tau = dp; dp += m;
  L.zhat = dp; dp += m;
  L.inv = dp; dp += m;
  L.vals = dp; dp += m;
  int* ip = reinterpret_cast<int*>(dp);
  L.perm = ip; ip += m;
  L.defl = ip; ip += m;
  L.nd = ip; ip += m;
  L.rp = ip; ip += m;
  L.ri = ip; ip += m;
  L.org = ip; ip += m;
  L.pos = ip; ip += m;
  return L;
}

// Root j of 1/rho + sum_i zeta_i^2 / (delta_i - lambda) = 0 for strictly
// increasing delta.  Returns the origin pole index and the offset tau from it.
__device__ void secular_root(const double* __restrict__ delta, const double* __restrict__ zeta,
                             int k, double rho, int j, int& org, double& tau_out) {
  double a, b;
  int o;
  if (j < k - 1) {
    const double gap = delta[j + 1] - delta[j];
    double w = 1.0 / rho;
    for (int i = 0; i < k; ++i) w += zeta[i] * zeta[i] / ((delta[i] - delta[j]) - 0.5 * gap);
    if (w >= 0.0) {
      o = j;
      a = 0.0;
      b = 0.5 * gap;
    } else {
      o = j + 1;
      a = -0.5 * gap;
      b = 0.0;
    }
  } else {
    double zz = 0.0;
    for (int i = 0; i < k; ++i) zz += zeta[i] * zeta[i];
    o = j;
    a = 0.0;
    b = rho * zz * (1.0 + 8.0 * DBL_EPSILON);
  }
  const double dlo = delta[o];
  const int jl = j;  // left pole of the interval is delta[j], right delta[j+1]
  double x = 0.5 * (a + b);
  for (int it = 0; it < 100; ++it) {
    double w = 1.0 / rho, err = 1.0 / rho, psi1 = 0.0, phi1 = 0.0, Dl = 0.0, Dr = 0.0;
    for (int i = 0; i < k; ++i) {
      const double Di = (delta[i] - dlo) - x;
      const double t = zeta[i] * zeta[i] / Di;
      w += t;
      err += fabs(t);
      if (i <= jl) psi1 += t / Di;
      else phi1 += t / Di;
      if (i == jl) Dl = Di;
      if (i == jl + 1) Dr = Di;
    }
    if (w < 0.0) a = x;
    else if (w > 0.0) b = x;
    if (fabs(w) <= 8.0 * DBL_EPSILON * err || b - a <= 2.0 * DBL_EPSILON * fmax(fabs(a), fabs(b)))
      break;
    double eta;
    if (j < k - 1) {
      const double c = w - Dl * psi1 - Dr * phi1;
      const double s = Dl * Dl * psi1, S = Dr * Dr * phi1;
      const double B = c * (Dl + Dr) + s + S;
      const double C = Dl * Dr * w;
      const double disc = sqrt(fabs(B * B - 4.0 * c * C));
      if (c == 0.0) eta = C / B;
      else if (B <= 0.0) eta = (B - disc) / (2.0 * c);
      else eta = 2.0 * C / (B + disc);
    } else {
      const double c = w - Dl * psi1;
      const double s = Dl * Dl * psi1;
      eta = c != 0.0 ? Dl + s / c : 0.5 * (a + b) - x;
    }
    double xn = x + eta;
    if (!(xn > a && xn < b)) xn = 0.5 * (a + b);
    if (xn == x) break;
    x = xn;
  }
  org = o;
  tau_out = x;
}

__global__ __launch_bounds__(kThreads) void k_dc_prep(
    const int32_t* __restrict__ merges, const int32_t* __restrict__ sub_orb_ptr,
    const int64_t* __restrict__ off2, const double* __restrict__ E, double* __restrict__ zbuf,
    double* __restrict__ lam, int32_t* __restrict__ md_k, int32_t* __restrict__ md_cols,
    int32_t* __restrict__ md_org, int32_t* __restrict__ md_pos, int32_t* __restrict__ md_dsrc,
    int32_t* __restrict__ md_dpos, double* __restrict__ md_delta, double* __restrict__ md_tau,
    double* __restrict__ md_zhat, double* __restrict__ md_inv) {
  extern __shared__ double smem[];
  __shared__ double red[8];
  __shared__ int sh_k, sh_nrot;
  const int mid = blockIdx.x;
  const int s = merges[4 * mid], lo = merges[4 * mid + 1];
  const int m1 = merges[4 * mid + 2], m2 = merges[4 * mid + 3];
  const int m = m1 + m2;
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  double* Z = zbuf + off2[s];
  PrepLds L = carve(smem, m);
  const int tid = threadIdx.x;

  const double beta = E[b + lo + m1 - 1];
  const double rho = fabs(beta);
  const double sg = beta >= 0.0 ? 1.0 : -1.0;

  for (int i = tid; i < m; i += kThreads) {
    L.D[i] = lam[b + lo + i];
    L.z[i] = i < m1 ? Z[(lo + m1 - 1) + (size_t)n * (lo + i)] : sg * Z[(lo + m1) + (size_t)n * (lo + i)];
  }
  // the off-diagonal child blocks hold stale data from earlier levels
  for (int idx = tid; idx < m1 * m2; idx += kThreads) {
    const int r = idx % m1, c = idx / m1;
    Z[(lo + r) + (size_t)n * (lo + m1 + c)] = 0.0;
  }
  for (int idx = tid; idx < m1 * m2; idx += kThreads) {
    const int r = idx % m2, c = idx / m2;
    Z[(lo + m1 + r) + (size_t)n * (lo + c)] = 0.0;
  }
  __syncthreads();
  double part = 0.0;
  for (int i = tid; i < m; i += kThreads) part += L.z[i] * L.z[i];
  const double zz = block_sum(part, red);
  const double zn = sqrt(zz);
  const double rho2 = rho * zz;
  // stable merge of the two ascending lists (first list wins ties)
  for (int i = tid; i < m; i += kThreads) {
    const double x = L.D[i];
    int rk;
    if (i < m1) {
      int a = m1, bb = m;
      while (a < bb) {
        const int md = (a + bb) >> 1;
        if (L.D[md] < x) a = md + 1;
        else bb = md;
      }
      rk = i + (a - m1);
    } else {
      int a = 0, bb = m1;
      while (a < bb) {
        const int md = (a + bb) >> 1;
        if (L.D[md] <= x) a = md + 1;
        else bb = md;
      }
      rk = (i - m1) + a;
    }
    L.perm[rk] = i;
  }
  __syncthreads();
  double mx = 0.0;
  for (int r = tid; r < m; r += kThreads) {
    L.dS[r] = L.D[L.perm[r]];
    L.zS[r] = zn > 0.0 ? L.z[L.perm[r]] / zn : 0.0;
    mx = fmax(mx, fabs(L.dS[r]));
  }
  const double dmax = block_max(mx, red);
  const double tol = 8.0 * DBL_EPSILON * fmax(dmax, rho2);

  // deflation (sequential scan over the sorted poles)
  if (tid == 0) {
    int p = -1, k = 0, nrot = 0;
    for (int i = 0; i < m; ++i) {
      L.defl[i] = 0;
      if (rho2 * fabs(L.zS[i]) <= tol) {
        L.defl[i] = 1;
        continue;
      }
      if (p < 0) {
        p = i;
        continue;
      }
      const double t = hypot(L.zS[p], L.zS[i]);
      const double c = L.zS[i] / t;
      const double sn = -L.zS[p] / t;
      if (fabs((L.dS[i] - L.dS[p]) * c * sn) <= tol) {
        L.rp[nrot] = p;
        L.ri[nrot] = i;
        L.rc[nrot] = c;
        L.rs[nrot] = sn;
        ++nrot;
        L.zS[i] = t;
        L.zS[p] = 0.0;
        const double dp = L.dS[p] * c * c + L.dS[i] * sn * sn;
        L.dS[i] = L.dS[p] * sn * sn + L.dS[i] * c * c;
        L.dS[p] = dp;
        L.defl[p] = 1;
      } else {
        L.nd[k++] = p;
      }
      p = i;
    }
    if (p >= 0) L.nd[k++] = p;
    sh_k = k;
    sh_nrot = nrot;
  }
  __syncthreads();
  const int k = sh_k, nrot = sh_nrot;
  // apply the deflating rotations to the columns of the children's vectors
  // Rotation t pairs sorted indices p_t < i_t with i_t strictly increasing in
  // t, so i_t is untouched before step t and p_t is either untouched or the
  // i of the previous step (then forwarded from a register).  Operands are
  // therefore loaded kPre steps ahead.
  constexpr int kPre = 8;
  for (int r = tid; r < m; r += kThreads) {
    double* row = Z + (lo + r);
    double qa[kPre], qb[kPre];
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      if (u < nrot) {
        qa[u] = row[(size_t)n * (lo + L.perm[L.rp[u]])];
        qb[u] = row[(size_t)n * (lo + L.perm[L.ri[u]])];
      }
    }
    double carry = 0.0;
    int carry_idx = -1;
    for (int t0 = 0; t0 < nrot; t0 += kPre) {
#pragma unroll
      for (int u = 0; u < kPre; ++u) {
        const int t = t0 + u;
        if (t < nrot) {
          const double a = (L.rp[t] == carry_idx) ? carry : qa[u];
          const double bb = qb[u];
          const double na = L.rc[t] * a + L.rs[t] * bb;
          const double nb = L.rc[t] * bb - L.rs[t] * a;
          row[(size_t)n * (lo + L.perm[L.rp[t]])] = na;
          row[(size_t)n * (lo + L.perm[L.ri[t]])] = nb;
          carry = nb;
          carry_idx = L.ri[t];
          const int tn = t + kPre;
          if (tn < nrot) {
            qa[u] = row[(size_t)n * (lo + L.perm[L.rp[tn]])];
            qb[u] = row[(size_t)n * (lo + L.perm[L.ri[tn]])];
          }
        }
      }
    }
  }
  for (int j = tid; j < k; j += kThreads) {
    L.delta[j] = L.dS[L.nd[j]];
    L.zeta[j] = L.zS[L.nd[j]];
  }
  __syncthreads();
  // secular roots
  for (int j = tid; j < k; j += kThreads) {
    int o;
    double t;
    secular_root(L.delta, L.zeta, k, rho2, j, o, t);
    L.org[j] = o;
    L.tau[j] = t;
  }
  __syncthreads();
  // recomputed z: zh_i^2 = (lambda_i - d_i)/rho * prod_{j != i} (d_i - lambda_j)/(d_i - d_j)
  for (int i = tid; i < k; i += kThreads) {
    const double di = L.delta[i];
    double prod = -((di - L.delta[L.org[i]]) - L.tau[i]) / rho2;
    for (int j = 0; j < k; ++j) {
      if (j == i) continue;
      prod *= ((di - L.delta[L.org[j]]) - L.tau[j]) / (di - L.delta[j]);
    }
    L.zhat[i] = copysign(sqrt(fmax(prod, 0.0)), L.zeta[i]);
  }
  __syncthreads();
  for (int j = tid; j < k; j += kThreads) {
    const double dO = L.delta[L.org[j]], tj = L.tau[j];
    double acc = 0.0;
    for (int i = 0; i < k; ++i) {
      const double u = L.zhat[i] / ((L.delta[i] - dO) - tj);
      acc += u * u;
    }
    L.inv[j] = 1.0 / sqrt(acc);
  }
  // output order: roots first (items 0..k-1), then deflated items
  for (int j = tid; j < k; j += kThreads) L.vals[j] = L.delta[L.org[j]] + L.tau[j];
  __syncthreads();
  if (tid == 0) {
    int q = k;
    for (int i = 0; i < m; ++i)
      if (L.defl[i]) {
        L.vals[q] = L.dS[i];
        L.nd[q] = i;  // the tail of nd lists the deflated sorted indices
        ++q;
      }
  }
  __syncthreads();
  for (int it = tid; it < m; it += kThreads) {
    const double x = L.vals[it];
    int rk = 0;
    for (int j = 0; j < m; ++j) rk += (L.vals[j] < x) || (L.vals[j] == x && j < it);
    L.pos[it] = rk;
  }
  __syncthreads();
  const int base = b + lo;
  for (int it = tid; it < m; it += kThreads) lam[base + L.pos[it]] = L.vals[it];
  for (int j = tid; j < k; j += kThreads) {
    md_cols[base + j] = L.perm[L.nd[j]];
    md_org[base + j] = L.org[j];
    md_pos[base + j] = L.pos[j];
    md_delta[base + j] = L.delta[j];
    md_tau[base + j] = L.tau[j];
    md_zhat[base + j] = L.zhat[j];
    md_inv[base + j] = L.inv[j];
  }
  for (int q = tid; q < m - k; q += kThreads) {
    md_dsrc[base + q] = L.perm[L.nd[k + q]];
    md_dpos[base + q] = L.pos[k + q];
  }
  if (tid == 0) md_k[mid] = k;
}

// Z_new[:, pos_j] = sum_i Z[:, cols_i] U_ij (j < k); deflated columns copied.
__global__ __launch_bounds__(kThreads) void k_dc_gemm(
    const int32_t* __restrict__ tiles, const int32_t* __restrict__ merges,
    const int32_t* __restrict__ sub_orb_ptr, const int64_t* __restrict__ off2,
    const double* __restrict__ zbuf, double* __restrict__ wbuf, const int32_t* __restrict__ md_k,
    const int32_t* __restrict__ md_cols, const int32_t* __restrict__ md_org,
    const int32_t* __restrict__ md_pos, const int32_t* __restrict__ md_dsrc,
    const int32_t* __restrict__ md_dpos, const double* __restrict__ md_delta,
    const double* __restrict__ md_tau, const double* __restrict__ md_zhat,
    const double* __restrict__ md_inv) {
  __shared__ double As[kKc][kTile + 1];
  __shared__ double Bs[kKc][kTile + 1];
  __shared__ double cdo[kTile], ctau[kTile], cinv[kTile];
  const int mid = tiles[3 * blockIdx.x], tr = tiles[3 * blockIdx.x + 1], tc = tiles[3 * blockIdx.x + 2];
  const int s = merges[4 * mid], lo = merges[4 * mid + 1];
  const int m = merges[4 * mid + 2] + merges[4 * mid + 3];
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  const int k = md_k[mid];
  const int base = b + lo;
  const double* Z = zbuf + off2[s];
  double* W = wbuf + off2[s];
  const int r0 = tr * kTile, c0 = tc * kTile;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  if (threadIdx.x < kTile) {
    const int c = c0 + threadIdx.x;
    if (c < k) {
      cdo[threadIdx.x] = md_delta[base + md_org[base + c]];
      ctau[threadIdx.x] = md_tau[base + c];
      cinv[threadIdx.x] = md_inv[base + c];
    } else {
      cdo[threadIdx.x] = 0.0;
      ctau[threadIdx.x] = 0.0;
      cinv[threadIdx.x] = 0.0;
    }
  }
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  if (c0 < k) {
    for (int i0 = 0; i0 < k; i0 += kKc) {
      __syncthreads();
      for (int idx = threadIdx.x; idx < kKc * kTile; idx += kThreads) {
        const int rr = idx % kTile, ii = idx / kTile;
        const int r = r0 + rr, i = i0 + ii;
        As[ii][rr] = (r < m && i < k) ? Z[(lo + r) + (size_t)n * (lo + md_cols[base + i])] : 0.0;
      }
      for (int idx = threadIdx.x; idx < kKc * kTile; idx += kThreads) {
        const int cc = idx % kTile, ii = idx / kTile;
        const int c = c0 + cc, i = i0 + ii;
        double u = 0.0;
        if (c < k && i < k) u = md_zhat[base + i] * cinv[cc] / ((md_delta[base + i] - cdo[cc]) - ctau[cc]);
        Bs[ii][cc] = u;
      }
      __syncthreads();
#pragma unroll 4
      for (int ii = 0; ii < kKc; ++ii) {
        double a[4], bv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] = As[ii][tx + 16 * q];
#pragma unroll
        for (int q = 0; q < 4; ++q) bv[q] = Bs[ii][ty + 16 * q];
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[p][q] += a[p] * bv[q];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = c0 + ty + 16 * q;
    if (c >= m) continue;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int r = r0 + tx + 16 * p;
      if (r >= m) continue;
      if (c < k) {
        W[(lo + r) + (size_t)n * (lo + md_pos[base + c])] = acc[p][q];
      } else {
        const int dq = c - k;
        W[(lo + r) + (size_t)n * (lo + md_dpos[base + dq])] =
            Z[(lo + r) + (size_t)n * (lo + md_dsrc[base + dq])];
      }
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_dc_copy(
    const int32_t* __restrict__ tiles, const int32_t* __restrict__ merges,
    const int32_t* __restrict__ sub_orb_ptr, const int64_t* __restrict__ off2,
    const double* __restrict__ wbuf, double* __restrict__ zbuf) {
  const int mid = tiles[3 * blockIdx.x], tr = tiles[3 * blockIdx.x + 1], tc = tiles[3 * blockIdx.x + 2];
  const int s = merges[4 * mid], lo = merges[4 * mid + 1];
  const int m = merges[4 * mid + 2] + merges[4 * mid + 3];
  const int n = sub_orb_ptr[s + 1] - sub_orb_ptr[s];
  const double* W = wbuf + off2[s];
  double* Z = zbuf + off2[s];
  for (int idx = threadIdx.x; idx < kTile * kTile; idx += kThreads) {
    const int r = tr * kTile + idx % kTile, c = tc * kTile + idx / kTile;
    if (r < m && c < m) Z[(lo + r) + (size_t)n * (lo + c)] = W[(lo + r) + (size_t)n * (lo + c)];
  }
}

// ------------------------------------------------------ back-transformation
// Q = H_0 H_1 ... H_{n-3} Z for a panel of kCb eigenvector columns held in LDS.
// Reflector k: H_k = I - tau_k v v^T, v = 1 at row k+1, A[k+2.., k] below.
__global__ __launch_bounds__(kThreads) void k_backtransform(
    const double* __restrict__ abuf, const double* __restrict__ TAU, double* __restrict__ zbuf,
    const int64_t* __restrict__ off2, const int32_t* __restrict__ sub_orb_ptr,
    const int32_t* __restrict__ n_core, const int32_t* __restrict__ order,
    double* __restrict__ wts) {
  extern __shared__ double zc[];  // [n][kCb]
  __shared__ double part[kThreads / 64][2 * kNb][kCb + 1];
  __shared__ double G[kNb][kNb + 1], Wm[kNb][kCb + 1], Tm[kNb][kNb + 1], W2[kNb][kCb + 1];
  const int s = order[blockIdx.x];
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  const int c0 = blockIdx.y * kCb;
  if (c0 >= n) return;
  const int ncol = min(kCb, n - c0);
  const double* A = abuf + off2[s];
  double* Z = zbuf + off2[s];
  const int tid = threadIdx.x;
  const int cl = tid % kCb, rg = tid / kCb;  // column, row group (16 groups)
  for (int idx = tid; idx < n * kCb; idx += kThreads) {
    const int r = idx % n, c = idx / n;
    zc[r * kCb + c] = c < ncol ? Z[r + (size_t)n * (c0 + c)] : 0.0;
  }
  __syncthreads();
  const int nref = n - 2;  // reflectors 0 .. n-3
  for (int kb = ((nref - 1) / kNb) * kNb; nref > 0 && kb >= 0; kb -= kNb) {
    const int nb = min(kNb, nref - kb);
    // V(r, q) for reflector kb+q: 0 above row kb+q+1, 1 there, A below
    auto V = [&](int r, int q) -> double {
      const int top = kb + q + 1;
      if (q >= nb || r < top) return 0.0;
      if (r == top) return 1.0;
      return A[r + (size_t)n * (kb + q)];
    };
    double g[kNb], w[kNb];
#pragma unroll
    for (int q = 0; q < kNb; ++q) g[q] = w[q] = 0.0;
    for (int r = kb + 1 + rg; r < n; r += 16) {
      const double vc = V(r, cl);
      const double zr = zc[r * kCb + cl];
#pragma unroll
      for (int q = 0; q < kNb; ++q) {
        const double vq = V(r, q);
        g[q] += vq * vc;
        w[q] += vq * zr;
      }
    }
    // the four row groups of a wave meet by shuffles, the waves in LDS
    const int wv = tid >> 6, lane = tid & 63;
#pragma unroll
    for (int q = 0; q < kNb; ++q) {
      g[q] += __shfl_xor(g[q], 16, 64);
      g[q] += __shfl_xor(g[q], 32, 64);
      w[q] += __shfl_xor(w[q], 16, 64);
      w[q] += __shfl_xor(w[q], 32, 64);
    }
    if (lane < kCb) {
#pragma unroll
      for (int q = 0; q < kNb; ++q) {
        part[wv][q][cl] = g[q];
        part[wv][kNb + q][cl] = w[q];
      }
    }
    __syncthreads();
    for (int idx = tid; idx < 2 * kNb * kCb; idx += kThreads) {
      const int q = idx / kCb, c = idx % kCb;
      double t = 0.0;
      for (int r = 0; r < kThreads / 64; ++r) t += part[r][q][c];
      if (q < kNb) G[q][c] = t;  // V^T V (column c of the Gram matrix)
      else Wm[q - kNb][c] = t;   // V^T Zc
    }
    __syncthreads();
    // T upper triangular: T_ii = tau_i, T[0:i, i] = -tau_i T[0:i, 0:i] G[0:i, i]
    if (tid == 0) {
      for (int i = 0; i < kNb; ++i)
        for (int j = 0; j < kNb; ++j) Tm[i][j] = 0.0;
      for (int i = 0; i < nb; ++i) {
        const double ti = TAU[b + kb + i];
        for (int r = 0; r < i; ++r) {
          double acc = 0.0;
          for (int q = r; q < i; ++q) acc += Tm[r][q] * G[q][i];
          Tm[r][i] = -ti * acc;
        }
        Tm[i][i] = ti;
      }
    }
    __syncthreads();
    // W2 = T W
    for (int idx = tid; idx < kNb * kCb; idx += kThreads) {
      const int q = idx / kCb, c = idx % kCb;
      double acc = 0.0;
      for (int p = q; p < kNb; ++p) acc += Tm[q][p] * Wm[p][c];
      W2[q][c] = acc;
    }
    __syncthreads();
    // Zc -= V W2
    for (int r = kb + 1 + rg; r < n; r += 16) {
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < kNb; ++q) acc += V(r, q) * W2[q][cl];
      zc[r * kCb + cl] -= acc;
    }
    __syncthreads();
  }
  for (int idx = tid; idx < n * kCb; idx += kThreads) {
    const int r = idx % n, c = idx / n;
    if (c < ncol) Z[r + (size_t)n * (c0 + c)] = zc[r * kCb + c];
  }
  // core weights of the finished columns
  if (tid < ncol) {
    const int c = n_core[s];
    double acc = 0.0;
    for (int r = 0; r < c; ++r) acc += zc[r * kCb + tid] * zc[r * kCb + tid];
    wts[b + c0 + tid] = acc;
  }
}

// T factors of the compact-WY blocks: H_kb ... H_{kb+nb-1} = I - V T V^T with
// T upper triangular (T_ii = tau_i, T[0:i, i] = -tau_i T[0:i, 0:i] V^T v_i).
// One workgroup per (subgraph, block); T stored as kNb x kNb row-major.
__device__ __forceinline__ double refl(const double* A, int n, int kb, int nb, int r, int q) {
  const int top = kb + q + 1;
  if (q >= nb || r < top) return 0.0;
  if (r == top) return 1.0;
  return A[r + (size_t)n * (kb + q)];
}

__global__ __launch_bounds__(kThreads) void k_bt_tfactors(
    const double* __restrict__ abuf, const double* __restrict__ TAU, const int64_t* __restrict__ off2,
    const int32_t* __restrict__ sub_orb_ptr, const int32_t* __restrict__ toff,
    double* __restrict__ tfac) {
  __shared__ double G[kNb][kNb + 1];
  __shared__ double T[kNb][kNb + 1];
  const int s = blockIdx.x;
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  const int kbi = blockIdx.y;
  const int kb = kbi * kNb;
  if (kb >= n - 2) return;
  const int nb = min(kNb, n - 2 - kb);
  const double* A = abuf + off2[s];
  const int q = threadIdx.x % kNb, p = threadIdx.x / kNb;  // G[p][q]
  double acc = 0.0;
  for (int r = kb + 1; r < n; ++r) acc += refl(A, n, kb, nb, r, p) * refl(A, n, kb, nb, r, q);
  G[p][q] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 0; i < kNb; ++i)
      for (int j = 0; j < kNb; ++j) T[i][j] = 0.0;
    for (int i = 0; i < nb; ++i) {
      const double ti = TAU[b + kb + i];
      for (int rr = 0; rr < i; ++rr) {
        double a = 0.0;
        for (int qq = rr; qq < i; ++qq) a += T[rr][qq] * G[qq][i];
        T[rr][i] = -ti * a;
      }
      T[i][i] = ti;
    }
    double* out = tfac + (size_t)(toff[s] + kbi) * kNb * kNb;
    for (int i = 0; i < kNb; ++i)
      for (int j = 0; j < kNb; ++j) out[i * kNb + j] = T[i][j];
  }
}

// Back-transformation of a 16-column panel with the reflector block staged in
// LDS (subgraphs of at most kBtSmall orbitals).
constexpr int kBtSmall = 512;

__global__ __launch_bounds__(kThreads) void k_backtransform_lds(
    const double* __restrict__ abuf, const double* __restrict__ tfac,
    const int32_t* __restrict__ toff, double* __restrict__ zbuf, const int64_t* __restrict__ off2,
    const int32_t* __restrict__ sub_orb_ptr, const int32_t* __restrict__ n_core,
    const int32_t* __restrict__ order, double* __restrict__ wts) {
  extern __shared__ double sm[];
  __shared__ double part[kThreads / 64][kNb][kCb + 1];
  __shared__ double Wm[kNb][kCb + 1], Tm[kNb][kNb + 1], W2[kNb][kCb + 1];
  const int s = order[blockIdx.x];
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  const int c0 = blockIdx.y * kCb;
  if (c0 >= n) return;
  const int ncol = min(kCb, n - c0);
  double* zc = sm;                       // [n][kCb]
  double* vb = sm + (size_t)n * kCb;     // [n][kNb] (rows kb+1.. used)
  const double* A = abuf + off2[s];
  double* Z = zbuf + off2[s];
  const int tid = threadIdx.x;
  const int cl = tid % kCb, rg = tid / kCb;
  const int wv = tid >> 6, lane = tid & 63;
  for (int idx = tid; idx < n * kCb; idx += kThreads) {
    const int r = idx % n, c = idx / n;
    zc[r * kCb + c] = c < ncol ? Z[r + (size_t)n * (c0 + c)] : 0.0;
  }
  const int nref = n - 2;
  for (int kbi = (nref - 1) / kNb; nref > 0 && kbi >= 0; --kbi) {
    const int kb = kbi * kNb;
    const int nb = min(kNb, nref - kb);
    const int nr = n - (kb + 1);
    __syncthreads();
    for (int idx = tid; idx < nr * kNb; idx += kThreads) {
      const int rr = idx % nr, q = idx / nr;
      vb[(kb + 1 + rr) * kNb + q] = refl(A, n, kb, nb, kb + 1 + rr, q);
    }
    if (tid < kNb * kNb) Tm[tid / kNb][tid % kNb] = tfac[(size_t)(toff[s] + kbi) * kNb * kNb + tid];
    __syncthreads();
    double w[kNb];
#pragma unroll
    for (int q = 0; q < kNb; ++q) w[q] = 0.0;
    for (int r = kb + 1 + rg; r < n; r += 16) {
      const double zr = zc[r * kCb + cl];
      const double* vr = vb + r * kNb;
#pragma unroll
      for (int q = 0; q < kNb; ++q) w[q] += vr[q] * zr;
    }
#pragma unroll
    for (int q = 0; q < kNb; ++q) {
      w[q] += __shfl_xor(w[q], 16, 64);
      w[q] += __shfl_xor(w[q], 32, 64);
    }
    if (lane < kCb) {
#pragma unroll
      for (int q = 0; q < kNb; ++q) part[wv][q][cl] = w[q];
    }
    __syncthreads();
    {
      const int q = tid / kCb, c = tid % kCb;
      Wm[q][c] = part[0][q][c] + part[1][q][c] + part[2][q][c] + part[3][q][c];
    }
    __syncthreads();
    {
      const int q = tid / kCb, c = tid % kCb;
      double acc = 0.0;
      for (int p = q; p < kNb; ++p) acc += Tm[q][p] * Wm[p][c];
      W2[q][c] = acc;
    }
    __syncthreads();
    double w2[kNb];
#pragma unroll
    for (int q = 0; q < kNb; ++q) w2[q] = W2[q][cl];
    for (int r = kb + 1 + rg; r < n; r += 16) {
      const double* vr = vb + r * kNb;
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < kNb; ++q) acc += vr[q] * w2[q];
      zc[r * kCb + cl] -= acc;
    }
  }
  __syncthreads();
  for (int idx = tid; idx < n * kCb; idx += kThreads) {
    const int r = idx % n, c = idx / n;
    if (c < ncol) Z[r + (size_t)n * (c0 + c)] = zc[r * kCb + c];
  }
  if (tid < ncol) {
    const int c = n_core[s];
    double acc = 0.0;
    for (int r = 0; r < c; ++r) acc += zc[r * kCb + tid] * zc[r * kCb + tid];
    wts[b + c0 + tid] = acc;
  }
}

}  // namespace

size_t dc_prep_lds(int m) { return (size_t)m * (12 * sizeof(double) + 7 * sizeof(int)); }

void dc_set_attributes() {
  (void)hipFuncSetAttribute((const void*)k_dc_prep, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)dc_prep_lds(kMaxN));
  (void)hipFuncSetAttribute((const void*)k_backtransform,
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(kMaxN * kCb * sizeof(double)));
  (void)hipFuncSetAttribute((const void*)k_backtransform_lds,
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(kBtSmall * (kCb + kNb) * sizeof(double)));
}

void launch_dc(gq_ctx* ctx, const gq_graph* g, gq_eigs* e) {
  const gq_graph_dev& dv = g->dev;
  hipStream_t st = ctx->stream;
  // Z lives in e->Q, the merge scratch in e->Y; eigenvalues in e->eps
  prof_begin(ctx, "k_dc_leaves");
  hipLaunchKernelGGL(k_dc_leaves, dim3(dv.n_leaves), dim3(64), 0, st, dv.dc_leaves, dv.sub_orb_ptr,
                     dv.off2, e->dd, e->ee, e->Q, e->eps, e->status);
  prof_end(ctx);
  for (int lv = 0; lv < (int)g->dc_level_merge_off.size() - 1; ++lv) {
    const int m0 = g->dc_level_merge_off[lv], m1 = g->dc_level_merge_off[lv + 1];
    const int t0 = g->dc_level_tile_off[lv], t1 = g->dc_level_tile_off[lv + 1];
    if (m1 == m0) continue;
    const int maxm = g->dc_level_maxm[lv];
    prof_begin(ctx, "k_dc_prep");
    hipLaunchKernelGGL(k_dc_prep, dim3(m1 - m0), dim3(kThreads), dc_prep_lds(maxm), st,
                       dv.dc_merges + 4 * m0, dv.sub_orb_ptr, dv.off2, e->ee, e->Q, e->eps,
                       e->md_k + m0, e->md_cols, e->md_org, e->md_pos, e->md_dsrc, e->md_dpos,
                       e->md_delta, e->md_tau, e->md_zhat, e->md_inv);
    prof_end(ctx);
    prof_begin(ctx, "k_dc_gemm");
    hipLaunchKernelGGL(k_dc_gemm, dim3(t1 - t0), dim3(kThreads), 0, st, dv.dc_tiles + 3 * t0,
                       dv.dc_merges + 4 * m0, dv.sub_orb_ptr, dv.off2, e->Q, e->Y, e->md_k + m0,
                       e->md_cols, e->md_org, e->md_pos, e->md_dsrc, e->md_dpos, e->md_delta,
                       e->md_tau, e->md_zhat, e->md_inv);
    prof_end(ctx);
    prof_begin(ctx, "k_dc_copy");
    hipLaunchKernelGGL(k_dc_copy, dim3(t1 - t0), dim3(kThreads), 0, st, dv.dc_tiles + 3 * t0,
                       dv.dc_merges + 4 * m0, dv.sub_orb_ptr, dv.off2, e->Y, e->Q);
    prof_end(ctx);
  }
  const int maxn = g->info.max_n;
  // subgraphs are ordered by decreasing size: the first n_big exceed kBtSmall
  int n_big = 0;
  while (n_big < g->n_sub && g->sub_orb_ptr[g->order[n_big] + 1] - g->sub_orb_ptr[g->order[n_big]] > kBtSmall) ++n_big;
  prof_begin(ctx, "k_bt_tfactors");
  hipLaunchKernelGGL(k_bt_tfactors, dim3(g->n_sub, (maxn + kNb - 1) / kNb), dim3(kThreads), 0, st,
                     e->A, e->tau, dv.off2, dv.sub_orb_ptr, dv.bt_toff, e->tfac);
  prof_end(ctx);
  prof_begin(ctx, "k_backtransform");
  if (n_big > 0)
    hipLaunchKernelGGL(k_backtransform, dim3(n_big, (maxn + kCb - 1) / kCb), dim3(kThreads),
                       (size_t)maxn * kCb * sizeof(double), st, e->A, e->tau, e->Q, dv.off2,
                       dv.sub_orb_ptr, dv.n_core, dv.order, e->wts);
  if (n_big < g->n_sub) {
    const int nsm = std::min(maxn, kBtSmall);
    hipLaunchKernelGGL(k_backtransform_lds, dim3(g->n_sub - n_big, (nsm + kCb - 1) / kCb),
                       dim3(kThreads), (size_t)nsm * (kCb + kNb) * sizeof(double), st, e->A,
                       e->tfac, dv.bt_toff, e->Q, dv.off2, dv.sub_orb_ptr, dv.n_core,
                       dv.order + n_big, e->wts);
  }
  prof_end(ctx);
}

}  // namespace gq
