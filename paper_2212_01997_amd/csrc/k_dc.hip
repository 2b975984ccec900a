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
//               (d_i - lambda_j) formed on the fly, plus the deflated columns.
// The vectors alternate between Q and a scratch of the same layout: a merge at
// depth d reads Q for odd d and the scratch for even d and writes the other,
// so the top merges (d = 0) leave them in Q, and every leaf is written where
// its parent merge reads.
// k_bt_mfma applies H_0 ... H_{n-3} to the eigenvectors of T in blocks of 16
// reflectors (compact WY, I - V T V^T; T factors from k_bt_tfactors) on
// 16-column panels held in registers, both products on FP64 MFMA, and forms
// the core weights of each eigenvector.
#include <algorithm>
#include <cfloat>

#include "gq_internal.hpp"

namespace gq {

namespace {

constexpr int kThreads = 256;
constexpr int kTile = 64;
constexpr int kNb = 16;   // reflectors per compact-WY block
// row stride of the staged reflector block: 17 doubles keep both the 16-row
// reads of the update and the 16-column reads of V^T Z in distinct LDS banks
constexpr int kLdv = kNb + 1;

// v_mfma_f64_4x4x4f64 (four blocks): lane l supplies A_b(l%4, l/16) and
// B_b(l/16, l%4) of block b = (l/4)%4 and receives D_b(l/16, l%4); with the
// blocks side by side along the columns one instruction yields a 4x16 strip.
__device__ __forceinline__ double mfma4b(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

// x from the lane given by the DPP control kCtrl (quad_perm, row_mirror, ...),
// both 32-bit halves moved by VALU permutes rather than the LDS crossbar.
template <int kCtrl>
__device__ __forceinline__ double dpp_f64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, kCtrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), kCtrl, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// 1/x from the hardware reciprocal and two Newton steps: within about an ulp,
// without the scaling and fix-up steps of an IEEE division
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

template <int NT>
__device__ double block_sum(double x, double* red) {
  x = wave_sum(x);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = x;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) t += red[i];
  return t;
}

template <int NT>
__device__ double block_max(double x, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = x;
  __syncthreads();
  double t = red[0];
#pragma unroll
  for (int i = 1; i < NT / 64; ++i) t = fmax(t, red[i]);
  return t;
}

// ------------------------------------------------------------------ leaves
// Sixteen lanes per leaf [lo, lo+m) of subgraph s, four leaves per wave:
// every lane of a group runs the scalar QL recurrence on the group's copy of
// (d, e) and applies each rotation to its own row of Z, kept in LDS.
__global__ __launch_bounds__(64) void k_dc_leaves(
    const int32_t* __restrict__ leaves, int n_leaves, const int32_t* __restrict__ sub_orb_ptr,
    const int64_t* __restrict__ off2, const double* __restrict__ D, const double* __restrict__ E,
    double* __restrict__ qbuf, double* __restrict__ sbuf, double* __restrict__ lam,
    int32_t* __restrict__ status, int iter_cap) {
  // four leaves per wave: lanes 16 gi .. 16 gi + 15 take leaf 4 blockIdx.x + gi
  // with arrays of their own (the QL loop below has no barrier, so the groups
  // may diverge)
  __shared__ double zls[4][kLeaf][kLeaf + 1];
  __shared__ double ds[4][kLeaf], es[4][kLeaf], css[4][2 * kLeaf];
  __shared__ int ranks[4][kLeaf];
  const int gi = threadIdx.x >> 4, lane = threadIdx.x & 15;
  const int leaf = 4 * blockIdx.x + gi;
  const bool live = leaf < n_leaves;
  const int lf = live ? leaf : n_leaves - 1;
  const int s = leaves[4 * lf], lo = leaves[4 * lf + 1], m = live ? leaves[4 * lf + 2] : 0;
  double* zbuf = leaves[4 * lf + 3] ? sbuf : qbuf;
  double(*zl)[kLeaf + 1] = zls[gi];
  double* d = ds[gi];
  double* e = es[gi];
  double* cs = css[gi];
  int* rank = ranks[gi];
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
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
      if (++iter > iter_cap) {
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
        const double ri = rcp_nr(r);
        sn = f * ri;
        c = g * ri;
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
  double *D, *z, *dS, *zS, *rc, *rs, *delta, *zeta, *z2, *tau, *zhat, *inv, *vals;
  int *perm, *defl, *nd, *rp, *ri, *org, *pos;
};

// Merges above kDcLdsMaxM: the arrays the O(k^2) loops read (delta, z2, tau,
// zhat, vals, org) in LDS, the others in the device scratch.
constexpr int kDcHotBytes = 5 * sizeof(double) + sizeof(int);  // per eigenvalue
__device__ PrepLds carve_split(void* lds, double* glob, int m) {
  PrepLds L;
  double* hp = reinterpret_cast<double*>(lds);
  L.delta = hp; hp += m;
  L.z2 = hp; hp += m;
  L.tau = hp; hp += m;
  L.zhat = hp; hp += m;
  L.vals = hp; hp += m;
  L.org = reinterpret_cast<int*>(hp);
  double* dp = glob;
  L.D = dp; dp += m;
  L.z = dp; dp += m;
  L.dS = dp; dp += m;
  L.zS = dp; dp += m;
  L.rc = dp; dp += m;
  L.rs = dp; dp += m;
  L.zeta = dp; dp += m;
  L.inv = dp; dp += m;
  int* ip = reinterpret_cast<int*>(dp);
  L.perm = ip; ip += m;
  L.defl = ip; ip += m;
  L.nd = ip; ip += m;
  L.rp = ip; ip += m;
  L.ri = ip; ip += m;
  L.pos = ip; ip += m;
  return L;
}

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
  L.z2 = dp; dp += m;
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
// increasing delta, evaluated by the G lanes g = 0..G-1 of a wave that share j
// (G a power of two up to 8, the group aligned to G): lane g sums the terms
// i = g, g+G, ...  The partial sums are combined pairwise, exchanging equal
// values at every step, which leaves the same bits in every lane of the
// group, so the group takes the same branches and returns the same root.  Returns the origin pole index and the offset tau
// from it.
__device__ void secular_root(const double* __restrict__ delta, const double* __restrict__ z2,
                             int k, double rho, int j, int G, int g, int& org, double& tau_out) {
  // sum over the group by DPP: quad_perm 1032 (pairs), quad_perm 2301
  // (quads), row_half_mirror (eights; after the quad steps it exchanges equal
  // quad sums); the lanes of a group are active together
  auto gsum = [G](double x) {
    if (G >= 2) x += dpp_f64<0xB1>(x);
    if (G >= 4) x += dpp_f64<0x4E>(x);
    if (G >= 8) x += dpp_f64<0x141>(x);
    return x;
  };
  double a, b;
  int o;
  if (j < k - 1) {
    const double gap = delta[j + 1] - delta[j];
    double w = 0.0;
    for (int i = g; i < k; i += G) w += z2[i] / ((delta[i] - delta[j]) - 0.5 * gap);
    w = 1.0 / rho + gsum(w);
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
    for (int i = g; i < k; i += G) zz += z2[i];
    zz = gsum(zz);
    o = j;
    a = 0.0;
    b = rho * zz * (1.0 + 8.0 * DBL_EPSILON);
  }
  const double dlo = delta[o];
  const int jl = j;  // left pole of the interval is delta[j], right delta[j+1]
  double x = 0.5 * (a + b);
  for (int it = 0; it < 100; ++it) {
    double w = 0.0, err = 0.0, psi1 = 0.0, phi1 = 0.0;
    // terms up to the left pole feed psi', the rest phi'; 1/Di within about an
    // ulp (enough for the iteration's tolerance tests), t / Di = t * ri
    int i = g;
    for (; i <= jl && i < k; i += G) {
      const double Di = (delta[i] - dlo) - x;
      const double ri = rcp_nr(Di);
      const double t = z2[i] * ri;
      w += t;
      err += fabs(t);
      psi1 += t * ri;
    }
    for (; i < k; i += G) {
      const double Di = (delta[i] - dlo) - x;
      const double ri = rcp_nr(Di);
      const double t = z2[i] * ri;
      w += t;
      err += fabs(t);
      phi1 += t * ri;
    }
    w = 1.0 / rho + gsum(w);
    err = 1.0 / rho + gsum(err);
    psi1 = gsum(psi1);
    phi1 = gsum(phi1);
    const double Dl = (delta[jl] - dlo) - x;
    const double Dr = jl + 1 < k ? (delta[jl + 1] - dlo) - x : 0.0;
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

// Stream compaction in index order over the workgroup: out[base + r] = i for
// every i < m with flag(i), r being the number of flagged j < i (wave ballots,
// then the wave totals in LDS).  Returns the count in every thread; ends with
// a barrier.
template <int NT, class F>
__device__ int compact(int m, F flag, int* out, int base, int* wtot) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int total = 0;
  for (int i0 = 0; i0 < m; i0 += NT) {
    const int i = i0 + (int)threadIdx.x;
    const bool f = i < m && flag(i);
    const unsigned long long bal = __ballot(f);
    if (lane == 0) wtot[w] = __popcll(bal);
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int ww = 0; ww < NT / 64; ++ww) {
      off += ww < w ? wtot[ww] : 0;
      tot += wtot[ww];
    }
    if (f) out[base + total + off + __popcll(bal & ((1ull << lane) - 1))] = i;
    __syncthreads();
    total += tot;
  }
  return total;
}

// GL: for merges above kDcLdsMaxM eigenvalues, the work arrays of the O(m)
// steps live in the device scratch gscr (kDcGlobalStride doubles per
// eigenvalue and workgroup) and only those the O(k^2) loops read in LDS.
template <int NT, bool GL>
__global__ __launch_bounds__(NT) void k_dc_prep(
    const int32_t* __restrict__ merges, const int32_t* __restrict__ sub_orb_ptr,
    const int64_t* __restrict__ off2, const double* __restrict__ E, double* __restrict__ zbuf,
    double* __restrict__ lam, int32_t* __restrict__ md_k, int32_t* __restrict__ md_cols,
    int32_t* __restrict__ md_org, int32_t* __restrict__ md_pos, int32_t* __restrict__ md_dsrc,
    int32_t* __restrict__ md_dpos, double* __restrict__ md_delta, double* __restrict__ md_tau,
    double* __restrict__ md_zhat, double* __restrict__ md_inv, double* __restrict__ gscr) {
  extern __shared__ double smem[];
  __shared__ double red[NT / 64];
  __shared__ int sh_k, sh_nrot, sh_rot;
  __shared__ int wtot[NT / 64];
  const int mid = blockIdx.x;
  const int s = merges[4 * mid], lo = merges[4 * mid + 1];
  const int m1 = merges[4 * mid + 2], m2 = merges[4 * mid + 3];
  const int m = m1 + m2;
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  double* Z = zbuf + off2[s];
  PrepLds L = GL ? carve_split(smem, gscr + (size_t)blockIdx.x * kMaxN * kDcGlobalStride, m)
                 : carve(smem, m);
  const int tid = threadIdx.x;

  const double beta = E[b + lo + m1 - 1];
  const double rho = fabs(beta);
  const double sg = beta >= 0.0 ? 1.0 : -1.0;

  for (int i = tid; i < m; i += NT) {
    L.D[i] = lam[b + lo + i];
    L.z[i] = i < m1 ? Z[(lo + m1 - 1) + (size_t)n * (lo + i)] : sg * Z[(lo + m1) + (size_t)n * (lo + i)];
  }
  // the off-diagonal child blocks hold stale data from earlier levels
  for (int idx = tid; idx < m1 * m2; idx += NT) {
    const int r = idx % m1, c = idx / m1;
    Z[(lo + r) + (size_t)n * (lo + m1 + c)] = 0.0;
  }
  for (int idx = tid; idx < m1 * m2; idx += NT) {
    const int r = idx % m2, c = idx / m2;
    Z[(lo + m1 + r) + (size_t)n * (lo + c)] = 0.0;
  }
  __syncthreads();
  double part = 0.0;
  for (int i = tid; i < m; i += NT) part += L.z[i] * L.z[i];
  const double zz = block_sum<NT>(part, red);
  const double zn = sqrt(zz);
  const double rho2 = rho * zz;
  // stable merge of the two ascending lists (first list wins ties)
  for (int i = tid; i < m; i += NT) {
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
  for (int r = tid; r < m; r += NT) {
    L.dS[r] = L.D[L.perm[r]];
    L.zS[r] = zn > 0.0 ? L.z[L.perm[r]] / zn : 0.0;
    mx = fmax(mx, fabs(L.dS[r]));
  }
  const double dmax = block_max<NT>(mx, red);
  const double tol = 8.0 * DBL_EPSILON * fmax(dmax, rho2);

  // deflation.  An entry with a negligible z deflates on its own; a kept entry
  // whose pole is close to that of the previous kept entry deflates by a
  // Givens rotation.  The kept entries are compacted in order first (the
  // scan's result when no rotation happens) and every consecutive pair is
  // tested with the scan's own arithmetic (the result kept per pair in pos);
  // only if some pair needs a rotation does thread 0 run the scan, over the
  // kept entries: a pair whose left entry no rotation has changed holds the
  // values the parallel test saw, so it takes that result, and only the pair
  // after a rotation is tested again.
  for (int i = tid; i < m; i += NT) L.defl[i] = rho2 * fabs(L.zS[i]) <= tol ? 1 : 0;
  if (tid == 0) sh_rot = 0;
  __syncthreads();
  const int kept = compact<NT>(m, [&](int i) { return L.defl[i] == 0; }, L.nd, 0, wtot);
  for (int q = 1 + tid; q < kept; q += NT) {
    const int p = L.nd[q - 1], i = L.nd[q];
    const double t = hypot(L.zS[p], L.zS[i]);
    const double c = L.zS[i] / t;
    const double sn = -L.zS[p] / t;
    const bool rot = fabs((L.dS[i] - L.dS[p]) * c * sn) <= tol;
    L.pos[q] = rot ? 1 : 0;
    if (rot) sh_rot = 1;
  }
  __syncthreads();
  const bool any_rot = sh_rot != 0;
  if (!any_rot && tid == 0) {
    sh_k = kept;
    sh_nrot = 0;
  }
  if (any_rot && tid == 0) {
    // nd is rewritten in place: entry q is read before any write reaches it
    int p = kept > 0 ? L.nd[0] : -1, k = 0, nrot = 0;
    bool pmod = false;  // p changed by the previous rotation
    for (int q = 1; q < kept; ++q) {
      const int i = L.nd[q];
      bool rot = false;
      double t = 0.0, c = 0.0, sn = 0.0;
      if (pmod || L.pos[q]) {
        t = hypot(L.zS[p], L.zS[i]);
        c = L.zS[i] / t;
        sn = -L.zS[p] / t;
        rot = fabs((L.dS[i] - L.dS[p]) * c * sn) <= tol;
      }
      if (rot) {
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
      pmod = rot;
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
  for (int r = tid; r < m; r += NT) {
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
  for (int j = tid; j < k; j += NT) {
    L.delta[j] = L.dS[L.nd[j]];
    const double zj = L.zS[L.nd[j]];
    L.zeta[j] = zj;
    L.z2[j] = zj * zj;
  }
  __syncthreads();
  // secular roots and the recomputed z, G lanes per root: G doubles (up to
  // 8) while G k fits the workgroup, so the roots take one or two rounds
  int G = 1;
  while (G < 8 && G * k <= NT) G *= 2;
  const int g = tid & (G - 1);
  {
    for (int j = tid / G; j < k; j += NT / G) {
      int o;
      double t;
      secular_root(L.delta, L.z2, k, rho2, j, G, g, o, t);
      if (g == 0) {
        L.org[j] = o;
        L.tau[j] = t;
      }
    }
  }
  __syncthreads();
  // recomputed z: zh_i^2 = (lambda_i - d_i)/rho * prod_{j != i} (d_i - lambda_j)/(d_i - d_j)
  // (numerators and denominators gathered in groups of four, one division per
  // group: every factor lies between about 1e-18 and 10, so a group cannot
  // leave the double range).  Lane g of root i's group takes j = g, g+G, ...;
  // the partial products are combined by DPP (quad_perm 1032, 2301,
  // row_half_mirror), as the secular sums are.
  for (int i = tid / G; i < k; i += NT / G) {
    const double di = L.delta[i];
    double prod = g == 0 ? -((di - L.delta[L.org[i]]) - L.tau[i]) / rho2 : 1.0;
    double num = 1.0, den = 1.0;
    int cnt = 0;
    for (int j = g; j < k; j += G) {
      if (j == i) continue;
      num *= (di - L.delta[L.org[j]]) - L.tau[j];
      den *= di - L.delta[j];
      if (++cnt == 4) {
        prod *= num / den;
        num = den = 1.0;
        cnt = 0;
      }
    }
    prod *= num / den;
    if (G >= 2) prod *= dpp_f64<0xB1>(prod);
    if (G >= 4) prod *= dpp_f64<0x4E>(prod);
    if (G >= 8) prod *= dpp_f64<0x141>(prod);
    if (g == 0) L.zhat[i] = copysign(sqrt(fmax(prod, 0.0)), L.zeta[i]);
  }
  __syncthreads();
  // sum_i (zh_i / D_i)^2 with pairs over a common denominator:
  // (za^2 Db^2 + zb^2 Da^2) / (Da^2 Db^2); lane g of root j's group takes the
  // pairs starting at i = 2g, 2g + 2G, ... (and the odd last term if it falls
  // to it), the partial sums combined by DPP
  for (int j = tid / G; j < k; j += NT / G) {
    const double dO = L.delta[L.org[j]], tj = L.tau[j];
    double acc = 0.0;
    int i = 2 * g;
    for (; i + 1 < k; i += 2 * G) {
      const double da = (L.delta[i] - dO) - tj, db = (L.delta[i + 1] - dO) - tj;
      const double za = L.zhat[i], zb = L.zhat[i + 1];
      const double da2 = da * da, db2 = db * db;
      acc += (za * za * db2 + zb * zb * da2) * rcp_nr(da2 * db2);
    }
    if (i == k - 1) {
      const double u = L.zhat[i] / ((L.delta[i] - dO) - tj);
      acc += u * u;
    }
    if (G >= 2) acc += dpp_f64<0xB1>(acc);
    if (G >= 4) acc += dpp_f64<0x4E>(acc);
    if (G >= 8) acc += dpp_f64<0x141>(acc);
    if (g == 0) L.inv[j] = 1.0 / sqrt(acc);
  }
  // output order: roots first (items 0..k-1), then the deflated items in
  // index order (the tail of nd lists their sorted indices)
  for (int j = tid; j < k; j += NT) L.vals[j] = L.delta[L.org[j]] + L.tau[j];
  compact<NT>(m, [&](int i) { return L.defl[i] != 0; }, L.nd, k, wtot);
  for (int q = k + tid; q < m; q += NT) L.vals[q] = L.dS[L.nd[q]];
  __syncthreads();
  // ranks of the output values, Gm lanes per value (counts combined by DPP)
  {
    int Gm = 1;
    while (Gm < 8 && 2 * Gm * m <= NT) Gm *= 2;
    const int gm = tid & (Gm - 1);
    for (int it = tid / Gm; it < m; it += NT / Gm) {
      const double x = L.vals[it];
      int rk = 0;
      for (int j = gm; j < m; j += Gm) rk += (L.vals[j] < x) || (L.vals[j] == x && j < it);
      if (Gm >= 2) rk += __builtin_amdgcn_update_dpp(0, rk, 0xB1, 0xF, 0xF, false);
      if (Gm >= 4) rk += __builtin_amdgcn_update_dpp(0, rk, 0x4E, 0xF, 0xF, false);
      if (Gm >= 8) rk += __builtin_amdgcn_update_dpp(0, rk, 0x141, 0xF, 0xF, false);
      if (gm == 0) L.pos[it] = rk;
    }
  }
  __syncthreads();
  const int base = b + lo;
  for (int it = tid; it < m; it += NT) lam[base + L.pos[it]] = L.vals[it];
  for (int j = tid; j < k; j += NT) {
    md_cols[base + j] = L.perm[L.nd[j]];
    md_org[base + j] = L.org[j];
    md_pos[base + j] = L.pos[j];
    md_delta[base + j] = L.delta[j];
    md_tau[base + j] = L.tau[j];
    md_zhat[base + j] = L.zhat[j];
    md_inv[base + j] = L.inv[j];
  }
  for (int q = tid; q < m - k; q += NT) {
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
  constexpr int kKg = 32;  // K chunk of the product
  __shared__ double As[kKg][kTile + 1];
  __shared__ double Bs[kKg][kTile + 1];
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
  // On the four-block 4x4x4 MFMA as the transposed product D = U^T Z^T: wave w
  // owns D rows (columns of W) 16w .. 16w+15 as four blocks of 4, and all 64 D
  // columns (rows of W) as four strips of 16; lane l holds W row
  // r0 + 16 s + l%16, W column c0 + 16 w + 4 b + l/16 in acc[b][s].
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lq = lane & 3, lr = lane >> 4, l15 = lane & 15;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  // the next chunk's gathered Z values and the roots' zhat, delta are loaded
  // (clamped, branch-free) while the current chunk's MFMAs run; U is formed
  // when they are written to LDS
  constexpr int kPf = kKg * kTile / kThreads;
  double pz[kPf], pzh[kPf], pdl[kPf];
  auto fetch = [&](int i0) {
#pragma unroll
    for (int u = 0; u < kPf; ++u) {
      const int idx = threadIdx.x + u * kThreads;
      const int i = min(i0 + idx / kTile, k - 1), r = min(r0 + idx % kTile, m - 1);
      pz[u] = Z[(lo + r) + (size_t)n * (lo + md_cols[base + i])];
      pzh[u] = md_zhat[base + i];
      pdl[u] = md_delta[base + i];
    }
  };
  if (c0 < k) {
    fetch(0);
    for (int i0 = 0; i0 < k; i0 += kKg) {
      __syncthreads();
#pragma unroll
      for (int u = 0; u < kPf; ++u) {
        const int idx = threadIdx.x + u * kThreads;
        const int rr = idx % kTile, ii = idx / kTile;
        const bool iok = i0 + ii < k;
        As[ii][rr] = (iok && r0 + rr < m) ? pz[u] : 0.0;
        Bs[ii][rr] = (iok && c0 + rr < k) ? pzh[u] * cinv[rr] * rcp_nr((pdl[u] - cdo[rr]) - ctau[rr]) : 0.0;
      }
      __syncthreads();
      if (i0 + kKg < k) fetch(i0 + kKg);
#pragma unroll
      for (int ks = 0; ks < kKg / 4; ++ks) {
        const int kk = 4 * ks + lr;
        double a[4], bv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] = Bs[kk][16 * w + 4 * q + lq];
#pragma unroll
        for (int q = 0; q < 4; ++q) bv[q] = As[kk][16 * q + l15];
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[p][q] = mfma4b(a[p], bv[q], acc[p][q]);
      }
    }
  }
  // destination columns (and sources of deflated ones) of this lane's four
  // columns, then every deflated value, all loaded from clamped (valid)
  // entries before the guarded stores
  int dst[4], src[4];
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int c = c0 + 16 * w + 4 * p + lr;
    const int ck = min(c, max(k - 1, 0));
    const int dq = max(min(c - k, m - k - 1), 0);
    const int pos = md_pos[base + ck], dpos = md_dpos[base + dq], dsrc = md_dsrc[base + dq];
    dst[p] = c < k ? pos : dpos;
    src[p] = min(max(dsrc, 0), m - 1);
  }
  double zc[4][4];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = min(r0 + 16 * q + l15, m - 1);
      zc[p][q] = Z[(lo + r) + (size_t)n * (lo + src[p])];
    }
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int c = c0 + 16 * w + 4 * p + lr;
    if (c >= m) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = r0 + 16 * q + l15;
      if (r < m) W[(lo + r) + (size_t)n * (lo + dst[p])] = c < k ? acc[p][q] : zc[p][q];
    }
  }
}

// T factors of the compact-WY blocks: H_kb ... H_{kb+nb-1} = I - V T V^T with
// T upper triangular (T_ii = tau_i, T[0:i, i] = -tau_i T[0:i, 0:i] V^T v_i).
// One workgroup per (subgraph, block); T stored as kNb x kNb row-major.
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// One workgroup per (subgraph, block): the Gram matrix G = V^T V on FP64 MFMA
// (the four waves take interleaved 4-row chunks; V^T as the A operand and V as
// the B operand are the same lane values), then the triangular recurrence.
__global__ __launch_bounds__(kThreads) void k_bt_tfactors(
    const double* __restrict__ abuf, const double* __restrict__ TAU, const int64_t* __restrict__ off2,
    const int32_t* __restrict__ sub_orb_ptr, const int32_t* __restrict__ toff,
    const int32_t* __restrict__ subs, double* __restrict__ tfac) {
  __shared__ double Gp[4][kNb][kNb + 1];
  __shared__ double T[kNb][kNb + 1];
  const int s = subs[blockIdx.x];
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  const int kbi = blockIdx.y;
  const int kb = kbi * kNb;
  if (kb >= n - 2) return;
  const int nb = min(kNb, n - 2 - kb);
  const double* A = abuf + off2[s];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  // Gram matrix V^T V: four row groups per step, their reflector entries
  // loaded from clamped (valid) addresses together and masked at use
  v4d G = {0.0, 0.0, 0.0, 0.0};
  const int qc = kb + min(li, nb - 1);
  const int top = kb + li + 1;
  for (int row0 = kb + 1 + 4 * w; row0 < n; row0 += 64) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = A[min(row0 + 16 * u + lk, n - 1) + (size_t)n * qc];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = row0 + 16 * u + lk;
      const double a = (li < nb && r < n && r >= top) ? (r == top ? 1.0 : v[u]) : 0.0;
      G = mfma16(a, a, G);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) Gp[w][4 * r + lk][li] = G[r];
  __syncthreads();
  if (tid < kNb * kNb) {
    const int p = tid / kNb, q = tid % kNb;
    Gp[0][p][q] = Gp[0][p][q] + Gp[1][p][q] + Gp[2][p][q] + Gp[3][p][q];
  }
  __syncthreads();
  // T column by column: T[rr][i] = -tau_i sum_{rr <= qq < i} T[rr][qq] G[qq][i],
  // T[i][i] = tau_i.  Lane rr of the first wave keeps row rr of T in
  // registers, so the 16 steps need no barrier.
  if (tid < kNb) {
    const int rr = tid;
    double trow[kNb];
#pragma unroll
    for (int i = 0; i < kNb; ++i) trow[i] = 0.0;
#pragma unroll
    for (int i = 0; i < kNb; ++i) {
      if (i < nb) {
        const double ti = TAU[b + kb + i];
        double acc = 0.0;
#pragma unroll
        for (int qq = 0; qq < i; ++qq) acc += (qq >= rr ? trow[qq] : 0.0) * Gp[0][qq][i];
        trow[i] = rr < i ? -ti * acc : (rr == i ? ti : 0.0);
      }
    }
#pragma unroll
    for (int i = 0; i < kNb; ++i) T[rr][i] = trow[i];
  }
  __syncthreads();
  if (tid < kNb * kNb)
    tfac[(size_t)(toff[s] + kbi) * kNb * kNb + tid] = T[tid / kNb][tid % kNb];
}

// ----------------------------------------- back-transformation on FP64 MFMA
// v_mfma_f64_16x16x4f64 on gfx950: lane l supplies A(l%16, l/16) and
// B(l/16, l%16); D(i, j) is returned in lane j + 16*(i%4), register i/4.  A
// 16x16 tile held in that D layout is, register by register, the B operand of
// four consecutive K steps (register r: rows 4r..4r+3).

// Q = H_0 ... H_{n-3} Z for a panel of 16 eigenvector columns, one compact-WY
// block of 16 reflectors at a time from the last: Z <- Z - V (T (V^T Z)).  The
// panel lives in registers as 16x16 tiles (wave w holds row blocks w, w+4,
// ...; at most MRB each), the reflector block is staged in LDS, and both
// products run on MFMA: W = V^T Z (partial per wave, summed in LDS), W2 = T W,
// Z -= V W2.  Also forms the core weights of the panel's columns.
template <int MRB>
__global__ __launch_bounds__(kThreads, MRB <= 4 ? 4 : MRB <= 6 ? 3 : MRB <= 10 ? 2 : 1) void k_bt_mfma(
    const double* __restrict__ abuf, const double* __restrict__ tfac,
    const int32_t* __restrict__ toff, double* __restrict__ zbuf, const int64_t* __restrict__ off2,
    const int32_t* __restrict__ sub_orb_ptr, const int32_t* __restrict__ n_core,
    const int32_t* __restrict__ list, double* __restrict__ wts, int count, int npanel) {
  extern __shared__ double vb[];  // [16 * nrb][kLdv]: reflector block, row-major
  __shared__ double Wp[4][16][17];
  __shared__ double Ts[16][17];
  __shared__ double csum[4][16];
  // workgroup id -> (subgraph, column panel): workgroup w runs on XCD w mod 8,
  // and the npanel panels of a subgraph take consecutive slots of one XCD, so
  // they stage the same reflector blocks through one L2
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int si = 8 * (slot / npanel) + xcd;
  if (si >= count) return;
  const int s = list[si];
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  const int c0 = (slot % npanel) * 16;
  if (c0 >= n) return;
  const int nrb = (n + 15) / 16;
  const double* A = abuf + off2[s];
  double* Z = zbuf + off2[s];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int col = c0 + li;
  v4d zt[MRB];
#pragma unroll
  for (int i = 0; i < MRB; ++i) {
    const int rb = w + 4 * i;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * rb + 4 * r + lk;
      zt[i][r] = (rb < nrb && row < n && col < n) ? Z[row + (size_t)n * col] : 0.0;
    }
  }
  const int nref = n - 2;
  for (int kbi = (nref - 1) / kNb; nref > 0 && kbi >= 0; --kbi) {
    const int kb = kbi * kNb;
    const int nb = min(kNb, nref - kb);
    const int rb0 = (kb + 1) / 16;  // first row block with a nonzero reflector row
    const int r0 = 16 * rb0;
    const int nrows = 16 * nrb - r0;
    __syncthreads();
    // stage the block: thread (q, rl) takes reflector q, rows r0 + rl + 16 i;
    // eight loads from clamped (valid) addresses are issued before their
    // stores, so they are in flight together
    {
      const int q = tid >> 4, rl = tid & 15;  // kThreads = 16 x 16
      const int colq = kb + min(q, nb - 1);
      const int top = kb + q + 1;
      const int nr16 = nrows / 16;
      for (int i0 = 0; i0 < nr16; i0 += 8) {
        double vv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int r = r0 + rl + 16 * min(i0 + u, nr16 - 1);
          vv[u] = A[min(r, n - 1) + (size_t)n * colq];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int r = r0 + rl + 16 * (i0 + u);
          if (i0 + u < nr16) {
            const double v = (q < nb && r < n && r >= top) ? ((r == top) ? 1.0 : vv[u]) : 0.0;
            vb[r * kLdv + q] = v;
          }
        }
      }
    }
    if (tid < kNb * kNb) Ts[tid / kNb][tid % kNb] = tfac[(size_t)(toff[s] + kbi) * kNb * kNb + tid];
    __syncthreads();
    // W = V^T Z over this wave's row blocks
    v4d W = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < MRB; ++i) {
      const int rb = w + 4 * i;
      if (rb < rb0 || rb >= nrb) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double a = vb[(16 * rb + 4 * r + lk) * kLdv + li];
        W = mfma16(a, zt[i][r], W);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) Wp[w][4 * r + lk][li] = W[r];
    __syncthreads();
    // W2 = T W (every wave, for its own use as the B operand below)
    v4d W2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      const int q = 4 * kc + lk;
      const double bw = Wp[0][q][li] + Wp[1][q][li] + Wp[2][q][li] + Wp[3][q][li];
      W2 = mfma16(Ts[li][q], bw, W2);
    }
    // Z -= V W2
#pragma unroll
    for (int i = 0; i < MRB; ++i) {
      const int rb = w + 4 * i;
      if (rb < rb0 || rb >= nrb) continue;
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) {
        const double a = vb[(16 * rb + li) * kLdv + 4 * kc + lk];
        zt[i] = mfma16(a, -W2[kc], zt[i]);
      }
    }
  }
  // write back and core weights of the panel's columns
  const int c = n_core[s];
  double cw = 0.0;
#pragma unroll
  for (int i = 0; i < MRB; ++i) {
    const int rb = w + 4 * i;
    if (rb >= nrb) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * rb + 4 * r + lk;
      if (row < n && col < n) {
        Z[row + (size_t)n * col] = zt[i][r];
        if (row < c) cw += zt[i][r] * zt[i][r];
      }
    }
  }
  cw += __shfl_xor(cw, 16, 64);
  cw += __shfl_xor(cw, 32, 64);
  if (lk == 0) csum[w][li] = cw;
  __syncthreads();
  if (tid < 16 && c0 + tid < n) wts[b + c0 + tid] = csum[0][tid] + csum[1][tid] + csum[2][tid] + csum[3][tid];
}

// The back-transformation of subgraphs above kTdMaxN orbitals (up to kMaxN):
// the products of k_bt_mfma on a 16-column panel held in registers by eight
// waves (wave w holds row blocks w, w + 8, ...), with the reflector block staged
// in LDS kBigHalf rows at a time: the first half, then the second for W =
// V^T Z; the update Z -= V W2 on the second half (still staged), then on the
// first, staged again.
constexpr int kBigThreads = 512;
constexpr int kBigHalf = 1024;
constexpr int kBigMRB = kMaxN / (16 * (kBigThreads / 64));  // row blocks per wave
static_assert(kBigMRB % 2 == 0 && 16 * (kBigThreads / 64) * (kBigMRB / 2) == kBigHalf,
              "half of each wave's row blocks per staged half");

__global__ __launch_bounds__(kBigThreads, 1) void k_bt_mfma_big(
    const double* __restrict__ abuf, const double* __restrict__ tfac,
    const int32_t* __restrict__ toff, double* __restrict__ zbuf, const int64_t* __restrict__ off2,
    const int32_t* __restrict__ sub_orb_ptr, const int32_t* __restrict__ n_core,
    const int32_t* __restrict__ list, double* __restrict__ wts, int count, int npanel) {
  extern __shared__ double vb[];  // [kBigHalf][kLdv]: half of the reflector block
  constexpr int NW = kBigThreads / 64;
  constexpr int HB = kBigMRB / 2;  // a wave's row blocks in one half
  __shared__ double Wp[NW][16][17];
  __shared__ double Ts[16][17];
  __shared__ double csum[NW][16];
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int si = 8 * (slot / npanel) + xcd;
  if (si >= count) return;
  const int s = list[si];
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  const int c0 = (slot % npanel) * 16;
  if (c0 >= n) return;
  const int nrb = (n + 15) / 16;
  const double* A = abuf + off2[s];
  double* Z = zbuf + off2[s];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int col = c0 + li;
  v4d zt[kBigMRB];
#pragma unroll
  for (int i = 0; i < kBigMRB; ++i) {
    const int rb = w + NW * i;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * rb + 4 * r + lk;
      zt[i][r] = (rb < nrb && row < n && col < n) ? Z[row + (size_t)n * col] : 0.0;
    }
  }
  const int nref = n - 2;
  for (int kbi = (nref - 1) / kNb; nref > 0 && kbi >= 0; --kbi) {
    const int kb = kbi * kNb;
    const int nb = min(kNb, nref - kb);
    const int rb0 = (kb + 1) / 16;  // first row block with a nonzero reflector row
    // rows [max(16 rb0, h kBigHalf), min(16 nrb, (h+1) kBigHalf)) of the block
    // into vb (row - h kBigHalf); thread (q, rl) takes reflector q, rows rl +
    // 32 i, eight loads in flight before their stores
    auto stage = [&](int h) {
      const int lo = max(16 * rb0, h * kBigHalf), hi = min(16 * nrb, (h + 1) * kBigHalf);
      const int q = tid >> 5, rl = tid & 31;
      const int colq = kb + min(q, nb - 1);
      const int top = kb + q + 1;
      for (int i0 = lo; i0 < hi; i0 += 8 * 32) {
        double vv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) vv[u] = A[min(i0 + rl + 32 * u, n - 1) + (size_t)n * colq];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int r = i0 + rl + 32 * u;
          if (r < hi) {
            const double v = (q < nb && r < n && r >= top) ? ((r == top) ? 1.0 : vv[u]) : 0.0;
            vb[(r - h * kBigHalf) * kLdv + q] = v;
          }
        }
      }
    };
    __syncthreads();
    stage(0);
    if (tid < kNb * kNb) Ts[tid / kNb][tid % kNb] = tfac[(size_t)(toff[s] + kbi) * kNb * kNb + tid];
    __syncthreads();
    // W = V^T Z over this wave's row blocks, first half then second
    v4d W = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < HB; ++i) {
      const int rb = w + NW * i;
      if (rb < rb0 || rb >= nrb) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) W = mfma16(vb[(16 * rb + 4 * r + lk) * kLdv + li], zt[i][r], W);
    }
    __syncthreads();
    stage(1);
    __syncthreads();
#pragma unroll
    for (int i = HB; i < kBigMRB; ++i) {
      const int rb = w + NW * i;
      if (rb < rb0 || rb >= nrb) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        W = mfma16(vb[(16 * rb - kBigHalf + 4 * r + lk) * kLdv + li], zt[i][r], W);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) Wp[w][4 * r + lk][li] = W[r];
    __syncthreads();
    // W2 = T W, the wave partials added in order
    v4d W2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      const int q = 4 * kc + lk;
      double bw = 0.0;
#pragma unroll
      for (int ww = 0; ww < NW; ++ww) bw += Wp[ww][q][li];
      W2 = mfma16(Ts[li][q], bw, W2);
    }
    // Z -= V W2: the second half (staged), then the first
#pragma unroll
    for (int i = HB; i < kBigMRB; ++i) {
      const int rb = w + NW * i;
      if (rb < rb0 || rb >= nrb) continue;
#pragma unroll
      for (int kc = 0; kc < 4; ++kc)
        zt[i] = mfma16(vb[(16 * rb - kBigHalf + li) * kLdv + 4 * kc + lk], -W2[kc], zt[i]);
    }
    __syncthreads();
    stage(0);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < HB; ++i) {
      const int rb = w + NW * i;
      if (rb < rb0 || rb >= nrb) continue;
#pragma unroll
      for (int kc = 0; kc < 4; ++kc)
        zt[i] = mfma16(vb[(16 * rb + li) * kLdv + 4 * kc + lk], -W2[kc], zt[i]);
    }
  }
  // write back and core weights of the panel's columns
  const int c = n_core[s];
  double cw = 0.0;
#pragma unroll
  for (int i = 0; i < kBigMRB; ++i) {
    const int rb = w + NW * i;
    if (rb >= nrb) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * rb + 4 * r + lk;
      if (row < n && col < n) {
        Z[row + (size_t)n * col] = zt[i][r];
        if (row < c) cw += zt[i][r] * zt[i][r];
      }
    }
  }
  cw += __shfl_xor(cw, 16, 64);
  cw += __shfl_xor(cw, 32, 64);
  if (lk == 0) csum[w][li] = cw;
  __syncthreads();
  if (tid < 16 && c0 + tid < n) {
    double t = 0.0;
#pragma unroll
    for (int ww = 0; ww < NW; ++ww) t += csum[ww][tid];
    wts[b + c0 + tid] = t;
  }
}

}  // namespace

size_t dc_prep_lds(int m) { return (size_t)m * (13 * sizeof(double) + 7 * sizeof(int)); }

void dc_set_attributes() {
  (void)hipFuncSetAttribute((const void*)k_dc_prep<kThreads, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)dc_prep_lds(kDcLdsMaxM));
  (void)hipFuncSetAttribute((const void*)k_dc_prep<512, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)dc_prep_lds(kDcLdsMaxM));
  (void)hipFuncSetAttribute((const void*)k_dc_prep<1024, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)dc_prep_lds(kDcLdsMaxM));
  (void)hipFuncSetAttribute((const void*)k_dc_prep<1024, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kMaxN * kDcHotBytes));
  (void)hipFuncSetAttribute((const void*)k_bt_mfma<4>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(256 * kLdv * sizeof(double)));
  (void)hipFuncSetAttribute((const void*)k_bt_mfma<6>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(384 * kLdv * sizeof(double)));
  (void)hipFuncSetAttribute((const void*)k_bt_mfma<8>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(512 * kLdv * sizeof(double)));
  (void)hipFuncSetAttribute((const void*)k_bt_mfma<10>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(640 * kLdv * sizeof(double)));
  (void)hipFuncSetAttribute((const void*)k_bt_mfma<16>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(kTdMaxN * kLdv * sizeof(double)));
  (void)hipFuncSetAttribute((const void*)k_bt_mfma_big, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(kBigHalf * kLdv * sizeof(double)));
}

void launch_dc(gq_ctx* ctx, const gq_graph* g, gq_eigs* e, int cls, hipStream_t st) {
  const gq_graph_dev& dv = g->dev;
  // size class cls: subgraphs order[i0..i1) with their leaves, merges and
  // tiles; the vectors alternate between e->Q and the scratch e->Y by merge
  // depth (the top merges write Q); eigenvalues in e->eps
  const int i0 = cls == 0 ? 0 : g->n_big, i1 = cls == 0 ? g->n_big : g->n_sub;
  if (i1 <= i0) return;
  const int l0 = g->dc_leaf_off[cls], nleaf = g->dc_leaf_off[cls + 1] - l0;
  prof_begin_on(ctx, "k_dc_leaves", st);
  hipLaunchKernelGGL(k_dc_leaves, dim3((nleaf + 3) / 4), dim3(64), 0, st, dv.dc_leaves + 4 * l0,
                     nleaf, dv.sub_orb_ptr, dv.off2, e->dd, e->ee, e->Q, e->Y, e->eps, e->status,
                     ctx->leaf_iter_cap);
  prof_end(ctx);
  const auto& mo = g->dc_level_merge_off[cls];
  const auto& to = g->dc_level_tile_off[cls];
  const int nlev = (int)mo.size() - 1;
  for (int lv = 0; lv < nlev; ++lv) {
    const int depth = nlev - 1 - lv;  // levels run from the deepest merges up
    double* zin = depth % 2 == 1 ? e->Q : e->Y;
    double* zout = depth % 2 == 1 ? e->Y : e->Q;
    const int m0 = mo[lv], m1 = mo[lv + 1];
    const int t0 = to[lv], t1 = to[lv + 1];
    if (m1 == m0) continue;
    prof_begin_on(ctx, "k_dc_prep", st);
    // the level's leading merges above kDcLdsMaxM eigenvalues keep their work
    // arrays in device scratch (one slot per workgroup)
    const int nglob = g->dc_level_nglob[cls][lv];
    if (nglob > 0)
      hipLaunchKernelGGL((k_dc_prep<1024, true>), dim3(nglob), dim3(1024),
                         (size_t)kMaxN * kDcHotBytes, st,
                         dv.dc_merges + 4 * m0, dv.sub_orb_ptr, dv.off2, e->ee, zin, e->eps,
                         e->md_k + m0, e->md_cols, e->md_org, e->md_pos, e->md_dsrc, e->md_dpos,
                         e->md_delta, e->md_tau, e->md_zhat, e->md_inv, e->dcg);
    if (m1 - m0 > nglob) {
      // levels whose merges average over 256 run on 1024 threads, over 128 on
      // 512, the rest on 256, so that a merge's roots take one or two rounds
      const int maxm = g->dc_level_maxm_lds[cls][lv];
      const int64_t msum = g->dc_level_msum[cls][lv], nm = m1 - m0;
      const int ntl = msum > 256 * nm ? 1024 : msum > 128 * nm ? 512 : kThreads;
      auto prep = ntl == 1024 ? k_dc_prep<1024, false>
                  : ntl == 512 ? k_dc_prep<512, false> : k_dc_prep<kThreads, false>;
      const int ms = m0 + nglob;
      hipLaunchKernelGGL(prep, dim3(m1 - ms), dim3(ntl), dc_prep_lds(maxm), st,
                         dv.dc_merges + 4 * ms, dv.sub_orb_ptr, dv.off2, e->ee, zin, e->eps,
                         e->md_k + ms, e->md_cols, e->md_org, e->md_pos, e->md_dsrc, e->md_dpos,
                         e->md_delta, e->md_tau, e->md_zhat, e->md_inv, nullptr);
    }
    prof_end(ctx);
    prof_begin_on(ctx, "k_dc_gemm", st);
    hipLaunchKernelGGL(k_dc_gemm, dim3(t1 - t0), dim3(kThreads), 0, st, dv.dc_tiles + 3 * t0,
                       dv.dc_merges + 4 * m0, dv.sub_orb_ptr, dv.off2, zin, zout, e->md_k + m0,
                       e->md_cols, e->md_org, e->md_pos, e->md_dsrc, e->md_dpos, e->md_delta,
                       e->md_tau, e->md_zhat, e->md_inv);
    prof_end(ctx);
  }
  const int maxn = g->sub_orb_ptr[g->order[i0] + 1] - g->sub_orb_ptr[g->order[i0]];
  prof_begin_on(ctx, "k_bt_tfactors", st);
  hipLaunchKernelGGL(k_bt_tfactors, dim3(i1 - i0, (maxn + kNb - 1) / kNb), dim3(kThreads), 0, st,
                     e->A, e->tau, dv.off2, dv.sub_orb_ptr, dv.bt_toff, dv.order + i0, e->tfac);
  prof_end(ctx);
  prof_begin_on(ctx, "k_backtransform", st);
  // subgraphs are ordered by decreasing size: classes n <= 256, <= 384, <= 512,
  // <= 640, <= 1024, <= kMaxN are contiguous ranges of that order, each
  // launched with its register panel (the smallest that holds its row blocks)
  static constexpr int kClassN[6] = {256, 384, 512, 640, kTdMaxN, kMaxN};
  static_assert(kTdMaxN == 1024, "the k_bt_mfma<16> class holds 1024 rows");
  int lo = i0;
  for (int c = 5; c >= 0; --c) {
    const int floor_n = c == 0 ? 0 : kClassN[c - 1];
    int hi = lo;
    while (hi < i1 && g->sub_orb_ptr[g->order[hi] + 1] - g->sub_orb_ptr[g->order[hi]] > floor_n) ++hi;
    if (hi > lo) {
      const int nmax = g->sub_orb_ptr[g->order[lo] + 1] - g->sub_orb_ptr[g->order[lo]];
      const int nrb = (nmax + 15) / 16;
      const int npanel = (nmax + 15) / 16, count = hi - lo;
      dim3 grid(8 * npanel * ((count + 7) / 8));
      if (c == 5) {
        hipLaunchKernelGGL(k_bt_mfma_big, grid, dim3(kBigThreads), kBigHalf * kLdv * sizeof(double),
                           st, e->A, e->tfac, dv.bt_toff, e->Q, dv.off2, dv.sub_orb_ptr,
                           dv.n_core, dv.order + lo, e->wts, count, npanel);
        lo = hi;
        continue;
      }
      const size_t lds = (size_t)16 * nrb * kLdv * sizeof(double);
      auto kern = c == 0 ? k_bt_mfma<4> : c == 1 ? k_bt_mfma<6> : c == 2 ? k_bt_mfma<8> : c == 3 ? k_bt_mfma<10> : k_bt_mfma<16>;
      hipLaunchKernelGGL(kern, grid, dim3(kThreads), lds, st, e->A, e->tfac, dv.bt_toff, e->Q,
                         dv.off2, dv.sub_orb_ptr, dv.n_core, dv.order + lo, e->wts, count, npanel);
    }
    lo = hi;
  }
  prof_end(ctx);
}

}  // namespace gq
