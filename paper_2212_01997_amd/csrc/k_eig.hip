// Principal submatrices and their FP64 eigendecomposition on gfx950.
//
// Fig. 1: each subgraph selects the principal submatrix h = H[orbs, orbs].
// Eq. (SmallKS): h = Q diag(eps) Q^T.  One 1024-thread workgroup per subgraph:
//   k_gather    CSR rows of H -> dense column-major h (binary search of each
//               column index in the subgraph's sorted orbital list, in LDS)
//   k_tridiag   blocked Householder reduction to tridiagonal form, reflectors
//               kept in the lower triangle (subgraphs below kMwgMinN
//               orbitals; larger ones take the multi-workgroup reduction
//               k_td_col / k_td_symv / k_td_update below)
//   then the tridiagonal eigenproblem by divide and conquer and the
//   back-transformation (k_dc.hip).
#include <algorithm>
#include <cfloat>
#include <utility>

#include "gq_internal.hpp"

namespace gq {

namespace {

// v_mfma_f64_16x16x4f64 on gfx950: lane l supplies A(l%16, l/16) and
// B(l/16, l%16); D(i, j) is returned in lane j + 16*(i%4), register i/4.
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kGaThreads = 1024;

__global__ __launch_bounds__(kGaThreads) void k_gather(
    const int32_t* __restrict__ h_rp, const int32_t* __restrict__ h_col,
    const double* __restrict__ h_val, double* __restrict__ abuf,
    const int64_t* __restrict__ off2, const int32_t* __restrict__ sub_orb_ptr,
    const int32_t* __restrict__ sub_orbs, const int32_t* __restrict__ sorted_orbs,
    const int32_t* __restrict__ sorted_local, const int32_t* __restrict__ order,
    int32_t* __restrict__ status) {
  extern __shared__ int32_t si[];
  const int s = order[blockIdx.x];
  if (status && threadIdx.x == 0) status[s] = 0;
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  int32_t* so = si;
  int32_t* sl = si + n;
  double* A = abuf + off2[s];
  for (int i = threadIdx.x; i < n; i += kGaThreads) {
    so[i] = sorted_orbs[b + i];
    sl[i] = sorted_local[b + i];
  }
  const size_t nn = (size_t)n * n;
  for (size_t i = threadIdx.x; i < nn; i += kGaThreads) A[i] = 0.0;
  __syncthreads();
  // T threads share a row (T = kGaThreads / next power of two >= n, at most 8)
  // and take its nonzeros p = start + h, start + h + T, ...  Four nonzeros at a
  // time: their column and value loads are issued together, then four
  // interleaved branch-free binary searches for the column in the sorted
  // orbital list (the trip count depends only on n).
  int np2 = 1;
  while (np2 < n) np2 <<= 1;
  const int T = min(8, max(1, kGaThreads / np2));
  const int h = threadIdx.x % T;
  for (int r = threadIdx.x / T; r < n; r += kGaThreads / T) {
    const int a = sub_orbs[b + r];
    const int p_end = h_rp[a + 1];
    for (int p0 = h_rp[a] + h; p0 < p_end; p0 += 4 * T) {
      int c[4], base[4];
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int pp = min(p0 + u * T, p_end - 1);
        c[u] = h_col[pp];
        v[u] = h_val[pp];
        base[u] = 0;
      }
      for (int len = n; len > 1;) {
        const int half = len >> 1;
#pragma unroll
        for (int u = 0; u < 4; ++u) base[u] = so[base[u] + half] < c[u] ? base[u] + half : base[u];
        len -= half;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int pos = base[u] + (so[base[u]] < c[u] ? 1 : 0);  // first index with so >= c
        if (p0 + u * T < p_end && pos < n && so[pos] == c[u]) A[r + (size_t)n * sl[pos]] = v[u];
      }
    }
  }
}

// Blocked Householder tridiagonalisation, one 1024-thread workgroup per
// subgraph.  Rows are owned by threads (H = 1024/next_pow2(n) threads share a
// row and split its columns).  A panel of kPanel reflectors is formed before
// the trailing matrix is touched: inside the panel the current column and the
// symmetric product use the stale trailing matrix plus the panel corrections
//   A_cur = A - sum_q (v_q w_q^T + w_q v_q^T);
// v_q is kept in A's column k0+q (v[0] = 1 stored at row k0+q+1); for the
// corrections the panel's v_q and w_q sit in LDS (subgraphs of up to
// kLdsPanelN orbitals) or are read back from A and a global scratch.  At the
// end of the panel the rank-2*kPanel update runs on FP64 MFMA.  d, e and tau
// go to D, E, TAU.
constexpr int kTdThreads = 1024;
constexpr int kPanel = 16;
constexpr int kUnroll = 8;

// x from the lane given by the DPP control kCtrl (quad_perm, row_mirror, ...),
// both 32-bit halves moved by VALU permutes rather than the LDS crossbar.
template <int kCtrl>
__device__ __forceinline__ double dpp_f64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, kCtrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), kCtrl, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the wave (all lanes active), the same in every lane: rows of 16
// lanes summed by DPP (quad_perm 1032, quad_perm 2301, row_half_mirror,
// row_mirror; after the quad steps a mirror is an exchange of equal sums),
// then the four row sums read out.
__device__ __forceinline__ double wave_total(double x) {
  x += dpp_f64<0xB1>(x);
  x += dpp_f64<0x4E>(x);
  x += dpp_f64<0x141>(x);
  x += dpp_f64<0x140>(x);
  const long long b = __double_as_longlong(x);
  double rs[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int lo = __builtin_amdgcn_readlane((int)b, 16 * i);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 16 * i);
    rs[i] = __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
  }
  return (rs[0] + rs[1]) + (rs[2] + rs[3]);
}

// Sum over the workgroup in a fixed order; every thread gets the total.  One
// barrier: each call site has a buffer of its own, and other barriers separate
// its uses, so no wave can overwrite red before every wave has read it.
__device__ double tsum(double x, double* red) {
  x = wave_total(x);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = x;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < kTdThreads / 64; ++i) t += red[i];
  return t;
}

// Row r of p = A22 v over columns > c, in chunks of kUnroll columns aligned
// to multiples of kUnroll (chunk g goes to the thread with h = g mod H).  v is
// 0 at columns <= c, so the chunk holding c+1 may start early, and 0 at the
// padding columns n .. n + kUnroll - 1, so the last, partial chunk is loaded
// like the others (columns clamped to n - 1) and all its loads are in flight
// together; the chunk's v values are one wave-uniform run of LDS, read two at
// a time.
// The thread with h = 0 also returns its row's entry in column c + 1 (first
// chunk), which the next column of the panel starts from.
// Rows from n0 on read their columns from n0 on (whole chunks: n0 is a
// multiple of 16) from the LDS corner cor (column-major, leading dimension
// ldc) instead of from A.
__device__ __forceinline__ double symv_row(const double* __restrict__ row,
                                           const double* __restrict__ vl, int n, int c, int h,
                                           int H, double& next_col, const double* cor_row,
                                           bool corner_row, int n0, int ldc) {
  double ac[kUnroll];
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) ac[u] = 0.0;
  const int g_end = (n + kUnroll - 1) / kUnroll;
  const int u1 = (c + 1) % kUnroll;
  bool first = true;
  for (int g = (c + 1) / kUnroll + h; g < g_end; g += H) {
    const int col = g * kUnroll;
    double x[kUnroll];
    if (corner_row && col >= n0) {
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) x[u] = cor_row[(size_t)ldc * (min(col + u, n - 1) - n0)];
    } else {
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) x[u] = row[(size_t)n * min(col + u, n - 1)];
    }
    if (first) {
#pragma unroll
      for (int u = 0; u < kUnroll; ++u)
        if (u == u1) next_col = x[u];
      first = false;
    }
    const double2* v2 = reinterpret_cast<const double2*>(vl + col);
#pragma unroll
    for (int u = 0; u < kUnroll / 2; ++u) {
      const double2 vv = v2[u];
      ac[2 * u] += x[2 * u] * vv.x;
      ac[2 * u + 1] += x[2 * u + 1] * vv.y;
    }
  }
#pragma unroll
  for (int u = 1; u < kUnroll; ++u) ac[0] += ac[u];
  return ac[0];
}

// Panel columns q < kPanel: V (v_q, rows > k0+q) and W (w_q).  Subgraphs of
// up to kLdsPanelN orbitals keep both in LDS (pan[q n + r], pan[(kPanel+q) n
// + r]); larger ones read V from A's columns and W from the global scratch.
constexpr int kLdsPanelN = 512;

// The trailing matrix's bottom-right corner, rows and columns n0 .. n - 1
// (n0 a multiple of 16, m = n - n0 as large as the LDS left after the panel
// allows; the whole matrix when it fits), lives in LDS (cor, column-major,
// leading dimension m) for the whole reduction: every column's symmetric
// product reads it there, the trailing updates write it there, and A's copy
// of it is not read again.  The reflectors are still stored in A for the
// back-transformation.
template <bool LP>
__device__ __forceinline__ void tridiag_body(double* __restrict__ A, double* __restrict__ Wg,
                                             double* __restrict__ pan, int n, int b,
                                             double* __restrict__ D, double* __restrict__ E,
                                             double* __restrict__ TAU, double* vl, double* part,
                                             double* red, double (*yp)[2 * kPanel + 1],
                                             double* yfin, double* rowc, double* alpha_sh,
                                             int lds_doubles) {
  const int tid = threadIdx.x;
  const int H = n <= 128 ? 8 : n <= 256 ? 4 : n <= 512 ? 2 : 1;
  const int P = kTdThreads / H;
  const int r = tid % P, h = tid / P;
  const bool own = (h == 0) && (r < n);
  const int lane = tid & 63, wv = tid >> 6;
  if (tid < kUnroll) vl[n + tid] = 0.0;  // padding of the last chunk (the first barrier orders it)
  double* cor = LP ? pan + 2 * kPanel * n : pan;
  // n0 a multiple of 16, so that no chunk of the symmetric product and no
  // 16x16 tile of a full panel's update straddles it; m^2 fits the LDS left
  const int m_fit = min((int)sqrt((double)max(lds_doubles - (LP ? 2 * kPanel * n : 0), 0)), n);
  const int n0 = min((n - m_fit + 15) & ~15, n);
  const int m = n - n0;
  for (int i = tid; i < m * m; i += kTdThreads)
    cor[i] = A[(n0 + i % m) + (size_t)n * (n0 + i / m)];
  __syncthreads();
  auto At = [&](int row, int col) -> double {
    return (row >= n0 && col >= n0) ? cor[(row - n0) + (size_t)m * (col - n0)]
                                    : A[row + (size_t)n * col];
  };

  for (int k0 = 0; k0 + 2 < n; k0 += kPanel) {
    const int nb = min(kPanel, n - 2 - k0);
    auto Vp = [&](int q, int row) -> double {
      if constexpr (LP) return pan[q * n + row];
      else return A[row + (size_t)n * (k0 + q)];
    };
    auto Wp = [&](int q, int row) -> double {
      if constexpr (LP) return pan[(kPanel + q) * n + row];
      else return Wg[q * n + row];
    };
    // A[r, c] of the panel's next column, taken from this column's symmetric
    // product (the row's first chunk holds column c + 1); the panel's first
    // column and a column after a skipped one load it
    double a_next = 0.0;
    bool have_next = false;
    for (int j = 0; j < nb; ++j) {
      const int c = k0 + j;
      if constexpr (!LP) {
        if (own && r == c) {
          for (int q = 0; q < j; ++q) {
            rowc[q] = Vp(q, r);
            rowc[kPanel + q] = Wp(q, r);
          }
        }
      }
      __syncthreads();
      double a = 0.0;
      if (own && r >= c) {
        a = have_next ? a_next : At(r, c);
#pragma unroll 4
        for (int q = 0; q < j; ++q) {
          const double vc = LP ? Vp(q, c) : rowc[q];
          const double wc = LP ? Wp(q, c) : rowc[kPanel + q];
          a -= Vp(q, r) * wc + Wp(q, r) * vc;
        }
        if (r == c) D[b + c] = a;
        if (r == c + 1) *alpha_sh = a;
      }
      const double sigma = tsum(own && r >= c + 2 ? a * a : 0.0, red);
      const double alpha = *alpha_sh;
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
        if constexpr (LP) pan[j * n + r] = v;
        if (r >= c + 1) A[r + (size_t)n * c] = v;
        if (r == c) {
          TAU[b + c] = tau;
          E[b + c] = beta;
        }
      }
      __syncthreads();
      have_next = false;
      if (tau == 0.0) {
        // H = I (column already reduced): it adds no correction to the panel
        if (own) {
          if constexpr (LP) pan[(kPanel + j) * n + r] = 0.0;
          else Wg[j * n + r] = 0.0;
        }
        if (own && r >= c + 1) A[r + (size_t)n * c] = 0.0;
        if constexpr (LP)
          if (own) pan[j * n + r] = 0.0;
        continue;
      }
      const double vr = r < n ? vl[r] : 0.0;
      // y1 = W^T v, y2 = V^T v over the panel so far (rows > c; V, W vanish
      // above): thread t sums panel column t mod 32 (W for q < kPanel, V
      // above) over rows c+1+seg, c+1+seg+32, ... of segment seg = t / 32
      {
        const int q = tid & 31, seg = tid >> 5;
        const int qp = q & (kPanel - 1);
        double t = 0.0;
        if (qp < j) {
          const bool isw = q < kPanel;
#pragma unroll 4
          for (int row = c + 1 + seg; row < n; row += kTdThreads / 32)
            t += (isw ? Wp(qp, row) : Vp(qp, row)) * vl[row];
        }
        yp[seg][q] = t;
      }
      // p = A22 v over the stale trailing matrix
      double acc = 0.0;
      if (r >= c + 1 && r < n)
        acc = symv_row(A + r, vl, n, c, h, H, a_next, cor + max(r - n0, 0), r >= n0, n0, m);
      have_next = true;
      part[tid] = acc;
      __syncthreads();
      if (tid < 2 * kPanel && (tid % kPanel) < j) {
        double t = 0.0;
        for (int sg = 0; sg < kTdThreads / 32; ++sg) t += yp[sg][tid];
        yfin[tid] = t;
      }
      __syncthreads();
      double p = 0.0;
      if (own && r >= c + 1) {
        for (int hh = 0; hh < H; ++hh) p += part[hh * P + r];
#pragma unroll 4
        for (int q = 0; q < j; ++q) p -= Vp(q, r) * yfin[q] + Wp(q, r) * yfin[kPanel + q];
        p *= tau;
      }
      const double K = 0.5 * tau * tsum(own && r >= c + 1 ? p * vr : 0.0, red + kTdThreads / 64);
      if (own) {
        const double w = r >= c + 1 ? p - K * vr : 0.0;
        if constexpr (LP) pan[(kPanel + j) * n + r] = w;
        else Wg[j * n + r] = w;
      }
    }
    __syncthreads();
    // trailing update A22 -= V W^T + W V^T of rows/cols >= k0 + nb on FP64
    // MFMA: 16x16 tiles dealt to the 16 waves, K = the panel's reflectors
    // (twice).  Tile element (row0 + j, col0 + i) sits in lane j + 16 (i%4),
    // register i/4, so every load and store of a register is a 128-byte run of
    // one column.
    {
      const int t0 = k0 + nb;
      const int nt = (n - t0 + 15) / 16;
      const int li = lane & 15, lk = lane >> 4;
      for (int tile = wv; tile < nt * nt; tile += kTdThreads / 64) {
        const int row0 = t0 + 16 * (tile / nt), col0 = t0 + 16 * (tile % nt);
        const int row = row0 + li;
        const bool rok = row < n;
        const int cl = col0 + li;
        const bool cok = cl < n;
        // every operand of the tile is loaded from a clamped (valid) address
        // first and zeroed where out of range afterwards, so the loads carry
        // no branches and are in flight together
        const int rowc_ = min(row, n - 1), clc = min(cl, n - 1);
        double a4[4], wcv[kPanel / 4], vcv[kPanel / 4], vrv[kPanel / 4], wrv[kPanel / 4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a4[i] = At(rowc_, min(col0 + 4 * i + lk, n - 1));
#pragma unroll
        for (int kq = 0; kq < kPanel / 4; ++kq) {
          const int qc = min(4 * kq + lk, nb - 1);
          wcv[kq] = Wp(qc, clc);
          vcv[kq] = Vp(qc, clc);
          vrv[kq] = Vp(qc, rowc_);
          wrv[kq] = Wp(qc, rowc_);
        }
        v4d acc;
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] = (rok && col0 + 4 * i + lk < n) ? a4[i] : 0.0;
#pragma unroll
        for (int kq = 0; kq < kPanel / 4; ++kq) {
          const bool qok = 4 * kq + lk < nb;
          const double wc = (qok && cok) ? wcv[kq] : 0.0;
          const double vc = (qok && cok) ? vcv[kq] : 0.0;
          const double vrr = (qok && rok) ? vrv[kq] : 0.0;
          const double wr = (qok && rok) ? wrv[kq] : 0.0;
          acc = mfma16(-wc, vrr, acc);
          acc = mfma16(-vc, wr, acc);
        }
        if (rok) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int col = col0 + 4 * i + lk;
            if (col < n) {
              if (row >= n0 && col >= n0) cor[(row - n0) + (size_t)m * (col - n0)] = acc[i];
              else A[row + (size_t)n * col] = acc[i];
            }
          }
        }
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (n >= 2) {
      D[b + n - 2] = At(n - 2, n - 2);
      E[b + n - 2] = At(n - 1, n - 2);
    }
    D[b + n - 1] = At(n - 1, n - 1);
    E[b + n - 1] = 0.0;
  }
}

__global__ __launch_bounds__(kTdThreads) void k_tridiag(
    double* __restrict__ abuf, double* __restrict__ wsc, const int64_t* __restrict__ off2,
    const int32_t* __restrict__ sub_orb_ptr, const int32_t* __restrict__ order,
    double* __restrict__ D, double* __restrict__ E, double* __restrict__ TAU, int lds_doubles) {
  extern __shared__ double pan[];  // the panel (n <= kLdsPanelN), then the corner
  __shared__ __align__(16) double vl[kTdMaxN + kUnroll];  // v, then kUnroll zeros
  __shared__ double part[kTdThreads];
  __shared__ double red[2 * (kTdThreads / 64)];  // the two sums of a column
  __shared__ double yp[kTdThreads / 32][2 * kPanel + 1];
  __shared__ double yfin[2 * kPanel];
  __shared__ double rowc[2 * kPanel];
  __shared__ double alpha_sh;
  const int s = order[blockIdx.x];
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  double* A = abuf + off2[s];
  double* W = wsc + (size_t)b * kPanel;  // W[q * n + r]
  if (n <= kLdsPanelN)
    tridiag_body<true>(A, W, pan, n, b, D, E, TAU, vl, part, red, yp, yfin, rowc, &alpha_sh,
                       lds_doubles);
  else
    tridiag_body<false>(A, W, pan, n, b, D, E, TAU, vl, part, red, yp, yfin, rowc, &alpha_sh,
                        lds_doubles);
}

// ---------------------------------------------------------------------------
// Multi-workgroup reduction of the subgraphs of kMwgMinN orbitals and more
// (up to kMaxN): the blocked algorithm of k_tridiag (panels of kPanel
// reflectors formed against the stale trailing matrix plus the panel
// corrections, then a rank-2 kPanel update on MFMA), with each step spread
// over workgroups and the kernel launches as the only synchronisation.  Only
// the lower triangle of the trailing matrix, in absolute 64x64 tiles (I >= J),
// is read and kept up to date; diagonal tiles are kept whole.
//   k_td_col     one 1024-thread workgroup per subgraph (two rows per
//                thread): completes the previous column's p from the tile
//                partials (fixed order), its panel corrections and tau, then
//                w = p - (tau/2)(p.v) v; forms the current column, its
//                reflector (v, tau, beta) and the panel products W^T v, V^T v;
//   k_td_symv    one workgroup per lower tile (I, J) of the trailing matrix:
//                the row partials A_IJ v_J and, off the diagonal, the column
//                partials A_IJ^T v_I (the upper tile's share by symmetry);
//   k_td_update  one workgroup per lower tile: A -= V W^T + W V^T on MFMA for
//                the rows and columns of the trailing matrix;
//   k_td_final   the last two diagonal entries and the last off-diagonal one.
// Every listed subgraph takes part in each launch (one whose reduction has
// ended returns at once).  Reflectors, d, e and tau are stored as k_tridiag
// stores them, so the divide and conquer and the back-transformation are
// shared.  Per subgraph the scratch slot holds v (rows < n; readers mask the
// rest), the panel products (W^T v, then V^T v) and the row and column
// partials of every lower tile.
constexpr int kTdRows = kMaxN / kTdThreads;
constexpr int kTdBlocks = kMaxN / 64;
constexpr int kTdTiles = kTdBlocks * (kTdBlocks + 1) / 2;

struct MwgSlot {
  double *v, *y, *rowp, *colp;
  __device__ MwgSlot(double* base) {
    v = base;               // [kMaxN]
    y = v + kMaxN;          // [2 kPanel]
    rowp = y + 2 * kPanel;  // [kTdTiles][64]
    colp = rowp + (size_t)kTdTiles * 64;
  }
};
static_assert(kMaxN + 2 * kPanel + 2 * kTdTiles * 64 <= kMwgSlot, "scratch slot too small");

// Index of the lower tile (I, J), J <= I, and its inverse.
__device__ __forceinline__ int tile_id(int I, int J) { return I * (I + 1) / 2 + J; }
__device__ __forceinline__ void tile_ij(int t, int& I, int& J) {
  int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while (i * (i + 1) / 2 > t) --i;
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  I = i;
  J = t - i * (i + 1) / 2;
}

__global__ __launch_bounds__(kTdThreads) void k_td_col(
    double* __restrict__ abuf, double* __restrict__ wsc, const int64_t* __restrict__ off2,
    const int32_t* __restrict__ sub_orb_ptr, const int32_t* __restrict__ order,
    double* __restrict__ D, double* __restrict__ E, double* __restrict__ TAU,
    double* __restrict__ mwg, int k0, int j) {
  __shared__ __align__(16) double vl[kMaxN];
  __shared__ double red[2][kTdThreads / 64];  // the two workgroup sums
  __shared__ double rowc[2 * kPanel];
  __shared__ double alpha_sh;
  const int s = order[blockIdx.x];
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  if (k0 + 2 >= n) return;
  const int nb = min(kPanel, n - 2 - k0);
  if (j > nb) return;
  double* A = abuf + off2[s];
  double* Wg = wsc + (size_t)b * kPanel;  // W[q * n + r]
  MwgSlot sl(mwg + (size_t)blockIdx.x * kMwgSlot);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // the previous column cp: p from the tile partials and the panel
  // corrections, then w; wprev keeps w of this thread's rows
  double wprev[kTdRows];
#pragma unroll
  for (int u = 0; u < kTdRows; ++u) wprev[u] = 0.0;
  if (j >= 1) {
    const int cp = k0 + j - 1;
    const double tp = TAU[b + cp];
    const int B0 = (cp + 1) / 64, NB = (n + 63) / 64;
    double pr[kTdRows], pv = 0.0;
#pragma unroll
    for (int u = 0; u < kTdRows; ++u) {
      const int r = tid + u * kTdThreads;
      pr[u] = 0.0;
      if (tp != 0.0 && r < n && r >= cp + 1) {
        // the partials of blocks B0 + t, t ascending: row partials of tiles
        // (I, B0 + t) up to the diagonal, column partials of tiles (B0 + t, I)
        // below it; all loads issued before the sum (unused terms read a
        // valid entry and are dropped)
        const int I = r >> 6, i = r & 63, cnt = NB - B0;
        double pt[kTdBlocks];
#pragma unroll
        for (int t = 0; t < kTdBlocks; ++t) {
          const int K2 = min(B0 + t, NB - 1);
          pt[t] = K2 <= I ? sl.rowp[(size_t)tile_id(I, K2) * 64 + i]
                          : sl.colp[(size_t)tile_id(K2, I) * 64 + i];
        }
        double acc = 0.0;
#pragma unroll
        for (int t = 0; t < kTdBlocks; ++t) acc += t < cnt ? pt[t] : 0.0;
        double cv[kPanel], cw[kPanel];
#pragma unroll
        for (int q = 0; q < kPanel; ++q) {
          const int qc = min(q, max(j - 2, 0));
          cv[q] = A[r + (size_t)n * (k0 + qc)];
          cw[q] = Wg[qc * n + r];
        }
#pragma unroll
        for (int q = 0; q < kPanel; ++q)
          if (q < j - 1) acc -= cv[q] * sl.y[q] + cw[q] * sl.y[kPanel + q];
        pr[u] = tp * acc;
        pv += pr[u] * sl.v[r];
      }
    }
    const double K = 0.5 * tp * tsum(pv, red[0]);
#pragma unroll
    for (int u = 0; u < kTdRows; ++u) {
      const int r = tid + u * kTdThreads;
      if (tp != 0.0 && r < n) {
        wprev[u] = r >= cp + 1 ? pr[u] - K * sl.v[r] : 0.0;
        Wg[(j - 1) * n + r] = wprev[u];
      }
    }
  }
  if (j == nb) return;
  const int c = k0 + j;
  // row c's panel entries: earlier columns from memory, column j - 1's w from
  // the thread that owns row c
  if (tid < j) rowc[tid] = A[c + (size_t)n * (k0 + tid)];
  if (tid + 1 < j) rowc[kPanel + tid] = Wg[tid * n + c];
  if (j >= 1 && (c % kTdThreads) == tid) rowc[kPanel + j - 1] = wprev[c / kTdThreads];
  __syncthreads();
  // the current column: A[r, c] - sum_q (v_q[r] w_q[c] + w_q[r] v_q[c]), r >= c
  double a[kTdRows];
  double sq = 0.0;
#pragma unroll
  for (int u = 0; u < kTdRows; ++u) {
    const int r = tid + u * kTdThreads;
    a[u] = 0.0;
    if (r < n && r >= c) {
      double x = A[r + (size_t)n * c];
      for (int q = 0; q + 1 < j; ++q)
        x -= A[r + (size_t)n * (k0 + q)] * rowc[kPanel + q] + Wg[q * n + r] * rowc[q];
      if (j >= 1)
        x -= A[r + (size_t)n * (k0 + j - 1)] * rowc[kPanel + j - 1] + wprev[u] * rowc[j - 1];
      a[u] = x;
      if (r == c) D[b + c] = x;
      if (r == c + 1) alpha_sh = x;
      if (r >= c + 2) sq += x * x;
    }
  }
  const double sigma = tsum(sq, red[1]);  // its barrier also publishes alpha_sh
  const double alpha = alpha_sh;
  double tau = 0.0, beta = alpha, scale = 0.0;
  if (sigma != 0.0) {
    const double nrm = sqrt(alpha * alpha + sigma);
    beta = alpha >= 0.0 ? -nrm : nrm;
    tau = (beta - alpha) / beta;
    scale = 1.0 / (alpha - beta);
  }
  // v (zero at rows <= c; all zero when H = I), into A's column c below the
  // diagonal, LDS and the slot
#pragma unroll
  for (int u = 0; u < kTdRows; ++u) {
    const int r = tid + u * kTdThreads;
    if (r < n) {
      const double v = tau == 0.0 ? 0.0 : (r == c + 1 ? 1.0 : (r >= c + 2 ? a[u] * scale : 0.0));
      vl[r] = v;
      sl.v[r] = v;
      if (r >= c + 1) A[r + (size_t)n * c] = v;
      if (tau == 0.0) Wg[j * n + r] = 0.0;
    }
  }
  if (tid == 0) {
    TAU[b + c] = tau;
    E[b + c] = beta;
  }
  if (tau == 0.0) return;
  __syncthreads();
  // y = (W^T v, V^T v) over the panel so far, rows > c: wave q takes panel
  // column q, its lanes 64-row strides, then a wave sum
  if (wv < j) {
    double t1 = 0.0, t2 = 0.0;
    for (int r = c + 1 + lane; r < n; r += 64) {
      t1 += Wg[wv * n + r] * vl[r];
      t2 += A[r + (size_t)n * (k0 + wv)] * vl[r];
    }
    t1 = wave_total(t1);
    t2 = wave_total(t2);
    if (lane == 0) {
      sl.y[wv] = t1;
      sl.y[kPanel + wv] = t2;
    }
  }
}

// Tile (I, J) of the trailing matrix (absolute 64-row blocks, B0 <= J <= I,
// B0 the block of row c + 1): wave w takes the tile's columns 16w .. 16w+15,
// lane l its row 64 I + l.  Row partials: sum over the tile's columns of
// A v; column partials (I > J): sum over the tile's rows of A^T v, reduced
// across the lanes by halving exchanges (each step keeps half of the columns
// and adds the partner's share), so lane l ends with column (l / 4) mod 16.
__global__ __launch_bounds__(256) void k_td_symv(
    const double* __restrict__ abuf, const int64_t* __restrict__ off2,
    const int32_t* __restrict__ sub_orb_ptr, const int32_t* __restrict__ order,
    const double* __restrict__ TAU, double* __restrict__ mwg, int k0, int j) {
  __shared__ double vr[64], vc[64];
  __shared__ double rp[4][64];
  const int s = order[blockIdx.y];
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  if (k0 + 2 >= n) return;
  const int nb = min(kPanel, n - 2 - k0);
  if (j >= nb) return;
  const int c = k0 + j;
  if (TAU[b + c] == 0.0) return;
  const int B0 = (c + 1) / 64, NB = (n + 63) / 64, nt = NB - B0;
  if ((int)blockIdx.x >= nt * (nt + 1) / 2) return;
  int I, J;
  tile_ij(blockIdx.x, I, J);
  I += B0;
  J += B0;
  MwgSlot sl(mwg + (size_t)blockIdx.y * kMwgSlot);
  const double* A = abuf + off2[s];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid < 64) {
    const int r = 64 * I + tid;
    vr[tid] = r < n ? sl.v[r] : 0.0;
  } else if (tid < 128) {
    const int k = 64 * J + tid - 64;
    vc[tid - 64] = k < n ? sl.v[k] : 0.0;
  }
  __syncthreads();
  const int rc = min(64 * I + lane, n - 1);
  double x[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) x[k] = A[rc + (size_t)n * min(64 * J + 16 * wv + k, n - 1)];
  double rs = 0.0;
#pragma unroll
  for (int k = 0; k < 16; ++k) rs += x[k] * vc[16 * wv + k];
  rp[wv][lane] = rs;
  const int t = tile_id(I, J);
  if (I > J) {
    const double vi = vr[lane];
    double y[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) y[k] = x[k] * vi;
    double y8[8], y4[4], y2[2];
    const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8, b2 = lane & 4;
#pragma unroll
    for (int k = 0; k < 8; ++k)
      y8[k] = (b5 ? y[k + 8] : y[k]) + __shfl_xor(b5 ? y[k] : y[k + 8], 32, 64);
#pragma unroll
    for (int k = 0; k < 4; ++k)
      y4[k] = (b4 ? y8[k + 4] : y8[k]) + __shfl_xor(b4 ? y8[k] : y8[k + 4], 16, 64);
#pragma unroll
    for (int k = 0; k < 2; ++k)
      y2[k] = (b3 ? y4[k + 2] : y4[k]) + __shfl_xor(b3 ? y4[k] : y4[k + 2], 8, 64);
    double z = (b2 ? y2[1] : y2[0]) + __shfl_xor(b2 ? y2[0] : y2[1], 4, 64);
    z += __shfl_xor(z, 2, 64);
    z += __shfl_xor(z, 1, 64);
    if ((lane & 3) == 0) sl.colp[(size_t)t * 64 + 16 * wv + ((lane >> 2) & 15)] = z;
  }
  __syncthreads();
  if (tid < 64) sl.rowp[(size_t)t * 64 + tid] = (rp[0][tid] + rp[1][tid]) + (rp[2][tid] + rp[3][tid]);
}

// Lower tile (BI, BJ), BT <= BJ <= BI with BT the block of row t0: the
// rank-2 kPanel update of its elements in rows and columns >= t0, by its
// sixteen 16x16 sub-tiles (four per wave); element (row0 + j, col0 + i) in
// lane j + 16 (i % 4), register i / 4, as in k_tridiag.
__global__ __launch_bounds__(256) void k_td_update(
    double* __restrict__ abuf, const double* __restrict__ wsc, const int64_t* __restrict__ off2,
    const int32_t* __restrict__ sub_orb_ptr, const int32_t* __restrict__ order, int k0) {
  const int s = order[blockIdx.y];
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  if (k0 + 2 >= n) return;
  const int nb = min(kPanel, n - 2 - k0);
  const int t0 = k0 + nb;
  const int BT = t0 / 64, NB = (n + 63) / 64, nt = NB - BT;
  if ((int)blockIdx.x >= nt * (nt + 1) / 2) return;
  int BI, BJ;
  tile_ij(blockIdx.x, BI, BJ);
  BI += BT;
  BJ += BT;
  double* A = abuf + off2[s];
  const double* Wg = wsc + (size_t)b * kPanel;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll 1
  for (int tile = wv; tile < 16; tile += 4) {
    const int row0 = 64 * BI + 16 * (tile / 4), col0 = 64 * BJ + 16 * (tile % 4);
    const int row = row0 + li;
    const bool rok = row >= t0 && row < n;
    const int cl = col0 + li;
    const bool cok = cl < n;
    const int rowc_ = min(row, n - 1), clc = min(cl, n - 1);
    double a4[4], wcv[kPanel / 4], vcv[kPanel / 4], vrv[kPanel / 4], wrv[kPanel / 4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a4[i] = A[rowc_ + (size_t)n * min(col0 + 4 * i + lk, n - 1)];
#pragma unroll
    for (int kq = 0; kq < kPanel / 4; ++kq) {
      const int qc = min(4 * kq + lk, nb - 1);
      wcv[kq] = Wg[qc * n + clc];
      vcv[kq] = A[clc + (size_t)n * (k0 + qc)];
      vrv[kq] = A[rowc_ + (size_t)n * (k0 + qc)];
      wrv[kq] = Wg[qc * n + rowc_];
    }
    v4d acc;
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = a4[i];
#pragma unroll
    for (int kq = 0; kq < kPanel / 4; ++kq) {
      const bool qok = 4 * kq + lk < nb;
      const double wc = (qok && cok) ? wcv[kq] : 0.0;
      const double vc = (qok && cok) ? vcv[kq] : 0.0;
      const double vrr = (qok && rok) ? vrv[kq] : 0.0;
      const double wr = (qok && rok) ? wrv[kq] : 0.0;
      acc = mfma16(-wc, vrr, acc);
      acc = mfma16(-vc, wr, acc);
    }
    if (rok) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int col = col0 + 4 * i + lk;
        if (col >= t0 && col < n) A[row + (size_t)n * col] = acc[i];
      }
    }
  }
}

__global__ void k_td_final(const double* __restrict__ abuf, const int64_t* __restrict__ off2,
                           const int32_t* __restrict__ sub_orb_ptr,
                           const int32_t* __restrict__ order, double* __restrict__ D,
                           double* __restrict__ E) {
  const int s = order[blockIdx.x];
  const int b = sub_orb_ptr[s];
  const int n = sub_orb_ptr[s + 1] - b;
  const double* A = abuf + off2[s];
  if (threadIdx.x == 0 && n >= 2) {
    D[b + n - 2] = A[(n - 2) + (size_t)n * (n - 2)];
    E[b + n - 2] = A[(n - 1) + (size_t)n * (n - 2)];
    D[b + n - 1] = A[(size_t)(n - 1) * (n + 1)];
    E[b + n - 1] = 0.0;
  }
}

}  // namespace

// The multi-workgroup reduction of order[first..first+count) (scratch slots
// from `first`) on stream st: per panel,
// kPanel column steps (k_td_col, k_td_symv) and one k_td_col that completes
// the panel's last w, then the trailing update of the lower tiles.
static void launch_tridiag_mwg(gq_ctx* ctx, const gq_graph* g, gq_eigs* e, hipStream_t st,
                               int first, int count, const char* label) {
  const gq_graph_dev& dv = g->dev;
  const int nh = count;
  const int32_t* order = dv.order + first;
  double* slots = e->mwg + (size_t)first * kMwgSlot;
  const int maxn = g->sub_orb_ptr[g->order[first] + 1] - g->sub_orb_ptr[g->order[first]];
  const int NB = (maxn + 63) / 64;
  prof_begin_on(ctx, label, st);
  for (int k0 = 0; k0 + 2 < maxn; k0 += kPanel) {
    const int nbmax = std::min(kPanel, maxn - 2 - k0);
    // lower tiles from the block of row k0 (an upper bound for every column
    // of the panel and for the update from row t0 > k0)
    const int nt = NB - k0 / 64, ntiles = nt * (nt + 1) / 2;
    for (int j = 0; j <= nbmax; ++j) {
      hipLaunchKernelGGL(k_td_col, dim3(nh), dim3(kTdThreads), 0, st, e->A, e->wsc, dv.off2,
                         dv.sub_orb_ptr, order, e->dd, e->ee, e->tau, slots, k0, j);
      if (j < nbmax)
        hipLaunchKernelGGL(k_td_symv, dim3(ntiles, nh), dim3(256), 0, st, e->A, dv.off2,
                           dv.sub_orb_ptr, order, e->tau, slots, k0, j);
    }
    hipLaunchKernelGGL(k_td_update, dim3(ntiles, nh), dim3(256), 0, st, e->A, e->wsc, dv.off2,
                       dv.sub_orb_ptr, order, k0);
  }
  hipLaunchKernelGGL(k_td_final, dim3(nh), dim3(64), 0, st, e->A, dv.off2, dv.sub_orb_ptr,
                     order, e->dd, e->ee);
  prof_end(ctx);
}

// Dynamic LDS of k_tridiag: the panel and the corner share what its 25.7 KB of
// static LDS leave of the CU's 160 KB (one workgroup per CU either way).
constexpr int kTdDynLds = 137216;

void eig_set_attributes() {
  (void)hipFuncSetAttribute((const void*)k_tridiag, hipFuncAttributeMaxDynamicSharedMemorySize,
                            kTdDynLds);
}

void launch_gather(gq_ctx* ctx, const gq_graph* g, const gq_csr* H, double* A, int32_t* status,
                   const char* label) {
  const gq_graph_dev& dv = g->dev;
  const int maxn = g->info.max_n;
  hipStream_t st = ctx->stream;
  prof_begin(ctx, label);
  hipLaunchKernelGGL(k_gather, dim3(g->n_sub), dim3(kGaThreads), 2 * maxn * sizeof(int32_t), st,
                     H->row_ptr, H->col, H->val, A, dv.off2, dv.sub_orb_ptr, dv.sub_orbs,
                     dv.sorted_orbs, dv.sorted_local, dv.order, status);
  prof_end(ctx);
}

void launch_eigensolve(gq_ctx* ctx, const gq_graph* g, gq_eigs* e) {
  const gq_graph_dev& dv = g->dev;
  // two size classes on two streams: the n_big largest subgraphs on the
  // caller's stream, the rest on a side stream forked from it and joined
  // back, so that the small subgraphs' divide and conquer and
  // back-transformation fill the CUs the long tridiagonalisations leave idle
  hipStream_t st = ctx->stream;
  const int nbig = g->n_big, nsmall = g->n_sub - g->n_big;
  if (nsmall > 0) {
    (void)hipEventRecord(ctx->ev_fork, st);
    (void)hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0);
    prof_begin_on(ctx, "k_tridiag", ctx->side);
    hipLaunchKernelGGL(k_tridiag, dim3(nsmall), dim3(kTdThreads), kTdDynLds, ctx->side,
                       e->A, e->wsc, dv.off2, dv.sub_orb_ptr, dv.order + nbig, e->dd, e->ee,
                       e->tau, kTdDynLds / 8);
    prof_end(ctx);
    launch_dc(ctx, g, e, 1, ctx->side);
  }
  // with no small class the side stream is free: the multi-workgroup
  // subgraphs go in two halves, the larger on the caller's stream and the
  // smaller on the side stream, so that one half's single-workgroup column
  // steps overlap the other half's tile products
  const bool mwg_split = nsmall == 0 && g->n_mwg >= 2;
  if (nbig > 0) {
    const int nh = g->n_mwg;
    if (mwg_split) {
      const int na = (nh + 1) / 2;
      (void)hipEventRecord(ctx->ev_fork, st);
      (void)hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0);
      launch_tridiag_mwg(ctx, g, e, ctx->side, na, nh - na, "k_tridiag_mwg_b");
      (void)hipEventRecord(ctx->ev_join, ctx->side);
      launch_tridiag_mwg(ctx, g, e, st, 0, na, "k_tridiag_mwg");
    } else if (nh > 0) {
      launch_tridiag_mwg(ctx, g, e, st, 0, nh, "k_tridiag_mwg");
    }
    if (nbig > nh) {
      prof_begin(ctx, "k_tridiag");
      hipLaunchKernelGGL(k_tridiag, dim3(nbig - nh), dim3(kTdThreads), kTdDynLds, st, e->A,
                         e->wsc, dv.off2, dv.sub_orb_ptr, dv.order + nh, e->dd, e->ee, e->tau,
                         kTdDynLds / 8);
      prof_end(ctx);
    }
    if (mwg_split) (void)hipStreamWaitEvent(st, ctx->ev_join, 0);
    launch_dc(ctx, g, e, 0, st);
  }
  if (nsmall > 0) {
    (void)hipEventRecord(ctx->ev_join, ctx->side);
    (void)hipStreamWaitEvent(st, ctx->ev_join, 0);
  }
}

}  // namespace gq
