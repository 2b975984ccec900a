// Charge response, subgraph preconditioner and the preconditioned low-rank
// Krylov kernel of graph-based shadow molecular dynamics (Sec. V), on top of
// the canonical response of k_response.hip.
//
// Atomic charges n act on every orbital of atom I through the potential
// (gamma n)_I, so a charge vector v perturbs the Hamiltonian by
// H1[v] = diag(gamma v) over the orbitals.  The core charges of a density
// (Eq. (assemble_rho0)) are the diagonal entries of its collected core rows
// summed per atom; for a response they are P_jj + mu1 M_jj (Eq. (D1)), which
// needs only the diagonal of P.
//
//   k_spmv          (gamma v)_I, one row per thread, fixed order
//   k_h1_atoms      the potential of every orbital of every subgraph
//   k_h1_unit       the potential of a unit charge on core atom q of each
//                   subgraph (Sec. V.A), restricted to that subgraph
//   k_atom_charges  per-atom charges from core-row blocks, or from the
//                   diagonal of P and mu1 M
//   k_unit_collect  the core-atom responses a_ij and mu responses b_i
//   k_k0            j = a + b mu1^T - I with the column sums over the core
//                   shifted to -1, k0 = (j - alpha I)^-1 (Gauss-Jordan)
//   k_k0_apply      K0 x, block-diagonal over the core atoms
//   k_kr_*          the Krylov vectors: normalisation, two-pass modified
//                   Gram-Schmidt, O = F F^T, M = O^-1 and the acceleration
//                   (one workgroup, fixed-order sums)
#include <algorithm>
#include <new>

#include "gq_internal.hpp"

struct gq_charge {
  gq_ctx* ctx = nullptr;
  const gq_graph* g = nullptr;
  int32_t n_atoms = 0, N = 0, n_sub = 0, max_m = 0;
  int64_t k0_len = 0;
  char* block = nullptr;
  bool in_arena = false;
  size_t arena_off = 0, arena_bytes = 0;
  // gamma (atoms x atoms, CSR)
  int32_t *g_rp = nullptr, *g_col = nullptr;
  double* g_val = nullptr;
  int32_t* atom_of = nullptr;     // [N] atom of each orbital
  int32_t* atom_sub = nullptr;    // [n_atoms] the subgraph whose core holds the atom
  int32_t* atom_j0 = nullptr;     // [n_atoms] its first local orbital there
  int32_t* atom_nk = nullptr;     // [n_atoms] its orbitals
  int32_t* atom_ci = nullptr;     // [n_atoms] its index among that core's atoms
  int32_t* core_ptr = nullptr;    // [n_sub+1]
  int32_t* core_atoms = nullptr;  // [n_atoms] core atoms, subgraph by subgraph
  int32_t* k0_off = nullptr;      // [n_sub+1] offsets of the m_s x m_s blocks
  double* pot = nullptr;          // [kmax][n_atoms] potentials
  double* a_all = nullptr;        // [k0_len] unit-charge responses
  double* bvec = nullptr;         // [n_atoms] mu responses per core atom
  double* vec = nullptr;          // [4][n_atoms] work vectors
  double* small = nullptr;        // [2 * 32 * 32 + 64] O, M and coefficients
  int32_t kmax = 0;
};

namespace gq {

namespace {

constexpr int kT = 256;     // threads of the elementwise kernels
constexpr int kRed = 1024;  // threads of the single-workgroup reductions
constexpr int kMaxKrylov = 32;

__global__ __launch_bounds__(kT) void k_spmv(const int32_t* __restrict__ rp,
                                             const int32_t* __restrict__ col,
                                             const double* __restrict__ val,
                                             const double* __restrict__ v, int n,
                                             double* __restrict__ out) {
  const int q = blockIdx.y;
  const double* vq = v + (size_t)q * n;
  for (int I = blockIdx.x * kT + threadIdx.x; I < n; I += gridDim.x * kT) {
    double acc = 0.0;
    for (int p = rp[I]; p < rp[I + 1]; ++p) acc += val[p] * vq[col[p]];
    out[(size_t)q * n + I] = acc;
  }
}

// hloc[q][b + m] = pot[q][atom of orbital orbs[b + m]]
__global__ __launch_bounds__(kT) void k_h1_atoms(const double* __restrict__ pot, int n_atoms,
                                                 const int32_t* __restrict__ atom_of,
                                                 const int32_t* __restrict__ sub_orbs,
                                                 int64_t sum_n, double* __restrict__ hloc) {
  const int q = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < sum_n;
       i += (int64_t)gridDim.x * kT)
    hloc[(size_t)q * sum_n + i] = pot[(size_t)q * n_atoms + atom_of[sub_orbs[i]]];
}

// Perturbation q of subgraph s: the potential gamma(I, J) on every orbital of
// atom I of the subgraph, J = core atom q0 + q of s (zero when s has fewer).
__global__ __launch_bounds__(kT) void k_h1_unit(
    const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
    const double* __restrict__ val, const int32_t* __restrict__ atom_of,
    const int32_t* __restrict__ sub_orb_ptr, const int32_t* __restrict__ sub_orbs,
    const int32_t* __restrict__ core_ptr, const int32_t* __restrict__ core_atoms, int q0,
    int64_t sum_n, double* __restrict__ hloc) {
  const int s = blockIdx.x, q = blockIdx.y;
  const int b = sub_orb_ptr[s], n = sub_orb_ptr[s + 1] - b;
  const int m = core_ptr[s + 1] - core_ptr[s];
  const int J = q0 + q < m ? core_atoms[core_ptr[s] + q0 + q] : -1;
  for (int i = threadIdx.x; i < n; i += kT) {
    double v = 0.0;
    if (J >= 0) {
      const int I = atom_of[sub_orbs[b + i]];
      int lo = rp[J], hi = rp[J + 1];  // gamma is symmetric: row J holds (J, I)
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (col[mid] < I) lo = mid + 1;
        else hi = mid;
      }
      if (lo < rp[J + 1] && col[lo] == I) v = val[lo];
    }
    hloc[(size_t)q * sum_n + b + i] = v;
  }
}

// Per-atom charges of K densities.  blocks != NULL: sum of the diagonal
// entries of the core-row blocks ([K][nnz]).  Otherwise the response form
// P_jj + mu1_q M_jj from pdiag ([K][sum_c]), M and mu1.
__global__ __launch_bounds__(kT) void k_atom_charges(
    const double* __restrict__ blocks, int64_t nnz, const double* __restrict__ pdiag,
    int sum_c, const double* __restrict__ M, const double* __restrict__ mu1,
    const int32_t* __restrict__ atom_sub, const int32_t* __restrict__ atom_j0,
    const int32_t* __restrict__ atom_nk, const int64_t* __restrict__ offc,
    const int32_t* __restrict__ offcd, const int32_t* __restrict__ sub_orb_ptr, int n_atoms,
    double* __restrict__ q_out) {
  const int q = blockIdx.y;
  for (int I = blockIdx.x * kT + threadIdx.x; I < n_atoms; I += gridDim.x * kT) {
    const int s = atom_sub[I], j0 = atom_j0[I], nk = atom_nk[I];
    const int n = sub_orb_ptr[s + 1] - sub_orb_ptr[s];
    double acc = 0.0;
    for (int j = j0; j < j0 + nk; ++j) {
      const size_t at = offc[s] + (size_t)j * n + j;
      if (blocks) acc += blocks[(size_t)q * nnz + at];
      else acc += pdiag[(size_t)q * sum_c + offcd[s] + j] + mu1[q] * M[at];
    }
    q_out[(size_t)q * n_atoms + I] = acc;
  }
}

// a[s](i, q0 + q) = sum over the orbitals of core atom i of P^(q)_jj (fixed mu);
// with q0 == 0 also b_i = the same sum of M_jj.
__global__ __launch_bounds__(kT) void k_unit_collect(
    const double* __restrict__ pdiag, int sum_c, const double* __restrict__ M, int K, int q0,
    const int32_t* __restrict__ atom_sub, const int32_t* __restrict__ atom_j0,
    const int32_t* __restrict__ atom_nk, const int32_t* __restrict__ atom_ci,
    const int32_t* __restrict__ core_ptr, const int32_t* __restrict__ k0_off,
    const int64_t* __restrict__ offc, const int32_t* __restrict__ offcd,
    const int32_t* __restrict__ sub_orb_ptr, int n_atoms, double* __restrict__ a_all,
    double* __restrict__ bvec) {
  for (int I = blockIdx.x * kT + threadIdx.x; I < n_atoms; I += gridDim.x * kT) {
    const int s = atom_sub[I], j0 = atom_j0[I], nk = atom_nk[I], ci = atom_ci[I];
    const int m = core_ptr[s + 1] - core_ptr[s];
    const int n = sub_orb_ptr[s + 1] - sub_orb_ptr[s];
    for (int q = 0; q < K && q0 + q < m; ++q) {
      double acc = 0.0;
      for (int j = j0; j < j0 + nk; ++j) acc += pdiag[(size_t)q * sum_c + offcd[s] + j];
      a_all[k0_off[s] + ci + (size_t)m * (q0 + q)] = acc;
    }
    if (q0 == 0) {
      double acc = 0.0;
      for (int j = j0; j < j0 + nk; ++j) acc += M[offc[s] + (size_t)j * n + j];
      bvec[I] = acc;
    }
  }
}

// In-place inverse of the m x m matrix A (LDS, row stride ld, m <= 32) by
// Gauss-Jordan elimination with partial pivoting on the augmented [A | I];
// the workgroup's threads share the row updates.  Returns false (uniformly)
// for a zero pivot.
__device__ bool gj_inverse(double* A, double* X, int m, int ld) {
  __shared__ int piv;
  for (int t = threadIdx.x; t < m * m; t += blockDim.x) {
    const int r = t / m, c = t % m;
    X[r * ld + c] = r == c ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int k = 0; k < m; ++k) {
    if (threadIdx.x == 0) {
      int p = k;
      double best = fabs(A[k * ld + k]);
      for (int r = k + 1; r < m; ++r)
        if (fabs(A[r * ld + k]) > best) {
          best = fabs(A[r * ld + k]);
          p = r;
        }
      piv = best > 0.0 ? p : -1;
    }
    __syncthreads();
    const int p = piv;
    if (p < 0) return false;
    if (p != k)
      for (int c = threadIdx.x; c < m; c += blockDim.x) {
        double t = A[k * ld + c];
        A[k * ld + c] = A[p * ld + c];
        A[p * ld + c] = t;
        t = X[k * ld + c];
        X[k * ld + c] = X[p * ld + c];
        X[p * ld + c] = t;
      }
    __syncthreads();
    const double inv = 1.0 / A[k * ld + k];
    __syncthreads();
    for (int c = threadIdx.x; c < m; c += blockDim.x) {
      A[k * ld + c] *= inv;
      X[k * ld + c] *= inv;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < m * m; t += blockDim.x) {
      const int r = t / m, c = t % m;
      if (r == k) continue;
      const double f = A[r * ld + k];
      if (c != k) A[r * ld + c] -= f * A[k * ld + c];
      X[r * ld + c] -= f * X[k * ld + c];
    }
    __syncthreads();
    for (int r = threadIdx.x; r < m; r += blockDim.x)
      if (r != k) A[r * ld + k] = 0.0;
    __syncthreads();
  }
  return true;
}

// k0 of subgraph s (one workgroup): a (column-major, m x m) and b give
// mu1_j = -sum_i a_ij / sum_i b_i, j = a + b mu1^T - I, k0 = (j - alpha I)^-1.
// A singular block leaves k0 as NaN and sets *bad.
__global__ __launch_bounds__(64) void k_k0(const double* __restrict__ a_all,
                                           const double* __restrict__ bvec,
                                           const int32_t* __restrict__ core_ptr,
                                           const int32_t* __restrict__ core_atoms,
                                           const int32_t* __restrict__ k0_off, double alpha,
                                           double* __restrict__ k0, int32_t* __restrict__ bad) {
  __shared__ double A[32 * 33], X[32 * 33], mu1[32], bs[32];
  constexpr int ld = 33;
  const int s = blockIdx.x;
  const int m = core_ptr[s + 1] - core_ptr[s];
  const double* a = a_all + k0_off[s];
  for (int i = threadIdx.x; i < m; i += 64) bs[i] = bvec[core_atoms[core_ptr[s] + i]];
  __syncthreads();
  if (threadIdx.x < m) {
    const int j = threadIdx.x;
    double ca = 0.0, cb = 0.0;
    for (int i = 0; i < m; ++i) {
      ca += a[i + (size_t)m * j];
      cb += bs[i];
    }
    mu1[j] = -ca / cb;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < m * m; t += 64) {
    const int r = t / m, c = t % m;
    A[r * ld + c] = a[r + (size_t)m * c] + bs[r] * mu1[c] - (r == c ? 1.0 + alpha : 0.0);
  }
  __syncthreads();
  const bool ok = gj_inverse(A, X, m, ld);
  double* out = k0 + k0_off[s];
  for (int t = threadIdx.x; t < m * m; t += 64) {
    const int r = t / m, c = t % m;
    out[r + (size_t)m * c] = ok ? X[r * ld + c] : __builtin_nan("");
  }
  if (!ok && threadIdx.x == 0) *bad = 1;
}

// y = K0 (x - z) (z may be NULL): atom I takes row ci of its core's block.
__global__ __launch_bounds__(kT) void k_k0_apply(
    const double* __restrict__ k0, const double* __restrict__ x, const double* __restrict__ z,
    const int32_t* __restrict__ atom_sub, const int32_t* __restrict__ atom_ci,
    const int32_t* __restrict__ core_ptr, const int32_t* __restrict__ core_atoms,
    const int32_t* __restrict__ k0_off, int n_atoms, double* __restrict__ y) {
  for (int I = blockIdx.x * kT + threadIdx.x; I < n_atoms; I += gridDim.x * kT) {
    const int s = atom_sub[I], ci = atom_ci[I];
    const int m = core_ptr[s + 1] - core_ptr[s];
    const double* blk = k0 + k0_off[s];
    double acc = 0.0;
    for (int j = 0; j < m; ++j) {
      const int J = core_atoms[core_ptr[s] + j];
      acc += blk[ci + (size_t)m * j] * (z ? x[J] - z[J] : x[J]);
    }
    y[I] = acc;
  }
}

__global__ __launch_bounds__(kT) void k_sub(const double* __restrict__ x,
                                            const double* __restrict__ z, int n,
                                            double* __restrict__ y) {
  for (int i = blockIdx.x * kT + threadIdx.x; i < n; i += gridDim.x * kT) y[i] = x[i] - z[i];
}

// Sum over the workgroup of kRed threads, the same in every thread; each
// thread's part is summed by the caller in a fixed order, so the total is
// reproducible.
__device__ double block_sum(double x, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = x;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < kRed / 64; ++i) t += red[i];
  return t;
}

__device__ double dot(const double* x, const double* y, int n, double* red) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += kRed) acc += x[i] * y[i];
  return block_sum(acc, red);
}

// V[i] = w / |w| with w = src orthogonalised against V[0..i) by two passes of
// modified Gram-Schmidt (w kept in wbuf).  One workgroup.
__global__ __launch_bounds__(kRed) void k_kr_gs(const double* __restrict__ src, double* V,
                                                int i, int n, double* wbuf) {
  __shared__ double red[kRed / 64];
  for (int t = threadIdx.x; t < n; t += kRed) wbuf[t] = src[t];
  __syncthreads();
  for (int pass = 0; pass < (i > 0 ? 2 : 0); ++pass)
    for (int j = 0; j < i; ++j) {
      const double* vj = V + (size_t)j * n;
      const double d = dot(wbuf, vj, n, red);
      for (int t = threadIdx.x; t < n; t += kRed) wbuf[t] -= d * vj[t];
      __syncthreads();
    }
  const double nrm = sqrt(dot(wbuf, wbuf, n, red));
  double* vi = V + (size_t)i * n;
  for (int t = threadIdx.x; t < n; t += kRed) vi[t] = wbuf[t] / nrm;
}

// O_ij = F_i . F_j, c_j = F_j . kf, M = O^-1, coef = M c and the acceleration
// ndd = -omega^2 sum_i coef_i V_i.  One workgroup; m <= 32.
__global__ __launch_bounds__(kRed) void k_kr_final(const double* __restrict__ V,
                                                   const double* __restrict__ F,
                                                   const double* __restrict__ kf, int m, int n,
                                                   double omega, double* __restrict__ Oout,
                                                   double* __restrict__ Mout,
                                                   double* __restrict__ ndd,
                                                   int32_t* __restrict__ bad) {
  __shared__ double red[kRed / 64];
  __shared__ double A[32 * 33], X[32 * 33], cvec[32], coef[32];
  constexpr int ld = 33;
  for (int i = 0; i < m; ++i) {
    for (int j = 0; j <= i; ++j) {
      const double d = dot(F + (size_t)i * n, F + (size_t)j * n, n, red);
      if (threadIdx.x == 0) A[i * ld + j] = A[j * ld + i] = d;
    }
    const double c = dot(F + (size_t)i * n, kf, n, red);
    if (threadIdx.x == 0) cvec[i] = c;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < m * m; t += kRed) Oout[t] = A[(t / m) * ld + t % m];
  __syncthreads();
  const bool ok = gj_inverse(A, X, m, ld);
  if (!ok && threadIdx.x == 0) *bad = 1;
  for (int t = threadIdx.x; t < m * m; t += kRed) Mout[t] = ok ? X[(t / m) * ld + t % m] : 0.0;
  if (threadIdx.x < m) {
    double acc = 0.0;
    for (int j = 0; j < m; ++j) acc += X[threadIdx.x * ld + j] * cvec[j];
    coef[threadIdx.x] = ok ? acc : 0.0;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < n; t += kRed) {
    double acc = 0.0;
    for (int i = 0; i < m; ++i) acc += coef[i] * V[(size_t)i * n + t];
    ndd[t] = -omega * omega * acc;
  }
}

// clears a status flag with a kernel (capturable, unlike a memset node)
__global__ void k_zero_flag(int32_t* flag) { *flag = 0; }

inline unsigned blocks_for(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, (n + kT - 1) / kT));
}

// Device arrays of a charge model carved from one block (sizes only when base is NULL).
struct CCarve {
  char* base = nullptr;
  size_t used = 0;
  template <class T>
  T* take(int64_t count) {
    const size_t at = (used + 255) & ~size_t(255);
    used = at + (size_t)std::max<int64_t>(1, count) * sizeof(T);
    return base ? reinterpret_cast<T*>(base + at) : nullptr;
  }
};

void charge_layout(gq_charge* c, int64_t gnnz, CCarve& cv) {
  c->g_rp = cv.take<int32_t>(c->n_atoms + 1);
  c->g_col = cv.take<int32_t>(gnnz);
  c->g_val = cv.take<double>(gnnz);
  c->atom_of = cv.take<int32_t>(c->N);
  c->atom_sub = cv.take<int32_t>(c->n_atoms);
  c->atom_j0 = cv.take<int32_t>(c->n_atoms);
  c->atom_nk = cv.take<int32_t>(c->n_atoms);
  c->atom_ci = cv.take<int32_t>(c->n_atoms);
  c->core_ptr = cv.take<int32_t>(c->n_sub + 1);
  c->core_atoms = cv.take<int32_t>(c->n_atoms);
  c->k0_off = cv.take<int32_t>(c->n_sub + 1);
  c->pot = cv.take<double>((int64_t)c->kmax * c->n_atoms);
  c->a_all = cv.take<double>(c->k0_len);
  c->bvec = cv.take<double>(c->n_atoms);
  c->vec = cv.take<double>(4 * (int64_t)c->n_atoms);
  c->small = cv.take<double>(2 * 32 * 32 + 64);
}

// Charge response of K = nq perturbations whose potentials are pot[0..nq):
// per-atom charges into q_out ([nq][n_atoms]) with the canonical mu1.
void charge_response_launch(gq_ctx* ctx, gq_charge* c, gq_eigs* e, int nq, uint32_t precision,
                            double* q_out) {
  const gq_graph* g = c->g;
  const gq_graph_dev& dv = g->dev;
  hipStream_t st = ctx->stream;
  hipLaunchKernelGGL(k_h1_atoms, dim3(blocks_for(g->info.sum_n), nq), dim3(kT), 0, st, c->pot,
                     c->n_atoms, c->atom_of, dv.sub_orbs, g->info.sum_n, e->hloc);
  const RespBufs rb{e->hloc, e->Y, e->G, e->T, e->pdiag, e->mu1};
  RespOpts opt;
  opt.local_h1 = true;
  opt.charge_only = true;
  launch_response(ctx, g, e, rb, H1Spec{GQ_H1_DIAG, nullptr, nullptr}, nq, precision, nullptr,
                  opt);
  hipLaunchKernelGGL(k_atom_charges, dim3(blocks_for(c->n_atoms), nq), dim3(kT), 0, st, nullptr,
                     g->info.nnz, e->pdiag, g->offcd[g->n_sub], e->M, e->mu1, c->atom_sub,
                     c->atom_j0, c->atom_nk, dv.offc, dv.offcd, dv.sub_orb_ptr, c->n_atoms, q_out);
}

gq_status check_ready(gq_ctx* ctx, gq_charge* c, gq_eigs* e, const char* who) {
  if (!ctx || !c || !e) {
    set_error("%s: NULL argument", who);
    return GQ_EINVAL;
  }
  if (e->g != c->g) {
    set_error("%s: the workspace and the charge model belong to different graphs", who);
    return GQ_EINVAL;
  }
  if (!e->have_density) {
    set_error("%s: call gq_density on this workspace first", who);
    return GQ_EINVAL;
  }
  if (e->overlap_solved) {
    set_error("%s: charges are defined for an orthogonal basis only (the workspace was "
              "solved with an overlap)", who);
    return GQ_EINVAL;
  }
  return GQ_OK;
}

}  // namespace
}  // namespace gq

using namespace gq;

extern "C" {

gq_status gq_charge_create(gq_ctx* ctx, const gq_graph* g, const gq_csr* gamma, int32_t kmax,
                           gq_charge** out) {
  if (!ctx || !g || !gamma || !out || kmax < 1) {
    set_error("gq_charge_create: bad argument");
    return GQ_EINVAL;
  }
  const int32_t na = g->n_atoms;
  if (gamma->n_rows != na || !gamma->row_ptr || gamma->row_ptr[0] != 0 ||
      gamma->row_ptr[na] != gamma->nnz || (gamma->nnz > 0 && (!gamma->col || !gamma->val))) {
    set_error("gq_charge_create: gamma must be an n_atoms x n_atoms CSR (n_atoms = %d)", na);
    return GQ_EINVAL;
  }
  for (int32_t I = 0; I < na; ++I)
    for (int32_t p = gamma->row_ptr[I]; p < gamma->row_ptr[I + 1]; ++p)
      if (gamma->col[p] < 0 || gamma->col[p] >= na ||
          (p > gamma->row_ptr[I] && gamma->col[p] <= gamma->col[p - 1])) {
        set_error("gq_charge_create: gamma row %d has columns out of range or not ascending", I);
        return GQ_EINVAL;
      }
  gq_charge* c = new (std::nothrow) gq_charge;
  if (!c) {
    set_error("gq_charge_create: out of host memory");
    return GQ_ENOMEM;
  }
  c->ctx = ctx;
  c->g = g;
  c->n_atoms = na;
  c->N = g->N;
  c->n_sub = g->n_sub;
  c->kmax = kmax;
  // host maps: each atom's core subgraph, local orbital range and core index
  std::vector<int32_t> atom_of(g->N), atom_sub(na), atom_j0(na), atom_nk(na), atom_ci(na);
  std::vector<int32_t> core_ptr(g->n_sub + 1, 0), core_atoms, k0_off(g->n_sub + 1, 0);
  for (int32_t I = 0; I < na; ++I)
    for (int32_t a = g->atom_orb_ptr[I]; a < g->atom_orb_ptr[I + 1]; ++a) atom_of[a] = I;
  for (int32_t s = 0; s < g->n_sub; ++s) {
    const int32_t m = g->n_core_atoms[s];
    int32_t j = 0;
    for (int32_t k = 0; k < m; ++k) {
      const int32_t I = g->sub_atoms[g->sub_ptr[s] + k];
      atom_sub[I] = s;
      atom_j0[I] = j;
      atom_nk[I] = g->atom_orb_ptr[I + 1] - g->atom_orb_ptr[I];
      atom_ci[I] = k;
      j += atom_nk[I];
      core_atoms.push_back(I);
    }
    core_ptr[s + 1] = core_ptr[s] + m;
    k0_off[s + 1] = k0_off[s] + m * m;
    c->max_m = std::max(c->max_m, m);
  }
  c->k0_len = k0_off[g->n_sub];
  CCarve cv;
  charge_layout(c, gamma->nnz, cv);
  const size_t bytes = cv.used + 256;
  gq_status st = GQ_OK;
  if (hipSetDevice(ctx->device) != hipSuccess) st = GQ_EDEVICE;
  if (st == GQ_OK && ctx->arena) {
    std::lock_guard<std::mutex> lk(ctx->arena_mu);
    if (ctx->arena->alloc(bytes, &c->arena_off)) {
      c->block = ctx->arena_mem + c->arena_off;
      c->in_arena = true;
      c->arena_bytes = bytes;
    }
  } else if (st == GQ_OK && hipMalloc((void**)&c->block, bytes) != hipSuccess) {
    (void)hipGetLastError();
    c->block = nullptr;
  }
  if (st == GQ_OK && !c->block) {
    set_error("gq_charge_create: %zu device bytes not available", bytes);
    st = GQ_ENOMEM;
  }
  if (st) {
    if (st == GQ_EDEVICE) set_error("gq_charge_create: cannot select device %d", ctx->device);
    delete c;
    return st;
  }
  cv = CCarve{};
  cv.base = c->block;
  charge_layout(c, gamma->nnz, cv);
  hipStream_t s = ctx->stream;
  auto up = [&](void* dst, const void* src, size_t b) {
    if (b && hipMemcpyAsync(dst, src, b, hipMemcpyHostToDevice, s) != hipSuccess) st = GQ_EDEVICE;
  };
  up(c->g_rp, gamma->row_ptr, (na + 1) * 4);
  up(c->g_col, gamma->col, (size_t)gamma->nnz * 4);
  up(c->g_val, gamma->val, (size_t)gamma->nnz * 8);
  up(c->atom_of, atom_of.data(), atom_of.size() * 4);
  up(c->atom_sub, atom_sub.data(), na * 4);
  up(c->atom_j0, atom_j0.data(), na * 4);
  up(c->atom_nk, atom_nk.data(), na * 4);
  up(c->atom_ci, atom_ci.data(), na * 4);
  up(c->core_ptr, core_ptr.data(), core_ptr.size() * 4);
  up(c->core_atoms, core_atoms.data(), core_atoms.size() * 4);
  up(c->k0_off, k0_off.data(), k0_off.size() * 4);
  if (st == GQ_OK && hipStreamSynchronize(s) != hipSuccess) st = GQ_EDEVICE;
  if (st) {
    set_error("gq_charge_create: upload failed: %s", hipGetErrorString(hipGetLastError()));
    gq_charge_destroy(c);
    return st;
  }
  *out = c;
  return GQ_OK;
}

void gq_charge_destroy(gq_charge* c) {
  if (!c) return;
  (void)hipSetDevice(c->ctx->device);
  if (c->in_arena) {
    (void)hipStreamSynchronize(c->ctx->stream);
    std::lock_guard<std::mutex> lk(c->ctx->arena_mu);
    c->ctx->arena->release(c->arena_off, c->arena_bytes);
  } else if (c->block) {
    (void)hipFree(c->block);
  }
  delete c;
}

gq_status gq_charge_core(gq_ctx* ctx, gq_charge* c, const double* blocks_dev, double* q_dev) {
  if (!ctx || !c || !blocks_dev || !q_dev) {
    set_error("gq_charge_core: NULL argument");
    return GQ_EINVAL;
  }
  const gq_graph* g = c->g;
  GQ_HIP(hipSetDevice(ctx->device));
  prof_begin(ctx, "k_atom_charges");
  hipLaunchKernelGGL(k_atom_charges, dim3(blocks_for(c->n_atoms), 1), dim3(kT), 0, ctx->stream,
                     blocks_dev, g->info.nnz, nullptr, 0, nullptr, nullptr, c->atom_sub,
                     c->atom_j0, c->atom_nk, g->dev.offc, g->dev.offcd, g->dev.sub_orb_ptr,
                     c->n_atoms, q_dev);
  prof_end(ctx);
  GQ_HIP(hipGetLastError());
  return GQ_OK;
}

gq_status gq_charge_response(gq_ctx* ctx, gq_charge* c, gq_eigs* e, const double* v_dev,
                             int32_t K, uint32_t precision, double* q1_dev, double* mu1_dev) {
  if (gq_status st = check_ready(ctx, c, e, "gq_charge_response")) return st;
  if (!v_dev || !q1_dev || K < 1 || K > e->max_k || K > c->kmax) {
    set_error("gq_charge_response: NULL vectors or K = %d outside [1, min(max_k %d, kmax %d)]",
              K, e->max_k, c->kmax);
    return GQ_EINVAL;
  }
  if (precision != GQ_PREC_FP64 && precision != GQ_PREC_SPLIT32) {
    set_error("gq_charge_response: precision %u not available", precision);
    return GQ_EINVAL;
  }
  GQ_HIP(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  prof_begin(ctx, "k_spmv");
  hipLaunchKernelGGL(k_spmv, dim3(blocks_for(c->n_atoms), K), dim3(kT), 0, st, c->g_rp,
                     c->g_col, c->g_val, v_dev, c->n_atoms, c->pot);
  prof_end(ctx);
  charge_response_launch(ctx, c, e, K, precision, q1_dev);
  if (mu1_dev)
    GQ_HIP(hipMemcpyAsync(mu1_dev, e->mu1, K * sizeof(double), hipMemcpyDeviceToDevice, st));
  GQ_HIP(hipGetLastError());
  return GQ_OK;
}

gq_status gq_preconditioner(gq_ctx* ctx, gq_charge* c, gq_eigs* e, double alpha, double* k0_dev,
                            int32_t* singular_dev) {
  if (gq_status st = check_ready(ctx, c, e, "gq_preconditioner")) return st;
  if (!k0_dev || !singular_dev || !(alpha >= 0.0)) {
    set_error("gq_preconditioner: NULL output or alpha < 0");
    return GQ_EINVAL;
  }
  if (c->max_m > 32) {
    set_error("gq_preconditioner: a core of %d atoms exceeds 32", c->max_m);
    return GQ_EINVAL;
  }
  GQ_HIP(hipSetDevice(ctx->device));
  const gq_graph* g = c->g;
  const gq_graph_dev& dv = g->dev;
  hipStream_t st = ctx->stream;
  const int kc = std::max(1, std::min(e->max_k, c->max_m));
  const RespBufs rb{e->hloc, e->Y, e->G, e->T, e->pdiag, e->mu1};
  RespOpts opt;
  opt.local_h1 = true;
  opt.charge_only = true;
  hipLaunchKernelGGL(k_zero_flag, dim3(1), dim3(1), 0, st, singular_dev);
  for (int q0 = 0; q0 < c->max_m; q0 += kc) {
    const int nq = std::min(kc, c->max_m - q0);
    prof_begin(ctx, "k_h1_unit");
    hipLaunchKernelGGL(k_h1_unit, dim3(g->n_sub, nq), dim3(kT), 0, st, c->g_rp, c->g_col,
                       c->g_val, c->atom_of, dv.sub_orb_ptr, dv.sub_orbs, c->core_ptr,
                       c->core_atoms, q0, g->info.sum_n, e->hloc);
    prof_end(ctx);
    launch_response(ctx, g, e, rb, H1Spec{GQ_H1_DIAG, nullptr, nullptr}, nq, GQ_PREC_FP64,
                    nullptr, opt);
    prof_begin(ctx, "k_k0");
    hipLaunchKernelGGL(k_unit_collect, dim3(blocks_for(c->n_atoms)), dim3(kT), 0, st, e->pdiag,
                       g->offcd[g->n_sub], e->M, nq, q0, c->atom_sub, c->atom_j0, c->atom_nk,
                       c->atom_ci, c->core_ptr, c->k0_off, dv.offc, dv.offcd, dv.sub_orb_ptr,
                       c->n_atoms, c->a_all, c->bvec);
    prof_end(ctx);
  }
  prof_begin(ctx, "k_k0");
  hipLaunchKernelGGL(k_k0, dim3(g->n_sub), dim3(64), 0, st, c->a_all, c->bvec, c->core_ptr,
                     c->core_atoms, c->k0_off, alpha, k0_dev, singular_dev);
  prof_end(ctx);
  GQ_HIP(hipGetLastError());
  return GQ_OK;
}

gq_status gq_krylov_kernel(gq_ctx* ctx, gq_charge* c, gq_eigs* e, const double* k0_dev,
                           const double* rho_blocks_dev, const double* n_dev, int32_t m,
                           double omega, uint32_t precision, double* ndd_dev, double* V_dev,
                           double* F_dev, double* O_dev, double* M_dev, int32_t* singular_dev) {
  if (gq_status st = check_ready(ctx, c, e, "gq_krylov_kernel")) return st;
  if (!k0_dev || !rho_blocks_dev || !n_dev || !ndd_dev || !V_dev || !F_dev || !O_dev ||
      !M_dev || !singular_dev) {
    set_error("gq_krylov_kernel: NULL argument");
    return GQ_EINVAL;
  }
  if (m < 1 || m > kMaxKrylov) {
    set_error("gq_krylov_kernel: rank m = %d outside [1, %d]", m, kMaxKrylov);
    return GQ_EINVAL;
  }
  if (precision != GQ_PREC_FP64 && precision != GQ_PREC_SPLIT32) {
    set_error("gq_krylov_kernel: precision %u not available", precision);
    return GQ_EINVAL;
  }
  GQ_HIP(hipSetDevice(ctx->device));
  const gq_graph* g = c->g;
  hipStream_t st = ctx->stream;
  const int na = c->n_atoms;
  double* q0 = c->vec;            // rho_0 per atom
  double* res = c->vec + na;      // f = rho_0 - n
  double* kf = c->vec + 2 * na;   // K0 f
  double* wbuf = c->vec + 3 * na; // Gram-Schmidt work vector, then each response's charges
  hipLaunchKernelGGL(k_zero_flag, dim3(1), dim3(1), 0, st, singular_dev);
  prof_begin(ctx, "k_krylov");
  hipLaunchKernelGGL(k_atom_charges, dim3(blocks_for(na), 1), dim3(kT), 0, st, rho_blocks_dev,
                     g->info.nnz, nullptr, 0, nullptr, nullptr, c->atom_sub, c->atom_j0,
                     c->atom_nk, g->dev.offc, g->dev.offcd, g->dev.sub_orb_ptr, na, q0);
  hipLaunchKernelGGL(k_sub, dim3(blocks_for(na)), dim3(kT), 0, st, q0, n_dev, na, res);
  hipLaunchKernelGGL(k_k0_apply, dim3(blocks_for(na)), dim3(kT), 0, st, k0_dev, res, nullptr,
                     c->atom_sub, c->atom_ci, c->core_ptr, c->core_atoms, c->k0_off, na, kf);
  hipLaunchKernelGGL(k_kr_gs, dim3(1), dim3(kRed), 0, st, kf, V_dev, 0, na, wbuf);
  prof_end(ctx);
  for (int i = 0; i < m; ++i) {
    double* vi = V_dev + (size_t)i * na;
    double* fi = F_dev + (size_t)i * na;
    prof_begin(ctx, "k_spmv");
    hipLaunchKernelGGL(k_spmv, dim3(blocks_for(na), 1), dim3(kT), 0, st, c->g_rp, c->g_col,
                       c->g_val, vi, na, c->pot);
    prof_end(ctx);
    // the response's charges land in wbuf, then f_{v_i} = K0 (wbuf - v_i)
    charge_response_launch(ctx, c, e, 1, precision, wbuf);
    prof_begin(ctx, "k_krylov");
    hipLaunchKernelGGL(k_k0_apply, dim3(blocks_for(na)), dim3(kT), 0, st, k0_dev, wbuf, vi,
                       c->atom_sub, c->atom_ci, c->core_ptr, c->core_atoms, c->k0_off, na, fi);
    if (i + 1 < m)
      hipLaunchKernelGGL(k_kr_gs, dim3(1), dim3(kRed), 0, st, fi, V_dev, i + 1, na, wbuf);
    prof_end(ctx);
  }
  prof_begin(ctx, "k_krylov");
  hipLaunchKernelGGL(k_kr_final, dim3(1), dim3(kRed), 0, st, V_dev, F_dev, kf, m, na, omega,
                     O_dev, M_dev, ndd_dev, singular_dev);
  prof_end(ctx);
  GQ_HIP(hipGetLastError());
  return GQ_OK;
}

}  // extern "C"
