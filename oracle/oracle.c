/*
 * Reference oracle for graph-based density and canonical response.
 *
 * TEST INFRASTRUCTURE ONLY: plain, slow, single-threaded FP64 code written
 * from the paper (arXiv:2212.01997) to check the GPU library.  No blocking,
 * fusion or reordering beyond what the definitions state; sums that feed the
 * chemical potentials run in a fixed order with compensated accumulation.
 * See oracle.h for the passages each function follows.
 */
#include "oracle.h"

#include <float.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static char g_err[512];

const char* orc_last_error(void) { return g_err; }

static int fail(int code, const char* msg) {
  snprintf(g_err, sizeof g_err, "%s", msg);
  return code;
}

/* ---------------------------------------------------------------- helpers */

/* Neumaier compensated sum, fixed order */
typedef struct { double s, c; } ksum;
static void ks_add(ksum* k, double x) {
  double t = k->s + x;
  if (fabs(k->s) >= fabs(x)) k->c += (k->s - t) + x;
  else k->c += (x - t) + k->s;
  k->s = t;
}
static double ks_val(const ksum* k) { return k->s + k->c; }

static int cmp_i64(const void* a, const void* b) {
  int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  return (x > y) - (x < y);
}
static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

static int csr_check(const orc_csr* X, int32_t n, const char* name) {
  if (!X || X->n_rows != n || !X->row_ptr || (X->nnz > 0 && (!X->col || !X->val))) {
    snprintf(g_err, sizeof g_err, "%s: bad CSR header", name);
    return ORC_EINVAL;
  }
  if (X->row_ptr[0] != 0 || X->row_ptr[n] != X->nnz) {
    snprintf(g_err, sizeof g_err, "%s: row_ptr does not span nnz", name);
    return ORC_EINVAL;
  }
  for (int32_t a = 0; a < n; ++a) {
    if (X->row_ptr[a + 1] < X->row_ptr[a]) {
      snprintf(g_err, sizeof g_err, "%s: row_ptr not monotone", name);
      return ORC_EINVAL;
    }
    for (int32_t p = X->row_ptr[a]; p < X->row_ptr[a + 1]; ++p) {
      if (X->col[p] < 0 || X->col[p] >= n || (p > X->row_ptr[a] && X->col[p] <= X->col[p - 1])) {
        snprintf(g_err, sizeof g_err, "%s: columns out of range or not ascending", name);
        return ORC_EINVAL;
      }
    }
  }
  return ORC_OK;
}

static int csr_has(const orc_csr* X, int32_t a, int32_t b) {
  int32_t lo = X->row_ptr[a], hi = X->row_ptr[a + 1];
  while (lo < hi) {
    int32_t mid = lo + (hi - lo) / 2;
    if (X->col[mid] < b) lo = mid + 1;
    else hi = mid;
  }
  return lo < X->row_ptr[a + 1] && X->col[lo] == b;
}

/* ------------------------------------------------------------- graph build
 * Sec. II.E: the graph is the nonzero structure of the thresholded density
 * matrix of a previous step, together with the elements of the thresholded
 * Hamiltonian; optionally extended by paths of length two.  Vertices are atoms
 * (all orbitals of an atom stay together).  Sec. II.C / Fig. 1: a subgraph is a
 * core plus the vertices directly connected to it (the halo).  Eq. (sub_f):
 * the collected result keeps the core rows of every subgraph function.
 */
int orc_graph_build(int32_t n_atoms, const int32_t* atom_orb_ptr, const orc_csr* H,
                    const orc_csr* rho_prev, const int32_t* core_of_atom, double tau,
                    int32_t flags, orc_graph* out) {
  memset(out, 0, sizeof *out);
  if (n_atoms <= 0 || !atom_orb_ptr || !core_of_atom) return fail(ORC_EINVAL, "empty system");
  if (!(tau >= 0.0)) return fail(ORC_EINVAL, "tau must be >= 0");
  if (atom_orb_ptr[0] != 0) return fail(ORC_EINVAL, "atom_orb_ptr[0] != 0");
  for (int32_t I = 0; I < n_atoms; ++I)
    if (atom_orb_ptr[I + 1] <= atom_orb_ptr[I])
      return fail(ORC_EINVAL, "atom_orb_ptr not strictly increasing");
  const int32_t N = atom_orb_ptr[n_atoms];
  int rc = csr_check(H, N, "H");
  if (rc) return rc;
  if (rho_prev) {
    rc = csr_check(rho_prev, N, "rho_prev");
    if (rc) return rc;
  }
  for (int32_t a = 0; a < N; ++a)
    for (int32_t p = H->row_ptr[a]; p < H->row_ptr[a + 1]; ++p)
      if (!csr_has(H, H->col[p], a)) return fail(ORC_EINVAL, "H pattern is not symmetric");

  int32_t n_sub = 0;
  for (int32_t I = 0; I < n_atoms; ++I) {
    if (core_of_atom[I] < 0) return fail(ORC_EINVAL, "negative core id");
    if (core_of_atom[I] + 1 > n_sub) n_sub = core_of_atom[I] + 1;
  }
  int32_t* core_cnt = calloc((size_t)n_sub, sizeof(int32_t));
  for (int32_t I = 0; I < n_atoms; ++I) core_cnt[core_of_atom[I]]++;
  for (int32_t s = 0; s < n_sub; ++s)
    if (core_cnt[s] == 0) { free(core_cnt); return fail(ORC_EINVAL, "core ids are not dense (empty core)"); }

  int32_t* atom_of = malloc(sizeof(int32_t) * (size_t)N);
  for (int32_t I = 0; I < n_atoms; ++I)
    for (int32_t a = atom_orb_ptr[I]; a < atom_orb_ptr[I + 1]; ++a) atom_of[a] = I;

  /* edges as 64-bit keys I*n_atoms+J, both orientations */
  int64_t cap = 1024, ne = 0;
  int64_t* keys = malloc(sizeof(int64_t) * (size_t)cap);
  const orc_csr* mats[2] = {H, rho_prev};
  for (int mi = 0; mi < 2; ++mi) {
    const orc_csr* X = mats[mi];
    if (!X) continue;
    for (int32_t a = 0; a < N; ++a) {
      for (int32_t p = X->row_ptr[a]; p < X->row_ptr[a + 1]; ++p) {
        int32_t I = atom_of[a], J = atom_of[X->col[p]];
        if (I == J || !(fabs(X->val[p]) >= tau)) continue;
        if (ne + 2 > cap) { cap *= 2; keys = realloc(keys, sizeof(int64_t) * (size_t)cap); }
        keys[ne++] = (int64_t)I * n_atoms + J;
        keys[ne++] = (int64_t)J * n_atoms + I;
      }
    }
  }
  qsort(keys, (size_t)ne, sizeof(int64_t), cmp_i64);
  int64_t nu = 0;
  for (int64_t q = 0; q < ne; ++q)
    if (q == 0 || keys[q] != keys[q - 1]) keys[nu++] = keys[q];
  int32_t* adj_ptr = calloc((size_t)n_atoms + 1, sizeof(int32_t));
  int32_t* adj = malloc(sizeof(int32_t) * (size_t)(nu > 0 ? nu : 1));
  for (int64_t q = 0; q < nu; ++q) {
    adj_ptr[keys[q] / n_atoms + 1]++;
    adj[q] = (int32_t)(keys[q] % n_atoms);
  }
  for (int32_t I = 0; I < n_atoms; ++I) adj_ptr[I + 1] += adj_ptr[I];
  free(keys);

  int32_t* mark = malloc(sizeof(int32_t) * (size_t)n_atoms);
  for (int32_t I = 0; I < n_atoms; ++I) mark[I] = -1;

  if (flags & ORC_PATHS2) {
    /* neighbours of neighbours: A u A^2 without self loops */
    int64_t cap2 = 1024, n2 = 0;
    int32_t* adj2 = malloc(sizeof(int32_t) * (size_t)cap2);
    int32_t* ptr2 = calloc((size_t)n_atoms + 1, sizeof(int32_t));
    int32_t* tmp = malloc(sizeof(int32_t) * (size_t)n_atoms);
    for (int32_t I = 0; I < n_atoms; ++I) {
      int32_t cnt = 0;
      mark[I] = I;
      for (int32_t p = adj_ptr[I]; p < adj_ptr[I + 1]; ++p) {
        int32_t J = adj[p];
        if (mark[J] != I) { mark[J] = I; tmp[cnt++] = J; }
        for (int32_t q = adj_ptr[J]; q < adj_ptr[J + 1]; ++q) {
          int32_t L = adj[q];
          if (mark[L] != I) { mark[L] = I; tmp[cnt++] = L; }
        }
      }
      qsort(tmp, (size_t)cnt, sizeof(int32_t), cmp_i32);
      while (n2 + cnt > cap2) { cap2 *= 2; adj2 = realloc(adj2, sizeof(int32_t) * (size_t)cap2); }
      memcpy(adj2 + n2, tmp, sizeof(int32_t) * (size_t)cnt);
      n2 += cnt;
      ptr2[I + 1] = (int32_t)n2;
    }
    free(tmp);
    free(adj);
    free(adj_ptr);
    adj = adj2;
    adj_ptr = ptr2;
    for (int32_t I = 0; I < n_atoms; ++I) mark[I] = -1;
  }

  /* cores: atoms ascending within each core */
  int32_t* core_ptr = calloc((size_t)n_sub + 1, sizeof(int32_t));
  for (int32_t s = 0; s < n_sub; ++s) core_ptr[s + 1] = core_ptr[s] + core_cnt[s];
  int32_t* core_atoms = malloc(sizeof(int32_t) * (size_t)n_atoms);
  int32_t* fill = calloc((size_t)n_sub, sizeof(int32_t));
  for (int32_t I = 0; I < n_atoms; ++I) {
    int32_t s = core_of_atom[I];
    core_atoms[core_ptr[s] + fill[s]++] = I;
  }
  free(fill);
  free(core_cnt);

  /* subgraph vertex lists: core ascending ++ halo ascending */
  int64_t cap_sa = n_atoms, n_sa = 0;
  int32_t* sub_atoms = malloc(sizeof(int32_t) * (size_t)cap_sa);
  int32_t* sub_ptr = calloc((size_t)n_sub + 1, sizeof(int32_t));
  int32_t* n_core_atoms = malloc(sizeof(int32_t) * (size_t)n_sub);
  int32_t* halo = malloc(sizeof(int32_t) * (size_t)n_atoms);
  for (int32_t s = 0; s < n_sub; ++s) {
    int32_t nc = core_ptr[s + 1] - core_ptr[s];
    for (int32_t q = core_ptr[s]; q < core_ptr[s + 1]; ++q) mark[core_atoms[q]] = s;
    int32_t nh = 0;
    if (flags & ORC_COMPLETE) {
      for (int32_t I = 0; I < n_atoms; ++I)
        if (mark[I] != s) halo[nh++] = I;
    } else {
      for (int32_t q = core_ptr[s]; q < core_ptr[s + 1]; ++q) {
        int32_t I = core_atoms[q];
        for (int32_t p = adj_ptr[I]; p < adj_ptr[I + 1]; ++p) {
          int32_t J = adj[p];
          if (mark[J] != s) { mark[J] = s; halo[nh++] = J; }
        }
      }
      qsort(halo, (size_t)nh, sizeof(int32_t), cmp_i32);
    }
    while (n_sa + nc + nh > cap_sa) { cap_sa *= 2; sub_atoms = realloc(sub_atoms, sizeof(int32_t) * (size_t)cap_sa); }
    memcpy(sub_atoms + n_sa, core_atoms + core_ptr[s], sizeof(int32_t) * (size_t)nc);
    memcpy(sub_atoms + n_sa + nc, halo, sizeof(int32_t) * (size_t)nh);
    n_sa += nc + nh;
    sub_ptr[s + 1] = (int32_t)n_sa;
    n_core_atoms[s] = nc;
  }
  free(halo);
  free(mark);
  free(adj);
  free(adj_ptr);
  free(core_atoms);
  free(core_ptr);

  /* orbital lists */
  int32_t* sub_orb_ptr = calloc((size_t)n_sub + 1, sizeof(int32_t));
  int32_t* n_core_orbs = malloc(sizeof(int32_t) * (size_t)n_sub);
  int64_t tot = 0;
  for (int32_t s = 0; s < n_sub; ++s) {
    int32_t nc = 0, nn = 0;
    for (int32_t q = sub_ptr[s]; q < sub_ptr[s + 1]; ++q) {
      int32_t I = sub_atoms[q];
      int32_t k = atom_orb_ptr[I + 1] - atom_orb_ptr[I];
      nn += k;
      if (q - sub_ptr[s] < n_core_atoms[s]) nc += k;
    }
    n_core_orbs[s] = nc;
    tot += nn;
    if (tot > INT32_MAX) { free(sub_orb_ptr); free(n_core_orbs); free(sub_atoms); free(sub_ptr); free(n_core_atoms); free(atom_of);
      return fail(ORC_ENOMEM, "orbital list exceeds int32"); }
    sub_orb_ptr[s + 1] = (int32_t)tot;
  }
  int32_t* sub_orbs = malloc(sizeof(int32_t) * (size_t)(tot > 0 ? tot : 1));
  for (int32_t s = 0; s < n_sub; ++s) {
    int32_t o = sub_orb_ptr[s];
    for (int32_t q = sub_ptr[s]; q < sub_ptr[s + 1]; ++q) {
      int32_t I = sub_atoms[q];
      for (int32_t a = atom_orb_ptr[I]; a < atom_orb_ptr[I + 1]; ++a) sub_orbs[o++] = a;
    }
  }

  /* collected pattern: row a holds the sorted orbitals of its owner subgraph */
  int32_t* rho_row_ptr = calloc((size_t)N + 1, sizeof(int32_t));
  int64_t nnz = 0;
  for (int32_t a = 0; a < N; ++a) {
    int32_t s = core_of_atom[atom_of[a]];
    nnz += sub_orb_ptr[s + 1] - sub_orb_ptr[s];
    if (nnz > INT32_MAX) { free(rho_row_ptr); free(sub_orbs); free(sub_orb_ptr); free(n_core_orbs); free(sub_atoms); free(sub_ptr); free(n_core_atoms); free(atom_of);
      return fail(ORC_ENOMEM, "collected pattern exceeds int32"); }
    rho_row_ptr[a + 1] = (int32_t)nnz;
  }
  int32_t* rho_col = malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  int32_t* sorted = malloc(sizeof(int32_t) * (size_t)N);
  for (int32_t s = 0; s < n_sub; ++s) {
    int32_t n = sub_orb_ptr[s + 1] - sub_orb_ptr[s];
    memcpy(sorted, sub_orbs + sub_orb_ptr[s], sizeof(int32_t) * (size_t)n);
    qsort(sorted, (size_t)n, sizeof(int32_t), cmp_i32);
    for (int32_t j = 0; j < n_core_orbs[s]; ++j) {
      int32_t a = sub_orbs[sub_orb_ptr[s] + j];
      memcpy(rho_col + rho_row_ptr[a], sorted, sizeof(int32_t) * (size_t)n);
    }
  }
  free(sorted);
  free(atom_of);

  out->n_atoms = n_atoms;
  out->n_orb = N;
  out->n_sub = n_sub;
  out->sub_ptr = sub_ptr;
  out->sub_atoms = sub_atoms;
  out->n_core_atoms = n_core_atoms;
  out->sub_orb_ptr = sub_orb_ptr;
  out->sub_orbs = sub_orbs;
  out->n_core_orbs = n_core_orbs;
  out->rho_row_ptr = rho_row_ptr;
  out->rho_col = rho_col;
  out->nnz = nnz;
  return ORC_OK;
}

void orc_graph_free(orc_graph* g) {
  if (!g) return;
  free(g->sub_ptr);
  free(g->sub_atoms);
  free(g->n_core_atoms);
  free(g->sub_orb_ptr);
  free(g->sub_orbs);
  free(g->n_core_orbs);
  free(g->rho_row_ptr);
  free(g->rho_col);
  memset(g, 0, sizeof *g);
}

/* ------------------------------------------------------------------ gather
 * Fig. 1: the principal submatrix is the restriction of X to the rows and
 * columns of the subgraph's vertices, in the subgraph's own order. */
int orc_gather(const orc_csr* X, int32_t n, const int32_t* orbs, double* h) {
  memset(h, 0, sizeof(double) * (size_t)n * (size_t)n);
  for (int32_t r = 0; r < n; ++r) {
    int32_t a = orbs[r];
    for (int32_t c = 0; c < n; ++c) {
      int32_t b = orbs[c];
      int32_t lo = X->row_ptr[a], hi = X->row_ptr[a + 1];
      while (lo < hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (X->col[mid] < b) lo = mid + 1;
        else hi = mid;
      }
      if (lo < X->row_ptr[a + 1] && X->col[lo] == b) h[r + (size_t)n * c] = X->val[lo];
    }
  }
  return ORC_OK;
}

/* --------------------------------------------------------------- eigensolve
 * Eq. (SmallKS): eigenpairs of each subgraph Hamiltonian.  Textbook route
 * (Golub & Van Loan, symmetric QR algorithm): Householder reduction to
 * tridiagonal form T = Q^T A Q, then implicit QL iterations with a Wilkinson
 * shift on T, accumulating the plane rotations into Q. */

/* Householder tridiagonalisation of the full symmetric matrix A (overwritten).
 * Reflector k is H_k = I - tau_k v v^T acting on indices k+1..n-1, v[0] = 1,
 * v[1..] stored in A[k+2.., k]. */
static void householder_tridiagonal(int32_t n, double* A, double* d, double* e, double* tau,
                                    double* v, double* p) {
  for (int32_t k = 0; k + 2 < n; ++k) {
    const int32_t m = n - k - 1;
    double* x = A + (k + 1) + (size_t)n * k;
    double alpha = x[0];
    double sigma = 0.0;
    for (int32_t i = 1; i < m; ++i) sigma += x[i] * x[i];
    d[k] = A[k + (size_t)n * k];
    if (sigma == 0.0) {
      tau[k] = 0.0;
      e[k] = alpha;
      continue;
    }
    double norm = sqrt(alpha * alpha + sigma);
    double beta = alpha >= 0.0 ? -norm : norm;
    double t = (beta - alpha) / beta;
    double scale = 1.0 / (alpha - beta);
    v[0] = 1.0;
    for (int32_t i = 1; i < m; ++i) v[i] = x[i] * scale;
    tau[k] = t;
    e[k] = beta;
    /* A22 <- H A22 H with p = t A22 v, w = p - (t/2)(p.v) v */
    double* A22 = A + (k + 1) + (size_t)n * (k + 1);
    for (int32_t i = 0; i < m; ++i) {
      double s = 0.0;
      for (int32_t j = 0; j < m; ++j) s += A22[i + (size_t)n * j] * v[j];
      p[i] = t * s;
    }
    double pv = 0.0;
    for (int32_t i = 0; i < m; ++i) pv += p[i] * v[i];
    double K = 0.5 * t * pv;
    for (int32_t i = 0; i < m; ++i) p[i] -= K * v[i];
    for (int32_t j = 0; j < m; ++j)
      for (int32_t i = 0; i < m; ++i)
        A22[i + (size_t)n * j] -= v[i] * p[j] + p[i] * v[j];
    for (int32_t i = 1; i < m; ++i) x[i] = v[i];
  }
  if (n >= 2) {
    d[n - 2] = A[(n - 2) + (size_t)n * (n - 2)];
    e[n - 2] = A[(n - 1) + (size_t)n * (n - 2)];
  }
  d[n - 1] = A[(n - 1) + (size_t)n * (n - 1)];
}

/* Q = H_0 H_1 ... H_{n-3}, accumulated from the last reflector backwards */
static void form_q(int32_t n, const double* A, const double* tau, double* Q) {
  memset(Q, 0, sizeof(double) * (size_t)n * (size_t)n);
  for (int32_t i = 0; i < n; ++i) Q[i + (size_t)n * i] = 1.0;
  for (int32_t k = n - 3; k >= 0; --k) {
    if (tau[k] == 0.0) continue;
    const int32_t m = n - k - 1;
    const double* vt = A + (k + 1) + (size_t)n * k; /* vt[0] is not v[0]; v[0] = 1 */
    for (int32_t j = k + 1; j < n; ++j) {
      double* q = Q + (k + 1) + (size_t)n * j;
      double s = q[0];
      for (int32_t i = 1; i < m; ++i) s += vt[i] * q[i];
      s *= tau[k];
      q[0] -= s;
      for (int32_t i = 1; i < m; ++i) q[i] -= s * vt[i];
    }
  }
}

/* implicit QL with Wilkinson shift on the symmetric tridiagonal (d, e);
 * e[i] couples d[i] and d[i+1]; rotations are applied to the columns of Z */
static int tridiagonal_ql(int32_t n, double* d, double* e, double* Z) {
  if (n > 0) e[n - 1] = 0.0;
  for (int32_t l = 0; l < n; ++l) {
    int32_t iter = 0;
    for (;;) {
      int32_t m = l;
      while (m < n - 1) {
        double dd = fabs(d[m]) + fabs(d[m + 1]);
        if (fabs(e[m]) <= DBL_EPSILON * dd) break;
        ++m;
      }
      if (m == l) break;
      if (++iter > 30 * (n > 8 ? n : 8)) return fail(ORC_ENOCONV, "QL iteration did not converge");
      /* shift: eigenvalue of the leading 2x2 block of the active part closer to d[l] */
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + copysign(r, g));
      double s = 1.0, c = 1.0, p = 0.0;
      int32_t i;
      int deflated_early = 0;
      for (i = m - 1; i >= l; --i) {
        double f = s * e[i];
        double b = c * e[i];
        r = hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= p;
          e[m] = 0.0;
          deflated_early = 1;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0 * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
        double* zi = Z + (size_t)n * i;
        double* zj = Z + (size_t)n * (i + 1);
        for (int32_t k = 0; k < n; ++k) {
          double t = zj[k];
          zj[k] = s * zi[k] + c * t;
          zi[k] = c * zi[k] - s * t;
        }
      }
      if (deflated_early) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  return ORC_OK;
}

int orc_eigh(int32_t n, const double* a, double* w, double* z) {
  if (n <= 0) return fail(ORC_EINVAL, "n must be positive");
  size_t nn = (size_t)n * (size_t)n;
  double* A = malloc(sizeof(double) * nn);
  double* e = malloc(sizeof(double) * (size_t)n);
  double* tau = malloc(sizeof(double) * (size_t)n);
  double* v = malloc(sizeof(double) * (size_t)n);
  double* p = malloc(sizeof(double) * (size_t)n);
  memcpy(A, a, sizeof(double) * nn);
  householder_tridiagonal(n, A, w, e, tau, v, p);
  form_q(n, A, tau, z);
  int rc = tridiagonal_ql(n, w, e, z);
  /* ascending order: selection sort with column swaps */
  for (int32_t i = 0; i < n - 1 && rc == ORC_OK; ++i) {
    int32_t k = i;
    for (int32_t j = i + 1; j < n; ++j)
      if (w[j] < w[k]) k = j;
    if (k != i) {
      double t = w[i];
      w[i] = w[k];
      w[k] = t;
      for (int32_t r = 0; r < n; ++r) {
        double q = z[r + (size_t)n * i];
        z[r + (size_t)n * i] = z[r + (size_t)n * k];
        z[r + (size_t)n * k] = q;
      }
    }
  }
  free(A);
  free(e);
  free(tau);
  free(v);
  free(p);
  return rc;
}

void orc_core_weights(int32_t n, int32_t c, const double* z, double* wts) {
  /* Sec. II.G: only the squares of the core elements of each eigenvector */
  for (int32_t k = 0; k < n; ++k) {
    double s = 0.0;
    for (int32_t j = 0; j < c; ++j) s += z[j + (size_t)n * k] * z[j + (size_t)n * k];
    wts[k] = s;
  }
}

/* ------------------------------------------------------- Fermi occupation */
double orc_fermi(double e, double mu, double kT) {
  double x = (e - mu) / kT;
  if (x > 0.0) {
    double t = exp(-x);
    return t / (1.0 + t);
  }
  return 1.0 / (1.0 + exp(x));
}

/* f (1 - f) without cancellation: t/(1+t)^2 with t = exp(-|x|) */
static double fermi_f1mf(double e, double mu, double kT) {
  double t = exp(-fabs((e - mu) / kT));
  return t / ((1.0 + t) * (1.0 + t));
}

/* Sec. II.G: Tr D(mu) collected over subgraphs is sum_{i,k} f_k^(i) w_k^(i);
 * the spin factor 2 makes its target N_e */
void orc_occupation(int64_t count, const double* e, const double* wts, double mu,
                    double kT, double n_elec, double* F, double* dF) {
  ksum s = {0, 0}, ds = {0, 0};
  for (int64_t q = 0; q < count; ++q) {
    ks_add(&s, wts[q] * orc_fermi(e[q], mu, kT));
    ks_add(&ds, wts[q] * fermi_f1mf(e[q], mu, kT));
  }
  if (F) *F = 2.0 * ks_val(&s) - n_elec;
  if (dF) *dF = 2.0 / kT * ks_val(&ds);
}

/* F(mu) is non-decreasing in mu, so the root is unique; bisection to the
 * last representable interval (the paper's Newton-Raphson reaches the same root) */
int orc_find_mu(int64_t count, const double* e, const double* wts, double kT,
                double n_elec, double* mu) {
  if (!(kT > 0.0)) return fail(ORC_EINVAL, "kT must be > 0");
  if (count <= 0) return fail(ORC_EINVAL, "no eigenvalues");
  double emin = e[0], emax = e[0], wsum = 0.0;
  for (int64_t q = 0; q < count; ++q) {
    if (e[q] < emin) emin = e[q];
    if (e[q] > emax) emax = e[q];
    wsum += wts[q];
  }
  if (!(n_elec > 0.0) || !(n_elec < 2.0 * wsum)) return fail(ORC_EINVAL, "N_e outside (0, 2N)");
  double lo = emin - 50.0 * kT, hi = emax + 50.0 * kT;
  double Flo, Fhi;
  orc_occupation(count, e, wts, lo, kT, n_elec, &Flo, NULL);
  orc_occupation(count, e, wts, hi, kT, n_elec, &Fhi, NULL);
  if (!(Flo < 0.0 && Fhi > 0.0)) return fail(ORC_ENOCONV, "chemical potential not bracketed");
  for (int it = 0; it < 400; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    double Fm;
    orc_occupation(count, e, wts, mid, kT, n_elec, &Fm, NULL);
    if (Fm == 0.0) { lo = hi = mid; break; }
    if (Fm < 0.0) lo = mid;
    else hi = mid;
  }
  *mu = 0.5 * (lo + hi);
  return ORC_OK;
}

/* ------------------------------------------------------ divided differences
 * The Frechet derivative of f(h) in the eigenbasis weights element (k,l) by
 * (f_k - f_l)/(e_k - e_l), and by f'(e_k) when e_k = e_l.  With
 * u = beta (e - mu) the Fermi function gives exactly
 *   (f_k - f_l)/(e_k - e_l) = -(beta/4) sinhc(x) / (cosh(u_k/2) cosh(u_l/2)),
 *   x = beta (e_k - e_l) / 2,  sinhc(x) = sinh(x)/x,  sinhc(0) = 1,
 * which is evaluated in log space (no overflow, no cancellation). */
static double log_cosh(double y) {
  double a = fabs(y);
  return a + log1p(exp(-2.0 * a)) - log(2.0);
}

static double log_sinhc(double x) {
  double a = fabs(x);
  if (a == 0.0) return 0.0;
  if (a < 20.0) return log(sinh(a) / a);
  return a + log1p(-exp(-2.0 * a)) - log(2.0) - log(a);
}

void orc_divided_differences(int32_t n, const double* e, double mu, double kT, double* dF) {
  double beta = 1.0 / kT;
  for (int32_t l = 0; l < n; ++l) {
    for (int32_t k = 0; k < n; ++k) {
      double x = 0.5 * beta * (e[k] - e[l]);
      double lg = log(0.25 * beta) + log_sinhc(x) - log_cosh(0.5 * beta * (e[k] - mu)) -
                  log_cosh(0.5 * beta * (e[l] - mu));
      dF[k + (size_t)n * l] = -exp(lg);
    }
  }
}

/* ----------------------------------------------------------- core rows
 * Eq. (DD): d = sum_k f(e_k) v_k v_k^T; only the core rows are kept. */
void orc_core_rows(int32_t n, int32_t c, const double* z, const double* e, double mu,
                   double kT, int32_t fn, double* rows) {
  double* g = malloc(sizeof(double) * (size_t)n);
  for (int32_t k = 0; k < n; ++k) {
    if (fn == ORC_FN_IDENT) g[k] = e[k];
    else if (fn == ORC_FN_SQUARE) g[k] = e[k] * e[k];
    else g[k] = 2.0 * orc_fermi(e[k], mu, kT);
  }
  for (int32_t j = 0; j < c; ++j)
    for (int32_t l = 0; l < n; ++l) {
      double s = 0.0;
      for (int32_t k = 0; k < n; ++k) s += z[j + (size_t)n * k] * g[k] * z[l + (size_t)n * k];
      rows[(size_t)j * n + l] = s;
    }
  free(g);
}

/* Eq. (dddmu): d1mu = beta d0 (I - d0) = Z diag(beta f(1-f)) Z^T; core rows x 2 */
void orc_mu_response_rows(int32_t n, int32_t c, const double* z, const double* e,
                          double mu, double kT, double* rows, double* trace) {
  double* g = malloc(sizeof(double) * (size_t)n);
  for (int32_t k = 0; k < n; ++k) g[k] = 2.0 / kT * fermi_f1mf(e[k], mu, kT);
  for (int32_t j = 0; j < c; ++j)
    for (int32_t l = 0; l < n; ++l) {
      double s = 0.0;
      for (int32_t k = 0; k < n; ++k) s += z[j + (size_t)n * k] * g[k] * z[l + (size_t)n * k];
      rows[(size_t)j * n + l] = s;
    }
  ksum t = {0, 0};
  for (int32_t j = 0; j < c; ++j) ks_add(&t, rows[(size_t)j * n + j]);
  *trace = ks_val(&t);
  free(g);
}

/* Eq. (ddlambda) in the eigenbasis: d1lambda = Z [(Z^T h1 Z) o dF] Z^T; core rows x 2 */
void orc_lambda_response_rows(int32_t n, int32_t c, const double* z, const double* dF,
                              const double* h1, double* rows, double* trace) {
  size_t nn = (size_t)n * (size_t)n;
  double* W = malloc(sizeof(double) * nn);  /* h1 Z */
  double* Y = malloc(sizeof(double) * nn);  /* (Z^T h1 Z) o dF */
  double* T = malloc(sizeof(double) * (size_t)c * (size_t)n); /* Z_c Y */
  for (int32_t l = 0; l < n; ++l)
    for (int32_t i = 0; i < n; ++i) {
      double s = 0.0;
      for (int32_t m = 0; m < n; ++m) s += h1[i + (size_t)n * m] * z[m + (size_t)n * l];
      W[i + (size_t)n * l] = s;
    }
  for (int32_t l = 0; l < n; ++l)
    for (int32_t k = 0; k < n; ++k) {
      double s = 0.0;
      for (int32_t m = 0; m < n; ++m) s += z[m + (size_t)n * k] * W[m + (size_t)n * l];
      Y[k + (size_t)n * l] = s * dF[k + (size_t)n * l];
    }
  for (int32_t j = 0; j < c; ++j)
    for (int32_t q = 0; q < n; ++q) {
      double s = 0.0;
      for (int32_t k = 0; k < n; ++k) s += z[j + (size_t)n * k] * Y[k + (size_t)n * q];
      T[(size_t)j * n + q] = s;
    }
  for (int32_t j = 0; j < c; ++j)
    for (int32_t l = 0; l < n; ++l) {
      double s = 0.0;
      for (int32_t q = 0; q < n; ++q) s += T[(size_t)j * n + q] * z[l + (size_t)n * q];
      rows[(size_t)j * n + l] = 2.0 * s;
    }
  ksum t = {0, 0};
  for (int32_t j = 0; j < c; ++j) ks_add(&t, rows[(size_t)j * n + j]);
  *trace = ks_val(&t);
  free(W);
  free(Y);
  free(T);
}

/* Eq. (dmu_1) */
double orc_mu1(int32_t n_sub, const double* tlam, const double* tmu) {
  ksum a = {0, 0}, b = {0, 0};
  for (int32_t i = 0; i < n_sub; ++i) {
    ks_add(&a, tlam[i]);
    ks_add(&b, tmu[i]);
  }
  return -ks_val(&a) / ks_val(&b);
}

/* Eq. (sub_f) / (dCollect): core row j of subgraph s becomes row orbs[j] of
 * the collected matrix; its columns are the subgraph orbitals in ascending order */
void orc_collect(const orc_graph* g, int32_t sub, const double* rows, double* vals) {
  int32_t n = g->sub_orb_ptr[sub + 1] - g->sub_orb_ptr[sub];
  const int32_t* orbs = g->sub_orbs + g->sub_orb_ptr[sub];
  for (int32_t j = 0; j < g->n_core_orbs[sub]; ++j) {
    int32_t a = orbs[j];
    const int32_t* cols = g->rho_col + g->rho_row_ptr[a];
    for (int32_t l = 0; l < n; ++l) {
      int32_t lo = 0, hi = n;
      while (lo < hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (cols[mid] < orbs[l]) lo = mid + 1;
        else hi = mid;
      }
      vals[g->rho_row_ptr[a] + lo] = rows[(size_t)j * n + l];
    }
  }
}

/* ------------------------------------------------------------- whole path */
int orc_solve(const orc_graph* g, const orc_csr* H, double kT, double n_elec, int32_t fn,
              int32_t K, const orc_csr* H1, double* rho_vals, double* mu_out,
              double* rho1_vals, double* mu1_out, double* eps_out) {
  if (!(kT > 0.0)) return fail(ORC_EINVAL, "kT must be > 0");
  const int32_t ns = g->n_sub;
  int64_t tot = g->sub_orb_ptr[ns];
  double* eps = calloc((size_t)(tot > 0 ? tot : 1), sizeof(double));
  double* wts = calloc((size_t)(tot > 0 ? tot : 1), sizeof(double));
  double** Z = calloc((size_t)ns, sizeof(double*));
  int rc = ORC_OK;
  for (int32_t s = 0; s < ns && rc == ORC_OK; ++s) {
    int32_t n = g->sub_orb_ptr[s + 1] - g->sub_orb_ptr[s];
    const int32_t* orbs = g->sub_orbs + g->sub_orb_ptr[s];
    double* h = malloc(sizeof(double) * (size_t)n * (size_t)n);
    Z[s] = malloc(sizeof(double) * (size_t)n * (size_t)n);
    orc_gather(H, n, orbs, h);
    rc = orc_eigh(n, h, eps + g->sub_orb_ptr[s], Z[s]);
    orc_core_weights(n, g->n_core_orbs[s], Z[s], wts + g->sub_orb_ptr[s]);
    free(h);
  }
  double mu = 0.0;
  if (rc == ORC_OK && fn == ORC_FN_FERMI) rc = orc_find_mu(tot, eps, wts, kT, n_elec, &mu);
  if (rc == ORC_OK) {
    *mu_out = mu;
    if (eps_out) memcpy(eps_out, eps, sizeof(double) * (size_t)tot);
    double* tmu = calloc((size_t)ns, sizeof(double));
    double* tlam = calloc((size_t)ns * (size_t)(K > 0 ? K : 1), sizeof(double));
    double** Mrows = calloc((size_t)ns, sizeof(double*));
    double** Prows = calloc((size_t)ns * (size_t)(K > 0 ? K : 1), sizeof(double*));
    for (int32_t s = 0; s < ns; ++s) {
      int32_t n = g->sub_orb_ptr[s + 1] - g->sub_orb_ptr[s];
      int32_t c = g->n_core_orbs[s];
      const int32_t* orbs = g->sub_orbs + g->sub_orb_ptr[s];
      const double* e = eps + g->sub_orb_ptr[s];
      double* rows = malloc(sizeof(double) * (size_t)c * (size_t)n);
      orc_core_rows(n, c, Z[s], e, mu, kT, fn, rows);
      orc_collect(g, s, rows, rho_vals);
      free(rows);
      if (K > 0 && fn == ORC_FN_FERMI) {
        Mrows[s] = malloc(sizeof(double) * (size_t)c * (size_t)n);
        orc_mu_response_rows(n, c, Z[s], e, mu, kT, Mrows[s], &tmu[s]);
        double* dF = malloc(sizeof(double) * (size_t)n * (size_t)n);
        double* h1 = malloc(sizeof(double) * (size_t)n * (size_t)n);
        orc_divided_differences(n, e, mu, kT, dF);
        for (int32_t q = 0; q < K; ++q) {
          orc_gather(&H1[q], n, orbs, h1);
          Prows[(size_t)q * ns + s] = malloc(sizeof(double) * (size_t)c * (size_t)n);
          orc_lambda_response_rows(n, c, Z[s], dF, h1, Prows[(size_t)q * ns + s],
                                   &tlam[(size_t)q * ns + s]);
        }
        free(dF);
        free(h1);
      }
    }
    if (K > 0 && fn == ORC_FN_FERMI) {
      for (int32_t q = 0; q < K; ++q) {
        double mu1 = orc_mu1(ns, tlam + (size_t)q * ns, tmu);
        mu1_out[q] = mu1;
        for (int32_t s = 0; s < ns; ++s) {
          int32_t n = g->sub_orb_ptr[s + 1] - g->sub_orb_ptr[s];
          int32_t c = g->n_core_orbs[s];
          double* P = Prows[(size_t)q * ns + s];
          for (size_t t = 0; t < (size_t)c * (size_t)n; ++t) P[t] += mu1 * Mrows[s][t];
          orc_collect(g, s, P, rho1_vals + (size_t)q * (size_t)g->nnz);
          free(P);
        }
      }
      for (int32_t s = 0; s < ns; ++s) free(Mrows[s]);
    }
    free(Mrows);
    free(Prows);
    free(tmu);
    free(tlam);
  }
  for (int32_t s = 0; s < ns; ++s) free(Z[s]);
  free(Z);
  free(eps);
  free(wts);
  return rc;
}
