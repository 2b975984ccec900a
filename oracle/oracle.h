/*
 * Reference oracle for graph-based density and canonical response.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded FP64 CPU
 * implementation written directly from the paper (Negre, Wall, Niklasson,
 * "Graph-based quantum response theory and shadow Born-Oppenheimer molecular
 * dynamics", arXiv:2212.01997).  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header or
 * table with the GPU library.
 *
 * Passages followed:
 *   graph, partition, principal submatrices ..... Sec. II.B-C, Fig. 1, Sec. II.E
 *   collect of core rows ......................... Eq. (sub_f), Eq. (dCollect)
 *   subgraph eigenbasis density .................. Eqs. (DD0), (DD), (SmallKS)
 *   shared chemical potential .................... Sec. II.G, Eq. (NewtonRaphson)
 *   canonical first-order response ............... Sec. IV.A, Eqs. (D1_a), (D1_b),
 *                                                  (D1), (ddlambda), (dddmu), (dmu_1)
 *
 * Conventions: matrices are column-major (a[i + n*j]); a density carries the
 * closed-shell spin factor 2, so Tr rho = N_e; energies in Hartree.
 */
#ifndef GQ_ORACLE_H
#define GQ_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_OK = 0,
  ORC_EINVAL = -1,
  ORC_ENOMEM = -2,
  ORC_ENOCONV = -3
};

enum {
  ORC_PATHS2 = 1,    /* add paths of length two to the estimated graph */
  ORC_COMPLETE = 2   /* every halo is the whole system */
};

enum {
  ORC_FN_FERMI = 0,  /* 2 * Fermi-Dirac occupation (the density) */
  ORC_FN_IDENT = 1,  /* f(e) = e, no spin factor (test of gather/collect) */
  ORC_FN_SQUARE = 2  /* f(e) = e^2, no spin factor */
};

typedef struct {
  int32_t n_rows;
  int32_t nnz;
  const int32_t* row_ptr;
  const int32_t* col;
  const double* val;
} orc_csr;

typedef struct {
  int32_t n_atoms, n_orb, n_sub;
  int32_t* sub_ptr;       /* [n_sub+1] offsets into sub_atoms */
  int32_t* sub_atoms;     /* core atoms ascending, then halo atoms ascending */
  int32_t* n_core_atoms;  /* [n_sub] */
  int32_t* sub_orb_ptr;   /* [n_sub+1] offsets into sub_orbs */
  int32_t* sub_orbs;      /* orbitals of the subgraph atoms, atom by atom */
  int32_t* n_core_orbs;   /* [n_sub] */
  int32_t* rho_row_ptr;   /* [n_orb+1]; row a holds the orbitals of a's subgraph */
  int32_t* rho_col;       /* ascending column indices */
  int64_t nnz;
} orc_graph;

const char* orc_last_error(void);

int orc_graph_build(int32_t n_atoms, const int32_t* atom_orb_ptr, const orc_csr* H,
                    const orc_csr* rho_prev, const int32_t* core_of_atom, double tau,
                    int32_t flags, orc_graph* out);
void orc_graph_free(orc_graph* g);

/* dense principal submatrix h = X[orbs, orbs] of a CSR matrix (n x n, col-major) */
int orc_gather(const orc_csr* X, int32_t n, const int32_t* orbs, double* h);

/* symmetric eigensolve a = Z diag(w) Z^T, w ascending; a is not modified */
int orc_eigh(int32_t n, const double* a, double* w, double* z);

/* core weights w_k = sum_{j<c} Z[j,k]^2 */
void orc_core_weights(int32_t n, int32_t c, const double* z, double* wts);

/* F(mu) = 2 sum w f(e;mu) - n_elec over `count` (e, w) pairs (fixed order,
 * compensated); dF = 2 beta sum w f (1-f) */
void orc_occupation(int64_t count, const double* e, const double* wts, double mu,
                    double kT, double n_elec, double* F, double* dF);

/* shared chemical potential by bisection on F(mu) = 0 */
int orc_find_mu(int64_t count, const double* e, const double* wts, double kT,
                double n_elec, double* mu);

/* Fermi occupation f(e; mu, kT), evaluated without overflow */
double orc_fermi(double e, double mu, double kT);

/* divided differences dF[k,l] = (f_k - f_l)/(e_k - e_l), dF[k,k] = f'(e_k) */
void orc_divided_differences(int32_t n, const double* e, double mu, double kT, double* dF);

/* core rows of g(h) = Z diag(g(e)) Z^T for the chosen function (c x n, row-major) */
void orc_core_rows(int32_t n, int32_t c, const double* z, const double* e, double mu,
                   double kT, int32_t fn, double* rows);

/* core rows of 2 d1mu = 2 beta d0 (I - d0) (c x n, row-major) and their trace */
void orc_mu_response_rows(int32_t n, int32_t c, const double* z, const double* e,
                          double mu, double kT, double* rows, double* trace);

/* core rows of 2 d1lambda = 2 Z[(Z^T h1 Z) o dF]Z^T (c x n, row-major) and trace;
 * h1 is the dense n x n principal submatrix of the perturbation (col-major) */
void orc_lambda_response_rows(int32_t n, int32_t c, const double* z, const double* dF,
                              const double* h1, double* rows, double* trace);

/* mu1 = - sum(tlam) / sum(tmu), both sums fixed order and compensated */
double orc_mu1(int32_t n_sub, const double* tlam, const double* tmu);

/* place a subgraph's c x n core-row block into CSR values (graph pattern) */
void orc_collect(const orc_graph* g, int32_t sub, const double* rows, double* vals);

/* whole path, serial: density values [nnz], mu, and for K perturbations given
 * as dense-gatherable CSR matrices the response values [K][nnz] and mu1[K] */
int orc_solve(const orc_graph* g, const orc_csr* H, double kT, double n_elec, int32_t fn,
              int32_t K, const orc_csr* H1, double* rho_vals, double* mu_out,
              double* rho1_vals, double* mu1_out, double* eps_out);

#ifdef __cplusplus
}
#endif

#endif
