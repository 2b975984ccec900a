/*
 * gq — graph-based density matrix and canonical first-order response on
 * AMD Instinct MI355X (gfx950).  C ABI of libgq.so.
 *
 * Method: Negre, Wall, Niklasson, "Graph-based quantum response theory and
 * shadow Born-Oppenheimer molecular dynamics", arXiv:2212.01997.
 *
 *   graph_build      Sec. II.E (graph estimate from a previous density and the
 *                    Hamiltonian, optional paths of length two), Sec. II.C and
 *                    Fig. 1 (core + halo subgraphs, principal submatrices)
 *   submatrix_solve  Fig. 1 (principal submatrix h of each subgraph) and
 *                    Eq. (SmallKS) (h = Q diag(eps) Q^T)
 *   density          Sec. II.G, Eq. (NewtonRaphson) (one chemical potential
 *                    shared by all subgraphs) and Eqs. (DD0), (DD) (core rows)
 *   response         Sec. IV.A, Eqs. (D1_a), (D1_b), (ddlambda), (dddmu),
 *                    (dmu_1) (canonical first-order response in the eigenbasis)
 *   assemble         Eqs. (sub_f), (dCollect), (D1) (collect core rows)
 *   purify           Sec. II.D, Eqs. (Step), (Recur) (zero-temperature density
 *                    of every subgraph by purification, products only)
 *   overlap          Sec. II.D, Eqs. (SmallKS), (ksSmall) (non-orthogonal basis:
 *                    inverse factor of each overlap submatrix, congruences)
 *   charges          Sec. V (charge response, subgraph preconditioner,
 *                    preconditioned Krylov kernel)
 *
 * Conventions
 *   - Orthogonal basis unless a workspace is solved with
 *     gq_submatrix_solve_overlap; energies in Hartree.  Densities carry the closed-shell
 *     spin factor 2: Tr rho = N_e.  beta = 1/kT.
 *   - A "subgraph" i has n_i orbitals, of which the first c_i are its core.
 *   - "Blocks" are ragged per-subgraph arrays of c_i x n_i doubles, row-major,
 *     subgraph after subgraph (offsets from gq_graph_block_offsets); the
 *     collected CSR pattern of rho and rho1 has the same nnz = sum c_i n_i.
 *   - Host pointers are borrowed for the call; the library copies what it
 *     keeps.  Device pointers named *_dev point to memory on the context's
 *     device; output buffers are allocated by the caller.
 *   - All device work is ordered on the context's stream (a hipStream_t
 *     given at gq_ctx_create).  The eigensolve runs its smaller subgraphs on
 *     a second stream that the context owns, forked from the context's
 *     stream by an event and joined back into it before the call's later
 *     work, so callers (and a HIP graph captured on the context's stream)
 *     see one stream.  A call blocks the host only where it returns a host
 *     scalar (noted per call).
 *   - Errors: every call returns gq_status; on error the outputs are
 *     unspecified, handles stay valid, and gq_last_error() gives a message
 *     (thread-local).  No exception crosses the ABI.
 */
#ifndef GQ_H
#define GQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gq_status;
#define GQ_OK 0
#define GQ_EINVAL (-1)   /* bad argument or input structure */
#define GQ_ENOMEM (-2)   /* device or host allocation failed, or size limit */
#define GQ_ENOCONV (-3)  /* eigensolver or chemical-potential bracket failed */
#define GQ_EDEVICE (-4)  /* HIP runtime error */
#define GQ_EBUSY (-5)    /* resource busy (serving admission) */

/* graph_build flags */
#define GQ_PATHS2 1u     /* extend the estimated graph by paths of length two */
#define GQ_COMPLETE 2u   /* every halo is the whole system (dense limit) */

/* submatrix_solve flags */
#define GQ_SOLVE_DEFAULT 0u

/* response precision */
#define GQ_PREC_FP64 0u       /* congruences in FP64 */
#define GQ_PREC_SPLIT32 1u    /* split-FP32 congruences + one FP64 refinement */
/* With GQ_PREC_SPLIT32, X = Q^T h1 Q is formed from the FP32 leading part of
 * Q on FP32 MFMA (FP64 sums of 32-deep FP32 chunks); X o dF amplifies its
 * rounding by dF, which is f'(eps) <= beta/4 for a pair of equal energies.
 * Every pair of states whose f' exceeds tau_F, i.e. with
 * |eps - mu| <= 2 acosh(sqrt(beta / (4 tau_F))) kT (none when
 * beta/4 <= tau_F), is recomputed on FP64 MFMA; a subgraph with more than
 * `cap` such states gets its whole X in FP64.  Defaults tau_F = 10 / Ha,
 * cap = 128 (gq_ctx_set_split_window). */

typedef struct gq_ctx gq_ctx;
typedef struct gq_graph gq_graph;
typedef struct gq_eigs gq_eigs;
typedef struct gq_exec gq_exec;

/* CSR matrix, 0-based, ascending columns in every row.  Host or device
 * memory as stated by the call that takes it. */
typedef struct {
  int32_t n_rows;
  int32_t nnz;
  const int32_t* row_ptr; /* [n_rows + 1] */
  const int32_t* col;     /* [nnz] */
  const double* val;      /* [nnz] */
} gq_csr;

typedef struct {
  int32_t n_atoms;
  int32_t n_orb;        /* N */
  int32_t n_sub;        /* number of subgraphs (= number of cores) */
  int32_t max_n;        /* largest subgraph, orbitals */
  int32_t min_n;
  int32_t max_c;        /* largest core, orbitals */
  int64_t nnz;          /* collected pattern = sum c_i n_i */
  int64_t sum_n;        /* sum n_i */
  int64_t sum_n2;       /* sum n_i^2 */
  int64_t sub_atoms_len;/* sum of subgraph vertex counts */
} gq_graph_info;

/* Message for the last non-OK status returned on this thread. */
const char* gq_last_error(void);
/* Library version string. */
const char* gq_version(void);

/* Context on HIP device `device`; `hip_stream` is a hipStream_t (NULL = the
 * default stream).  The stream is borrowed and must outlive the context.
 * arena_bytes > 0 allocates one device arena of that size here, once: every
 * eigen workspace later created on this context (gq_eigs_create), and the
 * device index maps of a graph first bound by such a call, then take a piece
 * of the arena (first fit, 256-byte aligned) and return it when destroyed, so
 * that no device allocation happens after this call.  gq_eigs_create reports
 * GQ_ENOMEM when no piece fits.  The context must outlive every workspace and
 * graph that holds a piece of its arena.  arena_bytes = 0: workspaces allocate
 * their own device memory.  GQ_ENOMEM if the arena cannot be allocated;
 * GQ_EINVAL if arena_bytes < 0. */
gq_status gq_ctx_create(int32_t device, void* hip_stream, int64_t arena_bytes, gq_ctx** out);
/* Bytes of the context's arena in use and its size (0, 0 without one). */
gq_status gq_ctx_arena_used(gq_ctx* ctx, int64_t* used, int64_t* size);
void gq_ctx_destroy(gq_ctx* ctx);

/* ---------------------------------------------------------- graph_build
 * Host, integer work, deterministic.  Atom graph: I != J are joined when some
 * orbital pair (a in I, b in J) has |H_ab| >= tau, or |rho_prev_ab| >= tau or
 * |rho_prev_ba| >= tau (Sec. II.E); GQ_PATHS2 adds every pair joined by a path
 * of length two.  Subgraph i: its core atoms (core_of_atom[I] == i) ascending,
 * then its halo (atoms joined to a core atom, not in the core) ascending
 * (Sec. II.C, Fig. 1); GQ_COMPLETE makes every halo the rest of the system.
 * Orbitals follow their atoms in native order.  The collected pattern holds,
 * for every orbital a, the ascending orbitals of a's subgraph.
 *
 * All pointers are host memory.  atom_orb_ptr[n_atoms+1] strictly increasing
 * from 0; H: N x N with a symmetric pattern; rho_prev: N x N or NULL;
 * core_of_atom[n_atoms]: ids 0..n_sub-1, each used.  GQ_EINVAL on any
 * violation, n_atoms < 1 or tau < 0; GQ_ENOMEM if a count exceeds int32.  *out is owned by
 * the caller (gq_graph_destroy). */
gq_status gq_graph_build(int32_t n_atoms, const int32_t* atom_orb_ptr, const gq_csr* H,
                         const gq_csr* rho_prev, const int32_t* core_of_atom, double tau,
                         uint32_t flags, gq_graph** out);
gq_status gq_graph_query(const gq_graph* g, gq_graph_info* info);
/* Copies the graph into caller arrays sized from gq_graph_info (any may be
 * NULL): sub_ptr[n_sub+1], sub_atoms[sub_atoms_len], n_core_atoms[n_sub],
 * sub_orb_ptr[n_sub+1], sub_orbs[sum_n], n_core_orbs[n_sub],
 * rho_row_ptr[N+1], rho_col[nnz]. */
gq_status gq_graph_export(const gq_graph* g, int32_t* sub_ptr, int32_t* sub_atoms,
                          int32_t* n_core_atoms, int32_t* sub_orb_ptr, int32_t* sub_orbs,
                          int32_t* n_core_orbs, int32_t* rho_row_ptr, int32_t* rho_col);
/* Block offsets: off[i] = sum_{j<i} c_j n_j, off[n_sub] = nnz (host array). */
gq_status gq_graph_block_offsets(const gq_graph* g, int64_t* off);
void gq_graph_destroy(gq_graph* g);

/* ------------------------------------------------------- eigen workspace
 * Device-resident state of one graph: eigenpairs, core weights, the mu
 * response rows and the divided differences, sized for up to `max_k`
 * perturbations per response call.  flags: GQ_EIGS_GENERAL_H1 also reserves
 * the buffer (max_k x sum n_i^2 doubles) that perturbations given as CSR
 * matrices need (GQ_H1_CSR); diagonal perturbations do not need it.
 * GQ_EIGS_OVERLAP reserves the non-orthogonal basis's inverse factors z_i
 * and atomic-orbital eigenvectors C_i = z_i Q_i (2 sum n_i^2 doubles), needed
 * by gq_submatrix_solve_overlap.  Allocates device memory, or takes a piece of the context's arena
 * (GQ_ENOMEM when neither is available); GQ_EINVAL for unknown flags, a
 * subgraph above 2048 orbitals or a core above 128 orbitals. */
#define GQ_EIGS_GENERAL_H1 1u
#define GQ_EIGS_OVERLAP 2u
gq_status gq_eigs_create(gq_ctx* ctx, const gq_graph* g, int32_t max_k, uint32_t flags,
                         gq_eigs** out);
/* Device bytes held by an eigen workspace for graph g, max_k and flags, plus
 * the graph's device index maps (for admission control); no allocation. */
gq_status gq_eigs_footprint(const gq_graph* g, int32_t max_k, uint32_t flags, int64_t* bytes);
/* As gq_eigs_create, with every device array of the workspace (and the
 * graph's device maps, if the graph is not bound to a device yet) placed in
 * caller-owned device memory `mem` of `bytes` >= gq_eigs_footprint(g, max_k,
 * flags), 256-byte aligned.  For allocators that hand out pieces of one arena
 * (the serving runtime): neither this call nor gq_eigs_destroy /
 * gq_graph_destroy allocate or free device memory for such a workspace.  mem
 * must outlive both handles. */
gq_status gq_eigs_create_in(gq_ctx* ctx, const gq_graph* g, int32_t max_k, uint32_t flags,
                            void* mem, int64_t bytes, gq_eigs** out);
void gq_eigs_destroy(gq_eigs* e);

/* ------------------------------------------------------ submatrix_solve
 * Gathers every principal submatrix h_i = H[orbs_i, orbs_i] from the device
 * CSR H (same N and a pattern containing the one given to graph_build) and
 * solves h_i = Q_i diag(eps_i) Q_i^T in FP64 (eps ascending), all on the
 * context stream.  Subgraphs below 768 orbitals are reduced to tridiagonal
 * form by one workgroup each; larger ones (up to 2048) on the lower 64x64
 * tiles of their trailing matrix, one workgroup per tile, two launches per
 * column (the tile products, then the column step), every such subgraph of
 * the graph in the same launches (in two halves on the context's two streams
 * when the graph has no smaller subgraphs).  Asynchronous; a later call that
 * syncs reports GQ_ENOCONV if an eigensolve hit its iteration cap. */
gq_status gq_submatrix_solve(gq_ctx* ctx, const gq_graph* g, const gq_csr* H_dev,
                             uint32_t flags, gq_eigs* e);

/* ------------------------------------------------ non-orthogonal basis
 * The same for a non-orthogonal (atomic-orbital) basis with overlap matrix S
 * (Sec. II.D, Eqs. (SmallKS), (ksSmall) and the atomic-orbital congruence
 * after them): for every subgraph, s_i = S[orbs_i, orbs_i] is solved as
 * s_i = U diag(sigma) U^T, z_i = s_i^(-1/2) = U diag(sigma^(-1/2)) U^T (the
 * Lowdin inverse factor, z^T s z = I), h_ao = H[orbs_i, orbs_i] is carried to
 * h_i = z_i h_ao z_i and solved as h_i = Q_i diag(eps_i) Q_i^T, and the
 * atomic-orbital eigenvectors C_i = z_i Q_i are kept.  All products run on
 * the batched FP64 MFMA kernel.  After this call, on this workspace:
 *   gq_density fixes mu on the orthogonalized core weights (Eq. (DD)) and
 *     writes the atomic-orbital core rows 2 C_c diag(f) C^T, the core rows of
 *     z d z^T (its mu-response rows likewise);
 *   gq_response and gq_response_static take h1 in the atomic-orbital basis
 *     (X = C^T h1 C = Q^T z h1 z Q), fix mu1 on the orthogonalized traces, and
 *     write the atomic-orbital response rows (the core rows of z d1 z^T),
 *     FP64 only (GQ_PREC_SPLIT32: GQ_EINVAL);
 *   the charge entry points return GQ_EINVAL.
 * A later gq_submatrix_solve returns the workspace to the orthogonal case.
 * S_dev: device CSR, N rows, symmetric, its pattern contained in the one
 * given to graph_build.  Needs a workspace created with GQ_EIGS_OVERLAP.
 * Waits for the stream once (after the overlap eigensolves): GQ_EINVAL if an
 * s_i is not positive definite (the message names the subgraph and its
 * smallest eigenvalue), GQ_ENOCONV if one of those eigensolves did not
 * converge.  Not while capturing. */
gq_status gq_submatrix_solve_overlap(gq_ctx* ctx, const gq_graph* g, const gq_csr* H_dev,
                                     const gq_csr* S_dev, uint32_t flags, gq_eigs* e);

/* -------------------------------------------------------------- density
 * Shared chemical potential: the root of 2 sum_{i,k} w_ik f(eps_ik; mu) = n_elec
 * with core weights w_ik = sum_{j<c_i} Q_i[j,k]^2 (Sec. II.G), found by
 * multisection on the device to the last representable interval.  Then the
 * core rows rho_i = 2 Q_i[0:c_i,:] diag(f) Q_i^T into rho_blocks_dev (device,
 * nnz doubles; may be NULL), and the mu-response rows
 * 2 beta Q_c diag(f(1-f)) Q^T kept in the workspace.  kT > 0 and
 * 0 < n_elec < 2N (GQ_EINVAL).
 * mu_inout (host, may be NULL): on entry a warm-start guess, as the previous
 * step's mu in Sec. II.G (NaN: none); on return the root, after waiting for
 * the stream.  With a guess the first pass places its points at
 * guess +- kT 4^j (j = -8..7, clipped to the eigenvalue span), so the passes
 * after it start from the bracket that holds the root, however far the guess
 * is; passes whose bracket has reached adjacent doubles do no work.  Twelve
 * passes run with a guess, eleven without.  NULL while capturing. */
gq_status gq_density(gq_ctx* ctx, gq_eigs* e, double kT, double n_elec, double* mu_inout,
                     double* rho_blocks_dev);

/* ---------------------------------------------------------------- purify
 * The zero-temperature density of every subgraph by recursive expansion
 * (Sec. II.D, Eqs. (Step), (Recur), (dCollect)), on matrix products only,
 * without an eigensolve: gathers h_i = H[orbs_i, orbs_i] from the device CSR
 * H_dev, maps it to X_0 = I/2 - (h_i - mu I)/(2 R_i) with R_i the Gershgorin
 * bound of |eig(h_i - mu I)|, and iterates X <- 3 X^2 - 2 X^3 (McWeeny),
 * which sends the eigenvalues of h_i below mu to 1 and above mu to 0.  A
 * subgraph stops once max |X_{k+1} - X_k| <= tol.  Writes the core rows
 * 2 X_i[0:c_i, :] (2 Theta(mu - h_i), spin included, as gq_density) into
 * rho_blocks_dev (device, nnz doubles, block layout).  mu (host) is given:
 * the grand-canonical form, as in Eq. (Step).  1 <= max_iter; tol > 0.
 * The workspace's eigenvectors and density are overwritten (a following
 * gq_response needs gq_submatrix_solve and gq_density again).  Waits for the
 * stream every fourth iteration to test convergence; not while capturing.
 * iterations (host, may be NULL): the iterations run.  GQ_ENOCONV (the rows
 * are still written) if a subgraph has not converged after max_iter, which
 * happens when an eigenvalue of h_i lies at or very close to mu: the step
 * function is then not defined or not reached at that precision. */
gq_status gq_purify(gq_ctx* ctx, const gq_graph* g, const gq_csr* H_dev, gq_eigs* e, double mu,
                    int32_t max_iter, double tol, double* rho_blocks_dev, int32_t* iterations);

/* ------------------------------------------------------------- response
 * K perturbations H1_q of the Hamiltonian, H(lambda) = H + lambda H1
 * (Sec. IV.A, Eq. (ddlambda)), each symmetric N x N, as
 *   GQ_H1_DIAG: h1 is `const double*`, diagonals h1[K][N] in device memory;
 *   GQ_H1_CSR:  h1 is `const gq_csr*`, a host array of K CSR matrices whose
 *               row_ptr/col/val arrays are device memory (N rows each, sorted
 *               columns, symmetric values); the workspace must have been
 *               created with GQ_EIGS_GENERAL_H1.
 * For each subgraph: h1_s = H1[orbs, orbs], X = Q^T h1_s Q (the molecular-
 * orbital representation, as remarked at the end of Sec. IV.A),
 * Y = X o dF with dF_kl = (f_k - f_l)/(e_k - e_l) (f'(e_k) when equal),
 * P = 2 Q_c Y Q^T, and the canonical mu1_q = -sum_i Tr_c P_i / sum_i Tr_c M_i
 * (Eq. (dmu_1)).  Writes p_blocks_dev[K][nnz] = P + mu1_q M (the collected
 * rho1 rows in block layout) and mu1_dev[K] (device; may be NULL).
 * `precision` is GQ_PREC_FP64 or GQ_PREC_SPLIT32.  Requires gq_density on the
 * same workspace first; 1 <= K <= max_k.  mu1_host (may be NULL) makes the
 * call wait for the stream; NULL while capturing. */
#define GQ_H1_DIAG 0u
#define GQ_H1_CSR 1u
gq_status gq_response(gq_ctx* ctx, gq_eigs* e, const void* h1, uint32_t h1_kind, int32_t K,
                      uint32_t precision, double* p_blocks_dev, double* mu1_dev,
                      double* mu1_host);

/* ------------------------------------------------- response, no allocation
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and the same results, bit for bit, as gq_response, with the
 * response's per-call buffers (perturbations gathered per subgraph,
 * X o dF, general-kind h1_s and W = h1_s Q, Q_c (X o dF), the core diagonals
 * of P, mu1) in the library's static device scratch of 2^25 doubles
 * (256 MiB) per device instead of the workspace, so K is not bounded by
 * max_k.  The perturbations run in chunks of as many as fit the scratch
 * (sum n_i^2 + 33 sum n_i + sum c_i doubles each, twice the n^2 term for
 * GQ_H1_CSR); GQ_ENOMEM with a message if one does not fit (sum n_i^2 above
 * about 3.2e7).  The scratch keeps the last call's contents and nothing in it
 * needs to start at zero.  It is shared by every context on the device:
 * calls that overlap in time on one GPU (concurrent streams or threads) race
 * on it and must be serialised by the caller.  Calls no hipMalloc, hipFree or
 * allocating library routine and does not wait for the stream (allowed while
 * capturing).  Arguments and errors as gq_response, without mu1_host; the
 * workspace needs no max_k >= K. */
gq_status gq_response_static(gq_ctx* ctx, gq_eigs* e, const void* h1, uint32_t h1_kind,
                             int32_t K, uint32_t precision, double* p_blocks_dev,
                             double* mu1_dev);

/* ------------------------------------------------------------- assemble
 * Scatters K block arrays (device, [K][nnz], block layout) into CSR value
 * arrays vals_dev[K][nnz] in the collected pattern of g (device). */
gq_status gq_assemble(gq_ctx* ctx, const gq_graph* g, const double* blocks_dev, int32_t K,
                      double* vals_dev);

/* -------------------------------------------------------------- charges
 * Sec. V: the charge response that the preconditioned Krylov kernel of the
 * electronic equations of motion needs.  Atomic charges n act on every
 * orbital of atom I through the potential (gamma n)_I, so a charge vector v
 * perturbs the Hamiltonian by H1[v] = diag(gamma v) over the orbitals; gamma
 * is an n_atoms x n_atoms symmetric kernel (the charge-charge interaction, a
 * Coulomb-type sum in SCC-DFTB).  Core charges of a density are the diagonal
 * entries of its collected core rows summed per atom (Eq. (assemble_rho0)).
 * Charge vectors are device arrays of n_atoms doubles; K of them are [K][n_atoms].
 *
 * gq_charge_create: device state of the charge model on graph g: gamma (host
 * CSR, ascending columns) and each atom's core subgraph, with work buffers
 * for up to kmax charge vectors per call (a piece of ctx's arena when it has
 * one).  GQ_EINVAL for a malformed gamma; GQ_ENOMEM.  The graph must outlive
 * the handle; the handle is destroyed before ctx.
 *
 * gq_charge_core: q[n_atoms] = per-atom core charges of the core-row blocks
 * `blocks_dev` (nnz, block layout, e.g. the rho blocks of gq_density).
 *
 * gq_charge_response: for each v_q, the derivative of the core charges along
 * H1[v_q] (Eq. (dfdv), first term): the canonical graph response (Eqs. (D1),
 * (dmu_1)) on the workspace's eigenbasis, of which only the diagonal of the
 * core rows is formed.  q1_dev [K][n_atoms]; mu1_dev [K] or NULL.
 * 1 <= K <= min(max_k of e, kmax).  Requires gq_density on e.
 *
 * gq_preconditioner: Sec. V.A, Eq. (PreCond).  For every subgraph k and each
 * of its m_k core atoms J, the fixed-mu response of the core charges to a
 * unit charge on J (H1 = gamma[., J] on every orbital, restricted to the
 * subgraph, Eq. (TwoDer)) and the core charges of the mu response; each
 * column's mu1 is set so that the column sums over the core are -1, giving
 * j^(k), and k0^(k) = (j^(k) - alpha I)^-1 (Gauss-Jordan, partial pivoting).
 * k0_dev receives the blocks subgraph after subgraph, each m_k x m_k
 * column-major over the subgraph's core atoms in ascending order (offsets
 * sum_{j<k} m_j^2).  *singular_dev (device int32) is set to 1 if a block is
 * singular (its entries are NaN then).  alpha >= 0; cores of at most 32 atoms.
 * The unit-charge perturbations run min(max_k, largest m_k) at a time.
 *
 * gq_krylov_kernel: Sec. V.B, Eqs. (v1_prim), (v1), (dfdv), (LowRankEEOM),
 * (ElEOM).  From the ground-state core rows rho_blocks_dev and the charges
 * n_dev: f = rho_0 - n, v_1 = K0 f / |K0 f|; for i = 1..m the charge response
 * along v_i and f_{v_i} = K0 (d rho_0 / d lambda - v_i) (F_dev row i), then
 * v_{i+1} = f_{v_i} orthogonalised against v_1..v_i by two passes of modified
 * Gram-Schmidt and normalised (V_dev row i+1); O_ij = f_{v_i} . f_{v_j}
 * (O_dev, m x m), M = O^-1 (M_dev) and the charge acceleration
 * ndd = -omega^2 sum_ij v_i M_ij (f_{v_j} . K0 f) (ndd_dev, n_atoms).  All
 * sums over the atoms run in a fixed order.  1 <= m <= 32; *singular_dev is
 * set to 1 if O is singular.  Requires gq_density on e; K0 from
 * gq_preconditioner. */
typedef struct gq_charge gq_charge;
gq_status gq_charge_create(gq_ctx* ctx, const gq_graph* g, const gq_csr* gamma, int32_t kmax,
                           gq_charge** out);
void gq_charge_destroy(gq_charge* c);
gq_status gq_charge_core(gq_ctx* ctx, gq_charge* c, const double* blocks_dev, double* q_dev);
gq_status gq_charge_response(gq_ctx* ctx, gq_charge* c, gq_eigs* e, const double* v_dev,
                             int32_t K, uint32_t precision, double* q1_dev, double* mu1_dev);
gq_status gq_preconditioner(gq_ctx* ctx, gq_charge* c, gq_eigs* e, double alpha, double* k0_dev,
                            int32_t* singular_dev);
gq_status gq_krylov_kernel(gq_ctx* ctx, gq_charge* c, gq_eigs* e, const double* k0_dev,
                           const double* rho_blocks_dev, const double* n_dev, int32_t m,
                           double omega, uint32_t precision, double* ndd_dev, double* V_dev,
                           double* F_dev, double* O_dev, double* M_dev, int32_t* singular_dev);

/* ------------------------------------------------------------ batching
 * Launch tuning and whole-step capture for batches of uneven subgraphs
 * (Sec. II.G: the subgraph problems are independent and are run as one
 * batch; the sizes follow from the graph).
 *
 * gq_autotune: times, on this workspace and for precision GQ_PREC_FP64 or
 * GQ_PREC_SPLIT32, each launch variant of the response's X kernel (64x64 or
 * 32x32 tiles; one workgroup per tile or a persistent grid) on every size bin
 * of the subgraphs (n <= 128, 256, 384, 512, 2048) and keeps the fastest per
 * bin in the graph handle, where later gq_response calls on any workspace of
 * that graph use it.  Requires gq_density first.  Overwrites the workspace's
 * response scratch; waits for the stream.  report (host, may be NULL)
 * receives up to report_len bytes of NUL-terminated text, one line per
 * variant and bin.  GQ_EINVAL while capturing.
 *
 * gq_capture_begin / gq_capture_end record every library call made on ctx in
 * between into one HIP graph instead of running it (the context's stream must
 * not be the legacy default stream).  Recorded calls must not return host
 * scalars (mu_out and mu1_host NULL, no gq_eigs_export or kernel times):
 * such calls fail with GQ_EINVAL while capturing.  Profiling is suspended.
 * gq_exec_launch replays the recorded work on ctx's stream with the buffers
 * and arguments of the recording (asynchronous); the handles and device
 * buffers it names must stay alive.  gq_exec_destroy frees the graph. */
gq_status gq_autotune(gq_ctx* ctx, gq_eigs* e, uint32_t precision, char* report,
                      size_t report_len);
/* Sets the X-kernel launch variant of one size bin by hand (diagnostics and
 * tests): bin 0..4 as above, variant bit 0 = 32x32 tiles, bit 1 = persistent
 * grid.  Every variant gives bit-identical results. */
gq_status gq_graph_set_launch(const gq_graph* g, uint32_t precision, int32_t bin,
                              int32_t variant);
gq_status gq_capture_begin(gq_ctx* ctx);
gq_status gq_capture_end(gq_ctx* ctx, gq_exec** out);
gq_status gq_exec_launch(gq_ctx* ctx, gq_exec* x);
void gq_exec_destroy(gq_exec* x);

/* ------------------------------------------------------------- serving
 * A runtime that admits whole-path requests continuously on one GPU.  One
 * device arena of arena_bytes is allocated at creation; n_slots executor
 * threads, each with a HIP stream and context of its own, take the oldest
 * waiting request, build its graph on the host, size its footprint (eigen
 * workspace, graph maps, H, the K perturbations, rho and rho1) and wait until
 * the arena has a contiguous piece of that size.  Admitted requests run
 * concurrently on their threads' streams; the K perturbations of a request
 * share its device-resident eigenbasis, mu and dF.  No device memory is
 * allocated or freed while serving.
 *
 * gq_server_submit copies the request (host memory) and returns at once with
 * its id.  gq_server_wait blocks until the request has finished and fills
 * info (times in seconds on the server clock, which starts at creation); it
 * returns the request's status (GQ_ENOMEM if it can never fit the arena).
 * gq_server_fetch copies the results to host arrays (any may be NULL):
 * mu1[K], rho[nnz], rho1[K][nnz], and the collected CSR pattern
 * rho_row_ptr[N+1], rho_col[nnz].  gq_server_release forgets a finished
 * request.  gq_server_destroy fails the requests still waiting (GQ_EBUSY),
 * waits for the running ones and frees the arena. */
typedef struct gq_server gq_server;
typedef struct {
  int32_t n_atoms;
  const int32_t* atom_orb_ptr; /* [n_atoms+1] */
  const gq_csr* H;             /* host CSR, N x N */
  const gq_csr* rho_prev;      /* host CSR or NULL (graph from H alone) */
  const int32_t* core_of_atom; /* [n_atoms] */
  double tau;
  uint32_t flags;              /* graph_build flags */
  double kT, n_elec;
  int32_t K;                   /* perturbations */
  const double* h1;            /* host [K][N], diagonal perturbations */
  uint32_t precision;          /* GQ_PREC_FP64 or GQ_PREC_SPLIT32 */
} gq_request;
typedef struct {
  gq_status status;
  double mu;
  int32_t n_sub, K;
  int64_t nnz, footprint;
  double t_submit, t_admit, t_done;
} gq_request_info;
gq_status gq_server_create(int32_t device, int32_t n_slots, int64_t arena_bytes,
                           gq_server** out);
gq_status gq_server_submit(gq_server* s, const gq_request* r, int64_t* id);
gq_status gq_server_wait(gq_server* s, int64_t id, gq_request_info* info);
gq_status gq_server_fetch(gq_server* s, int64_t id, double* mu1, double* rho, double* rho1,
                          int32_t* rho_row_ptr, int32_t* rho_col);
gq_status gq_server_release(gq_server* s, int64_t id);
gq_status gq_server_arena_used(gq_server* s, int64_t* used, int64_t* size);
double gq_server_clock(gq_server* s);
void gq_server_destroy(gq_server* s);

/* ---------------------------------------------------------- profiling
 * Diagnostics, not part of the method.  While enabled, every kernel launch
 * of the context is bracketed by a hipEvent pair on the stream it runs on
 * (launches on the two streams of the eigensolve overlap in time).
 * gq_ctx_kernel_times waits for the stream and reports per kernel name the
 * launch count and total milliseconds since profiling was last enabled
 * (arrays of `cap` entries, host; *count = entries filled; the name strings
 * are static).  Enabling resets the totals. */
gq_status gq_ctx_set_profiling(gq_ctx* ctx, int32_t enable);
gq_status gq_ctx_kernel_times(gq_ctx* ctx, const char** names, int64_t* launches,
                              double* total_ms, int32_t cap, int32_t* count);

/* ---------------------------------------------------------- diagnostics
 * Most QL iterations per eigenvalue in the divide-and-conquer leaves of the
 * eigensolves launched later on ctx (default 60; >= 0, else GQ_EINVAL).  A
 * leaf that needs more marks its subgraph as not converged, every kernel
 * still runs to its end, and the next call that synchronises (gq_density with
 * mu_inout, gq_response with mu1_host, gq_eigs_export) returns GQ_ENOCONV.
 * A small cap exercises that path from the host. */
gq_status gq_ctx_set_iteration_cap(gq_ctx* ctx, int32_t leaf_iterations);

/* Refinement window of the split-FP32 response on ctx: the divided-difference
 * threshold tau_F > 0 (1/Ha) and the largest window refined by itself
 * (cap >= 0; wider windows put the subgraph's X in FP64).  GQ_EINVAL
 * otherwise. */
gq_status gq_ctx_set_split_window(gq_ctx* ctx, double dF_threshold, int32_t max_states);

/* Diagnostics (continued).
 * Copies eigenvalues eps[sum_n] (subgraph by subgraph, ascending) and core
 * weights w[sum_n] to host arrays (either may be NULL); waits for the stream.
 * Returns GQ_ENOCONV if any eigensolve failed to converge. */
gq_status gq_eigs_export(gq_ctx* ctx, const gq_eigs* e, double* eps, double* w);
/* Device pointer to subgraph i's eigenvectors (n_i x n_i, column-major). */
gq_status gq_eigs_vectors(const gq_eigs* e, int32_t i, const double** q_dev, int32_t* n);

#ifdef __cplusplus
}
#endif

#endif
