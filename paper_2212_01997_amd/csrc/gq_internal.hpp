// Internal declarations of libgq (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <utility>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gq.h"

namespace gq {

// Largest subgraph the kernels accept (orbitals).  The one-workgroup
// reduction to tridiagonal form (a row per thread of a 1024-thread workgroup)
// takes subgraphs of up to kTdMaxN orbitals; subgraphs of kMwgMinN orbitals
// and more take the multi-workgroup reduction instead (the lower 64x64 tiles
// of a subgraph's trailing matrix on separate workgroups, two launches per
// column), whose scratch slot and register budgets end at kMaxN.  From about 700 orbitals one
// subgraph's reduction on one CU takes longer than the multi-workgroup one's
// two launches per column.
constexpr int kMaxN = 2048;
constexpr int kTdMaxN = 1024;
constexpr int kMwgMinN = 768;
// Divide-and-conquer merges of up to kDcLdsMaxM eigenvalues keep their work
// arrays in LDS; larger merges (the top merge of a subgraph above kTdMaxN)
// keep them in a device scratch of kDcGlobalStride doubles per eigenvalue.
constexpr int kDcLdsMaxM = 1024;
constexpr int kDcGlobalStride = 17;
// Device scratch of the multi-workgroup reduction per subgraph (doubles): v
// (kMaxN), the panel products (32), the row and column partials of the
// (kMaxN/64)(kMaxN/64 + 1)/2 lower 64x64 tiles (64 each).
constexpr int kMwgSlot = kMaxN + 32 + 2 * 64 * ((kMaxN / 64) * (kMaxN / 64 + 1) / 2);
// Largest tridiagonal block solved directly in the divide-and-conquer tree.
constexpr int kLeaf = 16;
// Largest core (orbitals).  The core-row products (density rows, T = Q_c Y,
// P = 2 T Q^T) run in blocks of 32 core rows, so the bound only caps the
// number of those blocks (4); 128 orbitals hold cores of about 50 atoms.
constexpr int kMaxCore = 128;
// Points per multisection pass of the chemical-potential search.
constexpr int kMuPoints = 32;  // chemical potentials per multisection pass
constexpr int kMuPasses = 11;  // the bracket shrinks 33^11 = 5e16 fold
// Size bins of the response's X kernel (upper bounds, orbitals).
constexpr int kXyBins = 5;
constexpr int kXyBinMax[kXyBins] = {128, 256, 384, 512, kMaxN};

// Tile-list ranges [off[x], off[x+1]) served by the workgroups of XCD x.
struct XcdSplit {
  int32_t off[9];
};

// Allocator whose value-initialisation leaves trivial elements uninitialised:
// large index arrays that are filled right after resize() skip the zero pass.
template <class T>
struct DefaultInitAllocator : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = DefaultInitAllocator<U>;
  };
  DefaultInitAllocator() = default;
  template <class U>
  DefaultInitAllocator(const DefaultInitAllocator<U>&) {}
  template <class U>
  void construct(U* p) {
    ::new (static_cast<void*>(p)) U;
  }
  template <class U, class... Args>
  void construct(U* p, Args&&... args) {
    ::new (static_cast<void*>(p)) U(std::forward<Args>(args)...);
  }
};

constexpr size_t kArenaAlign = 256;
inline size_t arena_align(size_t x) { return (x + kArenaAlign - 1) & ~(kArenaAlign - 1); }

// First-fit allocator over [0, size) with coalescing (host bookkeeping only;
// the caller serialises access).
class Arena {
 public:
  explicit Arena(size_t size) : size_(size) {
    if (size) free_[0] = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = arena_align(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = arena_align(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t size() const { return size_; }
  size_t used() const { return used_; }

 private:
  size_t size_, used_ = 0;
  std::map<size_t, size_t> free_;
};

void set_error(const char* fmt, ...);

#define GQ_HIP(call)                                                             \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess) {                                                      \
      ::gq::set_error("%s failed: %s", #call, hipGetErrorString(e_));            \
      return GQ_EDEVICE;                                                         \
    }                                                                            \
  } while (0)

}  // namespace gq

// Per-kernel timing on the context stream (hipEvent pairs), enabled on demand.
struct gq_prof_rec {
  const char* name;
  hipEvent_t start, stop;
  hipStream_t stream;
};
struct gq_prof_stat {
  const char* name;
  int64_t count;
  double total_ms;
};

struct gq_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  // second stream (default priority) for the eigensolve of the smaller
  // subgraphs, forked from and joined back into `stream` by events
  hipStream_t side = nullptr;
  // fork/join of the eigensolve's two size classes, and of the divided
  // differences beside the density rows: one event pair per fork point
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipEvent_t ev_fork_dd = nullptr, ev_join_dd = nullptr;
  bool profiling = false;
  bool capturing = false;
  int32_t leaf_iter_cap = 60;  // QL iterations per eigenvalue in the leaves
  // split-FP32 response: states with f'(eps) above win_dF (1/Ha) are refined
  // in FP64; windows above win_cap states put the subgraph's X in FP64
  double win_dF = 10.0;
  int32_t win_cap = 128;
  // optional device arena (gq_ctx_create with arena_bytes > 0): workspaces and
  // graph maps created on this context take pieces of it
  char* arena_mem = nullptr;
  gq::Arena* arena = nullptr;
  std::mutex arena_mu;
  std::vector<gq_prof_rec> pending;
  std::vector<gq_prof_stat> stats;
};

// Device copy of the index maps of a graph.
struct gq_graph_dev {
  int device = -1;
  char* block = nullptr;           // device block of the maps when owned by the graph
  gq_ctx* arena_ctx = nullptr;     // context whose arena holds `block`, if any
  size_t arena_off = 0, arena_bytes = 0;
  int32_t* sub_orb_ptr = nullptr;  // [n_sub+1]
  int32_t* sub_orbs = nullptr;     // [sum_n]
  int32_t* n_core = nullptr;       // [n_sub]
  int32_t* sorted_orbs = nullptr;  // [sum_n] ascending orbitals per subgraph
  int32_t* sorted_local = nullptr; // [sum_n] local index of each sorted entry
  int32_t* slot = nullptr;         // [sum_n] column slot of each local orbital
  int64_t* off2 = nullptr;         // [n_sub+1] offsets of n_i^2 arrays
  int64_t* offc = nullptr;         // [n_sub+1] offsets of c_i n_i blocks
  int32_t* offcd = nullptr;        // [n_sub+1] offsets of c_i arrays
  int32_t* order = nullptr;        // subgraphs by decreasing n
  int32_t* rho_row_ptr = nullptr;  // [N+1]
  int32_t* dc_leaves = nullptr;    // [n_leaves*4] (subgraph, lo, m, buffer: 0 Q, 1 scratch)
  int32_t* dc_merges = nullptr;    // [n_merges*4] (subgraph, lo, m1, m2), deepest level first
  int32_t* dc_tiles = nullptr;     // [*3] (merge index within its level, tile row, tile col)
  int32_t n_leaves = 0;
  int32_t* bt_toff = nullptr;      // [n_sub] first compact-WY block of each subgraph
  int32_t* xy_tiles[2] = {nullptr, nullptr};  // X tiles (subgraph, ti, tj): 64x64, 32x32
  int32_t* tri_tiles = nullptr;   // lower 64x64 tiles (subgraph, ti >= tj), by XCD range
};

struct gq_graph {
  int32_t n_atoms = 0, N = 0, n_sub = 0;
  std::vector<int32_t> atom_orb_ptr;  // [n_atoms+1] orbitals of each atom
  std::vector<int32_t> sub_ptr, sub_atoms, n_core_atoms;
  std::vector<int32_t> sub_orb_ptr, sub_orbs, n_core_orbs;
  std::vector<int32_t> rho_row_ptr;
  std::vector<int32_t, gq::DefaultInitAllocator<int32_t>> rho_col;
  std::vector<int32_t> sorted_orbs, sorted_local, slot;
  std::vector<int64_t> off2, offc;
  std::vector<int32_t> offcd;
  std::vector<int32_t> order;
  // divide-and-conquer plan of the tridiagonal eigensolves
  std::vector<int32_t> dc_leaves, dc_merges, dc_tiles;
  // two size classes: class 0 = the n_big largest subgraphs (order[0..n_big)),
  // class 1 = the rest; each has its own leaves and merge levels, stored one
  // after the other in dc_leaves / dc_merges / dc_tiles
  int32_t n_big = 0;
  // subgraphs of kMwgMinN orbitals and more (order[0..n_mwg), all in class
  // 0): the multi-workgroup reduction
  int32_t n_mwg = 0;
  int32_t dc_leaf_off[3] = {0, 0, 0};
  std::vector<int32_t> dc_level_merge_off[2], dc_level_tile_off[2];
  // per level: leading merges with device-memory work arrays, and the largest
  // of the other merges
  std::vector<int32_t> dc_level_nglob[2], dc_level_maxm_lds[2];
  int32_t dc_nglob_max = 0;  // most such merges in one level
  std::vector<int64_t> dc_level_msum[2];  // sum of the merge sizes of each level
  std::vector<int32_t> bt_toff;  // compact-WY block offsets (16 reflectors per block)
  int32_t bt_nblocks = 0;
  // response X tiles per shape (0: 64x64, 1: 32x32), binned by size, XCD ranges
  std::vector<int32_t> xy_tiles[2];
  gq::XcdSplit xy_split[2][gq::kXyBins];
  // every lower-triangular 64x64 tile of every subgraph (batched products of
  // symmetric results), cut into eight XCD ranges at subgraph boundaries
  std::vector<int32_t> tri_tiles;
  gq::XcdSplit tri_split;
  // launch variant per [precision][bin] (bit 0: 32x32 tiles, bit 1: persistent)
  mutable int8_t xy_choice[2][gq::kXyBins];
  gq_graph_info info{};
  mutable gq_graph_dev dev;
};

struct gq_eigs {
  char* block = nullptr;    // device block of every array below, when owned
  bool block_in_arena = false;  // block is a piece of ctx's arena
  size_t arena_off = 0, arena_bytes = 0;
  gq_ctx* ctx = nullptr;
  const gq_graph* g = nullptr;
  int32_t max_k = 0;
  uint32_t flags = 0;       // GQ_EIGS_* given at creation
  double* A = nullptr;      // [sum n^2] gathered matrix / tridiagonal work, then dF
  double* Q = nullptr;      // [sum n^2] eigenvectors, column-major per subgraph
  double* Y = nullptr;      // [max_k][sum n^2] response scratch (X o dF); eigensolver scratch
  double* T = nullptr;      // [max_k][sum n][32] response scratch (Q_c Y), column by column
  double* eps = nullptr;    // [sum n]
  double* wts = nullptr;    // [sum n]
  double* dd = nullptr;     // [sum n] tridiagonal diagonal
  double* ee = nullptr;     // [sum n] tridiagonal off-diagonal
  double* tau = nullptr;    // [sum n] reflector scalars
  double* M = nullptr;      // [sum c n] mu-response rows 2 beta Q_c diag(f(1-f)) Q^T
  double* tmu = nullptr;    // [n_sub]
  double* pdiag = nullptr;  // [max_k][sum c] diagonal of P (for the core traces)
  double* mu1 = nullptr;    // [max_k]
  double* mu_state = nullptr;  // lo, hi, mu, kT, n_elec, ...
  double* mu_part = nullptr;   // [blocks][kMuPoints]
  int32_t mu_blocks = 0;
  int32_t* status = nullptr;   // [n_sub] eigensolver status (0 ok)
  int32_t* wflag = nullptr;    // [n_sub] split response: 1 = window too wide, X in FP64
  // merge metadata of the divide-and-conquer levels
  int32_t *md_k = nullptr, *md_cols = nullptr, *md_org = nullptr, *md_pos = nullptr;
  int32_t *md_dsrc = nullptr, *md_dpos = nullptr;
  double *md_delta = nullptr, *md_tau = nullptr, *md_zhat = nullptr, *md_inv = nullptr;
  double* tfac = nullptr;  // [bt_nblocks][16*16] compact-WY T factors
  double* wsc = nullptr;   // [sum_n * 16] panel scratch of the tridiagonalisation
  double* mwg = nullptr;  // [n_mwg][kMwgSlot] multi-workgroup reduction scratch
  double* dcg = nullptr;   // [dc_nglob_max][kMaxN * kDcGlobalStride] large-merge work arrays
  double* hloc = nullptr;  // [max_k][sum_n] perturbations gathered into subgraph order
  double* G = nullptr;     // [max_k][sum n^2] general perturbations (GQ_EIGS_GENERAL_H1 only)
  double* Z = nullptr;     // [sum n^2] Lowdin factors s_i^(-1/2) (GQ_EIGS_OVERLAP only)
  double* C = nullptr;     // [sum n^2] atomic-orbital eigenvectors z_i Q_i (GQ_EIGS_OVERLAP only)
  bool overlap_solved = false;  // the last solve was gq_submatrix_solve_overlap
  float* Q32 = nullptr;    // [sum n^2] FP32 leading part of Q (split-FP32 congruences)
  bool q32_valid = false;  // Q32 matches the current Q
  bool have_density = false;
  double kT = 0, n_elec = 0;
};

namespace gq {

gq_status graph_build_host(int32_t n_atoms, const int32_t* atom_orb_ptr, const gq_csr* H,
                           const gq_csr* rho_prev, const int32_t* core_of_atom, double tau,
                           uint32_t flags, gq_graph* g);
gq_status graph_upload(const gq_graph* g, int device);
void graph_free_dev(const gq_graph* g);

// Marks the start / end of a timed launch on ctx->stream (no-ops unless profiling).
void prof_begin(gq_ctx* ctx, const char* name);
void prof_begin_on(gq_ctx* ctx, const char* name, hipStream_t st);
void prof_end(gq_ctx* ctx);

// kernel launchers (all asynchronous on ctx->stream)
// Principal submatrices of the device CSR matrix H for every subgraph into A
// (n_i x n_i column-major at off2[i]); resets the eigensolver status when
// status is not NULL.
void launch_gather(gq_ctx* ctx, const gq_graph* g, const gq_csr* H, double* A, int32_t* status,
                   const char* label = "k_gather");
// C = alpha A^T B + beta D + gamma I on every subgraph (n x n column-major at
// off2): SYM when A^T B is symmetric (lower tiles computed and mirrored),
// else general.  Subgraphs with
// conv[s] >= skip_level are skipped (B copied to C when copy_b); errbits
// (SYM only) gets max |C - B| per subgraph.  conv and errbits may be NULL.
// Non-orthogonal basis: smallest eigenvalue per subgraph of the solved
// overlap (into out[n_sub]); z = s^(-1/2) into Z from the eigenpairs in
// (Q, eps); A = z A z; C = z Q.
void launch_overlap_min(gq_ctx* ctx, const gq_graph* g, gq_eigs* e, double* out);
void launch_overlap_factor(gq_ctx* ctx, const gq_graph* g, gq_eigs* e);
void launch_overlap_congruence(gq_ctx* ctx, const gq_graph* g, gq_eigs* e);
void launch_overlap_vectors(gq_ctx* ctx, const gq_graph* g, gq_eigs* e);
template <bool SYM>
void launch_bgemm(gq_ctx* ctx, const gq_graph* g, const double* A, const double* B,
                  const double* D, double* C, double alpha, double beta, double gamma,
                  const int32_t* conv, int skip_level, int copy_b, unsigned long long* errbits);
void eig_set_attributes();
void dc_set_attributes();
void build_dc_plan(gq_graph* g);
void launch_dc(gq_ctx* ctx, const gq_graph* g, gq_eigs* e, int cls, hipStream_t st);
int mu_blocks_for(int64_t count);
void launch_eigensolve(gq_ctx* ctx, const gq_graph* g, gq_eigs* e);
// mu by multisection; `guess` (NaN: none) places the first pass's points
// around a warm-start value.
void launch_mu(gq_ctx* ctx, const gq_graph* g, gq_eigs* e, double guess);
void launch_density(gq_ctx* ctx, const gq_graph* g, gq_eigs* e, double* rho_blocks);
void launch_divided_differences(gq_ctx* ctx, const gq_graph* g, gq_eigs* e, hipStream_t st);
// Per-call buffers of the response for K perturbations: hloc [K][sum_n]
// (diagonal kind), Y [K][sum n^2], G [K][sum n^2] (general kind), T
// [K][sum_n][32], pdiag [K][sum_c], mu1 [K].
struct RespBufs {
  double *hloc, *Y, *G, *T, *pdiag, *mu1;
};
// Perturbations of one response call: diagonals h1[K][N] (device), or K
// device CSR matrices (host array of gq_csr with device pointers).
struct H1Spec {
  uint32_t kind;
  const double* diag;
  const gq_csr* csr;
};
// local_h1: rb.hloc already holds the perturbations in subgraph order (the
// kind in h1 is then ignored); charge_only: form only the diagonal of P (into
// rb.pdiag) and mu1, not the core rows (p_blocks may be NULL).
struct RespOpts {
  bool local_h1 = false;
  bool charge_only = false;
};
void launch_response(gq_ctx* ctx, const gq_graph* g, gq_eigs* e, const RespBufs& rb,
                     const H1Spec& h1, int32_t K, uint32_t precision, double* p_blocks,
                     RespOpts opt = RespOpts{});
// Doubles of response scratch one perturbation needs (RespBufs layout).
int64_t resp_doubles_per_k(const gq_graph* g, uint32_t kind);
// Device address of the library's static response scratch on the current
// device (taken once per device with hipGetSymbolAddress), and its size.
gq_status scratch_init(int device);
double* scratch_ptr(int device);
int64_t scratch_doubles();
void launch_assemble(gq_ctx* ctx, const gq_graph* g, const double* blocks, int32_t K,
                     double* vals);
void build_xy_tiles(gq_graph* g);
gq_status autotune_xy(gq_ctx* ctx, const gq_graph* g, gq_eigs* e, uint32_t precision,
                      std::string* report);

}  // namespace gq
