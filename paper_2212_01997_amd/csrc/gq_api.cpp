// C entry points of libgq: contexts, graphs, eigen workspaces and the five
// calls of the path (graph_build, submatrix_solve, density, response,
// assemble).  No exception crosses this boundary.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "gq_internal.hpp"

namespace gq {

namespace {
thread_local char g_err[1024] = "";
}

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

template <class T>
static gq_status dev_upload(T** dst, const std::vector<T>& src) {
  const size_t bytes = std::max<size_t>(1, src.size()) * sizeof(T);
  GQ_HIP(hipMalloc((void**)dst, bytes));
  if (!src.empty()) GQ_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
  return GQ_OK;
}

void graph_free_dev(const gq_graph* g) {
  gq_graph_dev& d = g->dev;
  void* ptrs[] = {d.sub_orb_ptr, d.sub_orbs, d.n_core, d.sorted_orbs, d.sorted_local, d.slot,
                  d.off2, d.offc, d.offcd, d.order, d.rho_row_ptr, d.tiles,
                  d.dc_leaves, d.dc_merges, d.dc_tiles, d.bt_toff};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  d = gq_graph_dev{};
}

gq_status graph_upload(const gq_graph* g, int device) {
  gq_graph_dev& d = g->dev;
  if (d.device == device) return GQ_OK;
  if (d.device >= 0) {
    set_error("graph already bound to device %d", d.device);
    return GQ_EINVAL;
  }
  std::vector<int32_t> tiles;
  for (int32_t s : g->order) {
    const int32_t n = g->sub_orb_ptr[s + 1] - g->sub_orb_ptr[s];
    const int32_t nt = (n + 63) / 64;
    for (int32_t ti = 0; ti < nt; ++ti)
      for (int32_t tj = 0; tj <= ti; ++tj) {
        tiles.push_back(s);
        tiles.push_back(ti);
        tiles.push_back(tj);
      }
  }
  gq_status st;
  if ((st = dev_upload(&d.sub_orb_ptr, g->sub_orb_ptr)) || (st = dev_upload(&d.sub_orbs, g->sub_orbs)) ||
      (st = dev_upload(&d.n_core, g->n_core_orbs)) || (st = dev_upload(&d.sorted_orbs, g->sorted_orbs)) ||
      (st = dev_upload(&d.sorted_local, g->sorted_local)) || (st = dev_upload(&d.slot, g->slot)) ||
      (st = dev_upload(&d.off2, g->off2)) || (st = dev_upload(&d.offc, g->offc)) ||
      (st = dev_upload(&d.offcd, g->offcd)) || (st = dev_upload(&d.order, g->order)) ||
      (st = dev_upload(&d.rho_row_ptr, g->rho_row_ptr)) || (st = dev_upload(&d.tiles, tiles)) ||
      (st = dev_upload(&d.dc_leaves, g->dc_leaves)) || (st = dev_upload(&d.dc_merges, g->dc_merges)) ||
      (st = dev_upload(&d.dc_tiles, g->dc_tiles)) || (st = dev_upload(&d.bt_toff, g->bt_toff))) {
    graph_free_dev(g);
    return st;
  }
  d.n_tiles = (int32_t)(tiles.size() / 3);
  d.n_leaves = (int32_t)(g->dc_leaves.size() / 3);
  d.device = device;
  return GQ_OK;
}

}  // namespace gq

using namespace gq;

extern "C" {

const char* gq_last_error(void) { return g_err; }

const char* gq_version(void) { return "gq 0.1 (gfx950, FP64)"; }

gq_status gq_ctx_create(int32_t device, void* hip_stream, gq_ctx** out) {
  if (!out) {
    set_error("gq_ctx_create: out is NULL");
    return GQ_EINVAL;
  }
  int count = 0;
  GQ_HIP(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) {
    set_error("gq_ctx_create: device %d not present (%d devices)", device, count);
    return GQ_EINVAL;
  }
  GQ_HIP(hipSetDevice(device));
  hipDeviceProp_t prop;
  GQ_HIP(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    set_error("gq_ctx_create: device %d is %s; this build targets gfx950", device, prop.gcnArchName);
    return GQ_EDEVICE;
  }
  eig_set_attributes();
  dc_set_attributes();
  gq_ctx* c = new (std::nothrow) gq_ctx;
  if (!c) {
    set_error("gq_ctx_create: out of host memory");
    return GQ_ENOMEM;
  }
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  *out = c;
  return GQ_OK;
}

void gq_ctx_destroy(gq_ctx* ctx) { delete ctx; }

gq_status gq_graph_build(int32_t n_atoms, const int32_t* atom_orb_ptr, const gq_csr* H,
                         const gq_csr* rho_prev, const int32_t* core_of_atom, double tau,
                         uint32_t flags, gq_graph** out) {
  if (!out) {
    set_error("gq_graph_build: out is NULL");
    return GQ_EINVAL;
  }
  if (flags & ~(GQ_PATHS2 | GQ_COMPLETE)) {
    set_error("gq_graph_build: unknown flags 0x%x", flags);
    return GQ_EINVAL;
  }
  gq_graph* g = new (std::nothrow) gq_graph;
  if (!g) {
    set_error("gq_graph_build: out of host memory");
    return GQ_ENOMEM;
  }
  gq_status st;
  try {
    st = graph_build_host(n_atoms, atom_orb_ptr, H, rho_prev, core_of_atom, tau, flags, g);
  } catch (const std::bad_alloc&) {
    set_error("gq_graph_build: out of host memory");
    st = GQ_ENOMEM;
  }
  if (st) {
    delete g;
    return st;
  }
  *out = g;
  return GQ_OK;
}

gq_status gq_graph_query(const gq_graph* g, gq_graph_info* info) {
  if (!g || !info) {
    set_error("gq_graph_query: NULL argument");
    return GQ_EINVAL;
  }
  *info = g->info;
  return GQ_OK;
}

gq_status gq_graph_export(const gq_graph* g, int32_t* sub_ptr, int32_t* sub_atoms,
                          int32_t* n_core_atoms, int32_t* sub_orb_ptr, int32_t* sub_orbs,
                          int32_t* n_core_orbs, int32_t* rho_row_ptr, int32_t* rho_col) {
  if (!g) {
    set_error("gq_graph_export: NULL graph");
    return GQ_EINVAL;
  }
  auto cp = [](int32_t* dst, const std::vector<int32_t>& v) {
    if (dst && !v.empty()) std::memcpy(dst, v.data(), v.size() * sizeof(int32_t));
  };
  cp(sub_ptr, g->sub_ptr);
  cp(sub_atoms, g->sub_atoms);
  cp(n_core_atoms, g->n_core_atoms);
  cp(sub_orb_ptr, g->sub_orb_ptr);
  cp(sub_orbs, g->sub_orbs);
  cp(n_core_orbs, g->n_core_orbs);
  cp(rho_row_ptr, g->rho_row_ptr);
  cp(rho_col, g->rho_col);
  return GQ_OK;
}

gq_status gq_graph_block_offsets(const gq_graph* g, int64_t* off) {
  if (!g || !off) {
    set_error("gq_graph_block_offsets: NULL argument");
    return GQ_EINVAL;
  }
  std::memcpy(off, g->offc.data(), g->offc.size() * sizeof(int64_t));
  return GQ_OK;
}

void gq_graph_destroy(gq_graph* g) {
  if (!g) return;
  graph_free_dev(g);
  delete g;
}

static int64_t footprint(const gq_graph* g, int32_t max_k) {
  const gq_graph_info& in = g->info;
  const int64_t sum_c = g->offcd[g->n_sub];
  int64_t b = 0;
  b += 3 * in.sum_n2 * 8;          // A, Q, Y
  b += in.nnz * 8 + in.sum_n * 32 * 8;  // M, T
  b += 5 * in.sum_n * 8;           // eps, wts, dd, ee, tau
  b += (int64_t)g->n_sub * (8 + 4);  // tmu, status
  b += (int64_t)std::max(max_k, 1) * (sum_c + 1) * 8;  // pdiag, mu1
  b += (int64_t)mu_blocks_for(in.sum_n) * kMuPoints * 8 + 16 * 8;
  b += in.sum_n * (4 * 8 + 5 * 4) + (int64_t)(g->dc_merges.size() / 4 + 1) * 4;  // merge metadata
  b += (int64_t)g->bt_nblocks * 256 * 8;                                          // WY factors
  b += in.sum_n * 17 * 8;                                                         // panel scratch, h1
  b += in.sum_n2 * 4;                                                             // FP32 part of Q
  return b;
}

gq_status gq_eigs_footprint(const gq_graph* g, int32_t max_k, int64_t* bytes) {
  if (!g || !bytes || max_k < 0) {
    set_error("gq_eigs_footprint: bad argument");
    return GQ_EINVAL;
  }
  *bytes = footprint(g, max_k);
  return GQ_OK;
}

void gq_eigs_destroy(gq_eigs* e) {
  if (!e) return;
  void* ptrs[] = {e->A, e->Q, e->Y, e->T, e->eps, e->wts, e->dd, e->ee, e->tau, e->M,
                  e->tmu, e->pdiag, e->mu1, e->mu_state, e->mu_part, e->status,
                  e->md_k, e->md_cols, e->md_org, e->md_pos, e->md_dsrc, e->md_dpos,
                  e->md_delta, e->md_tau, e->md_zhat, e->md_inv, e->tfac, e->wsc, e->hloc,
                  e->Q32};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete e;
}

gq_status gq_eigs_create(gq_ctx* ctx, const gq_graph* g, int32_t max_k, gq_eigs** out) {
  if (!ctx || !g || !out || max_k < 0) {
    set_error("gq_eigs_create: bad argument");
    return GQ_EINVAL;
  }
  if (g->info.max_n > kMaxN) {
    set_error("gq_eigs_create: subgraph of %d orbitals exceeds the limit %d", g->info.max_n, kMaxN);
    return GQ_EINVAL;
  }
  if (g->info.max_c > kMaxCore) {
    set_error("gq_eigs_create: core of %d orbitals exceeds the limit %d", g->info.max_c, kMaxCore);
    return GQ_EINVAL;
  }
  GQ_HIP(hipSetDevice(ctx->device));
  if (gq_status st = graph_upload(g, ctx->device)) return st;
  gq_eigs* e = new (std::nothrow) gq_eigs;
  if (!e) {
    set_error("gq_eigs_create: out of host memory");
    return GQ_ENOMEM;
  }
  e->ctx = ctx;
  e->g = g;
  e->max_k = max_k;
  const gq_graph_info& in = g->info;
  const int64_t sum_c = g->offcd[g->n_sub];
  e->mu_blocks = mu_blocks_for(in.sum_n);
  struct Req {
    double** p;
    int64_t count;
  } reqs[] = {{&e->A, in.sum_n2}, {&e->Q, in.sum_n2}, {&e->Y, in.sum_n2}, {&e->T, in.sum_n * 32},
              {&e->M, in.nnz}, {&e->eps, in.sum_n}, {&e->wts, in.sum_n}, {&e->dd, in.sum_n},
              {&e->ee, in.sum_n}, {&e->tau, in.sum_n}, {&e->tmu, g->n_sub},
              {&e->pdiag, (int64_t)std::max(max_k, 1) * std::max<int64_t>(sum_c, 1)},
              {&e->mu1, std::max(max_k, 1)}, {&e->mu_state, 16},
              {&e->mu_part, (int64_t)e->mu_blocks * kMuPoints},
              {&e->md_delta, in.sum_n}, {&e->md_tau, in.sum_n}, {&e->md_zhat, in.sum_n},
              {&e->md_inv, in.sum_n}, {&e->tfac, (int64_t)g->bt_nblocks * 256},
              {&e->wsc, in.sum_n * 16}, {&e->hloc, in.sum_n}};
  for (auto& r : reqs) {
    if (hipMalloc((void**)r.p, std::max<int64_t>(1, r.count) * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      set_error("gq_eigs_create: device allocation of %lld bytes failed",
                (long long)(r.count * 8));
      gq_eigs_destroy(e);
      return GQ_ENOMEM;
    }
  }
  struct ReqI {
    int32_t** p;
    int64_t count;
  } reqi[] = {{&e->status, g->n_sub}, {&e->md_k, (int64_t)(g->dc_merges.size() / 4)},
              {&e->md_cols, in.sum_n}, {&e->md_org, in.sum_n}, {&e->md_pos, in.sum_n},
              {&e->md_dsrc, in.sum_n}, {&e->md_dpos, in.sum_n}};
  for (auto& r : reqi) {
    if (hipMalloc((void**)r.p, std::max<int64_t>(1, r.count) * sizeof(int32_t)) != hipSuccess) {
      (void)hipGetLastError();
      set_error("gq_eigs_create: device allocation failed");
      gq_eigs_destroy(e);
      return GQ_ENOMEM;
    }
  }
  if (hipMalloc((void**)&e->Q32, std::max<int64_t>(1, in.sum_n2) * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    set_error("gq_eigs_create: device allocation failed");
    gq_eigs_destroy(e);
    return GQ_ENOMEM;
  }
  *out = e;
  return GQ_OK;
}

gq_status gq_submatrix_solve(gq_ctx* ctx, const gq_graph* g, const gq_csr* H_dev, uint32_t flags,
                             gq_eigs* e) {
  if (!ctx || !g || !H_dev || !e || e->g != g) {
    set_error("gq_submatrix_solve: bad argument (workspace must belong to this graph)");
    return GQ_EINVAL;
  }
  if (flags != GQ_SOLVE_DEFAULT) {
    set_error("gq_submatrix_solve: unknown flags 0x%x", flags);
    return GQ_EINVAL;
  }
  if (H_dev->n_rows != g->N || !H_dev->row_ptr || !H_dev->col || !H_dev->val) {
    set_error("gq_submatrix_solve: H has %d rows, graph has N = %d", H_dev->n_rows, g->N);
    return GQ_EINVAL;
  }
  GQ_HIP(hipSetDevice(ctx->device));
  launch_gather(ctx, g, H_dev, e->A, e->status);
  launch_eigensolve(ctx, g, e);
  GQ_HIP(hipGetLastError());
  e->have_density = false;
  e->q32_valid = false;
  return GQ_OK;
}

static gq_status check_status(gq_ctx* ctx, const gq_eigs* e) {
  std::vector<int32_t> st(e->g->n_sub);
  GQ_HIP(hipMemcpyAsync(st.data(), e->status, st.size() * sizeof(int32_t), hipMemcpyDeviceToHost,
                        ctx->stream));
  GQ_HIP(hipStreamSynchronize(ctx->stream));
  for (size_t i = 0; i < st.size(); ++i)
    if (st[i]) {
      set_error("eigensolver did not converge on subgraph %zu", i);
      return GQ_ENOCONV;
    }
  return GQ_OK;
}

gq_status gq_density(gq_ctx* ctx, gq_eigs* e, double kT, double n_elec, double* mu_out,
                     double* rho_blocks_dev) {
  if (!ctx || !e) {
    set_error("gq_density: NULL argument");
    return GQ_EINVAL;
  }
  if (!(kT > 0.0)) {
    set_error("gq_density: kT must be > 0 (got %g)", kT);
    return GQ_EINVAL;
  }
  if (!(n_elec > 0.0) || !(n_elec < 2.0 * e->g->N)) {
    set_error("gq_density: N_e = %g outside (0, 2N = %d)", n_elec, 2 * e->g->N);
    return GQ_EINVAL;
  }
  GQ_HIP(hipSetDevice(ctx->device));
  e->kT = kT;
  e->n_elec = n_elec;
  launch_mu(ctx, e->g, e);
  launch_density(ctx, e->g, e, rho_blocks_dev);
  launch_divided_differences(ctx, e->g, e);
  GQ_HIP(hipGetLastError());
  e->have_density = true;
  if (mu_out) {
    GQ_HIP(hipMemcpyAsync(mu_out, e->mu_state + 2, sizeof(double), hipMemcpyDeviceToHost,
                          ctx->stream));
    if (gq_status st = check_status(ctx, e)) return st;
  }
  return GQ_OK;
}

gq_status gq_response(gq_ctx* ctx, gq_eigs* e, const double* h1_dev, int32_t K, uint32_t precision,
                      double* p_blocks_dev, double* mu1_dev, double* mu1_host) {
  if (!ctx || !e || !h1_dev || !p_blocks_dev) {
    set_error("gq_response: NULL argument");
    return GQ_EINVAL;
  }
  if (!e->have_density) {
    set_error("gq_response: call gq_density on this workspace first");
    return GQ_EINVAL;
  }
  if (K < 1 || K > e->max_k) {
    set_error("gq_response: K = %d outside [1, max_k = %d]", K, e->max_k);
    return GQ_EINVAL;
  }
  if (precision != GQ_PREC_FP64 && precision != GQ_PREC_SPLIT32) {
    set_error("gq_response: precision %u not available", precision);
    return GQ_EINVAL;
  }
  GQ_HIP(hipSetDevice(ctx->device));
  launch_response(ctx, e->g, e, h1_dev, K, precision, p_blocks_dev);
  GQ_HIP(hipGetLastError());
  if (mu1_dev)
    GQ_HIP(hipMemcpyAsync(mu1_dev, e->mu1, K * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  if (mu1_host) {
    GQ_HIP(hipMemcpyAsync(mu1_host, e->mu1, K * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    if (gq_status st = check_status(ctx, e)) return st;
  }
  return GQ_OK;
}

gq_status gq_assemble(gq_ctx* ctx, const gq_graph* g, const double* blocks_dev, int32_t K,
                      double* vals_dev) {
  if (!ctx || !g || !blocks_dev || !vals_dev || K < 1) {
    set_error("gq_assemble: bad argument");
    return GQ_EINVAL;
  }
  GQ_HIP(hipSetDevice(ctx->device));
  if (gq_status st = graph_upload(g, ctx->device)) return st;
  launch_assemble(ctx, g, blocks_dev, K, vals_dev);
  GQ_HIP(hipGetLastError());
  return GQ_OK;
}

gq_status gq_eigs_export(gq_ctx* ctx, const gq_eigs* e, double* eps, double* w) {
  if (!ctx || !e) {
    set_error("gq_eigs_export: NULL argument");
    return GQ_EINVAL;
  }
  GQ_HIP(hipSetDevice(ctx->device));
  const size_t bytes = e->g->info.sum_n * sizeof(double);
  if (eps) GQ_HIP(hipMemcpyAsync(eps, e->eps, bytes, hipMemcpyDeviceToHost, ctx->stream));
  if (w) GQ_HIP(hipMemcpyAsync(w, e->wts, bytes, hipMemcpyDeviceToHost, ctx->stream));
  return check_status(ctx, e);
}

gq_status gq_eigs_vectors(const gq_eigs* e, int32_t i, const double** q_dev, int32_t* n) {
  if (!e || !q_dev || !n || i < 0 || i >= e->g->n_sub) {
    set_error("gq_eigs_vectors: bad argument");
    return GQ_EINVAL;
  }
  *q_dev = e->Q + e->g->off2[i];
  *n = e->g->sub_orb_ptr[i + 1] - e->g->sub_orb_ptr[i];
  return GQ_OK;
}

}  // extern "C"

// ------------------------------------------------------------- profiling

namespace gq {

void prof_begin(gq_ctx* ctx, const char* name) {
  if (!ctx->profiling) return;
  gq_prof_rec r{name, nullptr, nullptr};
  if (hipEventCreate(&r.start) != hipSuccess || hipEventCreate(&r.stop) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  (void)hipEventRecord(r.start, ctx->stream);
  ctx->pending.push_back(r);
}

void prof_end(gq_ctx* ctx) {
  if (!ctx->profiling || ctx->pending.empty()) return;
  (void)hipEventRecord(ctx->pending.back().stop, ctx->stream);
}

static void prof_drain(gq_ctx* ctx) {
  for (gq_prof_rec& r : ctx->pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(r.stop) == hipSuccess && hipEventElapsedTime(&ms, r.start, r.stop) == hipSuccess) {
      auto it = std::find_if(ctx->stats.begin(), ctx->stats.end(),
                             [&](const gq_prof_stat& s) { return std::strcmp(s.name, r.name) == 0; });
      if (it == ctx->stats.end()) ctx->stats.push_back({r.name, 1, ms});
      else {
        it->count += 1;
        it->total_ms += ms;
      }
    }
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  ctx->pending.clear();
}

}  // namespace gq

extern "C" {

gq_status gq_ctx_set_profiling(gq_ctx* ctx, int32_t enable) {
  if (!ctx) {
    set_error("gq_ctx_set_profiling: NULL context");
    return GQ_EINVAL;
  }
  GQ_HIP(hipSetDevice(ctx->device));
  prof_drain(ctx);
  ctx->stats.clear();
  ctx->profiling = enable != 0;
  return GQ_OK;
}

gq_status gq_ctx_kernel_times(gq_ctx* ctx, const char** names, int64_t* launches,
                              double* total_ms, int32_t cap, int32_t* count) {
  if (!ctx || !count || cap < 0) {
    set_error("gq_ctx_kernel_times: bad argument");
    return GQ_EINVAL;
  }
  GQ_HIP(hipSetDevice(ctx->device));
  prof_drain(ctx);
  int32_t k = 0;
  for (const gq_prof_stat& s : ctx->stats) {
    if (k >= cap) break;
    if (names) names[k] = s.name;
    if (launches) launches[k] = s.count;
    if (total_ms) total_ms[k] = s.total_ms;
    ++k;
  }
  *count = k;
  return GQ_OK;
}

}  // extern "C"
