// C entry points of libgq: contexts, graphs, eigen workspaces and the five
// calls of the path (graph_build, submatrix_solve, density, response,
// assemble).  No exception crosses this boundary.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <new>
#include <type_traits>

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

// Device arrays carved out of one block, each 256-byte aligned.  With a null
// base only the size is computed.
struct Carve {
  char* base = nullptr;
  size_t used = 0;
  template <class T>
  T* take(int64_t count) {
    const size_t at = (used + 255) & ~size_t(255);
    used = at + (size_t)std::max<int64_t>(1, count) * sizeof(T);
    return base ? reinterpret_cast<T*>(base + at) : nullptr;
  }
};

// Layout of a graph's device maps; copies the host maps in when `upload`.
static gq_status graph_maps(const gq_graph* g, gq_graph_dev& d, Carve& c, bool upload,
                            hipStream_t stream) {
  gq_status st = GQ_OK;
  auto put = [&](auto*& dst, const auto& src) {
    using T = typename std::decay_t<decltype(src)>::value_type;
    dst = c.template take<T>((int64_t)src.size());
    if (upload && st == GQ_OK && !src.empty() &&
        hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, stream) !=
            hipSuccess) {
      set_error("graph upload: %s", hipGetErrorString(hipGetLastError()));
      st = GQ_EDEVICE;
    }
  };
  put(d.sub_orb_ptr, g->sub_orb_ptr);
  put(d.sub_orbs, g->sub_orbs);
  put(d.n_core, g->n_core_orbs);
  put(d.sorted_orbs, g->sorted_orbs);
  put(d.sorted_local, g->sorted_local);
  put(d.slot, g->slot);
  put(d.off2, g->off2);
  put(d.offc, g->offc);
  put(d.offcd, g->offcd);
  put(d.order, g->order);
  put(d.rho_row_ptr, g->rho_row_ptr);
  put(d.dc_leaves, g->dc_leaves);
  put(d.dc_merges, g->dc_merges);
  put(d.dc_tiles, g->dc_tiles);
  put(d.bt_toff, g->bt_toff);
  put(d.xy_tiles[0], g->xy_tiles[0]);
  put(d.xy_tiles[1], g->xy_tiles[1]);
  put(d.tri_tiles, g->tri_tiles);
  d.n_leaves = (int32_t)(g->dc_leaves.size() / 4);  // both size classes
  return st;
}

static int64_t graph_maps_bytes(const gq_graph* g) {
  gq_graph_dev d;
  Carve c;
  (void)graph_maps(g, d, c, false, nullptr);
  return (int64_t)c.used + 256;
}

// Waits for the context's streams, so that a piece of its arena can be
// handed out again (hipFree waits for the device in the same way).
static void ctx_drain(gq_ctx* ctx) {
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->side);
  (void)hipStreamSynchronize(ctx->stream);
}

void graph_free_dev(const gq_graph* g) {
  gq_graph_dev& d = g->dev;
  if (d.arena_ctx) {
    ctx_drain(d.arena_ctx);
    std::lock_guard<std::mutex> lk(d.arena_ctx->arena_mu);
    d.arena_ctx->arena->release(d.arena_off, d.arena_bytes);
  } else if (d.block) {
    (void)hipFree(d.block);
  }
  d = gq_graph_dev{};
}

// Piece of ctx's arena (nullptr when the arena has no room).
static char* arena_take(gq_ctx* ctx, size_t bytes, size_t* off) {
  std::lock_guard<std::mutex> lk(ctx->arena_mu);
  if (!ctx->arena->alloc(bytes, off)) return nullptr;
  return ctx->arena_mem + *off;
}

static void arena_give(gq_ctx* ctx, size_t off, size_t bytes) {
  std::lock_guard<std::mutex> lk(ctx->arena_mu);
  ctx->arena->release(off, bytes);
}

// Binds the graph to `device`: its maps in `mem` (caller-owned, at least
// graph_maps_bytes) or, with mem == NULL, in a block of its own.
static gq_status graph_upload_at(const gq_graph* g, int device, char* mem, hipStream_t stream) {
  gq_graph_dev& d = g->dev;
  if (d.device == device) return GQ_OK;
  if (d.device >= 0) {
    set_error("graph already bound to device %d", d.device);
    return GQ_EINVAL;
  }
  Carve c;
  char* owned = nullptr;
  if (!mem) {
    (void)graph_maps(g, d, c, false, nullptr);
    if (hipMalloc((void**)&owned, c.used + 256) != hipSuccess) {
      (void)hipGetLastError();
      set_error("graph upload: device allocation of %zu bytes failed", c.used);
      d = gq_graph_dev{};
      return GQ_ENOMEM;
    }
    mem = owned;
  }
  c = Carve{};
  c.base = mem;
  gq_status st = graph_maps(g, d, c, true, stream);
  if (st == GQ_OK && hipStreamSynchronize(stream) != hipSuccess) {
    set_error("graph upload: %s", hipGetErrorString(hipGetLastError()));
    st = GQ_EDEVICE;
  }
  if (st) {
    if (owned) (void)hipFree(owned);
    d = gq_graph_dev{};
    return st;
  }
  d.block = owned;
  d.device = device;
  return GQ_OK;
}

gq_status graph_upload(const gq_graph* g, int device) {
  return graph_upload_at(g, device, nullptr, nullptr);
}

// Binds the graph to ctx's device, its maps in a piece of ctx's arena when the
// context has one.
static gq_status graph_upload_ctx(const gq_graph* g, gq_ctx* ctx) {
  if (!ctx->arena || g->dev.device >= 0) return graph_upload_at(g, ctx->device, nullptr, ctx->stream);
  const size_t bytes = (size_t)graph_maps_bytes(g);
  size_t off = 0;
  char* mem = arena_take(ctx, bytes, &off);
  if (!mem) {
    set_error("graph upload: %zu bytes do not fit the context's arena (%zu of %zu in use)", bytes,
              ctx->arena->used(), ctx->arena->size());
    return GQ_ENOMEM;
  }
  if (gq_status st = graph_upload_at(g, ctx->device, mem, ctx->stream)) {
    arena_give(ctx, off, bytes);
    return st;
  }
  g->dev.arena_ctx = ctx;
  g->dev.arena_off = off;
  g->dev.arena_bytes = bytes;
  return GQ_OK;
}

// Layout of an eigen workspace (pointers filled when c.base is set).
static void eigs_layout(gq_eigs* e, const gq_graph* g, int32_t max_k, uint32_t flags, Carve& c) {
  const gq_graph_info& in = g->info;
  const int64_t sum_c = g->offcd[g->n_sub];
  const int64_t kk = std::max(max_k, 1);
  gq_eigs tmp;
  gq_eigs& x = e ? *e : tmp;
  x.mu_blocks = mu_blocks_for(in.sum_n);
  x.A = c.take<double>(in.sum_n2);
  x.Q = c.take<double>(in.sum_n2);
  x.Y = c.take<double>(kk * in.sum_n2);
  x.T = c.take<double>(kk * in.sum_n * 32);
  x.M = c.take<double>(in.nnz);
  x.eps = c.take<double>(in.sum_n);
  x.wts = c.take<double>(in.sum_n);
  x.dd = c.take<double>(in.sum_n);
  x.ee = c.take<double>(in.sum_n);
  x.tau = c.take<double>(in.sum_n);
  x.tmu = c.take<double>(g->n_sub);
  x.pdiag = c.take<double>(kk * std::max<int64_t>(sum_c, 1));
  x.mu1 = c.take<double>(kk);
  x.mu_state = c.take<double>(16);
  x.mu_part = c.take<double>((int64_t)x.mu_blocks * kMuPoints);
  x.md_delta = c.take<double>(in.sum_n);
  x.md_tau = c.take<double>(in.sum_n);
  x.md_zhat = c.take<double>(in.sum_n);
  x.md_inv = c.take<double>(in.sum_n);
  x.tfac = c.take<double>((int64_t)g->bt_nblocks * 256);
  x.wsc = c.take<double>(in.sum_n * 16);
  x.mwg = g->n_mwg ? c.take<double>((int64_t)g->n_mwg * kMwgSlot) : nullptr;
  x.dcg = g->dc_nglob_max
              ? c.take<double>((int64_t)g->dc_nglob_max * kMaxN * kDcGlobalStride)
              : nullptr;
  x.hloc = c.take<double>(kk * in.sum_n);
  x.G = (flags & GQ_EIGS_GENERAL_H1) ? c.take<double>(kk * in.sum_n2) : nullptr;
  x.Z = (flags & GQ_EIGS_OVERLAP) ? c.take<double>(in.sum_n2) : nullptr;
  x.C = (flags & GQ_EIGS_OVERLAP) ? c.take<double>(in.sum_n2) : nullptr;
  x.Q32 = c.take<float>(in.sum_n2);
  x.status = c.take<int32_t>(g->n_sub);
  x.wflag = c.take<int32_t>(g->n_sub);
  x.md_k = c.take<int32_t>((int64_t)(g->dc_merges.size() / 4));
  x.md_cols = c.take<int32_t>(in.sum_n);
  x.md_org = c.take<int32_t>(in.sum_n);
  x.md_pos = c.take<int32_t>(in.sum_n);
  x.md_dsrc = c.take<int32_t>(in.sum_n);
  x.md_dpos = c.take<int32_t>(in.sum_n);
}

static int64_t eigs_bytes(const gq_graph* g, int32_t max_k, uint32_t flags) {
  Carve c;
  eigs_layout(nullptr, g, max_k, flags, c);
  return (int64_t)c.used + 256;
}

}  // namespace gq

using namespace gq;

extern "C" {

const char* gq_last_error(void) { return g_err; }

const char* gq_version(void) { return "gq 0.1 (gfx950, FP64)"; }

gq_status gq_ctx_create(int32_t device, void* hip_stream, int64_t arena_bytes, gq_ctx** out) {
  if (!out || arena_bytes < 0) {
    set_error("gq_ctx_create: out is NULL or arena_bytes < 0");
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
    set_error("gq_ctx_create: device %d is %s; libgq targets gfx950", device, prop.gcnArchName);
    return GQ_EDEVICE;
  }
  eig_set_attributes();
  dc_set_attributes();
  if (gq_status st = scratch_init(device)) return st;
  gq_ctx* c = new (std::nothrow) gq_ctx;
  if (!c) {
    set_error("gq_ctx_create: out of host memory");
    return GQ_ENOMEM;
  }
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_fork_dd, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_join_dd, hipEventDisableTiming) != hipSuccess) {
    set_error("gq_ctx_create: cannot create the side stream and its events");
    gq_ctx_destroy(c);
    return GQ_EDEVICE;
  }
  if (arena_bytes > 0) {
    if (hipMalloc((void**)&c->arena_mem, (size_t)arena_bytes) != hipSuccess) {
      (void)hipGetLastError();
      c->arena_mem = nullptr;
      set_error("gq_ctx_create: arena of %lld bytes not available", (long long)arena_bytes);
      gq_ctx_destroy(c);
      return GQ_ENOMEM;
    }
    c->arena = new (std::nothrow) Arena((size_t)arena_bytes);
    if (!c->arena) {
      set_error("gq_ctx_create: out of host memory");
      gq_ctx_destroy(c);
      return GQ_ENOMEM;
    }
  }
  *out = c;
  return GQ_OK;
}

gq_status gq_ctx_arena_used(gq_ctx* ctx, int64_t* used, int64_t* size) {
  if (!ctx) {
    set_error("gq_ctx_arena_used: NULL context");
    return GQ_EINVAL;
  }
  std::lock_guard<std::mutex> lk(ctx->arena_mu);
  if (used) *used = ctx->arena ? (int64_t)ctx->arena->used() : 0;
  if (size) *size = ctx->arena ? (int64_t)ctx->arena->size() : 0;
  return GQ_OK;
}

void gq_ctx_destroy(gq_ctx* ctx) {
  if (!ctx) return;
  if (ctx->arena_mem) {
    (void)hipSetDevice(ctx->device);
    (void)hipFree(ctx->arena_mem);
  }
  delete ctx->arena;
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  if (ctx->ev_fork_dd) (void)hipEventDestroy(ctx->ev_fork_dd);
  if (ctx->ev_join_dd) (void)hipEventDestroy(ctx->ev_join_dd);
  if (ctx->side) (void)hipStreamDestroy(ctx->side);
  delete ctx;
}

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
  auto cp = [](int32_t* dst, const auto& v) {
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

// Device bytes of a workspace plus the graph's device maps.
static int64_t footprint(const gq_graph* g, int32_t max_k, uint32_t flags) {
  return eigs_bytes(g, max_k, flags) + graph_maps_bytes(g);
}

gq_status gq_eigs_footprint(const gq_graph* g, int32_t max_k, uint32_t flags, int64_t* bytes) {
  if (!g || !bytes || max_k < 0 || (flags & ~(GQ_EIGS_GENERAL_H1 | GQ_EIGS_OVERLAP))) {
    set_error("gq_eigs_footprint: bad argument");
    return GQ_EINVAL;
  }
  *bytes = footprint(g, max_k, flags);
  return GQ_OK;
}

void gq_eigs_destroy(gq_eigs* e) {
  if (!e) return;
  if (e->block_in_arena) {
    ctx_drain(e->ctx);
    arena_give(e->ctx, e->arena_off, e->arena_bytes);
  }
  else if (e->block) (void)hipFree(e->block);
  delete e;
}

static gq_status eigs_check(gq_ctx* ctx, const gq_graph* g, int32_t max_k, uint32_t flags,
                            gq_eigs** out, const char* who) {
  if (!ctx || !g || !out || max_k < 0) {
    set_error("%s: bad argument", who);
    return GQ_EINVAL;
  }
  if (flags & ~(GQ_EIGS_GENERAL_H1 | GQ_EIGS_OVERLAP)) {
    set_error("%s: unknown flags 0x%x", who, flags);
    return GQ_EINVAL;
  }
  if (g->info.max_n > kMaxN) {
    set_error("%s: subgraph of %d orbitals exceeds the limit %d", who, g->info.max_n, kMaxN);
    return GQ_EINVAL;
  }
  if (g->info.max_c > kMaxCore) {
    set_error("%s: core of %d orbitals exceeds the limit %d", who, g->info.max_c, kMaxCore);
    return GQ_EINVAL;
  }
  return GQ_OK;
}

// mem: caller memory; otherwise a piece of ctx's arena or a block of its own.
static gq_status eigs_make(gq_ctx* ctx, const gq_graph* g, int32_t max_k, uint32_t flags,
                           char* mem, gq_eigs** out) {
  gq_eigs* e = new (std::nothrow) gq_eigs;
  if (!e) {
    set_error("gq_eigs_create: out of host memory");
    return GQ_ENOMEM;
  }
  e->ctx = ctx;
  e->g = g;
  e->max_k = max_k;
  e->flags = flags;
  if (!mem) {
    const size_t bytes = (size_t)eigs_bytes(g, max_k, flags);
    if (ctx->arena) {
      e->block = arena_take(ctx, bytes, &e->arena_off);
      if (!e->block) {
        set_error("gq_eigs_create: %zu bytes do not fit the context's arena (%zu of %zu in use)",
                  bytes, ctx->arena->used(), ctx->arena->size());
        delete e;
        return GQ_ENOMEM;
      }
      e->block_in_arena = true;
      e->arena_bytes = bytes;
    } else if (hipMalloc((void**)&e->block, bytes) != hipSuccess) {
      (void)hipGetLastError();
      set_error("gq_eigs_create: device allocation of %zu bytes failed", bytes);
      delete e;
      return GQ_ENOMEM;
    }
    mem = e->block;
  }
  Carve c;
  c.base = mem;
  eigs_layout(e, g, max_k, flags, c);
  *out = e;
  return GQ_OK;
}

gq_status gq_eigs_create(gq_ctx* ctx, const gq_graph* g, int32_t max_k, uint32_t flags,
                         gq_eigs** out) {
  if (gq_status st = eigs_check(ctx, g, max_k, flags, out, "gq_eigs_create")) return st;
  GQ_HIP(hipSetDevice(ctx->device));
  if (gq_status st = graph_upload_ctx(g, ctx)) return st;
  return eigs_make(ctx, g, max_k, flags, nullptr, out);
}

gq_status gq_eigs_create_in(gq_ctx* ctx, const gq_graph* g, int32_t max_k, uint32_t flags,
                            void* mem, int64_t bytes, gq_eigs** out) {
  if (gq_status st = eigs_check(ctx, g, max_k, flags, out, "gq_eigs_create_in")) return st;
  if (!mem || bytes < footprint(g, max_k, flags)) {
    set_error("gq_eigs_create_in: %lld bytes given, %lld needed", (long long)bytes,
              (long long)footprint(g, max_k, flags));
    return GQ_EINVAL;
  }
  if (reinterpret_cast<uintptr_t>(mem) % 256) {
    set_error("gq_eigs_create_in: memory must be 256-byte aligned");
    return GQ_EINVAL;
  }
  GQ_HIP(hipSetDevice(ctx->device));
  char* base = static_cast<char*>(mem);
  const bool bind = g->dev.device < 0;
  if (bind) {
    if (gq_status st = graph_upload_at(g, ctx->device, base, ctx->stream)) return st;
  } else if (g->dev.device != ctx->device) {
    set_error("gq_eigs_create_in: graph bound to device %d", g->dev.device);
    return GQ_EINVAL;
  }
  return eigs_make(ctx, g, max_k, flags, base + graph_maps_bytes(g), out);
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
  e->overlap_solved = false;
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

gq_status gq_submatrix_solve_overlap(gq_ctx* ctx, const gq_graph* g, const gq_csr* H_dev,
                                     const gq_csr* S_dev, uint32_t flags, gq_eigs* e) {
  if (!ctx || !g || !H_dev || !S_dev || !e || e->g != g) {
    set_error("gq_submatrix_solve_overlap: bad argument (workspace must belong to this graph)");
    return GQ_EINVAL;
  }
  if (flags != GQ_SOLVE_DEFAULT) {
    set_error("gq_submatrix_solve_overlap: unknown flags 0x%x", flags);
    return GQ_EINVAL;
  }
  if (!e->Z) {
    set_error("gq_submatrix_solve_overlap: the workspace was created without GQ_EIGS_OVERLAP");
    return GQ_EINVAL;
  }
  for (const gq_csr* m : {H_dev, S_dev})
    if (m->n_rows != g->N || !m->row_ptr || !m->col || !m->val) {
      set_error("gq_submatrix_solve_overlap: %s has %d rows, graph has N = %d",
                m == H_dev ? "H" : "S", m->n_rows, g->N);
      return GQ_EINVAL;
    }
  if (ctx->capturing) {
    set_error("gq_submatrix_solve_overlap: not available while capturing (it waits for the "
              "stream to check the overlap)");
    return GQ_EINVAL;
  }
  GQ_HIP(hipSetDevice(ctx->device));
  e->have_density = false;
  e->q32_valid = false;
  e->overlap_solved = false;
  // the overlap submatrices: eigenpairs, then their smallest eigenvalues
  launch_gather(ctx, g, S_dev, e->A, e->status, "k_s_gather");
  launch_eigensolve(ctx, g, e);
  launch_overlap_min(ctx, g, e, e->tmu);
  GQ_HIP(hipGetLastError());
  gq_status rc = check_status(ctx, e);
  if (rc != GQ_OK) return rc;
  std::vector<double> smin(g->n_sub);
  GQ_HIP(hipMemcpy(smin.data(), e->tmu, smin.size() * sizeof(double), hipMemcpyDeviceToHost));
  for (int32_t i = 0; i < g->n_sub; ++i)
    if (!(smin[i] > 0.0)) {
      set_error("gq_submatrix_solve_overlap: overlap submatrix of subgraph %d is not positive "
                "definite (smallest eigenvalue %g)", i, smin[i]);
      return GQ_EINVAL;
    }
  launch_overlap_factor(ctx, g, e);
  launch_gather(ctx, g, H_dev, e->A, e->status);
  launch_overlap_congruence(ctx, g, e);
  launch_eigensolve(ctx, g, e);
  launch_overlap_vectors(ctx, g, e);
  GQ_HIP(hipGetLastError());
  e->overlap_solved = true;
  return GQ_OK;
}

gq_status gq_density(gq_ctx* ctx, gq_eigs* e, double kT, double n_elec, double* mu_inout,
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
  if (mu_inout && ctx->capturing) {
    set_error("gq_density: mu_inout must be NULL while capturing");
    return GQ_EINVAL;
  }
  GQ_HIP(hipSetDevice(ctx->device));
  e->kT = kT;
  e->n_elec = n_elec;
  const double guess = mu_inout ? *mu_inout : std::numeric_limits<double>::quiet_NaN();
  launch_mu(ctx, e->g, e, guess);
  // the divided differences (eigenvalues and mu only, written over the
  // reflectors in A) run on the side stream beside the density rows (Q, into
  // rho), joined back before the call returns
  GQ_HIP(hipEventRecord(ctx->ev_fork_dd, ctx->stream));
  GQ_HIP(hipStreamWaitEvent(ctx->side, ctx->ev_fork_dd, 0));
  launch_divided_differences(ctx, e->g, e, ctx->side);
  launch_density(ctx, e->g, e, rho_blocks_dev);
  GQ_HIP(hipEventRecord(ctx->ev_join_dd, ctx->side));
  GQ_HIP(hipStreamWaitEvent(ctx->stream, ctx->ev_join_dd, 0));
  GQ_HIP(hipGetLastError());
  e->have_density = true;
  if (mu_inout) {
    GQ_HIP(hipMemcpyAsync(mu_inout, e->mu_state + 2, sizeof(double), hipMemcpyDeviceToHost,
                          ctx->stream));
    if (gq_status st = check_status(ctx, e)) return st;
  }
  return GQ_OK;
}

// Validation shared by the response entry points.
static gq_status response_check(gq_ctx* ctx, gq_eigs* e, const void* h1, uint32_t kind,
                                int32_t K, uint32_t precision, double* p_blocks_dev,
                                const char* who, H1Spec* spec) {
  if (!ctx || !e || !h1 || !p_blocks_dev) {
    set_error("%s: NULL argument", who);
    return GQ_EINVAL;
  }
  if (!e->have_density) {
    set_error("%s: call gq_density on this workspace first", who);
    return GQ_EINVAL;
  }
  if (precision != GQ_PREC_FP64 && precision != GQ_PREC_SPLIT32) {
    set_error("%s: precision %u not available", who, precision);
    return GQ_EINVAL;
  }
  if (e->overlap_solved && precision != GQ_PREC_FP64) {
    set_error("%s: a non-orthogonal basis takes FP64 congruences only", who);
    return GQ_EINVAL;
  }
  if (K < 1) {
    set_error("%s: K = %d < 1", who, K);
    return GQ_EINVAL;
  }
  *spec = H1Spec{kind, nullptr, nullptr};
  if (kind == GQ_H1_DIAG) {
    spec->diag = static_cast<const double*>(h1);
  } else if (kind == GQ_H1_CSR) {
    spec->csr = static_cast<const gq_csr*>(h1);
    for (int32_t q = 0; q < K; ++q) {
      const gq_csr& m = spec->csr[q];
      if (m.n_rows != e->g->N || m.nnz < 0 || !m.row_ptr || (m.nnz > 0 && (!m.col || !m.val))) {
        set_error("%s: perturbation %d: %d rows (N = %d) or missing arrays", who, q, m.n_rows,
                  e->g->N);
        return GQ_EINVAL;
      }
    }
  } else {
    set_error("%s: unknown perturbation kind %u", who, kind);
    return GQ_EINVAL;
  }
  return GQ_OK;
}

gq_status gq_response(gq_ctx* ctx, gq_eigs* e, const void* h1, uint32_t h1_kind, int32_t K,
                      uint32_t precision, double* p_blocks_dev, double* mu1_dev,
                      double* mu1_host) {
  H1Spec spec;
  if (gq_status st = response_check(ctx, e, h1, h1_kind, K, precision, p_blocks_dev,
                                    "gq_response", &spec))
    return st;
  if (K > e->max_k) {
    set_error("gq_response: K = %d above max_k = %d", K, e->max_k);
    return GQ_EINVAL;
  }
  if (h1_kind == GQ_H1_CSR && !e->G) {
    set_error("gq_response: CSR perturbations need a workspace created with GQ_EIGS_GENERAL_H1");
    return GQ_EINVAL;
  }
  if (mu1_host && ctx->capturing) {
    set_error("gq_response: mu1_host must be NULL while capturing");
    return GQ_EINVAL;
  }
  GQ_HIP(hipSetDevice(ctx->device));
  const RespBufs rb{e->hloc, e->Y, e->G, e->T, e->pdiag, e->mu1};
  launch_response(ctx, e->g, e, rb, spec, K, precision, p_blocks_dev);
  GQ_HIP(hipGetLastError());
  if (mu1_dev)
    GQ_HIP(hipMemcpyAsync(mu1_dev, e->mu1, K * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  if (mu1_host) {
    GQ_HIP(hipMemcpyAsync(mu1_host, e->mu1, K * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    if (gq_status st = check_status(ctx, e)) return st;
  }
  return GQ_OK;
}

gq_status gq_response_static(gq_ctx* ctx, gq_eigs* e, const void* h1, uint32_t h1_kind,
                             int32_t K, uint32_t precision, double* p_blocks_dev,
                             double* mu1_dev) {
  H1Spec spec;
  if (gq_status st = response_check(ctx, e, h1, h1_kind, K, precision, p_blocks_dev,
                                    "gq_response_static", &spec))
    return st;
  double* base = scratch_ptr(ctx->device);
  if (!base) {
    set_error("gq_response_static: no static scratch on device %d", ctx->device);
    return GQ_EDEVICE;
  }
  const gq_graph* g = e->g;
  const int64_t per_k = resp_doubles_per_k(g, h1_kind);
  const int64_t cap = scratch_doubles();
  if (per_k > cap) {
    set_error("gq_response_static: one perturbation needs %lld doubles of scratch, the static "
              "scratch holds %lld (sum n_i^2 = %lld)",
              (long long)per_k, (long long)cap, (long long)g->info.sum_n2);
    return GQ_ENOMEM;
  }
  GQ_HIP(hipSetDevice(ctx->device));
  const int64_t sum_n = g->info.sum_n, sum_n2 = g->info.sum_n2, nnz = g->info.nnz;
  const int64_t sum_c = std::max<int64_t>(g->offcd[g->n_sub], 1);
  auto up = [](int64_t x) { return (x + 31) & ~int64_t(31); };
  const int32_t kc = (int32_t)std::min<int64_t>(K, cap / per_k);
  for (int32_t q0 = 0; q0 < K; q0 += kc) {
    const int32_t nq = std::min(kc, K - q0);
    // carve nq perturbations' buffers out of the scratch (the layout that
    // resp_doubles_per_k counts, for nq at once)
    double* at = base;
    auto take = [&](int64_t count) {
      double* p = at;
      at += up(count);
      return p;
    };
    RespBufs rb;
    rb.hloc = take(nq * sum_n);
    rb.Y = take(nq * sum_n2);
    rb.G = h1_kind == GQ_H1_CSR ? take(nq * sum_n2) : nullptr;
    rb.T = take(nq * sum_n * 32);
    rb.pdiag = take(nq * sum_c);
    rb.mu1 = take(nq);
    H1Spec sub = spec;
    if (h1_kind == GQ_H1_DIAG) sub.diag = spec.diag + (size_t)q0 * g->N;
    else sub.csr = spec.csr + q0;
    launch_response(ctx, g, e, rb, sub, nq, precision, p_blocks_dev + (size_t)q0 * nnz);
    GQ_HIP(hipGetLastError());
    if (mu1_dev)
      GQ_HIP(hipMemcpyAsync(mu1_dev + q0, rb.mu1, nq * sizeof(double), hipMemcpyDeviceToDevice,
                            ctx->stream));
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
  if (ctx->capturing) {
    set_error("gq_eigs_export: not available while capturing");
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

void prof_begin_on(gq_ctx* ctx, const char* name, hipStream_t st) {
  if (!ctx->profiling || ctx->capturing) return;
  gq_prof_rec r{name, nullptr, nullptr, st};
  if (hipEventCreate(&r.start) != hipSuccess || hipEventCreate(&r.stop) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  (void)hipEventRecord(r.start, st);
  ctx->pending.push_back(r);
}

void prof_begin(gq_ctx* ctx, const char* name) { prof_begin_on(ctx, name, ctx->stream); }

void prof_end(gq_ctx* ctx) {
  if (!ctx->profiling || ctx->capturing || ctx->pending.empty()) return;
  (void)hipEventRecord(ctx->pending.back().stop, ctx->pending.back().stream);
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

struct gq_exec {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int device = 0;
};

gq_status gq_autotune(gq_ctx* ctx, gq_eigs* e, uint32_t precision, char* report,
                      size_t report_len) {
  if (!ctx || !e) {
    set_error("gq_autotune: NULL argument");
    return GQ_EINVAL;
  }
  if (ctx->capturing) {
    set_error("gq_autotune: not available while capturing");
    return GQ_EINVAL;
  }
  if (!e->have_density) {
    set_error("gq_autotune: call gq_density on this workspace first");
    return GQ_EINVAL;
  }
  if (precision != GQ_PREC_FP64 && precision != GQ_PREC_SPLIT32) {
    set_error("gq_autotune: precision %u not available", precision);
    return GQ_EINVAL;
  }
  GQ_HIP(hipSetDevice(ctx->device));
  std::string text;
  gq_status st = autotune_xy(ctx, e->g, e, precision, &text);
  if (report && report_len > 0) {
    const size_t m = std::min(report_len - 1, text.size());
    std::memcpy(report, text.data(), m);
    report[m] = 0;
  }
  return st;
}

gq_status gq_graph_set_launch(const gq_graph* g, uint32_t precision, int32_t bin,
                              int32_t variant) {
  if (!g || (precision != GQ_PREC_FP64 && precision != GQ_PREC_SPLIT32) || bin < 0 ||
      bin >= kXyBins || variant < 0 || variant > 3) {
    set_error("gq_graph_set_launch: bad argument");
    return GQ_EINVAL;
  }
  g->xy_choice[precision == GQ_PREC_SPLIT32 ? 1 : 0][bin] = (int8_t)variant;
  return GQ_OK;
}

gq_status gq_capture_begin(gq_ctx* ctx) {
  if (!ctx) {
    set_error("gq_capture_begin: NULL context");
    return GQ_EINVAL;
  }
  if (ctx->capturing) {
    set_error("gq_capture_begin: already capturing");
    return GQ_EINVAL;
  }
  if (ctx->stream == nullptr) {
    set_error("gq_capture_begin: the legacy default stream cannot be captured; create the "
              "context on a stream of its own");
    return GQ_EINVAL;
  }
  GQ_HIP(hipSetDevice(ctx->device));
  GQ_HIP(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
  ctx->capturing = true;
  return GQ_OK;
}

gq_status gq_capture_end(gq_ctx* ctx, gq_exec** out) {
  if (!ctx || !out) {
    set_error("gq_capture_end: NULL argument");
    return GQ_EINVAL;
  }
  if (!ctx->capturing) {
    set_error("gq_capture_end: not capturing");
    return GQ_EINVAL;
  }
  ctx->capturing = false;
  GQ_HIP(hipSetDevice(ctx->device));
  hipGraph_t graph = nullptr;
  GQ_HIP(hipStreamEndCapture(ctx->stream, &graph));
  gq_exec* x = new (std::nothrow) gq_exec;
  if (!x) {
    (void)hipGraphDestroy(graph);
    set_error("gq_capture_end: out of host memory");
    return GQ_ENOMEM;
  }
  x->graph = graph;
  x->device = ctx->device;
  if (hipGraphInstantiate(&x->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    set_error("gq_capture_end: hipGraphInstantiate failed: %s",
              hipGetErrorString(hipGetLastError()));
    (void)hipGraphDestroy(graph);
    delete x;
    return GQ_EDEVICE;
  }
  *out = x;
  return GQ_OK;
}

gq_status gq_exec_launch(gq_ctx* ctx, gq_exec* x) {
  if (!ctx || !x) {
    set_error("gq_exec_launch: NULL argument");
    return GQ_EINVAL;
  }
  if (ctx->capturing) {
    set_error("gq_exec_launch: not available while capturing");
    return GQ_EINVAL;
  }
  GQ_HIP(hipSetDevice(ctx->device));
  GQ_HIP(hipGraphLaunch(x->exec, ctx->stream));
  return GQ_OK;
}

void gq_exec_destroy(gq_exec* x) {
  if (!x) return;
  if (x->exec) (void)hipGraphExecDestroy(x->exec);
  if (x->graph) (void)hipGraphDestroy(x->graph);
  delete x;
}

gq_status gq_ctx_set_iteration_cap(gq_ctx* ctx, int32_t leaf_iterations) {
  if (!ctx || leaf_iterations < 0) {
    set_error("gq_ctx_set_iteration_cap: bad argument");
    return GQ_EINVAL;
  }
  ctx->leaf_iter_cap = leaf_iterations;
  return GQ_OK;
}

gq_status gq_ctx_set_split_window(gq_ctx* ctx, double dF_threshold, int32_t max_states) {
  if (!ctx || !(dF_threshold > 0.0) || max_states < 0) {
    set_error("gq_ctx_set_split_window: bad argument");
    return GQ_EINVAL;
  }
  ctx->win_dF = dF_threshold;
  ctx->win_cap = max_states;
  return GQ_OK;
}

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
  if (ctx->capturing) {
    set_error("gq_ctx_kernel_times: not available while capturing");
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
