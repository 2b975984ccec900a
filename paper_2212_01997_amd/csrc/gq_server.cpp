// Serving runtime: continuous admission of whole-path requests on one GPU.
//
// Each request is one system (H, previous density, cores) with K diagonal
// perturbations; the runtime builds its graph (Sec. II.E), solves every
// subgraph (Fig. 1, Eq. (SmallKS)), fixes mu (Sec. II.G), applies the K
// perturbations to the one device-resident eigenbasis (Sec. IV.A) and collects
// rho and rho1 (Eqs. (sub_f), (D1)).
//
// Design: one device arena allocated at start; n_slots executor threads, each
// with a HIP stream (default priority) and a context of its own.  A thread
// takes the oldest waiting request, builds its graph on the host, sizes its
// footprint (workspace + graph maps + inputs and outputs) and waits until the
// arena has a contiguous piece of that size; the request is then admitted and
// its kernels run on the thread's stream, overlapping with the requests of the
// other threads.  Completion frees the piece and wakes waiting threads.  No
// device memory is allocated or freed after start, so no call of the serving
// loop synchronises the device.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "gq_internal.hpp"

namespace gq {
namespace {

struct Request {
  int64_t id = 0;
  // inputs (owned copies)
  int32_t n_atoms = 0, N = 0, K = 0;
  std::vector<int32_t> atom_orb_ptr, core;
  std::vector<int32_t> h_rp, h_col, p_rp, p_col;
  std::vector<double> h_val, p_val, h1;
  bool has_prev = false;
  double tau = 0, kT = 0, n_elec = 0;
  uint32_t flags = 0, precision = 0;
  // outputs
  gq_status status = GQ_OK;
  std::string error;
  double mu = 0;
  std::vector<double> mu1, rho, rho1;
  std::vector<int32_t> rho_row_ptr, rho_col;
  int32_t n_sub = 0;
  int64_t nnz = 0, footprint = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  bool done = false;
};

}  // namespace
}  // namespace gq

using namespace gq;

struct gq_server {
  int device = 0;
  char* arena_mem = nullptr;
  std::unique_ptr<Arena> arena;
  std::mutex mu;
  std::condition_variable cv_queue, cv_mem, cv_done;
  std::deque<std::shared_ptr<Request>> queue;
  std::unordered_map<int64_t, std::shared_ptr<Request>> reqs;
  int64_t next_id = 1;
  bool stop = false;
  std::vector<std::thread> workers;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  void worker();
  void run(Request& r, gq_ctx* ctx);
};

namespace {

struct Fail {
  gq_status st;
};

void ok(gq_status st) {
  if (st != GQ_OK) throw Fail{st};
}

void hip_ok(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    set_error("%s: %s", what, hipGetErrorString(e));
    throw Fail{GQ_EDEVICE};
  }
}

}  // namespace

void gq_server::run(Request& r, gq_ctx* ctx) {
  // graph estimate on the host (this thread)
  gq_csr H{r.N, (int32_t)r.h_col.size(), r.h_rp.data(), r.h_col.data(), r.h_val.data()};
  gq_csr P{r.N, (int32_t)r.p_col.size(), r.p_rp.data(), r.p_col.data(), r.p_val.data()};
  gq_graph* g = nullptr;
  ok(gq_graph_build(r.n_atoms, r.atom_orb_ptr.data(), &H, r.has_prev ? &P : nullptr,
                    r.core.data(), r.tau, r.flags, &g));
  std::unique_ptr<gq_graph, void (*)(gq_graph*)> gh(g, gq_graph_destroy);
  const int64_t nnz = g->info.nnz;
  r.n_sub = g->n_sub;
  r.nnz = nnz;
  int64_t ws = 0;
  ok(gq_eigs_footprint(g, r.K, 0u, &ws));
  // footprint: workspace + graph maps, H, h1, rho blocks and values, P blocks and rho1
  size_t bytes = arena_align((size_t)ws);
  const size_t o_hrp = bytes;
  bytes = arena_align(bytes + r.h_rp.size() * 4);
  const size_t o_hcol = bytes;
  bytes = arena_align(bytes + r.h_col.size() * 4);
  const size_t o_hval = bytes;
  bytes = arena_align(bytes + r.h_val.size() * 8);
  const size_t o_h1 = bytes;
  bytes = arena_align(bytes + r.h1.size() * 8);
  const size_t o_rb = bytes;
  bytes = arena_align(bytes + (size_t)nnz * 8);
  const size_t o_rho = bytes;
  bytes = arena_align(bytes + (size_t)nnz * 8);
  const size_t o_pb = bytes;
  bytes = arena_align(bytes + (size_t)r.K * nnz * 8);
  const size_t o_rho1 = bytes;
  bytes = arena_align(bytes + (size_t)r.K * nnz * 8);
  r.footprint = (int64_t)bytes;
  if (bytes > arena->size()) {
    set_error("request %lld needs %zu bytes, the arena holds %zu", (long long)r.id, bytes,
              arena->size());
    throw Fail{GQ_ENOMEM};
  }
  // admission: wait for a contiguous piece of the arena
  size_t off = 0;
  {
    std::unique_lock<std::mutex> lk(mu);
    cv_mem.wait(lk, [&] { return stop || arena->alloc(bytes, &off); });
    if (stop) throw Fail{GQ_EBUSY};
  }
  r.t_admit = now();
  struct Piece {
    gq_server* s;
    size_t off, bytes;
    hipStream_t stream;
    ~Piece() {
      // the piece is reused only after every kernel of this request has ended
      (void)hipStreamSynchronize(stream);
      {
        std::lock_guard<std::mutex> lk(s->mu);
        s->arena->release(off, bytes);
      }
      s->cv_mem.notify_all();
    }
  } piece{this, off, bytes, ctx->stream};
  char* base = arena_mem + off;
  gq_eigs* e = nullptr;
  ok(gq_eigs_create_in(ctx, g, r.K, 0u, base, ws, &e));
  std::unique_ptr<gq_eigs, void (*)(gq_eigs*)> eh(e, gq_eigs_destroy);
  hipStream_t st = ctx->stream;
  hip_ok(hipMemcpyAsync(base + o_hrp, r.h_rp.data(), r.h_rp.size() * 4, hipMemcpyHostToDevice, st),
         "upload H");
  hip_ok(hipMemcpyAsync(base + o_hcol, r.h_col.data(), r.h_col.size() * 4, hipMemcpyHostToDevice,
                        st),
         "upload H");
  hip_ok(hipMemcpyAsync(base + o_hval, r.h_val.data(), r.h_val.size() * 8, hipMemcpyHostToDevice,
                        st),
         "upload H");
  hip_ok(hipMemcpyAsync(base + o_h1, r.h1.data(), r.h1.size() * 8, hipMemcpyHostToDevice, st),
         "upload h1");
  gq_csr Hd{r.N, (int32_t)r.h_col.size(), reinterpret_cast<const int32_t*>(base + o_hrp),
            reinterpret_cast<const int32_t*>(base + o_hcol),
            reinterpret_cast<const double*>(base + o_hval)};
  double* rb = reinterpret_cast<double*>(base + o_rb);
  double* rho = reinterpret_cast<double*>(base + o_rho);
  double* pb = reinterpret_cast<double*>(base + o_pb);
  double* rho1 = reinterpret_cast<double*>(base + o_rho1);
  ok(gq_submatrix_solve(ctx, g, &Hd, GQ_SOLVE_DEFAULT, e));
  r.mu = std::numeric_limits<double>::quiet_NaN();  // no warm start
  ok(gq_density(ctx, e, r.kT, r.n_elec, &r.mu, rb));
  r.mu1.assign(r.K, 0.0);
  ok(gq_response(ctx, e, base + o_h1, GQ_H1_DIAG, r.K, r.precision, pb, nullptr, r.mu1.data()));
  ok(gq_assemble(ctx, g, rb, 1, rho));
  ok(gq_assemble(ctx, g, pb, r.K, rho1));
  r.rho.resize(nnz);
  r.rho1.resize((size_t)r.K * nnz);
  hip_ok(hipMemcpyAsync(r.rho.data(), rho, nnz * 8, hipMemcpyDeviceToHost, st), "download rho");
  hip_ok(hipMemcpyAsync(r.rho1.data(), rho1, (size_t)r.K * nnz * 8, hipMemcpyDeviceToHost, st),
         "download rho1");
  hip_ok(hipStreamSynchronize(st), "request stream");
  r.rho_row_ptr = g->rho_row_ptr;
  r.rho_col.assign(g->rho_col.begin(), g->rho_col.end());
  r.t_done = now();  // before the arena piece is released below
}

void gq_server::worker() {
  (void)hipSetDevice(device);
  hipStream_t st = nullptr;
  gq_ctx* ctx = nullptr;
  bool ready = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess &&
               gq_ctx_create(device, st, 0, &ctx) == GQ_OK;
  for (;;) {
    std::shared_ptr<Request> r;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_queue.wait(lk, [&] { return stop || !queue.empty(); });
      if (stop && queue.empty()) break;
      r = queue.front();
      queue.pop_front();
    }
    gq_status status = GQ_OK;
    bool stopping;
    {
      std::lock_guard<std::mutex> lk(mu);
      stopping = stop;
    }
    if (stopping) {
      set_error("server shutting down");
      status = GQ_EBUSY;
    } else if (!ready) {
      set_error("serving thread could not create its stream/context");
      status = GQ_EDEVICE;
    } else {
      try {
        run(*r, ctx);
      } catch (const Fail& f) {
        status = f.st;
      } catch (const std::bad_alloc&) {
        set_error("out of host memory");
        status = GQ_ENOMEM;
      }
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      r->status = status;
      if (status != GQ_OK) {
        r->error = gq_last_error();
        r->t_done = now();
      }
      r->done = true;
      r->h1.clear();
      r->h1.shrink_to_fit();
    }
    cv_done.notify_all();
  }
  if (ctx) gq_ctx_destroy(ctx);
  if (st) (void)hipStreamDestroy(st);
}

extern "C" {

gq_status gq_server_create(int32_t device, int32_t n_slots, int64_t arena_bytes, gq_server** out) {
  if (!out || n_slots < 1 || n_slots > 64 || arena_bytes <= 0) {
    set_error("gq_server_create: bad argument");
    return GQ_EINVAL;
  }
  gq_ctx* probe = nullptr;
  if (gq_status st = gq_ctx_create(device, nullptr, 0, &probe)) return st;  // checks the device
  gq_ctx_destroy(probe);
  gq_server* s = new (std::nothrow) gq_server;
  if (!s) {
    set_error("gq_server_create: out of host memory");
    return GQ_ENOMEM;
  }
  s->device = device;
  if (hipMalloc((void**)&s->arena_mem, (size_t)arena_bytes) != hipSuccess) {
    (void)hipGetLastError();
    set_error("gq_server_create: arena of %lld bytes not available", (long long)arena_bytes);
    delete s;
    return GQ_ENOMEM;
  }
  s->arena = std::make_unique<Arena>((size_t)arena_bytes);
  for (int i = 0; i < n_slots; ++i) s->workers.emplace_back(&gq_server::worker, s);
  *out = s;
  return GQ_OK;
}

gq_status gq_server_submit(gq_server* s, const gq_request* q, int64_t* id) {
  if (!s || !q || !id || !q->atom_orb_ptr || !q->H || !q->core_of_atom || !q->h1 || q->K < 1 ||
      q->n_atoms < 1) {
    set_error("gq_server_submit: bad argument");
    return GQ_EINVAL;
  }
  if (!(q->kT > 0.0)) {
    set_error("gq_server_submit: kT must be > 0");
    return GQ_EINVAL;
  }
  if (q->precision != GQ_PREC_FP64 && q->precision != GQ_PREC_SPLIT32) {
    set_error("gq_server_submit: precision %u not available", q->precision);
    return GQ_EINVAL;
  }
  auto r = std::make_shared<Request>();
  const int32_t N = q->atom_orb_ptr[q->n_atoms];
  if (q->H->n_rows != N) {
    set_error("gq_server_submit: H has %d rows, the atoms carry %d orbitals", q->H->n_rows, N);
    return GQ_EINVAL;
  }
  r->n_atoms = q->n_atoms;
  r->N = N;
  r->K = q->K;
  r->atom_orb_ptr.assign(q->atom_orb_ptr, q->atom_orb_ptr + q->n_atoms + 1);
  r->core.assign(q->core_of_atom, q->core_of_atom + q->n_atoms);
  auto copy_csr = [](const gq_csr* c, std::vector<int32_t>& rp, std::vector<int32_t>& col,
                     std::vector<double>& val) {
    const int32_t* p = static_cast<const int32_t*>(c->row_ptr);
    rp.assign(p, p + c->n_rows + 1);
    const int32_t* cl = static_cast<const int32_t*>(c->col);
    col.assign(cl, cl + c->nnz);
    const double* v = static_cast<const double*>(c->val);
    val.assign(v, v + c->nnz);
  };
  copy_csr(q->H, r->h_rp, r->h_col, r->h_val);
  if (q->rho_prev) {
    r->has_prev = true;
    copy_csr(q->rho_prev, r->p_rp, r->p_col, r->p_val);
  }
  r->tau = q->tau;
  r->flags = q->flags;
  r->kT = q->kT;
  r->n_elec = q->n_elec;
  r->precision = q->precision;
  r->h1.assign(q->h1, q->h1 + (size_t)q->K * N);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    r->id = s->next_id++;
    r->t_submit = s->now();
    s->reqs[r->id] = r;
    s->queue.push_back(r);
    *id = r->id;
  }
  s->cv_queue.notify_one();
  return GQ_OK;
}

gq_status gq_server_wait(gq_server* s, int64_t id, gq_request_info* info) {
  if (!s || !info) {
    set_error("gq_server_wait: bad argument");
    return GQ_EINVAL;
  }
  std::shared_ptr<Request> r;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) {
      set_error("gq_server_wait: unknown request %lld", (long long)id);
      return GQ_EINVAL;
    }
    r = it->second;
    s->cv_done.wait(lk, [&] { return r->done; });
  }
  info->status = r->status;
  info->mu = r->mu;
  info->n_sub = r->n_sub;
  info->K = r->K;
  info->nnz = r->nnz;
  info->footprint = r->footprint;
  info->t_submit = r->t_submit;
  info->t_admit = r->t_admit;
  info->t_done = r->t_done;
  if (r->status != GQ_OK) set_error("request %lld: %s", (long long)id, r->error.c_str());
  return r->status;
}

gq_status gq_server_fetch(gq_server* s, int64_t id, double* mu1, double* rho, double* rho1,
                          int32_t* rho_row_ptr, int32_t* rho_col) {
  if (!s) {
    set_error("gq_server_fetch: bad argument");
    return GQ_EINVAL;
  }
  std::shared_ptr<Request> r;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end() || !it->second->done) {
      set_error("gq_server_fetch: request %lld unknown or not finished", (long long)id);
      return GQ_EINVAL;
    }
    r = it->second;
  }
  if (r->status != GQ_OK) {
    set_error("request %lld: %s", (long long)id, r->error.c_str());
    return r->status;
  }
  if (mu1) std::memcpy(mu1, r->mu1.data(), r->mu1.size() * 8);
  if (rho) std::memcpy(rho, r->rho.data(), r->rho.size() * 8);
  if (rho1) std::memcpy(rho1, r->rho1.data(), r->rho1.size() * 8);
  if (rho_row_ptr) std::memcpy(rho_row_ptr, r->rho_row_ptr.data(), r->rho_row_ptr.size() * 4);
  if (rho_col) std::memcpy(rho_col, r->rho_col.data(), r->rho_col.size() * 4);
  return GQ_OK;
}

gq_status gq_server_release(gq_server* s, int64_t id) {
  if (!s) {
    set_error("gq_server_release: bad argument");
    return GQ_EINVAL;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end() || !it->second->done) {
    set_error("gq_server_release: request %lld unknown or not finished", (long long)id);
    return GQ_EINVAL;
  }
  s->reqs.erase(it);
  return GQ_OK;
}

double gq_server_clock(gq_server* s) { return s ? s->now() : 0.0; }

gq_status gq_server_arena_used(gq_server* s, int64_t* used, int64_t* size) {
  if (!s) {
    set_error("gq_server_arena_used: bad argument");
    return GQ_EINVAL;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (used) *used = (int64_t)s->arena->used();
  if (size) *size = (int64_t)s->arena->size();
  return GQ_OK;
}

void gq_server_destroy(gq_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_queue.notify_all();
  s->cv_mem.notify_all();
  for (auto& t : s->workers) t.join();
  (void)hipSetDevice(s->device);
  if (s->arena_mem) (void)hipFree(s->arena_mem);
  delete s;
}

}  // extern "C"
