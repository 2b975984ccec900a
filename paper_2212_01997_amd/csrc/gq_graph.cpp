// Graph estimate and core/halo partition (host, integer work).
//
// Sec. II.E: the data-dependency graph is estimated from the thresholded
// density of a previous step together with the thresholded Hamiltonian, and
// optionally widened by paths of length two.  Sec. II.C / Fig. 1: each core
// (a set of atoms) with every atom joined to it forms a subgraph, whose
// orbitals select a principal submatrix.  Eq. (sub_f): the collected result
// keeps the core rows of each subgraph, so the collected pattern of orbital a
// is the orbital set of the subgraph owning a.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <numeric>
#include <thread>

#include "gq_internal.hpp"

namespace gq {

namespace {

// Host threads for the graph build: every task writes only its own output
// region, so the result does not depend on the thread count.
int build_threads() {
  const unsigned hc = std::thread::hardware_concurrency();
  return (int)std::min(16u, std::max(1u, hc));
}

// A pool of host worker threads kept for the life of the process, so that the
// dozen parallel phases of a graph build do not each start and join threads.
// One job at a time: a caller that finds the pool busy (graph builds on
// several threads at once, as in the serving runtime) runs its job with
// threads of its own instead.  Never destroyed: the workers wait on a
// condition variable and end with the process.
class BuildPool {
 public:
  static BuildPool& get() {
    static BuildPool* p = new BuildPool;
    return *p;
  }
  // work(tid) for tid in [0, nt), tid 0 on the calling thread; false (nothing
  // run) if another job holds the pool
  bool run(int nt, const std::function<void(int)>& work) {
    std::unique_lock<std::mutex> own(run_mu_, std::try_to_lock);
    if (!own.owns_lock()) return false;
    {
      std::lock_guard<std::mutex> lk(mu_);
      while ((int)workers_ < nt - 1) {
        const int id = ++workers_;
        std::thread([this, id] { loop(id); }).detach();
      }
      job_ = &work;
      want_ = nt - 1;
      done_ = 0;
      ++gen_;
    }
    cv_.notify_all();
    work(0);
    std::unique_lock<std::mutex> lk(mu_);
    done_cv_.wait(lk, [&] { return done_ == want_; });
    job_ = nullptr;
    return true;
  }

 private:
  void loop(int id) {
    uint64_t seen = 0;
    for (;;) {
      const std::function<void(int)>* job;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return gen_ != seen && id <= want_; });
        seen = gen_;
        job = job_;
      }
      (*job)(id);
      {
        std::lock_guard<std::mutex> lk(mu_);
        ++done_;
      }
      done_cv_.notify_one();
    }
  }
  std::mutex run_mu_, mu_;
  std::condition_variable cv_, done_cv_;
  const std::function<void(int)>* job_ = nullptr;
  int workers_ = 0, want_ = 0, done_ = 0;
  uint64_t gen_ = 0;
};

// fn(tid, i) for i in [0, n), items dealt in blocks of `grain` from a shared
// counter; tid in [0, threads) names the calling thread's scratch.
template <class F>
void parallel_for(int64_t n, int64_t grain, int threads, F&& fn) {
  if (threads <= 1 || n <= grain) {
    for (int64_t i = 0; i < n; ++i) fn(0, i);
    return;
  }
  std::atomic<int64_t> next{0};
  const std::function<void(int)> work = [&](int tid) {
    for (;;) {
      const int64_t b = next.fetch_add(grain);
      if (b >= n) break;
      const int64_t e = std::min(n, b + grain);
      for (int64_t i = b; i < e; ++i) fn(tid, i);
    }
  };
  const int nt = (int)std::min<int64_t>(threads, (n + grain - 1) / grain);
  if (BuildPool::get().run(nt, work)) return;
  std::vector<std::thread> pool;
  for (int t = 1; t < nt; ++t) pool.emplace_back(work, t);
  work(0);
  for (auto& t : pool) t.join();
}

// Structure checks of a host CSR matrix of n rows in one parallel pass: the
// first row where row_ptr decreases, the first row with columns out of range
// or not ascending, and (symmetric) the first row holding an entry (a, b)
// whose mirror (b, a) is missing.  They are reported in that order, so each
// is the first such row of a matrix that passed the checks before it.  Every
// read is bounds-checked first: a row whose range lies outside [0, nnz] (only
// possible where row_ptr decreases elsewhere) is not read, and another row's
// search does not enter it.  The mirror search keeps one cursor per row b and
// thread: a thread takes its rows a in ascending order, so the a it looks for
// in row b only grow and each cursor only moves forward.
gq_status check_csr(const gq_csr* X, int32_t n, const char* name, bool symmetric, int threads) {
  if (!X || X->n_rows != n || !X->row_ptr || (X->nnz > 0 && (!X->col || !X->val))) {
    set_error("%s: CSR header does not match N = %d", name, n);
    return GQ_EINVAL;
  }
  if (X->row_ptr[0] != 0 || X->row_ptr[n] != X->nnz) {
    set_error("%s: row_ptr must run from 0 to nnz", name);
    return GQ_EINVAL;
  }
  const int32_t* rp = X->row_ptr;
  const int32_t* col = X->col;
  const int32_t nnz = X->nnz;
  auto readable = [&](int32_t a) { return rp[a] >= 0 && rp[a] <= rp[a + 1] && rp[a + 1] <= nnz; };
  std::atomic<int32_t> bad_ptr{INT32_MAX}, bad_col{INT32_MAX}, bad_sym{INT32_MAX};
  auto lower = [](std::atomic<int32_t>& f, int32_t a) {
    int32_t cur = f.load();
    while (a < cur && !f.compare_exchange_weak(cur, a)) {
    }
  };
  std::vector<std::vector<int32_t>> cursor(symmetric ? threads : 0);
  parallel_for(n, 512, threads, [&](int tid, int64_t ai) {
    const int32_t a = (int32_t)ai;
    if (rp[a + 1] < rp[a]) {
      lower(bad_ptr, a);
      return;
    }
    if (!readable(a)) return;
    for (int32_t p = rp[a]; p < rp[a + 1]; ++p) {
      const int32_t c = col[p];
      if (c < 0 || c >= n || (p > rp[a] && c <= col[p - 1])) {
        lower(bad_col, a);
        return;
      }
    }
    if (!symmetric) return;
    std::vector<int32_t>& cu = cursor[tid];
    if (cu.empty()) cu.assign(rp, rp + n);
    for (int32_t p = rp[a]; p < rp[a + 1]; ++p) {
      const int32_t c = col[p];
      if (!readable(c)) {
        lower(bad_sym, a);
        return;
      }
      int32_t q = std::max(cu[c], rp[c]);
      while (q < rp[c + 1] && col[q] < a) ++q;
      cu[c] = q;
      if (q == rp[c + 1] || col[q] != a) {
        lower(bad_sym, a);
        return;
      }
    }
  });
  if (bad_ptr.load() != INT32_MAX) {
    set_error("%s: row_ptr decreases at row %d", name, bad_ptr.load());
    return GQ_EINVAL;
  }
  if (bad_col.load() != INT32_MAX) {
    set_error("%s: row %d has columns out of range or not ascending", name, bad_col.load());
    return GQ_EINVAL;
  }
  if (bad_sym.load() != INT32_MAX) {
    set_error("graph_build: the pattern of %s is not symmetric", name);
    return GQ_EINVAL;
  }
  return GQ_OK;
}

}  // namespace

gq_status graph_build_host(int32_t n_atoms, const int32_t* atom_orb_ptr, const gq_csr* H,
                           const gq_csr* rho_prev, const int32_t* core_of_atom, double tau,
                           uint32_t flags, gq_graph* g) {
  if (n_atoms <= 0 || !atom_orb_ptr || !core_of_atom || !H) {
    set_error("graph_build: empty system or NULL input");
    return GQ_EINVAL;
  }
  if (!(tau >= 0.0)) {
    set_error("graph_build: tau must be >= 0 (got %g)", tau);
    return GQ_EINVAL;
  }
  if (atom_orb_ptr[0] != 0) {
    set_error("graph_build: atom_orb_ptr[0] must be 0");
    return GQ_EINVAL;
  }
  for (int32_t I = 0; I < n_atoms; ++I) {
    if (atom_orb_ptr[I + 1] <= atom_orb_ptr[I]) {
      set_error("graph_build: atom_orb_ptr must be strictly increasing (atom %d)", I);
      return GQ_EINVAL;
    }
  }
  const int32_t N = atom_orb_ptr[n_atoms];
  const int threads = build_threads();
  if (gq_status st = check_csr(H, N, "H", true, threads)) return st;
  if (rho_prev)
    if (gq_status st = check_csr(rho_prev, N, "rho_prev", false, threads)) return st;

  int32_t n_sub = 0;
  for (int32_t I = 0; I < n_atoms; ++I) {
    if (core_of_atom[I] < 0) {
      set_error("graph_build: negative core id at atom %d", I);
      return GQ_EINVAL;
    }
    n_sub = std::max(n_sub, core_of_atom[I] + 1);
  }
  std::vector<std::vector<int32_t>> cores(n_sub);
  for (int32_t I = 0; I < n_atoms; ++I) cores[core_of_atom[I]].push_back(I);
  for (int32_t s = 0; s < n_sub; ++s) {
    if (cores[s].empty()) {
      set_error("graph_build: core ids must be dense; core %d is empty", s);
      return GQ_EINVAL;
    }
  }

  std::vector<int32_t> atom_of(N);
  for (int32_t I = 0; I < n_atoms; ++I)
    std::fill(atom_of.begin() + atom_orb_ptr[I], atom_of.begin() + atom_orb_ptr[I + 1], I);

  // atom adjacency: every thresholded element joins its two atoms (both ways).
  // fwd[I]: atoms J != I holding a thresholded element of a row of atom I
  // (ascending); the graph is fwd united with its transpose.
  std::vector<std::vector<int32_t>> stamp_t(threads, std::vector<int32_t>(n_atoms, -1));
  std::vector<std::vector<int32_t>> fwd(n_atoms);
  parallel_for(n_atoms, 64, threads, [&](int tid, int64_t Ii) {
    const int32_t I = (int32_t)Ii;
    std::vector<int32_t>& stamp = stamp_t[tid];
    std::vector<int32_t>& out = fwd[I];
    auto rows = [&](const gq_csr* X) {
      for (int32_t a = atom_orb_ptr[I]; a < atom_orb_ptr[I + 1]; ++a)
        for (int32_t p = X->row_ptr[a]; p < X->row_ptr[a + 1]; ++p) {
          if (!(std::fabs(X->val[p]) >= tau)) continue;
          const int32_t J = atom_of[X->col[p]];
          if (J != I && stamp[J] != I) {
            stamp[J] = I;
            out.push_back(J);
          }
        }
    };
    rows(H);
    if (rho_prev) rows(rho_prev);
    std::sort(out.begin(), out.end());
  });
  // transpose of fwd: rev[J] lists the I with J in fwd[I], ascending (each
  // thread owns a contiguous range of I and fills its own slots of every rev[J])
  std::vector<int32_t> rev_ptr(n_atoms + 1, 0), rev;
  {
    const int nt = threads;
    const int64_t span = (n_atoms + nt - 1) / nt;
    std::vector<std::vector<int32_t>> cnt(nt, std::vector<int32_t>(n_atoms, 0));
    parallel_for(nt, 1, nt, [&](int, int64_t t) {
      const int32_t i0 = (int32_t)std::min<int64_t>(n_atoms, t * span);
      const int32_t i1 = (int32_t)std::min<int64_t>(n_atoms, (t + 1) * span);
      for (int32_t I = i0; I < i1; ++I)
        for (int32_t J : fwd[I]) ++cnt[t][J];
    });
    // slot of thread t in rev[J]: after the entries of rev[J] from threads < t
    for (int32_t J = 0; J < n_atoms; ++J) {
      int32_t c = 0;
      for (int t = 0; t < nt; ++t) {
        const int32_t k = cnt[t][J];
        cnt[t][J] = c;
        c += k;
      }
      rev_ptr[J + 1] = rev_ptr[J] + c;
    }
    rev.resize(rev_ptr[n_atoms]);
    parallel_for(nt, 1, nt, [&](int, int64_t t) {
      const int32_t i0 = (int32_t)std::min<int64_t>(n_atoms, t * span);
      const int32_t i1 = (int32_t)std::min<int64_t>(n_atoms, (t + 1) * span);
      for (int32_t I = i0; I < i1; ++I)
        for (int32_t J : fwd[I]) rev[rev_ptr[J] + cnt[t][J]++] = I;
    });
  }
  std::vector<std::vector<int32_t>> nbr(n_atoms);
  parallel_for(n_atoms, 64, threads, [&](int, int64_t Ii) {
    const int32_t I = (int32_t)Ii;
    const auto& f = fwd[I];
    std::vector<int32_t>& out = nbr[I];
    out.resize(f.size() + (rev_ptr[I + 1] - rev_ptr[I]));
    auto end = std::set_union(f.begin(), f.end(), rev.begin() + rev_ptr[I],
                              rev.begin() + rev_ptr[I + 1], out.begin());
    out.resize(end - out.begin());
  });
  fwd.clear();

  // subgraphs: core ascending (already, atoms were visited in order) ++ halo ascending
  g->n_atoms = n_atoms;
  g->N = N;
  g->n_sub = n_sub;
  g->atom_orb_ptr.assign(atom_orb_ptr, atom_orb_ptr + n_atoms + 1);
  g->sub_ptr.assign(n_sub + 1, 0);
  g->n_core_atoms.resize(n_sub);
  g->sub_atoms.clear();
  std::vector<std::vector<int32_t>> halos(n_sub);
  for (auto& st : stamp_t) std::fill(st.begin(), st.end(), -1);
  parallel_for(n_sub, 16, threads, [&](int tid, int64_t si) {
    const int32_t s = (int32_t)si;
    std::vector<int32_t>& mark = stamp_t[tid];
    std::vector<int32_t>& halo = halos[s];
    if (flags & GQ_COMPLETE) {
      for (int32_t I = 0; I < n_atoms; ++I)
        if (core_of_atom[I] != s) halo.push_back(I);
      return;
    }
    // the halo: every atom within one edge of a core atom, or within two
    // with paths of length two (the neighbours J of a core atom and, with
    // GQ_PATHS2, the neighbours of every such J), minus the core; gathered
    // per subgraph with marks, so the two-step neighbour lists of single
    // atoms are never formed
    const bool two = flags & GQ_PATHS2;
    for (int32_t I : cores[s]) mark[I] = s;
    for (int32_t I : cores[s])
      for (int32_t J : nbr[I]) {
        if (mark[J] != s) { mark[J] = s; halo.push_back(J); }
        if (two)
          for (int32_t L : nbr[J])
            if (mark[L] != s) { mark[L] = s; halo.push_back(L); }
      }
    std::sort(halo.begin(), halo.end());
  });
  for (int32_t s = 0; s < n_sub; ++s) {
    g->sub_atoms.insert(g->sub_atoms.end(), cores[s].begin(), cores[s].end());
    g->sub_atoms.insert(g->sub_atoms.end(), halos[s].begin(), halos[s].end());
    g->n_core_atoms[s] = (int32_t)cores[s].size();
    if (g->sub_atoms.size() > (size_t)INT32_MAX) {
      set_error("graph_build: subgraph vertex lists exceed int32");
      return GQ_ENOMEM;
    }
    g->sub_ptr[s + 1] = (int32_t)g->sub_atoms.size();
  }
  halos.clear();

  // orbital maps: counts per subgraph, offsets, then the lists in parallel
  g->sub_orb_ptr.assign(n_sub + 1, 0);
  g->n_core_orbs.resize(n_sub);
  std::vector<int64_t> norb(n_sub);
  parallel_for(n_sub, 64, threads, [&](int, int64_t si) {
    const int32_t s = (int32_t)si;
    int64_t n = 0;
    int32_t c = 0;
    for (int32_t q = g->sub_ptr[s]; q < g->sub_ptr[s + 1]; ++q) {
      const int32_t I = g->sub_atoms[q];
      const int32_t k = atom_orb_ptr[I + 1] - atom_orb_ptr[I];
      n += k;
      if (q - g->sub_ptr[s] < g->n_core_atoms[s]) c += k;
    }
    norb[s] = n;
    g->n_core_orbs[s] = c;
  });
  int64_t tot = 0;
  for (int32_t s = 0; s < n_sub; ++s) {
    tot += norb[s];
    if (tot > INT32_MAX) {
      set_error("graph_build: orbital lists exceed int32");
      return GQ_ENOMEM;
    }
    g->sub_orb_ptr[s + 1] = (int32_t)tot;
  }
  g->sub_orbs.resize(tot);
  parallel_for(n_sub, 64, threads, [&](int, int64_t si) {
    const int32_t s = (int32_t)si;
    int32_t* out = g->sub_orbs.data() + g->sub_orb_ptr[s];
    for (int32_t q = g->sub_ptr[s]; q < g->sub_ptr[s + 1]; ++q) {
      const int32_t I = g->sub_atoms[q];
      for (int32_t a = atom_orb_ptr[I]; a < atom_orb_ptr[I + 1]; ++a) *out++ = a;
    }
  });

  // sorted orbital lists, their local indices, and the column slot of every local orbital
  const size_t sum_n = g->sub_orbs.size();
  g->sorted_orbs.resize(sum_n);
  g->sorted_local.resize(sum_n);
  g->slot.resize(sum_n);
  parallel_for(n_sub, 16, threads, [&](int, int64_t si) {
    const int32_t s = (int32_t)si;
    const int32_t b = g->sub_orb_ptr[s], n = g->sub_orb_ptr[s + 1] - b;
    int32_t* loc = g->sorted_local.data() + b;
    const int32_t* orbs = g->sub_orbs.data() + b;
    // the core orbitals (ascending) come first, then the halo's (ascending),
    // and no orbital is in both: the sorted order is the merge of the two runs
    const int32_t nc = g->n_core_orbs[s];
    int32_t i = 0, j = nc, r = 0;
    while (i < nc && j < n) loc[r++] = orbs[i] < orbs[j] ? i++ : j++;
    while (i < nc) loc[r++] = i++;
    while (j < n) loc[r++] = j++;
    for (int32_t r = 0; r < n; ++r) {
      g->sorted_orbs[b + r] = orbs[loc[r]];
      g->slot[b + loc[r]] = r;
    }
  });

  // collected pattern
  g->rho_row_ptr.assign(N + 1, 0);
  int64_t nnz = 0;
  for (int32_t a = 0; a < N; ++a) {
    const int32_t s = core_of_atom[atom_of[a]];
    nnz += g->sub_orb_ptr[s + 1] - g->sub_orb_ptr[s];
    if (nnz > INT32_MAX) {
      set_error("graph_build: collected pattern exceeds int32 nonzeros");
      return GQ_ENOMEM;
    }
    g->rho_row_ptr[a + 1] = (int32_t)nnz;
  }
  g->rho_col.resize(nnz);
  parallel_for(n_sub, 16, threads, [&](int, int64_t si) {
    const int32_t s = (int32_t)si;
    const int32_t b = g->sub_orb_ptr[s], n = g->sub_orb_ptr[s + 1] - b;
    for (int32_t j = 0; j < g->n_core_orbs[s]; ++j) {
      const int32_t a = g->sub_orbs[b + j];
      std::copy(g->sorted_orbs.begin() + b, g->sorted_orbs.begin() + b + n,
                g->rho_col.begin() + g->rho_row_ptr[a]);
    }
  });

  // per-subgraph offsets and a largest-first order
  g->off2.assign(n_sub + 1, 0);
  g->offc.assign(n_sub + 1, 0);
  g->offcd.assign(n_sub + 1, 0);
  int32_t max_n = 0, min_n = INT32_MAX, max_c = 0;
  for (int32_t s = 0; s < n_sub; ++s) {
    const int64_t n = g->sub_orb_ptr[s + 1] - g->sub_orb_ptr[s];
    const int64_t c = g->n_core_orbs[s];
    g->off2[s + 1] = g->off2[s] + n * n;
    g->offc[s + 1] = g->offc[s] + c * n;
    g->offcd[s + 1] = g->offcd[s] + (int32_t)c;
    max_n = std::max<int32_t>(max_n, (int32_t)n);
    min_n = std::min<int32_t>(min_n, (int32_t)n);
    max_c = std::max<int32_t>(max_c, (int32_t)c);
  }
  g->order.resize(n_sub);
  std::iota(g->order.begin(), g->order.end(), 0);
  std::stable_sort(g->order.begin(), g->order.end(), [&](int32_t x, int32_t y) {
    return (g->sub_orb_ptr[x + 1] - g->sub_orb_ptr[x]) > (g->sub_orb_ptr[y + 1] - g->sub_orb_ptr[y]);
  });

  gq_graph_info& in = g->info;
  in.n_atoms = n_atoms;
  in.n_orb = N;
  in.n_sub = n_sub;
  in.max_n = max_n;
  in.min_n = min_n;
  in.max_c = max_c;
  in.nnz = nnz;
  in.sum_n = (int64_t)sum_n;
  in.sum_n2 = g->off2[n_sub];
  in.sub_atoms_len = (int64_t)g->sub_atoms.size();
  build_dc_plan(g);
  build_xy_tiles(g);
  return GQ_OK;
}

}  // namespace gq

namespace gq {

// Halving tree of every subgraph's tridiagonal down to blocks of at most
// kLeaf rows.  Merges are grouped by depth, deepest first, so each level only
// needs the results of the levels before it; every level carries its list of
// 64x64 output tiles.
void build_dc_plan(gq_graph* g) {
  struct Node {
    int32_t lo, m, depth;
  };
  // class 0: the largest fifth of the subgraphs (order[0..n_big)), class 1:
  // the rest; the eigensolve runs the two classes on two streams (a larger
  // first class leaves fewer small subgraphs to fill the CUs while the
  // largest are reduced, a smaller one puts more of them in its way)
  g->n_big = std::min(g->n_sub, std::max(1, (g->n_sub + 2) / 5));
  // the subgraphs of the multi-workgroup reduction lead the order and stay in
  // class 0
  g->n_mwg = 0;
  while (g->n_mwg < g->n_sub &&
         g->sub_orb_ptr[g->order[g->n_mwg] + 1] - g->sub_orb_ptr[g->order[g->n_mwg]] >= kMwgMinN)
    ++g->n_mwg;
  g->n_big = std::max(g->n_big, g->n_mwg);
  g->dc_leaves.clear();
  g->dc_merges.clear();
  g->dc_nglob_max = 0;
  g->dc_tiles.clear();
  for (int cls = 0; cls < 2; ++cls) {
    const int32_t i0 = cls == 0 ? 0 : g->n_big, i1 = cls == 0 ? g->n_big : g->n_sub;
    std::vector<std::vector<int32_t>> by_depth;
    g->dc_leaf_off[cls] = (int32_t)(g->dc_leaves.size() / 4);
    for (int32_t oi = i0; oi < i1; ++oi) {
      const int32_t s = g->order[oi];
      const int32_t n = g->sub_orb_ptr[s + 1] - g->sub_orb_ptr[s];
      std::vector<Node> stack{{0, n, 0}};
      while (!stack.empty()) {
        const Node nd = stack.back();
        stack.pop_back();
        if (nd.m > kLeaf) {
          const int32_t m1 = nd.m / 2;
          if ((int32_t)by_depth.size() <= nd.depth) by_depth.resize(nd.depth + 1);
          auto& v = by_depth[nd.depth];
          v.insert(v.end(), {s, nd.lo, m1, nd.m - m1});
          stack.push_back({nd.lo, m1, nd.depth + 1});
          stack.push_back({nd.lo + m1, nd.m - m1, nd.depth + 1});
        } else {
          // the leaf goes where its parent merge reads: a merge at depth d
          // reads Q for odd d and the scratch for even d (and writes the other
          // one), so the top merges write Q; a subgraph that is one leaf
          // writes Q
          const int32_t tgt = nd.depth == 0 ? 0 : ((nd.depth - 1) % 2 == 1 ? 0 : 1);
          g->dc_leaves.insert(g->dc_leaves.end(), {s, nd.lo, nd.m, tgt});
        }
      }
    }
    auto& mo = g->dc_level_merge_off[cls];
    auto& to = g->dc_level_tile_off[cls];
    mo.assign(1, (int32_t)(g->dc_merges.size() / 4));
    to.assign(1, (int32_t)(g->dc_tiles.size() / 3));
    g->dc_level_msum[cls].clear();
    g->dc_level_nglob[cls].clear();
    g->dc_level_maxm_lds[cls].clear();
    for (int d = (int)by_depth.size() - 1; d >= 0; --d) {
      const auto& v = by_depth[d];
      int32_t maxm_lds = 0, nglob = 0;
      int64_t msum = 0;
      int64_t ntiles = 0;
      for (size_t q = 0; q < v.size(); q += 4) {
        const int32_t li = (int32_t)(q / 4);
        const int32_t m = v[q + 2] + v[q + 3];
        msum += m;
        // merges above the LDS bound come first in their level (subgraphs in
        // decreasing size; only a top merge can exceed it)
        if (m > kDcLdsMaxM) nglob = li + 1;
        else maxm_lds = std::max(maxm_lds, m);
        const int64_t nt = (m + 63) / 64;
        ntiles += nt * nt;
      }
      size_t at = g->dc_tiles.size();
      g->dc_tiles.resize(at + 3 * (size_t)ntiles);
      int32_t* t = g->dc_tiles.data();
      for (size_t q = 0; q < v.size(); q += 4) {
        const int32_t li = (int32_t)(q / 4);
        const int32_t nt = (v[q + 2] + v[q + 3] + 63) / 64;
        for (int32_t tr = 0; tr < nt; ++tr)
          for (int32_t tc = 0; tc < nt; ++tc) {
            t[at++] = li;
            t[at++] = tr;
            t[at++] = tc;
          }
      }
      g->dc_merges.insert(g->dc_merges.end(), v.begin(), v.end());
      mo.push_back((int32_t)(g->dc_merges.size() / 4));
      to.push_back((int32_t)(g->dc_tiles.size() / 3));
      g->dc_level_msum[cls].push_back(msum);
      g->dc_level_nglob[cls].push_back(nglob);
      g->dc_nglob_max = std::max(g->dc_nglob_max, nglob);
      g->dc_level_maxm_lds[cls].push_back(maxm_lds);
    }
  }
  g->dc_leaf_off[2] = (int32_t)(g->dc_leaves.size() / 4);
  g->bt_toff.assign(g->n_sub, 0);
  int32_t nb = 0;
  for (int32_t s = 0; s < g->n_sub; ++s) {
    const int32_t n = g->sub_orb_ptr[s + 1] - g->sub_orb_ptr[s];
    g->bt_toff[s] = nb;
    nb += n > 2 ? (n - 2 + 15) / 16 : 0;
  }
  g->bt_nblocks = nb;
}

}  // namespace gq
