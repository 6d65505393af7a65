// Serving loop: continuous batching of solve requests on one GPU.
//
// The server owns an arena (one allocation of the HBM budget, first-fit free
// list) shared by its lanes.  A lane is a worker thread with its own HIP
// stream: at every GMRES restart-cycle boundary it retires finished requests
// (inverse transform, copy to host, free state) and admits queued ones whose
// state -- and operator, unless cached -- fits the arena; then it runs one
// cycle of its engine over every admitted request.  With the large lane on,
// requests whose stored dense operator would exceed a size limit are solved
// in the compressed form on a second lane, so their work overlaps the other
// lane's on the device.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "internal.h"

namespace cqm {
void h2_release(Problem& p);
}
using namespace cqm;

namespace {
using clk = std::chrono::steady_clock;

struct Arena {
  char* base = nullptr;
  size_t size = 0, used = 0, peak = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  void init(char* b, size_t n) {
    base = b;
    size = n;
    free_.clear();
    free_[0] = n;
  }
  // first fit, 256-byte granularity; returns size_t(-1) when nothing fits
  size_t alloc(size_t n) {
    n = (n + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= n) {
        const size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > n) free_[off + n] = len - n;
        used += n;
        peak = std::max(peak, used);
        return off;
      }
    return size_t(-1);
  }
  void release(size_t off, size_t n) {
    n = (n + 255) & ~size_t(255);
    used -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

struct OpEntry {
  uint64_t key = 0;
  Problem* prob = nullptr;
  size_t off = 0, bytes = 0;
  int users = 0;
  bool ready = false;
  clk::time_point last;
};

struct Request {
  uint64_t ticket = 0;
  std::vector<double> verts;
  std::vector<int32_t> tris;
  int N = 0;
  double T = 0;
  Incident inc;
  clk::time_point t_submit, t_done;
  int state = 0;  // 0 queued, 1 active, 2 done, 3 rejected
  int rc = CQM_OK;
  std::vector<double> q;
  cqm_diag diag{};
  OpEntry* op = nullptr;
  SolveState st;
  size_t off = 0, bytes = 0;
  int cycles = 0;
  int lane = 0;  // 1: large request, compressed form on the second lane
};

uint64_t fnv(const void* data, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char* p = (const unsigned char*)data;
  for (size_t k = 0; k < n; ++k) h = (h ^ p[k]) * 1099511628211ull;
  return h;
}
}  // namespace

struct cqm_server_s {
  // One lane: a worker thread with its own stream, engine buffers, queue and
  // active set.  Lane 0 serves ordinary requests; lane 1 (optional) the large
  // ones, in the compressed form, so that their long cycles run beside
  // lane 0's work instead of holding it back.
  struct Lane {
    int id = 0;
    hipStream_t stream = nullptr;
    EngineBufs eb;
    std::deque<Request*> queue;    // guarded by mu
    std::vector<Request*> active;  // owned by the lane's worker
    std::thread worker;
    bool dead = false;             // guarded by mu: the worker stopped on an error
  };

  cqm_ctx_t ctx = nullptr;
  cqm_server_opts opts{};
  char* arena_mem = nullptr;
  Arena arena;               // guarded by amu (with the operator cache)
  std::mutex mu, amu;
  std::condition_variable cv, cv_done;
  bool stop = false;
  uint64_t next_ticket = 1;
  Lane lanes[2];
  int nlanes = 1;
  std::map<uint64_t, std::unique_ptr<Request>> all;
  std::vector<std::unique_ptr<OpEntry>> cache;
  cqm_server_stats_t st{};
  std::string worker_error;

  // Stored dense operator bytes of a request in the plain form (the decision
  // between the lanes and forms is taken on this figure).
  int64_t dense_bytes(const Request& r) const {
    const int M = (int)(r.tris.size() / 3);
    const int64_t F = r.N + 1, Fh = F / 2 + 1;
    return Fh * sym_slice(M) * 24;
  }

  // ---------------------------------------------------------------- worker
  // Operator of the request (cached by mesh, N, T and lane).  Called with amu.
  OpEntry* find_or_build(Request& r, bool* cannot_fit) {
    *cannot_fit = false;
    uint64_t key = fnv(r.verts.data(), r.verts.size() * sizeof(double));
    key = fnv(r.tris.data(), r.tris.size() * sizeof(int32_t), key);
    key = fnv(&r.N, sizeof(r.N), key);
    key = fnv(&r.T, sizeof(r.T), key);
    key = fnv(&r.lane, sizeof(r.lane), key);
    if (opts.cache_operators)
      for (auto& e : cache)
        if (e->key == key && e->ready) {
          std::lock_guard<std::mutex> lk(mu);
          ++st.operator_cache_hits;
          return e.get();
        }
    cqm_options so = opts.solver;
    if (r.lane == 1) so.mode = mode_is_mixed(so.mode) ? CQM_MIXED_H2ACA : CQM_FP64_H2ACA;
    cqm_problem_t h = nullptr;
    int rc = cqm_problem_create(ctx, r.verts.data(), (int64_t)r.verts.size() / 3, r.tris.data(),
                                (int64_t)r.tris.size() / 3, r.N, r.T, &so, &h);
    if (rc != CQM_OK) throw Error(rc, cqm_last_error());
    Problem* p = h;
    const size_t need = p->lay.total;
    size_t off = arena.alloc(need);
    while (off == size_t(-1) && evict_one()) off = arena.alloc(need);
    if (off == size_t(-1)) {
      *cannot_fit = need > arena.size;
      cqm_problem_destroy(h);
      return nullptr;
    }
    p->ws = arena.base + off;
    p->ws_bytes = need;
    p->own.p = p;
    p->own.base = p->ws;
    auto e = std::make_unique<OpEntry>();
    e->key = key;
    e->prob = p;
    e->off = off;
    e->bytes = need;
    cache.push_back(std::move(e));
    std::lock_guard<std::mutex> lk(mu);
    ++st.operators_built;
    return cache.back().get();
  }
  bool evict_one() {  // least recently used operator without users (amu held)
    int best = -1;
    for (int k = 0; k < (int)cache.size(); ++k)
      if (cache[k]->users == 0 && cache[k]->ready &&
          (best < 0 || cache[k]->last < cache[best]->last))
        best = k;
    if (best < 0) return false;
    arena.release(cache[best]->off, cache[best]->bytes);
    cqm_problem_destroy(static_cast<cqm_problem_t>(cache[best]->prob));
    cache.erase(cache.begin() + best);
    return true;
  }

  // admit from the lane's queue; returns true if the active set changed
  bool admit(Lane& L) {
    bool changed = false;
    while ((int)L.active.size() < opts.max_active) {
      Request* r;
      {
        std::lock_guard<std::mutex> lk(mu);
        if (L.queue.empty()) break;
        r = L.queue.front();
      }
      std::unique_lock<std::mutex> ak(amu);
      bool never = false;
      OpEntry* op = nullptr;
      try {
        op = find_or_build(*r, &never);
      } catch (const Error& e) {
        ak.unlock();
        reject(L, r, e.code);
        continue;
      }
      if (!op) {
        ak.unlock();
        if (never || (L.active.empty() && other_lanes_idle(L))) reject(L, r, CQM_ENOMEM);
        break;  // wait for memory
      }
      Problem& p = *op->prob;
      SolveState& s = r->st;
      s = SolveState{};
      s.p = &p;
      const size_t sbytes = state_layout(p, s);
      const size_t need = sbytes + sizeof(double) * (size_t)(r->N + 1) * p.M;
      size_t off = arena.alloc(need);
      if (off == size_t(-1) && L.active.empty()) {
        // drop idle operators other than this one
        op->users++;
        while (off == size_t(-1) && evict_one()) off = arena.alloc(need);
        op->users--;
      }
      if (off == size_t(-1)) {
        if (!op->ready && op->users == 0) {
          // an operator built for this request alone: give its memory back
          for (int q = 0; q < (int)cache.size(); ++q)
            if (cache[q].get() == op) {
              arena.release(cache[q]->off, cache[q]->bytes);
              cqm_problem_destroy(static_cast<cqm_problem_t>(cache[q]->prob));
              cache.erase(cache.begin() + q);
              break;
            }
        }
        ak.unlock();
        if (L.active.empty() && other_lanes_idle(L)) reject(L, r, CQM_ENOMEM);
        break;
      }
      r->off = off;
      r->bytes = need;
      s.base = arena.base + off;
      s.inc = r->inc;
      s.q_out = reinterpret_cast<double*>(s.base + sbytes);
      op->users++;
      op->last = clk::now();
      r->op = op;
      const bool prepare = !op->ready;
      ak.unlock();
      try {
        pre_solve(s, L.stream, prepare);
      } catch (...) {
        std::lock_guard<std::mutex> a2(amu);
        arena.release(r->off, r->bytes);
        op->users--;
        r->op = nullptr;
        throw;
      }
      {
        std::lock_guard<std::mutex> a2(amu);
        op->ready = true;
      }
      changed = true;
      std::lock_guard<std::mutex> lk(mu);
      L.queue.pop_front();
      r->state = 1;
      L.active.push_back(r);
      int64_t act = 0;
      for (int k = 0; k < nlanes; ++k) act += (int64_t)lanes[k].active.size();
      st.peak_active = std::max<int64_t>(st.peak_active, act);
    }
    return changed;
  }
  bool other_lanes_idle(const Lane& L) {
    std::lock_guard<std::mutex> lk(mu);
    for (int k = 0; k < nlanes; ++k)
      if (&lanes[k] != &L && !lanes[k].active.empty()) return false;
    return true;
  }
  void reject(Lane& L, Request* r, int code) {
    std::lock_guard<std::mutex> lk(mu);
    if (!L.queue.empty() && L.queue.front() == r) L.queue.pop_front();
    r->state = 3;
    r->rc = code;
    r->t_done = clk::now();
    ++st.rejected;
    cv_done.notify_all();
  }
  void retire(Lane& L, Engine& E, int k) {
    Request* r = L.active[k];
    E.finish_diag(k, L.stream);
    post_solve(r->st, L.stream);
    r->q.resize((size_t)(r->N + 1) * r->st.p->M);
    CQM_HIP(hipMemcpyAsync(r->q.data(), r->st.q_out, sizeof(double) * r->q.size(),
                           hipMemcpyDeviceToHost, L.stream));
    CQM_HIP(hipStreamSynchronize(L.stream));
    r->diag = r->st.diag;
    r->diag.cycles = r->cycles;
    {
      std::lock_guard<std::mutex> ak(amu);
      arena.release(r->off, r->bytes);
      r->op->users--;
      r->op->last = clk::now();
      if (!opts.cache_operators && r->op->users == 0) {
        for (int q = 0; q < (int)cache.size(); ++q)
          if (cache[q].get() == r->op) {
            arena.release(cache[q]->off, cache[q]->bytes);
            cqm_problem_destroy(static_cast<cqm_problem_t>(cache[q]->prob));
            cache.erase(cache.begin() + q);
            break;
          }
      }
    }
    std::lock_guard<std::mutex> lk(mu);
    r->rc = diag_status(r->diag);
    r->state = 2;
    r->t_done = clk::now();
    ++st.completed;
    ++st.lane_completed[L.id];
    cv_done.notify_all();
  }

  void run(Lane& L) {
    try {
      CQM_HIP(hipSetDevice(ctx->device));
      Engine E(*ctx, L.eb);
      bool dirty = true;
      int64_t lane_cycles = 0;
      for (;;) {
        {
          std::unique_lock<std::mutex> lk(mu);
          cv.wait(lk, [&] { return stop || !L.queue.empty() || !L.active.empty(); });
          if (stop && L.queue.empty() && L.active.empty()) break;
        }
        const size_t before = L.active.size();
        if (admit(L)) dirty = true;
        if (L.active.empty()) {
          std::unique_lock<std::mutex> lk(mu);
          cv.wait_for(lk, std::chrono::milliseconds(1));
          continue;
        }
        if (dirty) {
          std::vector<SolveState*> S;
          for (Request* r : L.active) S.push_back(&r->st);
          E.set(S, L.stream);
          for (size_t k = before; k < L.active.size(); ++k) E.init((int)k, L.stream);
          dirty = false;
        }
        E.cycle(L.stream);
        {
          std::lock_guard<std::mutex> lk(mu);
          ++st.cycles;
        }
        ++lane_cycles;
        if (L.id == 0 && opts.fail_after_cycles > 0 && lane_cycles >= opts.fail_after_cycles) {
          CQM_HIP(hipStreamSynchronize(L.stream));
          throw Error(CQM_EDEVICE, "lane 0 stopped by the fail_after_cycles test hook");
        }
        E.status(L.stream);
        for (Request* r : L.active) r->cycles++;
        // retire finished (or out-of-cycles) requests, highest index first
        for (int k = (int)L.active.size() - 1; k >= 0; --k) {
          Request* r = L.active[k];
          if (E.state_done(k) || r->cycles >= r->st.p->opt.max_cycles) {
            retire(L, E, k);
            std::lock_guard<std::mutex> lk(mu);
            L.active.erase(L.active.begin() + k);
            dirty = true;
          }
        }
        if (dirty && !L.active.empty()) {
          // keep the survivors' descriptors valid for the next cycle
          std::vector<SolveState*> S;
          for (Request* r : L.active) S.push_back(&r->st);
          E.set(S, L.stream);
          dirty = false;
        }
      }
    } catch (const std::exception& e) {
      // The lane stops: give back the arena regions and operator uses of
      // its active requests (operators left half-built are dropped), reject
      // everything it holds, and mark it dead so that submit refuses new
      // requests for it and drain/destroy do not wait on it.  (Operators
      // without users are kept only when caching is on.)
      (void)hipStreamSynchronize(L.stream);
      {
        std::lock_guard<std::mutex> ak(amu);
        for (Request* r : L.active)
          if (r->op) {
            arena.release(r->off, r->bytes);
            r->op->users--;
            r->op = nullptr;
          }
        for (int q = (int)cache.size() - 1; q >= 0; --q)
          if ((!cache[q]->ready || !opts.cache_operators) && cache[q]->users == 0) {
            arena.release(cache[q]->off, cache[q]->bytes);
            cqm_problem_destroy(static_cast<cqm_problem_t>(cache[q]->prob));
            cache.erase(cache.begin() + q);
          }
      }
      std::lock_guard<std::mutex> lk(mu);
      L.dead = true;
      worker_error = e.what();
      const auto now = clk::now();
      for (Request* r : L.queue) {
        r->state = 3;
        r->rc = CQM_EDEVICE;
        r->t_done = now;
        ++st.rejected;
      }
      L.queue.clear();
      for (Request* r : L.active) {
        r->state = 3;
        r->rc = CQM_EDEVICE;
        r->t_done = now;
        ++st.rejected;
      }
      L.active.clear();
      cv_done.notify_all();
    }
  }
  bool idle() const {  // mu held; a dead lane holds nothing
    for (int k = 0; k < nlanes; ++k)
      if (!lanes[k].queue.empty() || !lanes[k].active.empty()) return false;
    return (int64_t)(st.completed + st.rejected) == st.submitted;
  }
};

namespace {
thread_local std::string g_srv_err;
}

extern "C" {

int cqm_server_default_options(cqm_server_opts* o) {
  if (!o) return CQM_EINVAL;
  std::memset(o, 0, sizeof(*o));
  o->max_active = 16;
  o->cache_operators = 1;
  o->large_cu_percent = 50;
  cqm_default_options(&o->solver);
  o->solver.reuse_operator = 1;
  return CQM_OK;
}

int cqm_server_create(cqm_ctx_t ctx, size_t hbm_budget, const cqm_server_opts* opts, cqm_server_t* out) {
  if (!ctx || !out || hbm_budget < (1u << 20))
    return fail_with(CQM_EINVAL, "cqm_server_create: NULL argument or budget under 1 MiB");
  auto* s = new cqm_server_s();
  s->ctx = ctx;
  if (opts) s->opts = *opts;
  else cqm_server_default_options(&s->opts);
  s->opts.solver.reuse_operator = 1;
  s->opts.solver.profile = 0;
  if (s->opts.max_active < 1) s->opts.max_active = 1;
  if (s->opts.large_lane && s->opts.large_bytes <= 0) s->opts.large_bytes = (int64_t)(hbm_budget / 4);
  s->nlanes = s->opts.large_lane ? 2 : 1;
  bool ok = hipSetDevice(ctx->device) == hipSuccess;
  for (int k = 0; ok && k < s->nlanes; ++k) {
    s->lanes[k].id = k;
    const int pct = s->opts.large_cu_percent;
    if (k == 1 && pct > 0 && pct < 100) {
      // the large lane's long-running kernels would otherwise fill every CU
      // and hold the first lane's launches back: confine them to every
      // k-th CU (an even spread over the chip's dies and shader engines)
      int cus = 0;
      ok = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) ==
           hipSuccess;
      if (ok && cus > 0) {
        std::vector<uint32_t> mask((cus + 31) / 32, 0u);
        const int keep = std::max(1, cus * pct / 100);
        for (int j = 0; j < keep; ++j) {
          const int cu = (int)((int64_t)j * cus / keep);
          mask[cu / 32] |= 1u << (cu % 32);
        }
        if (hipExtStreamCreateWithCUMask(&s->lanes[k].stream, (uint32_t)mask.size(),
                                         mask.data()) == hipSuccess)
          continue;
        (void)hipGetLastError();
      }
    }
    ok = ok && hipStreamCreateWithFlags(&s->lanes[k].stream, hipStreamNonBlocking) == hipSuccess;
  }
  const char* what = ok ? nullptr : "cqm_server_create: device or stream set-up failed";
  if (ok && hipMalloc(&s->arena_mem, hbm_budget) != hipSuccess) {
    (void)hipGetLastError();  // clear the sticky allocation error for later checks
    ok = false;
    what = "cqm_server_create: the arena (hbm_budget bytes) could not be allocated";
  }
  if (!ok) {
    for (int k = 0; k < s->nlanes; ++k)
      if (s->lanes[k].stream) (void)hipStreamDestroy(s->lanes[k].stream);
    delete s;
    return fail_with(CQM_ENOMEM, what);
  }
  s->arena.init(s->arena_mem, hbm_budget);
  for (int k = 0; k < s->nlanes; ++k) {
    cqm_server_s::Lane* L = &s->lanes[k];
    L->worker = std::thread([s, L] { s->run(*L); });
  }
  *out = s;
  return CQM_OK;
}

int cqm_server_submit(cqm_server_t s, const cqm_request* q, uint64_t* ticket) {
  if (!s || !q || !ticket || !q->vertices || !q->tris || q->nv < 3 || q->M < 1 || q->N < 2 || !(q->T > 0))
    return CQM_EINVAL;
  auto r = std::make_unique<Request>();
  r->verts.assign(q->vertices, q->vertices + 3 * q->nv);
  r->tris.assign(q->tris, q->tris + 3 * q->M);
  r->N = q->N;
  r->T = q->T;
  const double n = std::sqrt(q->direction[0] * q->direction[0] + q->direction[1] * q->direction[1] +
                             q->direction[2] * q->direction[2]);
  if (!(n > 0) || !(q->sigma > 0)) return CQM_EINVAL;
  r->inc.kind = 1;
  for (int k = 0; k < 3; ++k) r->inc.dir[k] = q->direction[k] / n;
  r->inc.sigma = q->sigma;
  r->inc.t0 = q->t0;
  r->inc.amp = q->amplitude;
  r->t_submit = clk::now();
  r->lane = (s->nlanes > 1 && s->dense_bytes(*r) > s->opts.large_bytes) ? 1 : 0;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->lanes[r->lane].dead) return CQM_EDEVICE;
  r->ticket = s->next_ticket++;
  *ticket = r->ticket;
  s->lanes[r->lane].queue.push_back(r.get());
  s->all[r->ticket] = std::move(r);
  ++s->st.submitted;
  s->cv.notify_all();
  return CQM_OK;
}

int cqm_server_poll(cqm_server_t s, uint64_t ticket, int32_t* done, double* q_out, cqm_diag* diag,
                    double* latency_ms) {
  if (!s || !done) return CQM_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return CQM_EINVAL;
  Request& r = *it->second;
  if (r.state < 2) {
    *done = 0;
    return CQM_OK;
  }
  *done = r.state == 2 ? 1 : -1;
  if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r.t_done - r.t_submit).count();
  if (r.state == 2) {
    if (q_out) std::memcpy(q_out, r.q.data(), sizeof(double) * r.q.size());
    if (diag) *diag = r.diag;
  }
  return r.rc;
}

int cqm_server_drain(cqm_server_t s) {
  if (!s) return CQM_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->idle(); });
  return s->worker_error.empty() ? CQM_OK : CQM_EDEVICE;
}

int cqm_server_stats(cqm_server_t s, cqm_server_stats_t* out) {
  if (!s || !out) return CQM_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    out->active = out->queued = 0;
    for (int k = 0; k < s->nlanes; ++k) {
      out->active += (int64_t)s->lanes[k].active.size();
      out->queued += (int64_t)s->lanes[k].queue.size();
    }
  }
  std::lock_guard<std::mutex> ak(s->amu);
  out->arena_used = (int64_t)s->arena.used;
  out->arena_bytes = (int64_t)s->arena.size;
  out->peak_arena_bytes = (int64_t)s->arena.peak;
  return CQM_OK;
}

int cqm_server_destroy(cqm_server_t s) {
  if (!s) return CQM_OK;
  cqm_server_drain(s);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv.notify_all();
  }
  for (int k = 0; k < s->nlanes; ++k)
    if (s->lanes[k].worker.joinable()) s->lanes[k].worker.join();
  (void)hipSetDevice(s->ctx->device);
  for (auto& e : s->cache) cqm_problem_destroy(static_cast<cqm_problem_t>(e->prob));
  s->cache.clear();
  if (s->arena_mem) (void)hipFree(s->arena_mem);
  for (int k = 0; k < s->nlanes; ++k) {
    release_engine_bufs(s->lanes[k].eb);
    if (s->lanes[k].stream) (void)hipStreamDestroy(s->lanes[k].stream);
  }
  delete s;
  return CQM_OK;
}

}  // extern "C"
