// server.hip -- request server: continuous batching of exact solves.
//
// One worker thread per server owns a HIP stream and runs rounds:
//   1. admit queued requests, first come first served, while a slot is free and
//      the request's workspace fits the free part of the HBM budget (first-fit
//      allocator over one device allocation);
//   2. write the device header (per-slot descriptors and three tile tables:
//      the new systems, all running systems, the systems to retire);
//   3. set up the new systems, then advance every running system by `chunk`
//      iterations, one launch per phase for all of them (batch.h kernels);
//   4. read every slot's device state; systems that stopped get their exact true
//      residual, their results are published and their slots and memory freed.
// A system's arithmetic never depends on its neighbours in the batch (exact
// reductions, per-system scalars), so every result equals the solve alone.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <thread>
#include <unordered_map>

#include "host.h"

using namespace rpk;
using namespace rpkhost;

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

// First-fit allocator of 256-byte-aligned blocks inside [0, size).
class Arena {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
    used_ = peak_ = 0;
  }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used_ += bytes;
        if (used_ > peak_) peak_ = used_;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
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
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0, peak_ = 0;
};

struct Req {
  uint64_t id = 0;
  const rpk_matrix* A = nullptr;
  const double* b = nullptr;
  double* x = nullptr;
  int64_t n = 0;
  int gcap = 0;
  size_t bytes = 0, off = 0;
  int slot = -1;
  bool finished = false;
  bool streamed = false;  // some round ran it with the far vectors streamed
  Clock::time_point t_submit, t_admit;
  rpk_info info;
};

// A view of the header: which tiles / systems one launch sequence covers.
// A request runs the Unif instantiations (Csr::unif) exactly when its matrix's
// Jacobi vector is uniform, from its set-up to its last iteration, so each round
// launches the uniform requests and the others as two views.
enum : int { V_NEW_U = 0, V_NEW_N = 1, V_RUN_U = 2, V_RUN_N = 3, V_FIN = 4, NVIEW = 5 };

}  // namespace

struct rpk_server {
  rpk_server_opts o{};
  int device = 0;
  int N = 4, tile = 4096, block = 512, nvec = 8, nph = 8;
  hipStream_t stream = nullptr;
  char* budget = nullptr;  // device allocation of o.hbm_budget bytes
  Arena arena;
  State* d_states = nullptr;  // [max_slots] device state of each slot (never moves)
  // device header, rewritten every round: counts[NVIEW][2] | SysDesc[max_slots] |
  // order[NVIEW][max_slots] | tiles[NVIEW][tile_cap]
  char* hdr = nullptr;
  size_t hdr_bytes = 0, off_descs = 0, off_order = 0, off_tiles = 0;
  int64_t tile_cap = 0;
  std::vector<char> h_hdr;   // host image of the header
  State* h_states = nullptr; // pinned
  std::vector<Req*> slots;
  std::vector<int> free_slots;
  int view_far[NVIEW] = {};   // per view: its systems' vectors do not fit in the Infinity Cache
  int view_unif[NVIEW] = {};  // per view: every system's Jacobi vector is uniform

  mutable std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> queue;
  std::unordered_map<uint64_t, Req*> reqs;
  uint64_t next_id = 1;
  bool stop = false;
  rpk_status failure = RPK_OK;
  rpk_server_stats st{};
  std::thread worker;
};

namespace {

rpk_status layout_header(rpk_server* S, int64_t tile_cap) {
  const size_t ms = (size_t)S->o.max_slots;
  size_t off = up(NVIEW * 2 * sizeof(int));
  S->off_descs = off;
  off += up(ms * sizeof(SysDesc));
  S->off_order = off;
  off += up(NVIEW * ms * sizeof(int));
  S->off_tiles = off;
  off += up((size_t)NVIEW * tile_cap * sizeof(Tile));
  if (S->hdr) (void)hipFree(S->hdr);
  S->hdr = nullptr;
  if (hipMalloc((void**)&S->hdr, off) != hipSuccess) return RPK_ERR_NOMEM;
  S->hdr_bytes = off;
  S->tile_cap = tile_cap;
  std::vector<char> h(off, 0);
  // keep the descriptors of running systems across a re-layout
  if (!S->h_hdr.empty()) std::memcpy(h.data() + S->off_descs, S->h_hdr.data() + S->off_descs, ms * sizeof(SysDesc));
  S->h_hdr.swap(h);
  return RPK_OK;
}

Batch view(const rpk_server* S, int v) {
  Batch B;
  B.count = (const int*)(S->hdr) + 2 * v;
  B.sys = (const SysDesc*)(S->hdr + S->off_descs);
  B.order = (const int*)(S->hdr + S->off_order) + (size_t)v * S->o.max_slots;
  B.tiles = (const Tile*)(S->hdr + S->off_tiles) + (size_t)v * S->tile_cap;
  B.far = S->view_far[v];
  B.unif = S->view_unif[v];
  return B;
}

// Fill view v of the host header image with the systems in `slots_v` (launched
// with the Unif / Far instantiations when unif / far); returns the number of
// tiles (a multiple of 8) through *ntiles.
rpk_status set_view(rpk_server* S, int v, const std::vector<int>& slots_v, bool unif, bool far, int* ntiles) {
  std::vector<int64_t> n;
  for (int k : slots_v) n.push_back(S->slots[k]->n);
  S->view_far[v] = far ? 1 : 0;
  S->view_unif[v] = unif ? 1 : 0;
  Plan p;
  if (!slots_v.empty()) p = make_plan(n, S->tile, &slots_v);
  if ((int64_t)p.tiles.size() > S->tile_cap) {
    // grow the tile tables (no kernel is running between rounds)
    const std::vector<char> keep = S->h_hdr;
    const int64_t need = (int64_t)p.tiles.size() * 2;
    const size_t old_tiles = S->off_tiles;
    const int64_t old_cap = S->tile_cap;
    RET_IF(layout_header(S, need));
    for (int w = 0; w < NVIEW; ++w) {  // keep the other views (rewritten below when used)
      std::memcpy(S->h_hdr.data() + S->off_tiles + (size_t)w * need * sizeof(Tile),
                  keep.data() + old_tiles + (size_t)w * old_cap * sizeof(Tile), (size_t)old_cap * sizeof(Tile));
    }
    std::memcpy(S->h_hdr.data(), keep.data(), NVIEW * 2 * sizeof(int));
    std::memcpy(S->h_hdr.data() + S->off_order, keep.data() + S->off_order,
                (size_t)NVIEW * S->o.max_slots * sizeof(int));
  }
  int* cnt = (int*)S->h_hdr.data() + 2 * v;
  cnt[0] = (int)p.tiles.size();
  cnt[1] = (int)slots_v.size();
  int* order = (int*)(S->h_hdr.data() + S->off_order) + (size_t)v * S->o.max_slots;
  for (size_t k = 0; k < slots_v.size(); ++k) order[k] = slots_v[k];
  Tile* t = (Tile*)(S->h_hdr.data() + S->off_tiles) + (size_t)v * S->tile_cap;
  if (!p.tiles.empty()) std::memcpy(t, p.tiles.data(), p.tiles.size() * sizeof(Tile));
  *ntiles = (int)p.tiles.size();
  return RPK_OK;
}

rpk_status upload(rpk_server* S) {
  HIPCHK(hipMemcpyAsync(S->hdr, S->h_hdr.data(), S->hdr_bytes, hipMemcpyHostToDevice, S->stream));
  HIPCHK(hipStreamSynchronize(S->stream));
  return RPK_OK;
}

int gf_of(size_t ns) { return (int)std::min<size_t>((ns + 7) & ~size_t(7), 1024); }
// tile-walking workgroups: one per tile up to a limit
int g_of(int ntiles) { return std::min(ntiles, 64000); }

template <int N>
struct SPhaseF {
  static rpk_status call(int variant, int ph, int G, int Gf, int B, hipStream_t s, Batch b) {
    return KernB<N>::phase(variant, ph, G, Gf, B, s, b);
  }
};
template <int N>
struct SStartF {
  static rpk_status call(int variant, int G, int Gf, int B, hipStream_t s, Batch b, double tol, int maxit) {
    RET_IF(KernB<N>::setup(Gf, s, b, tol, maxit, variant));
    return KernB<N>::init(variant, G, Gf, B, s, b);
  }
};

// One round of the worker (called without the lock held).
rpk_status round(rpk_server* S, const std::vector<int>& fresh, const std::vector<int>& running,
                 std::vector<int>* stopped) {
  const int variant = S->o.solve.variant;
  for (int k : fresh) {
    Req* r = S->slots[k];
    const int G = (int)std::max<int64_t>(1, (r->n + S->tile - 1) / S->tile);
    ((SysDesc*)(S->h_hdr.data() + S->off_descs))[k] =
        make_desc(r->A, r->b, r->x, S->budget + r->off, r->gcap, G, variant, S->d_states + k, nullptr);
  }
  // [0]: requests whose Jacobi vector is uniform, [1]: the others
  std::vector<int> fresh_v[2], run_v[2];
  int64_t rows = 0;
  for (int k : fresh) fresh_v[S->slots[k]->A->unif ? 0 : 1].push_back(k);
  for (int k : running) {
    run_v[S->slots[k]->A->unif ? 0 : 1].push_back(k);
    rows += S->slots[k]->n;
  }
  // the two views share the Infinity Cache: one decision on all rows in flight
  const bool far = rows_stream_far(rows, variant, run_v[1].empty());
  int nt_new[2] = {0, 0}, nt_run[2] = {0, 0};
  for (int u = 0; u < 2; ++u) {
    RET_IF(set_view(S, V_NEW_U + u, fresh_v[u], u == 0, far, &nt_new[u]));
    RET_IF(set_view(S, V_RUN_U + u, run_v[u], u == 0, far, &nt_run[u]));
  }
  if (far)
    for (int k : running) S->slots[k]->streamed = true;
  RET_IF(upload(S));
  for (int u = 0; u < 2; ++u)
    if (!fresh_v[u].empty())
      RET_IF(by_fpe<SStartF>(S->N, variant, g_of(nt_new[u]), gf_of(fresh_v[u].size()), S->block, S->stream,
                             view(S, V_NEW_U + u), S->o.solve.tol, S->o.solve.maxit));
  const int chunk = S->o.chunk > 0 ? S->o.chunk : 4;
  const Batch run[2] = {view(S, V_RUN_U), view(S, V_RUN_N)};
  for (int it = 0; it < chunk; ++it)
    for (int ph = 0; ph < S->nph; ++ph)
      for (int u = 0; u < 2; ++u)
        if (!run_v[u].empty())
          RET_IF(by_fpe<SPhaseF>(S->N, variant, ph, g_of(nt_run[u]), gf_of(run_v[u].size()), S->block, S->stream,
                                 run[u]));
  S->st.iterations += chunk;
  HIPCHK(hipMemcpyAsync(S->h_states, S->d_states, (size_t)S->o.max_slots * sizeof(State),
                        hipMemcpyDeviceToHost, S->stream));
  HIPCHK(hipStreamSynchronize(S->stream));
  stopped->clear();
  for (int k : running)
    if (S->h_states[k].done) stopped->push_back(k);
  if (stopped->empty()) return RPK_OK;
  // exact true residual of the stopped systems
  int nt_fin = 0;
  RET_IF(set_view(S, V_FIN, *stopped, false, false, &nt_fin));
  RET_IF(upload(S));
  RET_IF(KernB<4>::resid(g_of(nt_fin), gf_of(stopped->size()), S->block, S->stream, view(S, V_FIN)));
  HIPCHK(hipMemcpyAsync(S->h_states, S->d_states, (size_t)S->o.max_slots * sizeof(State),
                        hipMemcpyDeviceToHost, S->stream));
  HIPCHK(hipStreamSynchronize(S->stream));
  return RPK_OK;
}

void fail_all(rpk_server* S, rpk_status why) {
  // with S->mu held
  S->failure = why;
  for (auto& kv : S->reqs) {
    Req* r = kv.second;
    if (!r->finished) {
      r->finished = true;
      r->info.status = why;
    }
  }
  S->queue.clear();
  S->cv_done.notify_all();
}

void worker_main(rpk_server* S) {
  if (hipSetDevice(S->device) != hipSuccess) {
    std::lock_guard<std::mutex> lk(S->mu);
    fail_all(S, RPK_ERR_HIP);
    return;
  }
  std::vector<int> running, fresh, stopped;
  for (;;) {
    fresh.clear();
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty() || !running.empty(); });
      if (S->failure != RPK_OK) return;
      if (S->stop && S->queue.empty() && running.empty()) return;
      // admission: first come, first served, by HBM footprint and free slots
      while (!S->queue.empty() && !S->free_slots.empty()) {
        Req* r = S->queue.front();
        size_t off = 0;
        if (!S->arena.alloc(r->bytes, &off)) break;
        S->queue.pop_front();
        r->off = off;
        r->slot = S->free_slots.back();
        S->free_slots.pop_back();
        S->slots[r->slot] = r;
        r->t_admit = Clock::now();
        fresh.push_back(r->slot);
        S->st.admitted += 1;
        S->st.bytes_in_use = S->arena.used();
        S->st.bytes_peak = S->arena.peak();
      }
    }
    for (int k : fresh) running.push_back(k);
    rpk_status rs = running.empty() ? RPK_OK : round(S, fresh, running, &stopped);
    std::lock_guard<std::mutex> lk(S->mu);
    S->st.rounds += 1;
    if (rs != RPK_OK) {
      fail_all(S, rs);
      return;
    }
    if (running.empty()) continue;
    const Clock::time_point now = Clock::now();
    for (int k : stopped) {
      Req* r = S->slots[k];
      const State& h = S->h_states[k];
      rpk_info& I = r->info;
      I.status = h.status;
      I.iters = h.iter;
      I.tau0 = h.tau0;
      I.tau = h.tau;
      I.true_res = h.true_res;
      I.used.block = S->block;
      I.used.fpe = S->N;
      I.used.tile = S->tile;
      I.used.graph = -1;
      I.streamed = r->streamed ? 1 : 0;
      I.queue_ms = ms_between(r->t_submit, r->t_admit);
      I.latency_ms = ms_between(r->t_submit, now);
      r->finished = true;
      S->arena.release(r->off, r->bytes);
      S->slots[k] = nullptr;
      S->free_slots.push_back(k);
      S->st.completed += 1;
      running.erase(std::find(running.begin(), running.end(), k));
    }
    S->st.bytes_in_use = S->arena.used();
    if (!stopped.empty()) S->cv_done.notify_all();
  }
}

size_t footprint(const rpk_server* S, int64_t n) {
  const int gcap = (int)std::max<int64_t>(1, (n + S->tile - 1) / S->tile);
  return sys_bytes(n, gcap, S->nvec);
}

rpk_status take(rpk_server* S, std::unique_lock<std::mutex>& lk, uint64_t ticket, rpk_info* info, bool block) {
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return RPK_ERR_ARG;
  Req* r = it->second;
  if (!r->finished) {
    if (!block) return RPK_PENDING;
    S->cv_done.wait(lk, [&] { return r->finished; });
  }
  *info = r->info;
  S->reqs.erase(it);
  delete r;
  return RPK_OK;
}

}  // namespace

extern "C" {

rpk_status rpk_server_create(const rpk_server_opts* o, rpk_server** out) {
  if (!o || !out) return RPK_ERR_ARG;
  *out = nullptr;
  const rpk_opts& so = o->solve;
  if (o->hbm_budget < 4096 || o->max_slots < 1 || o->max_slots > 65536 || o->chunk < 0) return RPK_ERR_ARG;
  if (so.variant != RPK_STD && so.variant != RPK_PIPELINED && so.variant != RPK_PCG) return RPK_ERR_ARG;
  if (so.dots != RPK_DOT_EXACT && so.dots != RPK_DOT_PLAIN) return RPK_ERR_ARG;
  if (so.maxit < 0 || !(so.tol >= 0.0) || so.hist || so.xr_hist || so.timing || so.resume) return RPK_ERR_ARG;
  const rpk_launch& l = so.launch;
  if (l.block && (l.block < 64 || l.block > 1024 || l.block % 64)) return RPK_ERR_ARG;
  if (l.fpe && l.fpe != 1 && l.fpe != 2 && l.fpe != 3 && l.fpe != 4 && l.fpe != 8) return RPK_ERR_ARG;
  if (l.tile && (l.tile < 64 || l.tile > (1 << 20) || l.tile % 64)) return RPK_ERR_ARG;
  rpk_server* S = new (std::nothrow) rpk_server();
  if (!S) return RPK_ERR_NOMEM;
  S->o = *o;
  S->block = l.block ? l.block : 512;
  S->tile = l.tile ? l.tile : 4096;
  S->N = (so.dots == RPK_DOT_PLAIN) ? 0 : (l.fpe ? l.fpe : 3);
  S->nvec = nvec_of(so.variant);
  S->nph = (so.variant == RPK_STD) ? 5 : (so.variant == RPK_PCG) ? 3 : 4;
  rpk_status st = RPK_OK;
  do {
    if (hipGetDevice(&S->device) != hipSuccess) { st = RPK_ERR_HIP; break; }
    if (hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess) { st = RPK_ERR_HIP; break; }
    if (hipMalloc((void**)&S->budget, o->hbm_budget) != hipSuccess) { st = RPK_ERR_NOMEM; break; }
    if (hipMalloc((void**)&S->d_states, (size_t)o->max_slots * sizeof(State)) != hipSuccess) {
      st = RPK_ERR_NOMEM;
      break;
    }
    if (hipHostMalloc((void**)&S->h_states, (size_t)o->max_slots * sizeof(State), hipHostMallocDefault) != hipSuccess) {
      st = RPK_ERR_NOMEM;
      break;
    }
    st = layout_header(S, 8 * ((int64_t)o->max_slots + 64));
  } while (0);
  if (st != RPK_OK) {
    if (S->hdr) (void)hipFree(S->hdr);
    if (S->d_states) (void)hipFree(S->d_states);
    if (S->budget) (void)hipFree(S->budget);
    if (S->h_states) (void)hipHostFree(S->h_states);
    if (S->stream) (void)hipStreamDestroy(S->stream);
    delete S;
    return st;
  }
  S->arena.reset(o->hbm_budget / kAlign * kAlign);
  S->slots.assign((size_t)o->max_slots, nullptr);
  for (int k = o->max_slots - 1; k >= 0; --k) S->free_slots.push_back(k);
  S->worker = std::thread(worker_main, S);
  *out = S;
  return RPK_OK;
}

rpk_status rpk_server_footprint(const rpk_server* s, const rpk_matrix* A, size_t* bytes) {
  if (!s || !A || !bytes) return RPK_ERR_ARG;
  *bytes = footprint(s, A->n);
  return RPK_OK;
}

rpk_status rpk_server_submit(rpk_server* s, const rpk_matrix* A, const double* b, double* x, uint64_t* ticket) {
  if (!s || !A || !b || !x || !ticket) return RPK_ERR_ARG;
  const int64_t gcap = std::max<int64_t>(1, (A->n + s->tile - 1) / s->tile);
  // the request's reduction records (its tiles) must fit the carry budget
  if (!records_fit(gcap, std::min(s->block, s->tile), s->N)) return RPK_ERR_ARG;
  const size_t bytes = footprint(s, A->n);
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->failure != RPK_OK) return s->failure;
  if (s->stop) return RPK_ERR_ARG;
  if (bytes > s->o.hbm_budget / kAlign * kAlign) {
    s->st.rejected += 1;
    return RPK_REJECTED;
  }
  Req* r = new (std::nothrow) Req();
  if (!r) return RPK_ERR_NOMEM;
  r->id = s->next_id++;
  r->A = A;
  r->b = b;
  r->x = x;
  r->n = A->n;
  r->gcap = (int)gcap;
  r->bytes = bytes;
  r->t_submit = Clock::now();
  std::memset(&r->info, 0, sizeof(r->info));
  s->reqs[r->id] = r;
  s->queue.push_back(r);
  s->st.submitted += 1;
  *ticket = r->id;
  s->cv_work.notify_one();
  return RPK_OK;
}

rpk_status rpk_server_poll(rpk_server* s, uint64_t ticket, rpk_info* info) {
  if (!s || !info) return RPK_ERR_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  return take(s, lk, ticket, info, false);
}

rpk_status rpk_server_wait(rpk_server* s, uint64_t ticket, rpk_info* info) {
  if (!s || !info) return RPK_ERR_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  return take(s, lk, ticket, info, true);
}

rpk_status rpk_server_get_stats(const rpk_server* s, rpk_server_stats* out) {
  if (!s || !out) return RPK_ERR_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  out->queued = (int32_t)s->queue.size();
  int inflight = 0;
  for (const Req* r : s->slots) inflight += (r != nullptr);
  out->in_flight = inflight;
  out->bytes_in_use = s->arena.used();
  out->bytes_peak = s->arena.peak();
  return RPK_OK;
}

rpk_status rpk_server_destroy(rpk_server* s) {
  if (!s) return RPK_ERR_ARG;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  rpk_status st = s->failure;
  for (auto& kv : s->reqs) delete kv.second;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  if (s->hdr) (void)hipFree(s->hdr);
  if (s->d_states) (void)hipFree(s->d_states);
  if (s->budget) (void)hipFree(s->budget);
  if (s->h_states) (void)hipHostFree(s->h_states);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
  return st;
}

}  // extern "C"
