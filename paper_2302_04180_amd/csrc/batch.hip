// batch.hip -- rpk_solve_batched: many independent systems, one launch per
// phase for all of them, iterations replayed from HIP graphs, tile shape picked
// by a small autotuner.
//
// Workspace (256-byte aligned pieces):
//   header : tile/system counts | States[nsys] | SysDesc[nsys] | order[nsys] | Tile[cap]
//   per system k: tickets+flags | long accumulators | plain-mode tile sums
//                 (cap_k tiles) | solver vectors
//   trial  : one x per system (only when the autotuner may run)
// The header is written with one host-to-device copy per call; everything the
// kernels need is found through it, so a cached graph only depends on the
// workspace address, the launch shape and whether the batch's far vectors are
// streamed (which picks the kernel instantiations captured).
#include <algorithm>
#include <cstring>
#include <numeric>

#include "host.h"

using namespace rpk;
using namespace rpkhost;

namespace {

constexpr int kTileMinAuto = 1024;  // smallest tile the autotuner tries
constexpr int kMaxSys = 65536;

struct BCfg {
  int tile, block, fpe, graph, grid_cap;
};

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

namespace rpkhost {

// Cut every system into tiles of at most T rows (64-aligned starts, near-equal
// sizes), give whole systems to the 8 XCDs (largest first, to the XCD with the
// fewest tiles so far) so that a system's SpMV gathers stay in one L2, and
// interleave the 8 lists so that tile t lands on XCD t % 8 (workgroups are
// dispatched to XCDs round-robin).  Short lists are padded with empty tiles.
Plan make_plan(const std::vector<int64_t>& n, int T, const std::vector<int>* ids) {
  const int ns = (int)n.size();
  Plan p;
  p.G.resize(ns);
  std::vector<int64_t> chunk(ns);
  for (int k = 0; k < ns; ++k) {
    const int64_t g = std::max<int64_t>(1, cdiv(n[k], T));
    p.G[k] = (int)g;
    chunk[k] = (cdiv(n[k], g) + 63) / 64 * 64;
  }
  std::vector<int> idx(ns);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return p.G[a] > p.G[b]; });
  std::vector<int64_t> load(8, 0);
  std::vector<std::vector<int>> bins(8);
  for (int k : idx) {
    const int bin = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    load[bin] += p.G[k];
    bins[bin].push_back(k);
  }
  const int64_t rows = *std::max_element(load.begin(), load.end());
  p.tiles.assign((size_t)(8 * rows), Tile{-1, 0, 0, 0});
  for (int bin = 0; bin < 8; ++bin) {
    int64_t pos = 0;
    for (int k : bins[bin])
      for (int j = 0; j < p.G[k]; ++j, ++pos) {
        const int64_t lo = j * chunk[k], hi = std::min<int64_t>(n[k], lo + chunk[k]);
        p.tiles[(size_t)(8 * pos + bin)] = Tile{ids ? (*ids)[k] : k, (int)lo, (int)hi, j};
      }
  }
  return p;
}

int64_t tile_capacity(const std::vector<int64_t>& n, int Tcap) {
  int64_t sum = 0, mx = 0;
  for (int64_t v : n) {
    const int64_t g = std::max<int64_t>(1, cdiv(v, Tcap));
    sum += g;
    mx = std::max(mx, g);
  }
  return 8 * (cdiv(sum, 8) + mx);
}

size_t sys_bytes(int64_t n, int gcap, int nvec) {
  return up(kFlagsBytes) + up((size_t)MAX_DOTS * SA_D * 8) + up((size_t)MAX_DOTS * gcap * 8) +
         (size_t)nvec * up((size_t)n * 8);
}

SysDesc make_desc(const rpk_matrix* A, const double* b, double* x, char* base, int gcap, int G, int variant,
                  State* st, double* hist) {
  Red r;
  r.tickets = (unsigned*)base;
  r.gflags = (int*)(base + 8 * sizeof(unsigned));
  r.gsa = (long long*)(base + up(kFlagsBytes));
  r.partials = (double*)(base + up(kFlagsBytes) + up((size_t)MAX_DOTS * SA_D * 8));
  r.G = G;
  char* vec = (char*)r.partials + up((size_t)MAX_DOTS * gcap * 8);
  const size_t step = up((size_t)A->n * 8);
  double* p[16];
  for (int j = 0; j < nvec_of(variant); ++j) p[j] = (double*)(vec + j * step);
  Vecs V;
  std::memset(&V, 0, sizeof(V));
  if (variant == RPK_PCG) {  // r, p, d (in s), y
    V.r = p[0]; V.p = p[1]; V.s = p[2]; V.y = p[3];
  } else {
    V.r0 = p[0]; V.r = p[1]; V.p = p[2]; V.ph = p[3]; V.s = p[4]; V.q = p[5]; V.qh = p[6]; V.y = p[7];
  }
  if (variant == RPK_PIPELINED) {
    V.rh = p[8]; V.w = p[9]; V.wh = p[10]; V.t = p[11]; V.sh = p[12]; V.z = p[13]; V.zh = p[14]; V.v = p[15];
  }
  V.x = x;
  V.b = b;
  V.st = st;
  V.hist = hist;
  V.xr = nullptr;
  SysDesc D;
  D.A = csr_of(A);
  D.V = V;
  D.red = r;
  return D;
}

}  // namespace rpkhost

namespace {

struct BLayout {
  size_t count, states, descs, order, tiles, header;
  std::vector<size_t> sys;  // per-system block offsets
  std::vector<int> gcap;    // record capacity per system
  size_t trial, total;
  int64_t cap_tiles;
};

BLayout blayout(const std::vector<int64_t>& n, int nvec, int Tcap, bool trial) {
  BLayout L;
  const size_t ns = n.size();
  size_t off = 0;
  L.count = off;
  off += up(2 * sizeof(int));
  L.states = off;
  off += up(ns * sizeof(State));
  L.descs = off;
  off += up(ns * sizeof(SysDesc));
  L.order = off;
  off += up(ns * sizeof(int));
  L.cap_tiles = tile_capacity(n, Tcap);
  L.tiles = off;
  off += up((size_t)L.cap_tiles * sizeof(Tile));
  L.header = off;
  L.sys.resize(ns);
  L.gcap.resize(ns);
  for (size_t k = 0; k < ns; ++k) {
    L.gcap[k] = (int)std::max<int64_t>(1, cdiv(n[k], Tcap));
    L.sys[k] = off;
    off += sys_bytes(n[k], L.gcap[k], nvec);
  }
  L.trial = off;
  if (trial)
    for (size_t k = 0; k < ns; ++k) off += up((size_t)n[k] * 8);
  L.total = off;
  return L;
}

rpk_status check_opts(const rpk_opts* o) {
  if (!o) return RPK_ERR_ARG;
  if (o->variant != RPK_STD && o->variant != RPK_PIPELINED && o->variant != RPK_PCG) return RPK_ERR_ARG;
  if (o->dots != RPK_DOT_EXACT && o->dots != RPK_DOT_PLAIN) return RPK_ERR_ARG;
  if (o->maxit < 0 || !(o->tol >= 0.0) || o->xr_hist || o->resume) return RPK_ERR_ARG;
  const rpk_launch& l = o->launch;
  if (l.block && (l.block < 64 || l.block > 1024 || l.block % 64)) return RPK_ERR_ARG;
  if (l.fpe && l.fpe != 1 && l.fpe != 2 && l.fpe != 3 && l.fpe != 4 && l.fpe != 8) return RPK_ERR_ARG;
  if (l.graph < -1 || l.grid < 0 || l.grid > 65535) return RPK_ERR_ARG;
  if (l.tile && (l.tile < 64 || l.tile > (1 << 20) || l.tile % 64)) return RPK_ERR_ARG;
  return RPK_OK;
}

template <int N>
struct BSetupF {
  static rpk_status call(int Gf, hipStream_t s, Batch b, double tol, int maxit, int variant) {
    return KernB<N>::setup(Gf, s, b, tol, maxit, variant);
  }
};
template <int N>
struct BInitF {
  static rpk_status call(int variant, int G, int Gf, int B, hipStream_t s, Batch b) {
    return KernB<N>::init(variant, G, Gf, B, s, b);
  }
};
template <int N>
struct BPhaseF {
  static rpk_status call(int variant, int ph, int G, int Gf, int B, hipStream_t s, Batch b) {
    return KernB<N>::phase(variant, ph, G, Gf, B, s, b);
  }
};

struct Ctx {
  int ns;
  const rpk_matrix* const* A;
  const double* const* b;
  double* const* x;
  const rpk_opts* o;
  char* ws;
  hipStream_t s;
  std::vector<int64_t> n;
  BLayout L;
};

Batch batch_of(const Ctx& c) {
  Batch B;
  B.count = (const int*)(c.ws + c.L.count);
  B.sys = (const SysDesc*)(c.ws + c.L.descs);
  B.order = (const int*)(c.ws + c.L.order);
  B.tiles = (const Tile*)(c.ws + c.L.tiles);
  int64_t rows = 0;
  bool unif = true;
  for (int k = 0; k < c.ns; ++k) {
    rows += c.n[k];
    unif = unif && c.A[k]->unif != 0;
  }
  B.far = rows_stream_far(rows, c.o->variant, unif) ? 1 : 0;
  B.unif = unif ? 1 : 0;
  return B;
}

// Write the header (counts, descriptors, order, tile table) for `plan`.
rpk_status upload(const Ctx& c, const Plan& plan, bool trial) {
  if ((int64_t)plan.tiles.size() > c.L.cap_tiles) return RPK_ERR_ARG;
  std::vector<char> h(c.L.header, 0);
  int cnt[2] = {(int)plan.tiles.size(), c.ns};
  std::memcpy(h.data() + c.L.count, cnt, sizeof(cnt));
  SysDesc* D = (SysDesc*)(h.data() + c.L.descs);
  int* order = (int*)(h.data() + c.L.order);
  size_t trial_off = c.L.trial;
  const int variant = c.o->variant;
  for (int k = 0; k < c.ns; ++k) {
    order[k] = k;
    if (plan.G[k] > c.L.gcap[k]) return RPK_ERR_ARG;
    double* x = c.x[k];
    if (trial) {
      x = (double*)(c.ws + trial_off);
      trial_off += up((size_t)c.n[k] * 8);
    }
    double* hist = (!trial && c.o->hist) ? c.o->hist + (size_t)k * c.o->maxit * HIST_W : nullptr;
    D[k] = make_desc(c.A[k], c.b[k], x, c.ws + c.L.sys[k], c.L.gcap[k], plan.G[k], variant,
                     (State*)(c.ws + c.L.states) + k, hist);
  }
  std::memcpy(h.data() + c.L.tiles, plan.tiles.data(), plan.tiles.size() * sizeof(Tile));
  HIPCHK(hipMemcpyAsync(c.ws, h.data(), c.L.header, hipMemcpyHostToDevice, c.s));
  HIPCHK(hipStreamSynchronize(c.s));  // h goes out of scope
  return RPK_OK;
}

struct Shape {
  int G, Gf, B, N, nph;
};

Shape shape_of(const Ctx& c, const BCfg& cfg, const Plan& plan) {
  Shape sh;
  const int nt = (int)plan.tiles.size();  // a multiple of 8
  const int cap = cfg.grid_cap ? std::min((cfg.grid_cap + 7) & ~7, 64000) : 64000;
  sh.G = std::max(8, std::min(nt, cap));
  sh.Gf = std::min((c.ns + 7) & ~7, 1024);
  sh.B = cfg.block;
  sh.N = (c.o->dots == RPK_DOT_PLAIN) ? 0 : cfg.fpe;
  sh.nph = (c.o->variant == RPK_STD) ? 5 : (c.o->variant == RPK_PCG) ? 3 : 4;
  return sh;
}

rpk_status read_states(const Ctx& c, State** out) {
  State* h = pinned_states((size_t)c.ns);
  if (!h) return RPK_ERR_NOMEM;
  HIPCHK(hipMemcpyAsync(h, c.ws + c.L.states, (size_t)c.ns * sizeof(State), hipMemcpyDeviceToHost, c.s));
  HIPCHK(hipStreamSynchronize(c.s));
  *out = h;
  return RPK_OK;
}

bool all_done(const State* h, int ns) {
  for (int k = 0; k < ns; ++k)
    if (!h[k].done) return false;
  return true;
}

// Set-up + first reduction for every system (x from the caller, or from the
// trial copies of x0).
rpk_status start(const Ctx& c, const BCfg& cfg, const Plan& plan, bool trial, Shape* out) {
  RET_IF(upload(c, plan, trial));
  const Shape sh = shape_of(c, cfg, plan);
  const Batch bt = batch_of(c);
  if (trial) {
    size_t off = c.L.trial;
    for (int k = 0; k < c.ns; ++k) {
      HIPCHK(hipMemcpyAsync(c.ws + off, c.x[k], (size_t)c.n[k] * 8, hipMemcpyDeviceToDevice, c.s));
      off += up((size_t)c.n[k] * 8);
    }
  } else if (c.o->hist) {
    HIPCHK(hipMemsetAsync(c.o->hist, 0, (size_t)c.ns * c.o->maxit * HIST_W * sizeof(double), c.s));
  }
  RET_IF(by_fpe<BSetupF>(sh.N, sh.Gf, c.s, bt, c.o->tol, c.o->maxit, c.o->variant));
  RET_IF(by_fpe<BInitF>(sh.N, c.o->variant, sh.G, sh.Gf, sh.B, c.s, bt));
  *out = sh;
  return RPK_OK;
}

rpk_status iterate_direct(const Ctx& c, const Shape& sh, int iters) {
  const Batch bt = batch_of(c);
  for (int k = 0; k < iters; ++k)
    for (int ph = 0; ph < sh.nph; ++ph) RET_IF(by_fpe<BPhaseF>(sh.N, c.o->variant, ph, sh.G, sh.Gf, sh.B, c.s, bt));
  return RPK_OK;
}

// Average time of one batch iteration (ms) for a candidate configuration, on
// scratch copies of x0 and without the caller's histories.
rpk_status trial_time(const Ctx& c, const BCfg& cfg, float* ms) {
  const Plan plan = make_plan(c.n, cfg.tile);
  Shape sh;
  RET_IF(start(c, cfg, plan, true, &sh));
  RET_IF(iterate_direct(c, sh, 1));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return RPK_ERR_HIP;
  }
  constexpr int kIters = 3;
  rpk_status st = RPK_OK;
  if (hipEventRecord(e0, c.s) != hipSuccess) st = RPK_ERR_HIP;
  if (st == RPK_OK) st = iterate_direct(c, sh, kIters);
  if (st == RPK_OK && (hipEventRecord(e1, c.s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
    st = RPK_ERR_HIP;
  float t = 0.f;
  if (st == RPK_OK && hipEventElapsedTime(&t, e0, e1) != hipSuccess) st = RPK_ERR_HIP;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = t / kIters;
  return st;
}

std::map<std::vector<int64_t>, BCfg> g_tuned;  // guarded by lib_mutex()

// Every system's reduction records (its tiles) fit the carry budget of the long
// accumulators at this tile / workgroup / FPE length (plain sums have none).
bool plan_fits(const Plan& plan, const BCfg& cfg, bool plain) {
  const int64_t lanes = std::min(cfg.block, cfg.tile);
  for (int g : plan.G)
    if (!records_fit(g, lanes, plain ? 0 : cfg.fpe)) return false;
  return true;
}

// The configurations rpk_solve_batched may run: the caller's tile, or the
// autotuner's candidates (tile rows x workgroup size x FPE length, with the
// caller's workgroup size / FPE length where given), those that fit the carry
// budget for systems of n rows.
std::vector<BCfg> configs_for(const std::vector<int64_t>& n, const rpk_opts* o) {
  const bool plain = o->dots == RPK_DOT_PLAIN;
  std::vector<BCfg> out;
  if (o->launch.tile) {
    out.push_back(BCfg{o->launch.tile, o->launch.block ? o->launch.block : 512, o->launch.fpe ? o->launch.fpe : 3,
                       o->launch.graph, o->launch.grid});
  } else {
    struct Cand {
      int tile, block, fpe;
    };
    const Cand all[] = {{1024, 256, 3}, {2048, 512, 3}, {4096, 512, 3}, {8192, 512, 3},
                        {4096, 1024, 3}, {16384, 1024, 3}, {4096, 512, 4}, {4096, 512, 2}};
    for (const Cand& cd : all) {
      if (plain && cd.fpe != 3) continue;  // the FPE length does not exist in plain mode
      if (cd.tile < kTileMinAuto) continue;
      out.push_back(BCfg{cd.tile, o->launch.block ? o->launch.block : cd.block,
                         o->launch.fpe ? o->launch.fpe : cd.fpe, -1, o->launch.grid});
    }
  }
  std::vector<BCfg> fit;
  for (const BCfg& cfg : out)
    if (plan_fits(make_plan(n, cfg.tile), cfg, plain)) fit.push_back(cfg);
  return fit;
}

rpk_status autotune(const Ctx& c, BCfg* best) {
  int64_t sum_n = 0, sum_nnz = 0, max_n = 0;
  for (int k = 0; k < c.ns; ++k) {
    sum_n += c.n[k];
    sum_nnz += c.A[k]->nnz;
    max_n = std::max(max_n, c.n[k]);
  }
  const bool plain = c.o->dots == RPK_DOT_PLAIN;
  const std::vector<int64_t> key{c.ns, sum_n, sum_nnz, max_n, c.o->variant, plain, c.o->launch.block,
                                 c.o->launch.fpe, c.o->launch.grid};
  auto it = g_tuned.find(key);
  if (it != g_tuned.end()) {
    *best = it->second;
    best->graph = c.o->launch.graph;
    return RPK_OK;
  }
  const std::vector<BCfg> cands = configs_for(c.n, c.o);
  if (cands.empty()) return RPK_ERR_ARG;
  float best_ms = -1.f;
  for (const BCfg& cfg : cands) {
    float ms = 0.f;
    RET_IF(trial_time(c, cfg, &ms));
    if (best_ms < 0.f || ms < best_ms) {
      best_ms = ms;
      *best = cfg;
    }
  }
  g_tuned[key] = *best;
  best->graph = c.o->launch.graph;
  return RPK_OK;
}

rpk_status run(const Ctx& c, const BCfg& cfg, rpk_info* infos) {
  const Plan plan = make_plan(c.n, cfg.tile);
  Shape sh;
  const bool timing = c.o->timing != 0;
  hipEvent_t ev[RPK_NPHASE + 1] = {};
  rpk_status st = RPK_OK;
  if (timing)
    for (int k = 0; k <= RPK_NPHASE && st == RPK_OK; ++k)
      if (hipEventCreate(&ev[k]) != hipSuccess) st = RPK_ERR_HIP;
  auto elapsed = [&](int a, int b, int slot) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev[a], ev[b]);
    infos[0].phase_ms[slot] += ms;
    infos[0].phase_launches[slot] += 1;
  };
  State* h = nullptr;
  const int bt_far = batch_of(c).far;
  do {
    if (st != RPK_OK) break;
    if (timing && hipEventRecord(ev[0], c.s) != hipSuccess) { st = RPK_ERR_HIP; break; }
    st = start(c, cfg, plan, false, &sh);
    if (st != RPK_OK) break;
    if (timing) {
      if (hipEventRecord(ev[1], c.s) != hipSuccess || hipEventSynchronize(ev[1]) != hipSuccess) { st = RPK_ERR_HIP; break; }
      elapsed(0, 1, 8);
    }
    const Batch bt = batch_of(c);
    const bool use_graph = !timing && cfg.graph >= 0;
    int chunk = cfg.graph > 0 ? cfg.graph : 4;
    long long launched = 0;
    for (;;) {
      st = read_states(c, &h);
      if (st != RPK_OK || all_done(h, c.ns)) break;
      if (launched > (long long)c.o->maxit + 8) { st = RPK_ERR_HIP; break; }  // the device stops at maxit
      if (timing) {
        for (int ph = 0; ph < sh.nph && st == RPK_OK; ++ph) {
          if (hipEventRecord(ev[ph], c.s) != hipSuccess) st = RPK_ERR_HIP;
          if (st == RPK_OK) st = by_fpe<BPhaseF>(sh.N, c.o->variant, ph, sh.G, sh.Gf, sh.B, c.s, bt);
        }
        if (st != RPK_OK) break;
        if (hipEventRecord(ev[sh.nph], c.s) != hipSuccess || hipEventSynchronize(ev[sh.nph]) != hipSuccess) {
          st = RPK_ERR_HIP;
          break;
        }
        for (int ph = 0; ph < sh.nph; ++ph) elapsed(ph, ph + 1, ph);
        launched += 1;
      } else if (use_graph) {
        const std::vector<uint64_t> key{0, (uint64_t)(uintptr_t)c.ws, (uint64_t)c.L.count, (uint64_t)c.L.descs,
                                        (uint64_t)c.L.order, (uint64_t)c.L.tiles, (uint64_t)c.o->variant,
                                        (uint64_t)sh.N, (uint64_t)sh.G, (uint64_t)sh.Gf, (uint64_t)sh.B,
                                        (uint64_t)chunk, (uint64_t)bt.far, 0xba7c4ull};
        hipGraphExec_t exec = nullptr;
        st = graph_get(key, [&](hipStream_t cs) {
          rpk_status cst = RPK_OK;
          for (int k = 0; k < chunk && cst == RPK_OK; ++k)
            for (int ph = 0; ph < sh.nph && cst == RPK_OK; ++ph)
              cst = by_fpe<BPhaseF>(sh.N, c.o->variant, ph, sh.G, sh.Gf, sh.B, cs, bt);
          return cst;
        }, &exec);
        if (st != RPK_OK) break;
        if (hipGraphLaunch(exec, c.s) != hipSuccess) { st = RPK_ERR_HIP; break; }
        launched += chunk;
        if (cfg.graph == 0 && chunk < 32) chunk *= 2;
      } else {
        st = iterate_direct(c, sh, chunk);
        if (st != RPK_OK) break;
        launched += chunk;
      }
    }
    if (st != RPK_OK) break;
    // true residual of every returned iterate, exact
    if (timing && hipEventRecord(ev[0], c.s) != hipSuccess) { st = RPK_ERR_HIP; break; }
    st = KernB<4>::resid(sh.G, sh.Gf, sh.B, c.s, bt);
    if (st != RPK_OK) break;
    if (timing) {
      if (hipEventRecord(ev[1], c.s) != hipSuccess || hipEventSynchronize(ev[1]) != hipSuccess) { st = RPK_ERR_HIP; break; }
      elapsed(0, 1, 9);
    }
    st = read_states(c, &h);
  } while (0);
  if (timing)
    for (int k = 0; k <= RPK_NPHASE; ++k)
      if (ev[k]) (void)hipEventDestroy(ev[k]);
  if (st != RPK_OK) return st;
  rpk_status first = RPK_OK;
  for (int k = 0; k < c.ns; ++k) {
    rpk_info& I = infos[k];
    I.status = h[k].status;
    I.iters = h[k].iter;
    I.tau0 = h[k].tau0;
    I.tau = h[k].tau;
    I.true_res = h[k].true_res;
    I.used.block = sh.B;
    I.used.grid = sh.G;
    I.used.fpe = sh.N;
    I.used.graph = cfg.graph;
    I.used.tile = cfg.tile;
    I.streamed = bt_far;
    if (first == RPK_OK && h[k].status != RPK_OK) first = (rpk_status)h[k].status;
  }
  return first;
}

rpk_status prepare(int32_t nsys, const rpk_matrix* const* A, const rpk_opts* o, std::vector<int64_t>* n) {
  if (nsys < 1 || nsys > kMaxSys || !A) return RPK_ERR_ARG;
  RET_IF(check_opts(o));
  n->resize(nsys);
  for (int k = 0; k < nsys; ++k) {
    if (!A[k]) return RPK_ERR_ARG;
    (*n)[k] = A[k]->n;
  }
  if (configs_for(*n, o).empty()) return RPK_ERR_ARG;  // over the carry budget
  return RPK_OK;
}

}  // namespace

extern "C" {

rpk_status rpk_plan_tiles(int32_t nsys, const int64_t* n, int32_t tile, int32_t* tiles, int64_t cap,
                          int64_t* ntiles) {
  if (nsys < 1 || nsys > kMaxSys || !n || !tiles || !ntiles || tile < 64 || tile % 64) return RPK_ERR_ARG;
  std::vector<int64_t> nv(n, n + nsys);
  for (int64_t v : nv)
    if (v < 1 || v >= (1ll << 31)) return RPK_ERR_ARG;
  const Plan p = make_plan(nv, tile);
  *ntiles = (int64_t)p.tiles.size();
  if ((int64_t)p.tiles.size() > cap) return RPK_ERR_ARG;
  for (size_t t = 0; t < p.tiles.size(); ++t) {
    tiles[4 * t + 0] = p.tiles[t].sys;
    tiles[4 * t + 1] = p.tiles[t].lo;
    tiles[4 * t + 2] = p.tiles[t].hi;
    tiles[4 * t + 3] = p.tiles[t].rec;
  }
  return RPK_OK;
}

rpk_status rpk_batched_check(int32_t nsys, const int64_t* n, const rpk_opts* opts) {
  if (nsys < 1 || nsys > kMaxSys || !n) return RPK_ERR_ARG;
  RET_IF(check_opts(opts));
  std::vector<int64_t> nv(n, n + nsys);
  for (int64_t v : nv)
    if (v < 1 || v >= (1ll << 31)) return RPK_ERR_ARG;
  return configs_for(nv, opts).empty() ? RPK_ERR_ARG : RPK_OK;
}

rpk_status rpk_solve_batched_workspace_bytes(int32_t nsys, const rpk_matrix* const* A, const rpk_opts* o,
                                             size_t* bytes) {
  if (!bytes) return RPK_ERR_ARG;
  std::vector<int64_t> n;
  RET_IF(prepare(nsys, A, o, &n));
  const int tile = o->launch.tile;
  *bytes = blayout(n, nvec_of(o->variant), tile ? tile : kTileMinAuto, tile == 0).total;
  return RPK_OK;
}

rpk_status rpk_solve_batched(int32_t nsys, const rpk_matrix* const* A, const double* const* b, double* const* x,
                             const rpk_opts* o, void* ws, size_t ws_bytes, void* stream, rpk_info* infos) {
  if (!b || !x || !ws || !infos) return RPK_ERR_ARG;
  Ctx c;
  RET_IF(prepare(nsys, A, o, &c.n));
  for (int k = 0; k < nsys; ++k)
    if (!b[k] || !x[k]) return RPK_ERR_ARG;
  std::memset(infos, 0, sizeof(rpk_info) * (size_t)nsys);
  const int tile = o->launch.tile;
  c.L = blayout(c.n, nvec_of(o->variant), tile ? tile : kTileMinAuto, tile == 0);
  if (ws_bytes < c.L.total) return RPK_ERR_ARG;
  c.ns = nsys;
  c.A = A;
  c.b = b;
  c.x = x;
  c.o = o;
  c.ws = (char*)ws;
  c.s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(lib_mutex());
  RET_IF(ensure_globals());
  BCfg cfg;
  if (tile) {
    cfg = configs_for(c.n, o)[0];  // prepare() checked that it fits
  } else {
    RET_IF(autotune(c, &cfg));
  }
  return run(c, cfg, infos);
}

}  // extern "C"
