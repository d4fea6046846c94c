// host.h -- host-side pieces shared by the single-system solver (rpk.hip), the
// batched solver (batch.hip) and the request server (server.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <vector>

#include "kern.h"
#include "rpk.h"

struct rpk_matrix {
  int64_t n = 0, nnz = 0;
  int* rp = nullptr;  // CSR as given (validated), kept for reference
  int* ci = nullptr;
  double* v = nullptr;
  double* dinv = nullptr;
  int nslices = 0;    // SELL-64 copy used by the kernels
  long long* sptr = nullptr;
  int* scol = nullptr;
  double* sval = nullptr;
  long long sell_entries = 0;      // entries of the SELL copy, padding included
  int cert = 0;                    // rows of wide slices try the certified sum (see Csr)
  int unif = 0;                    // every dinv_i has the bits of du (see Csr)
  double du = 0.0;
};

namespace rpkhost {

using namespace rpk;

#define HIPCHK(call)                              \
  do {                                            \
    if ((call) != hipSuccess) return RPK_ERR_HIP; \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Carry budget of the exact reductions.  Long-accumulator digits are int64
// words that receive signed 32-bit chunks and propagate no carry until the final
// rounding, so the number of chunks a digit can receive is what bounds a sum
// (Sec. 3.2 bounds the merges of its 52+12 split the same way):
//   - a workgroup's LDS accumulator takes, per digit, at most two chunks per
//     product it sums (the twoprod terms p and e) plus one per FPE component it
//     flushes: kMaxPerGroup elements per workgroup keep 2^30 + 8*1024 chunks of
//     < 2^32 below 2^63;
//   - a global accumulator takes, per digit and per published record, at most
//     one chunk per FPE component of every lane that had data, plus one digit of
//     the workgroup's normalised LDS accumulator: a reduction of R records from
//     L lanes with FPE length N stays below 2^63 when R (L N + 1) < 2^31.
// Single solves always fit the second rule (grid <= 65535, L <= 1024, N <= 8);
// the batched solver and the server check it per system (records = tiles).
constexpr int64_t kMaxPerGroup = int64_t(1) << 29;
// Solves of at most this many rows with the automatic launch shape run in one
// workgroup (standard and PCG loops, exact and plain dots): with exact dots
// measured faster at 512 rows and slower from 1,000 on, where one CU's share of
// the exact rows and dots outweighs the launches it saves (the pipelined loop
// ran slower in one workgroup already at 512 rows)
constexpr int64_t kOneGroupRows = 512;
// Solves of fewer rows with the automatic launch shape use workgroups of 256
// threads instead of 512: measured 3-12 % faster from 1,728 to 32,768 rows
// (7-point Poisson, all three loops), slower from 110,592 on
constexpr int64_t kSmallBlockRows = 65536;
// Largest automatic chunk of iterations between two looks at a solve's state
constexpr int kMaxChunk = 64;
constexpr int64_t kCarryChunks = (int64_t(1) << 31) - 1;
inline bool records_fit(int64_t records, int64_t lanes, int fpe) {
  return records * (lanes * (int64_t)fpe + 1) <= kCarryChunks;
}

inline Csr csr_of(const rpk_matrix* A) {
  return Csr{A->sptr, A->scol, A->sval, A->dinv, (int)A->n, A->cert, 0, A->unif, A->du};
}

inline int nvec_of(int variant) { return variant == RPK_STD ? 8 : variant == RPK_PCG ? 4 : 16; }

// MI355X's Infinity Cache: 256 MiB in front of HBM, shared by all XCDs.
constexpr double kInfinityCacheBytes = 256.0 * 1024 * 1024;

// Leading SELL slices of A read with ordinary loads (Csr::keep): as much of
// the matrix as fits in nine tenths of the Infinity Cache next to `nvec`
// n-vectors (those one solver iteration touches, or x and y of a lone SpMV),
// so that the next SpMV finds it there.  Slices are counted in proportion to
// the SELL entries.
inline int keep_slices(const rpk_matrix* A, int nvec) {
  const double vecs = (double)nvec * (double)A->n * 8.0;
  const double room = 0.9 * kInfinityCacheBytes - vecs;
  const double sell = (double)A->sell_entries * 12.0;
  if (room <= 0.0 || sell <= 0.0) return 0;
  if (room >= sell) return A->nslices;
  return (int)((double)A->nslices * (room / sell));
}

// Vectors one standard iteration touches: its eight work vectors, x and the
// Jacobi vector; with a uniform Jacobi vector p^ and q^ are never stored and
// dinv is a scalar, which leaves seven.
inline int std_vectors(bool unif) { return unif ? 7 : nvec_of(RPK_STD) + 2; }
// Vectors the pipelined loop keeps cached when they fit: p^, q, q^, y, r, r^, w,
// t, v and z^, w^ (its other six, s, s^, z, x, r0 and dinv, are always
// streamed); with a uniform Jacobi vector z^ and w^ are never stored and z
// (gathered by P2) is kept instead: ten.
inline int pipe_kept(bool unif) { return unif ? 10 : 11; }

// Whether a solve streams vectors past the Infinity Cache beyond what it always
// does (Vecs::far): the standard loop when the vectors it touches do not fit in
// nine tenths of the cache, the pipelined loop when the eleven it otherwise
// keeps do not.  A batch of systems decides the same way on its total number of
// rows (unif: every system's Jacobi vector is uniform).
inline bool rows_stream_far(int64_t rows, int variant, bool unif) {
  const int kept = variant == RPK_STD ? std_vectors(unif) : variant == RPK_PIPELINED ? pipe_kept(unif) : 0;
  return kept > 0 && (double)kept * (double)rows * 8.0 > 0.9 * kInfinityCacheBytes;
}
inline bool streams_far(const rpk_matrix* A, int variant) { return rows_stream_far(A->n, variant, A->unif != 0); }

// Vectors of one iteration that stay in the Infinity Cache (those it touches,
// less those streamed past it: x, p, r0 and dinv in the standard loop, x and r0
// with a uniform Jacobi vector)
inline int cached_vectors(int variant, bool far, bool unif) {
  if (variant == RPK_PIPELINED) return far ? 4 : pipe_kept(unif);
  if (variant == RPK_STD) return std_vectors(unif) - (far ? (unif ? 2 : 4) : 0);
  return unif ? nvec_of(variant) : nvec_of(variant) + 2;  // PCG: r, p, d, y, x, dinv (r, p, d, x)
}

template <template <int> class F, typename... Args>
rpk_status by_fpe(int N, Args&&... args) {
  switch (N) {
    case 0: return F<0>::call(args...);
    case 1: return F<1>::call(args...);
    case 2: return F<2>::call(args...);
    case 3: return F<3>::call(args...);
    case 4: return F<4>::call(args...);
    case 8: return F<8>::call(args...);
  }
  return RPK_ERR_ARG;
}

// ---------------------------------------------------------------------------
// Batches of systems (batch.hip; also used by the server)
// ---------------------------------------------------------------------------
struct Plan {
  std::vector<Tile> tiles;  // XCD-interleaved: tile t runs on XCD t % 8
  std::vector<int> G;       // tiles per listed system
};

// Tiles of at most T rows for the listed systems (sizes n); Tile.sys is ids[k]
// (or k when ids is null) and Tile.rec the tile's index inside its system.
Plan make_plan(const std::vector<int64_t>& n, int T, const std::vector<int>* ids = nullptr);
// upper bound of make_plan(n, T).tiles.size() for every T >= Tcap
int64_t tile_capacity(const std::vector<int64_t>& n, int Tcap);

// Device block of one system: tickets + flags | long accumulators | plain-mode
// sums of gcap tiles | nvec solver vectors of n doubles.
constexpr size_t kFlagsBytes = 8 * sizeof(unsigned) + MAX_DOTS * sizeof(int);
size_t sys_bytes(int64_t n, int gcap, int nvec);
// Descriptor of a system whose block starts at `base` (device address).
SysDesc make_desc(const rpk_matrix* A, const double* b, double* x, char* base, int gcap, int G, int variant,
                  State* st, double* hist);

// Library-wide state, guarded by g_mu: the capture stream, pinned state
// buffers, and the cache of instantiated iteration graphs.  A graph key lists
// every kernel argument the graph bakes in; key[0] is the matrix handle the
// graph refers to (0 when its kernels find their systems through device memory).
std::mutex& lib_mutex();
hipStream_t capture_stream();
rpk_status ensure_globals();
// pinned host buffer of at least `count` States (valid until the next call)
State* pinned_states(size_t count);
hipGraphExec_t graph_find(const std::vector<uint64_t>& key);
void graph_put(const std::vector<uint64_t>& key, hipGraphExec_t g);
void graph_drop_owner(uint64_t owner);

// Capture `body(capture_stream)` into a graph and instantiate it (cached by key).
template <class Body>
rpk_status graph_get(const std::vector<uint64_t>& key, Body body, hipGraphExec_t* out) {
  hipGraphExec_t exec = graph_find(key);
  if (!exec) {
    hipGraph_t graph = nullptr;
    hipStream_t cs = capture_stream();
    HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    const rpk_status cst = body(cs);
    const hipError_t ec = hipStreamEndCapture(cs, &graph);
    if (cst != RPK_OK || ec != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return RPK_ERR_HIP;
    }
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return RPK_ERR_HIP;
    graph_put(key, exec);
  }
  *out = exec;
  return RPK_OK;
}

}  // namespace rpkhost
