// Launch sequences behind the C-ABI, one instantiation per (dtype, model).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/mapscan.h"
#include "counters.h"

namespace ms {

struct WsLayout {
  int64_t n_lanes;   // padded to whole tiles (passes after the filter up-sweep)
  int64_t n_tiles;
  int64_t n_lanes1;  // the same for the filter up-sweep
  int64_t n_tiles1;
  size_t off[10];    // counters, lane_pre, tile_agg, tile_carry, slane_pre, stile_agg, stile_carry, tile_pre,
                     // stile_suf, lane_half
  size_t total;
};

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Work tiles: 64 lanes of `chunk` states (chunk = 4, 8, 16 or 32), one per
// wavefront.  A final work tile of at most kMergeStates states is not given a
// wavefront of its own: the last lane of the tile before it runs those states
// after its own (a grid of 2^k steps has 2^k + 1 states, and a one-state tile
// would otherwise make a block that can only start once an earlier block has
// left its compute unit).  The storage layout of state-indexed arrays does
// not depend on this.
constexpr int64_t kMergeStates = 8;
constexpr int kChunks[4] = {32, 16, 8, 4};  // flat schedules, largest first
constexpr int kMinChunk = 4;
// Segment-local schedule of the fused step (map_smooth): one wavefront per
// segment, in rounds of 64 lanes x 16 states (segwave.h).
constexpr int kSchedSegWave = MAP_SCHED_SEGMENT_WAVE;
inline bool valid_flat_chunk(int c) { return c == 4 || c == 8 || c == 16 || c == 32; }
inline bool valid_chunk(int c) { return valid_flat_chunk(c) || c == kSchedSegWave; }
// Schedule 32 is split: the filter up-sweep folds 32 states per lane (its
// wavefront scan, block tree and arrival then cost half as much per state)
// and also keeps the fold of each lane's first 16; the passes after it run 16
// per lane, which keeps their streamed accesses on whole cache lines.
inline int later_chunk(int chunk) { return chunk == 32 ? 16 : chunk; }

// Workspace of the segment-local schedule: the control words and the segment
// queue (one int per segment).
inline size_t seg_ws_order_offset() { return align256(size_t(kCounterWords) * 4); }
inline size_t seg_ws_bytes(int64_t n_seg) {
  return seg_ws_order_offset() + align256(size_t(n_seg) * sizeof(int));
}

inline int64_t work_tiles(int64_t n_states, int64_t chunk) {
  const int64_t ts = 64 * chunk;
  const int64_t full = n_states / ts, rem = n_states % ts;
  if (full > 0 && rem > 0 && rem <= kMergeStates) return full;
  return (n_states + ts - 1) / ts;
}

inline WsLayout ws_layout(int nx, int64_t n_states, size_t sz, int64_t chunk) {
  WsLayout w;
  w.n_tiles = work_tiles(n_states, later_chunk(int(chunk)));
  w.n_lanes = w.n_tiles * 64;
  w.n_tiles1 = work_tiles(n_states, chunk);  // <= n_tiles
  w.n_lanes1 = w.n_tiles1 * 64;
  const int64_t sym = nx * (nx + 1) / 2;
  const int64_t elem = nx * nx + 2 * nx + 2 * sym;
  const int64_t aff = nx * nx + nx + sym;
  // the reverse-scan regions serve the trajectory maps (RTS form) and the
  // flagged backward-filter runs (two-filter form)
  const int64_t rlane = aff > elem + 1 ? aff : elem + 1;
  const int64_t rcarry = nx + sym > elem ? nx + sym : elem;
  const size_t sizes[10] = {size_t(kCounterWords) * 4,
                           size_t(elem * w.n_lanes) * sz,
                           size_t(elem * w.n_tiles) * sz,
                           size_t((sym + nx) * w.n_tiles) * sz,
                           size_t(rlane * w.n_lanes) * sz,
                           size_t(rlane * w.n_tiles) * sz,
                           size_t(rcarry * w.n_tiles) * sz,
                           size_t(elem * w.n_tiles) * sz,
                           size_t(rlane * w.n_tiles) * sz,
                           chunk == 32 ? size_t(elem * w.n_lanes1) * sz : size_t(0)};
  size_t o = 0;
  for (int i = 0; i < 10; ++i) {
    w.off[i] = o;
    o += align256(sizes[i]);
  }
  w.total = o;
  return w;
}

// Values in a filter checkpoint: (S, v) before every block of four tiles of
// the filter up-sweep's decomposition (the carries its last block scans).
inline int64_t checkpoint_values(int nx, int64_t n_states, int chunk) {
  const int64_t sym = nx * (nx + 1) / 2;
  return (sym + nx) * ((work_tiles(n_states, chunk) + 3) / 4);
}

struct SmoothArgs {
  void* S;
  void* v;
  void* m;
  void* P;
  void* xs;
  void* Ps;
  double* loglik;
  double* obj;
  double* g_loglik;
  double* g_obj;
  void* ws;
  hipStream_t stream;
  int chunk;  // states per lane (4, 8, 16 or 32)
  double* g_elems = nullptr;  // map_backward: per-step element cotangents (flat schedules)
  // filter checkpoint (checkpoint_values of the arithmetic type): written by
  // the fused step, read by the adjoint, which then rebuilds S, v into a.S, a.v
  void* ckpt = nullptr;
};

// Implicit-function VJP (map_backward with a cotangent of x*).
struct IftArgs {
  const void* gx;   // tiled [nx] per state: cotangent of x*
  void* mu;         // out, tiled [nx] per state: mu = H^{-1} g
  void* vmu;        // out, tiled [nx] per state: the adjoint problem's second filter plane
  double* g_theta;  // out [n_seg][n_theta]
};

// Profiling hook: kernel kinds timed by HIP events when enabled.
enum ProfKind : int {
  kProfFilterUp = 0,
  kProfFilterDown = 1,
  kProfFused = 2,
  kProfTrajUp = 3,
  kProfTrajDown = 4,
  kProfTrajDownGrad = 5,
  kProfAux = 6,
  kProfTwoFilterUp = 7,
  kProfTwoFilterDown = 8,
  kProfIftSolve = 9,
  kProfIftGrad = 10,
  kProfSegWave = 11,
  kProfDense = 12,
  kProfKinds = 13
};
void prof_begin(int kind, hipStream_t st);
void prof_end(int kind, hipStream_t st);

// TS: storage type of the caller's arrays; T: arithmetic (and workspace) type.
template <typename TS, typename T, class M>
struct Runner {
  static hipError_t build(const map_problem& p, void* elems, hipStream_t st);
  static hipError_t filter(const map_problem& p, const SmoothArgs& a);
  static hipError_t smoother(const map_problem& p, const SmoothArgs& a, bool grad);
  static hipError_t smooth(const map_problem& p, const SmoothArgs& a);
  static hipError_t two_filter(const map_problem& p, const SmoothArgs& a);
  // needs a.S, a.v (the filter planes) and a.xs (x*) of the problem
  static hipError_t ift(const map_problem& p, const SmoothArgs& a, const IftArgs& b);
  // sub-stepped blocks: filter and MAP state at the interior substeps
  static hipError_t dense(const map_problem& p, const void* S, const void* v, const void* xs,
                          void* xd, void* Sd, void* vd, hipStream_t st);
  static hipError_t init_xbar(const map_problem& p, void* xbar, hipStream_t st);
};

}  // namespace ms
