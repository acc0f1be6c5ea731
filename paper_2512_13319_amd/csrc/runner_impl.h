// Definitions of the launch sequences (included by the instantiation units).
#pragma once
#include "kernels.h"
#include "runner.h"
#include "segwave.h"
#include "blocks.h"

namespace ms {

template <typename T>
inline Prob<T> make_prob(const map_problem& q) {
  Prob<T> p;
  p.n_seg = q.n_seg;
  p.n_steps = q.n_steps;
  p.n_states = q.n_steps + q.n_seg;
  p.seg_off = q.seg_off;
  p.dt = static_cast<const T*>(q.dt);
  p.dt_stride = q.dt_stride;
  p.y = static_cast<const T*>(q.y);
  p.m0 = static_cast<const T*>(q.m0);
  p.m0_stride = q.m0_stride;
  p.P0 = static_cast<const T*>(q.P0);
  p.P0_stride = q.P0_stride;
  p.theta = static_cast<const T*>(q.theta);
  p.th_stride = q.theta_stride;
  p.xbar = static_cast<const T*>(q.xbar);
  p.gx = nullptr;
  p.om_div = (q.flags & MAP_OM_DIVERGENCE) ? 1 : 0;
  p.n_sub = q.n_sub > 1 ? q.n_sub : 1;
  p.ny_in = q.ny;
  p.nw_in = q.nw;
  p.F = static_cast<const T*>(q.F);
  p.c = static_cast<const T*>(q.c);
  p.L = static_cast<const T*>(q.L);
  p.W = static_cast<const T*>(q.W);
  p.H = static_cast<const T*>(q.H);
  p.r = static_cast<const T*>(q.r);
  p.R = static_cast<const T*>(q.R);
  p.sF = q.F_stride;
  p.sc = q.c_stride;
  p.sL = q.L_stride;
  p.sW = q.W_stride;
  p.sH = q.H_stride;
  p.sr = q.r_stride;
  p.sR = q.R_stride;
  return p;
}

template <typename T>
inline Ws<T> make_ws(int nx, int64_t n_states, void* base, int chunk, int flags) {
  WsLayout l = ws_layout(nx, n_states, sizeof(T), chunk);
  char* b = static_cast<char*>(base);
  Ws<T> w;
  w.counters = reinterpret_cast<unsigned int*>(b + l.off[0]);
  w.lane_pre = reinterpret_cast<T*>(b + l.off[1]);
  w.tile_agg = reinterpret_cast<T*>(b + l.off[2]);
  w.tile_carry = reinterpret_cast<T*>(b + l.off[3]);
  w.slane_pre = reinterpret_cast<T*>(b + l.off[4]);
  w.stile_agg = reinterpret_cast<T*>(b + l.off[5]);
  w.stile_carry = reinterpret_cast<T*>(b + l.off[6]);
  w.tile_pre = reinterpret_cast<T*>(b + l.off[7]);
  w.stile_suf = reinterpret_cast<T*>(b + l.off[8]);
  w.lane_half = chunk == 32 ? reinterpret_cast<T*>(b + l.off[9]) : nullptr;
  w.n_lanes = l.n_lanes;
  w.n_tiles = l.n_tiles;
  w.chunk = later_chunk(chunk);
  w.n_lanes1 = l.n_lanes1;
  w.n_tiles1 = l.n_tiles1;
  w.chunk1 = chunk;
  w.k1_shift = chunk == 32 ? 1 : 0;
  w.up_tail = 1;
  w.status = (flags & MAP_CHECK_FINITE) ? w.counters + kStatusWord : nullptr;
  return w;
}

// The workspace as the filter up-sweep sees it: its own decomposition.
template <typename T>
inline Ws<T> up_view(const Ws<T>& w) {
  Ws<T> u = w;
  u.n_lanes = w.n_lanes1;
  u.n_tiles = w.n_tiles1;
  u.chunk = w.chunk1;
  return u;
}

inline unsigned grid_for(int64_t n_tiles) { return unsigned((n_tiles + 3) / 4); }

// SIMDs of the current device (compute units x 4), read once per device.
inline int64_t device_simds() {
  static int64_t cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 1024;
  if (cache[dev] == 0) {
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cu <= 0)
      cu = 256;
    cache[dev] = int64_t(cu) * 4;
  }
  return cache[dev];
}

// The filter up-sweep, in the variant for the grid's wavefront count (see
// k_filter_up).
template <typename TS, typename T, class M>
void launch_filter_up(unsigned grid, hipStream_t s, const Prob<TS>& p, const Ws<T>& w,
                      const Acc& acc) {
  if constexpr (M::kWaves == 2) {
    if (int64_t(grid) * (kBlock / kWave) > device_simds()) {
      k_filter_up<TS, T, M, 2><<<grid, kBlock, 0, s>>>(p, w, acc);
      return;
    }
  }
  k_filter_up<TS, T, M, 1><<<grid, kBlock, 0, s>>>(p, w, acc);
}

inline hipError_t zero(const Acc& a, int64_t n_seg, int64_t nth, hipStream_t st) {
  if (!a.loglik && !a.obj && !a.g_loglik && !a.g_obj) return hipSuccess;
  const int64_t n = n_seg * (nth > 1 ? nth : 1);
  const int64_t nb = (n + kBlock - 1) / kBlock;
  const unsigned g = unsigned(nb < 1024 ? nb : 1024);
  prof_begin(kProfAux, st);
  k_zero_acc<<<g, kBlock, 0, st>>>(a, n_seg, nth);
  prof_end(kProfAux, st);
  return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_init_xbar(Prob<T> p, int nx, T* xb) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= p.n_states) return;
  int64_t lo = 0, hi = p.n_seg - 1;
  while (lo < hi) {
    int64_t mid = (lo + hi + 1) >> 1;
    if (p.seg_off[mid] + mid <= i) lo = mid; else hi = mid - 1;
  }
  for (int c = 0; c < nx; ++c) xb[tix(i, c, nx)] = p.m0[lo * p.m0_stride + c];
}

#define MS_CHECK(x)                         \
  do {                                      \
    hipError_t e_ = (x);                    \
    if (e_ != hipSuccess) return e_;        \
  } while (0)

template <typename TS, typename T, class M>
hipError_t Runner<TS, T, M>::build(const map_problem& q, void* elems, hipStream_t st) {
  Prob<TS> p = make_prob<TS>(q);
  const unsigned g = unsigned((p.n_states + kBlock - 1) / kBlock);
  k_build_elements<TS, T, M><<<g, kBlock, 0, st>>>(p, static_cast<TS*>(elems));
  return hipGetLastError();
}

template <typename TS, typename T, class M>
hipError_t Runner<TS, T, M>::init_xbar(const map_problem& q, void* xbar, hipStream_t st) {
  Prob<TS> p = make_prob<TS>(q);
  const unsigned g = unsigned((p.n_states + kBlock - 1) / kBlock);
  k_init_xbar<TS><<<g, kBlock, 0, st>>>(p, M::NX, static_cast<TS*>(xbar));
  return hipGetLastError();
}

// Trajectory fix-up with three states prefetched (see k_traj_down; five,
// for grids of at most one wavefront per SIMD, measured no faster at
// T = 2^20: 58-59 against 50-57 us with the adjoint).
template <typename TS, typename T, class M, bool kGrad, bool kCov>
void launch_traj_depth(const Prob<TS>& p, const Ws<T>& w, const TrajOut& to, const Acc& acc,
                       unsigned g, hipStream_t st) {
  k_traj_down<TS, T, M, kGrad, kCov, 3><<<g, kBlock, 0, st>>>(p, w, to, acc);
}

// Trajectory fix-up, instantiated for (adjoint, covariance output).
template <typename TS, typename T, class M>
hipError_t launch_traj_down(const Prob<TS>& p, const Ws<T>& w, TrajOut to, const Acc& acc, bool grad,
                            unsigned g, hipStream_t st) {
  const bool cov = to.Ps != nullptr;
  if constexpr (M::kAdjoint) {
    if (grad) {
      prof_begin(kProfTrajDownGrad, st);
      if (cov)
        launch_traj_depth<TS, T, M, true, true>(p, w, to, acc, g, st);
      else
        launch_traj_depth<TS, T, M, true, false>(p, w, to, acc, g, st);
      prof_end(kProfTrajDownGrad, st);
      return hipGetLastError();
    }
  }
  to.want_grad = 0;
  prof_begin(kProfTrajDown, st);
  if (cov)
    launch_traj_depth<TS, T, M, false, true>(p, w, to, acc, g, st);
  else
    launch_traj_depth<TS, T, M, false, false>(p, w, to, acc, g, st);
  prof_end(kProfTrajDown, st);
  return hipGetLastError();
}

template <typename TS, typename T, class M>
hipError_t Runner<TS, T, M>::filter(const map_problem& q, const SmoothArgs& a) {
  Prob<TS> p = make_prob<TS>(q);
  Ws<T> w = make_ws<T>(M::NX, p.n_states, a.ws, a.chunk, q.flags);
  const unsigned g = grid_for(w.n_tiles);
  prof_begin(kProfFilterUp, a.stream);
  launch_filter_up<TS, T, M>(grid_for(w.n_tiles1), a.stream, p, up_view(w),
      Acc{a.loglik, nullptr, nullptr, nullptr});
  prof_end(kProfFilterUp, a.stream);
  MS_CHECK(hipGetLastError());
  FilterOut fo{a.S, a.v, a.m, a.P, a.loglik != nullptr};
  Acc acc{a.loglik, nullptr, nullptr, nullptr};
  prof_begin(kProfFilterDown, a.stream);
  k_filter_down<TS, T, M, kModeFilter><<<g, kBlock, 0, a.stream>>>(p, w, fo, acc);
  prof_end(kProfFilterDown, a.stream);
  return hipGetLastError();
}

template <typename TS, typename T, class M>
hipError_t Runner<TS, T, M>::smoother(const map_problem& q, const SmoothArgs& a, bool grad) {
  Prob<TS> p = make_prob<TS>(q);
  Ws<T> w = make_ws<T>(M::NX, p.n_states, a.ws, a.chunk, q.flags);
  const int64_t nth = M::NTH;
  const unsigned g = grid_for(w.n_tiles);
  FilterOut fo{a.S, a.v, nullptr, nullptr, 0};
  Acc acc{nullptr, a.obj, a.g_loglik, a.g_obj};
  const Acc zacc{nullptr, a.obj, grad ? a.g_loglik : nullptr, grad ? a.g_obj : nullptr};
  if (a.ckpt != nullptr) {
    // From a filter checkpoint: the up-sweep rebuilds the lane and tile
    // prefixes inside each block (and zeroes the accumulators), the block
    // carries are the checkpoint's, and the fused fix-up writes S, v again
    // while it builds the trajectory maps.
    w.tile_carry = static_cast<T*>(a.ckpt);
    w.up_tail = 0;
    prof_begin(kProfFilterUp, a.stream);
    launch_filter_up<TS, T, M>(grid_for(w.n_tiles1), a.stream, p, up_view(w), zacc);
    prof_end(kProfFilterUp, a.stream);
    MS_CHECK(hipGetLastError());
    prof_begin(kProfFused, a.stream);
    k_filter_down<TS, T, M, kModeFused><<<g, kBlock, 0, a.stream>>>(p, w, fo, acc);
    prof_end(kProfFused, a.stream);
  } else {
    MS_CHECK(zero(zacc, q.n_seg, nth, a.stream));
    prof_begin(kProfTrajUp, a.stream);
    k_filter_down<TS, T, M, kModeTrajOnly><<<g, kBlock, 0, a.stream>>>(p, w, fo, acc);
    prof_end(kProfTrajUp, a.stream);
  }
  MS_CHECK(hipGetLastError());
  TrajOut to{a.S, a.v, a.xs, a.Ps, a.obj != nullptr, grad, grad ? a.g_elems : nullptr};
  return launch_traj_down<TS, T, M>(p, w, to, acc, grad, g, a.stream);
}

// Blocks of k_seg_wave<...> resident on the whole device (its persistent grid).
template <typename TS, typename T, class M, bool kGrad, bool kCov>
unsigned seg_wave_grid(int64_t n_seg) {
  static int resident = 0;
  if (resident == 0) {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_seg_wave<TS, T, M, kGrad, kCov>,
                                                     kBlock, 0) != hipSuccess || per_cu < 1)
      per_cu = 1;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
      cus = 256;
    resident = per_cu * cus;
  }
  const int64_t want = (n_seg + kBlock / kWave - 1) / (kBlock / kWave);
  return unsigned(want < resident ? want : resident);
}

template <typename TS, typename T, class M, bool kGrad, bool kCov>
hipError_t launch_seg_wave(const Prob<TS>& p, const SegOut& o, hipStream_t st) {
  prof_begin(kProfSegWave, st);
  k_seg_wave<TS, T, M, kGrad, kCov>
      <<<seg_wave_grid<TS, T, M, kGrad, kCov>(p.n_seg), kBlock, 0, st>>>(p, o);
  prof_end(kProfSegWave, st);
  return hipGetLastError();
}

// Segment-local schedule of the fused step (segwave.h): the queue of segments
// by decreasing length, then the persistent wavefronts.
template <typename TS, typename T, class M>
hipError_t smooth_seg_wave(const map_problem& q, const SmoothArgs& a) {
  Prob<TS> p = make_prob<TS>(q);
  char* base = static_cast<char*>(a.ws);
  unsigned int* ctl = reinterpret_cast<unsigned int*>(base);
  int* order = reinterpret_cast<int*>(base + seg_ws_order_offset());
  prof_begin(kProfAux, a.stream);
  k_seg_order<<<1, kBlock, 0, a.stream>>>(q.seg_off, q.n_seg, order, ctl + kQueueWord);
  prof_end(kProfAux, a.stream);
  MS_CHECK(hipGetLastError());
  const bool grad = a.g_loglik != nullptr || a.g_obj != nullptr;
  SegOut o{a.S, a.v, a.xs, a.Ps, a.loglik, a.obj, a.g_loglik, a.g_obj, order,
           ctl + kQueueWord, (q.flags & MAP_CHECK_FINITE) ? ctl + kStatusWord : nullptr};
  if constexpr (M::kAdjoint) {
    if (grad)
      return a.Ps ? launch_seg_wave<TS, T, M, true, true>(p, o, a.stream)
                  : launch_seg_wave<TS, T, M, true, false>(p, o, a.stream);
  }
  return a.Ps ? launch_seg_wave<TS, T, M, false, true>(p, o, a.stream)
              : launch_seg_wave<TS, T, M, false, false>(p, o, a.stream);
}

// General linear models above nx = 4 (their matrices no longer fit in
// registers; the kernels run from scratch memory): flat schedules and the RTS
// form only, which keeps their compilation within bounds.
template <class M>
constexpr bool kLargeLinear = M::kPadded && M::NX > 4;

template <typename TS, typename T, class M>
hipError_t Runner<TS, T, M>::smooth(const map_problem& q, const SmoothArgs& a) {
  if constexpr (!kLargeLinear<M>) {
    if (a.chunk == kSchedSegWave) return smooth_seg_wave<TS, T, M>(q, a);
  }
  Prob<TS> p = make_prob<TS>(q);
  Ws<T> w = make_ws<T>(M::NX, p.n_states, a.ws, a.chunk, q.flags);
  // checkpointed: the up-sweep's block carries go straight to the checkpoint
  if (a.ckpt != nullptr) w.tile_carry = static_cast<T*>(a.ckpt);
  const bool grad = a.g_loglik != nullptr || a.g_obj != nullptr;
  const unsigned g = grid_for(w.n_tiles);
  prof_begin(kProfFilterUp, a.stream);
  launch_filter_up<TS, T, M>(grid_for(w.n_tiles1), a.stream, p, up_view(w),
      Acc{a.loglik, a.obj, grad ? a.g_loglik : nullptr, grad ? a.g_obj : nullptr});
  prof_end(kProfFilterUp, a.stream);
  MS_CHECK(hipGetLastError());
  FilterOut fo{a.S, a.v, nullptr, nullptr, a.loglik != nullptr};
  Acc acc{a.loglik, a.obj, a.g_loglik, a.g_obj};
  prof_begin(kProfFused, a.stream);
  k_filter_down<TS, T, M, kModeFused><<<g, kBlock, 0, a.stream>>>(p, w, fo, acc);
  prof_end(kProfFused, a.stream);
  MS_CHECK(hipGetLastError());
  TrajOut to{a.S, a.v, a.xs, a.Ps, a.obj != nullptr, grad, grad ? a.g_elems : nullptr};
  return launch_traj_down<TS, T, M>(p, w, to, acc, grad, g, a.stream);
}

// Two-filter smoother: filter up-sweep, filter fix-up with the backward
// filter's up-sweep, two-filter combination.
template <typename TS, typename T, class M>
hipError_t Runner<TS, T, M>::dense(const map_problem& q, const void* S, const void* v,
                                   const void* xs, void* xd, void* Sd, void* vd, hipStream_t st) {
  if constexpr (!M::kBlocked) {
    return hipErrorInvalidValue;  // rejected by the entry point before this
  } else {
    Prob<TS> p = make_prob<TS>(q);
    prof_begin(kProfDense, st);
    k_dense<TS, T, M><<<unsigned((p.n_states + kBlock - 1) / kBlock), kBlock, 0, st>>>(
        p, DenseIO{S, v, xs, xd, Sd, vd});
    prof_end(kProfDense, st);
    return hipGetLastError();
  }
}

template <typename TS, typename T, class M>
hipError_t Runner<TS, T, M>::two_filter(const map_problem& q, const SmoothArgs& a) {
  if constexpr (M::kBlocked || kLargeLinear<M>) {
    return hipErrorInvalidValue;  // rejected by the entry point
  } else {
    Prob<TS> p = make_prob<TS>(q);
    Ws<T> w = make_ws<T>(M::NX, p.n_states, a.ws, a.chunk, q.flags);
    const unsigned g = grid_for(w.n_tiles);
    prof_begin(kProfFilterUp, a.stream);
    launch_filter_up<TS, T, M>(grid_for(w.n_tiles1), a.stream, p, up_view(w),
        Acc{a.loglik, nullptr, nullptr, nullptr});
    prof_end(kProfFilterUp, a.stream);
    MS_CHECK(hipGetLastError());
    FilterOut fo{a.S, a.v, nullptr, nullptr, a.loglik != nullptr};
    Acc acc{a.loglik, nullptr, nullptr, nullptr};
    prof_begin(kProfTwoFilterUp, a.stream);
    k_filter_down<TS, T, M, kModeTwoFilter><<<g, kBlock, 0, a.stream>>>(p, w, fo, acc);
    prof_end(kProfTwoFilterUp, a.stream);
    MS_CHECK(hipGetLastError());
    TrajOut to{a.S, a.v, a.xs, a.Ps, 0, 0};
    prof_begin(kProfTwoFilterDown, a.stream);
    if (a.Ps != nullptr)
      k_two_filter_down<TS, T, M, true><<<g, kBlock, 0, a.stream>>>(p, w, to);
    else
      k_two_filter_down<TS, T, M, false><<<g, kBlock, 0, a.stream>>>(p, w, to);
    prof_end(kProfTwoFilterDown, a.stream);
    return hipGetLastError();
  }
}

// Implicit-function VJP: mu = H^{-1} g by the smoother's three passes on the
// adjoint problem Ift<M> (the problem's own S is read, not stored again), then
// the per-step cotangents reduced per segment (k_ift_grad).
template <typename TS, typename T, class M>
hipError_t Runner<TS, T, M>::ift(const map_problem& q, const SmoothArgs& a, const IftArgs& b) {
  if constexpr (!M::kAdjoint) {
    return hipErrorInvalidValue;  // rejected by the entry point before this
  } else {
    using MI = Ift<M>;
    Prob<TS> p = make_prob<TS>(q);
    p.gx = static_cast<const TS*>(b.gx);
    Ws<T> w = make_ws<T>(M::NX, p.n_states, a.ws, a.chunk, q.flags);
    const unsigned g = grid_for(w.n_tiles);
    prof_begin(kProfIftSolve, a.stream);
    // also zeroes g_theta (the accumulator of the last kernel)
    launch_filter_up<TS, T, MI>(grid_for(w.n_tiles1), a.stream, p, up_view(w),
        Acc{nullptr, nullptr, b.g_theta, nullptr});
    prof_end(kProfIftSolve, a.stream);
    MS_CHECK(hipGetLastError());
    FilterOut fo{a.S, b.vmu, nullptr, nullptr, 0};
    const Acc none{nullptr, nullptr, nullptr, nullptr};
    prof_begin(kProfIftSolve, a.stream);
    k_filter_down<TS, T, MI, kModeFused><<<g, kBlock, 0, a.stream>>>(p, w, fo, none);
    prof_end(kProfIftSolve, a.stream);
    MS_CHECK(hipGetLastError());
    TrajOut to{a.S, b.vmu, b.mu, nullptr, 0, 0};
    prof_begin(kProfIftSolve, a.stream);
    k_traj_down<TS, T, MI, false, false, 3><<<g, kBlock, 0, a.stream>>>(p, w, to, none);
    prof_end(kProfIftSolve, a.stream);
    MS_CHECK(hipGetLastError());
    IftIn in{a.S, a.v, b.vmu, a.xs, b.mu};
    const int64_t lanes = (p.n_states + kRow - 1) / kRow;
    prof_begin(kProfIftGrad, a.stream);
    k_ift_grad<TS, T, M><<<unsigned((lanes + kBlock - 1) / kBlock), kBlock, 0, a.stream>>>(
        p, in, b.g_theta);
    prof_end(kProfIftGrad, a.stream);
    return hipGetLastError();
  }
}

#define MS_COMMA ,
#define MS_INSTANTIATE(M)                 \
  template struct Runner<double, double, M>; \
  template struct Runner<float, double, M>;  \
  template struct Runner<float, float, M>;
// general linear model padded to NX, NX > 4: FP64 arithmetic only, one
// storage type per unit
#define MS_INSTANTIATE_LARGE(TS, M) template struct Runner<TS, double, M>;
// sub-stepped blocks: FP64 arithmetic only
#define MS_INSTANTIATE_BLOCKED(M)            \
  template struct Runner<double, double, Blocked<M>>; \
  template struct Runner<float, double, Blocked<M>>;

}  // namespace ms
