// C-ABI front end: host-side validation, schedule choice, dispatch to the
// (dtype, model) instantiation, error reporting.  Only map_autotune allocates
// device memory (temporary outputs, freed before it returns).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <iterator>
#include <string>
#include <vector>

#include "models.h"
#include "runner.h"
#include "lti.h"

// Fixed workspace of map_smooth_noalloc (one copy per device, held until the
// process ends).  64 MiB fits the fused step of a 2^20-step nx = 4 problem at
// the schedules the library picks for it.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace ms {

__global__ void k_clear_words(unsigned int* w, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) w[i] = 0u;
}

// ---------------------------------------------------------------- profiling hook
// When enabled, every kernel launch is bracketed by two HIP events recorded on
// the launch stream.  Events are created once (no device memory is involved).
namespace prof {
struct Rec {
  hipEvent_t a, b;
  int kind;
};
static std::vector<Rec> g_recs;
static size_t g_used = 0;
static bool g_on = false;
static int g_open_kind = -1;
}  // namespace prof

void prof_begin(int kind, hipStream_t st) {
  if (!prof::g_on || prof::g_used >= prof::g_recs.size()) return;
  prof::Rec& r = prof::g_recs[prof::g_used];
  r.kind = kind;
  hipEventRecord(r.a, st);
  prof::g_open_kind = kind;
}

void prof_end(int kind, hipStream_t st) {
  if (!prof::g_on || prof::g_open_kind != kind || prof::g_used >= prof::g_recs.size()) return;
  hipEventRecord(prof::g_recs[prof::g_used].b, st);
  ++prof::g_used;
  prof::g_open_kind = -1;
}

namespace {

thread_local std::string g_err;

map_status fail(map_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

map_status hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return MAP_OK;
  return fail(MAP_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Models built into this library: (model, nx, ny, nw, n_theta).
struct Entry {
  int model, nx, ny, nw, nth;
};

#define MS_MODELS(X)                              \
  X(MAP_MODEL_CV, 2, 1, 1, 3, ModelCV<1>)         \
  X(MAP_MODEL_CV, 4, 2, 2, 3, ModelCV<2>)         \
  X(MAP_MODEL_CV, 6, 3, 3, 3, ModelCV<3>)         \
  X(MAP_MODEL_VDP, 2, 1, 2, 3, ModelVdP)          \
  X(MAP_MODEL_LORENZ63, 3, 3, 3, 5, ModelLorenz63) \
  X(MAP_MODEL_CT, 5, 2, 3, 4, ModelCT)            \
  X(MAP_MODEL_LINEAR, 1, 1, 1, 0, ModelLinear<1 MS_COMMA 1 MS_COMMA 1>) \
  X(MAP_MODEL_LINEAR, 2, 1, 1, 0, ModelLinear<2 MS_COMMA 1 MS_COMMA 1>) \
  X(MAP_MODEL_LINEAR, 2, 1, 2, 0, ModelLinear<2 MS_COMMA 1 MS_COMMA 2>) \
  X(MAP_MODEL_LINEAR, 2, 2, 2, 0, ModelLinear<2 MS_COMMA 2 MS_COMMA 2>) \
  X(MAP_MODEL_LINEAR, 3, 2, 2, 0, ModelLinear<3 MS_COMMA 2 MS_COMMA 2>) \
  X(MAP_MODEL_LINEAR, 3, 2, 3, 0, ModelLinear<3 MS_COMMA 2 MS_COMMA 3>) \
  X(MAP_MODEL_LINEAR, 3, 3, 3, 0, ModelLinear<3 MS_COMMA 3 MS_COMMA 3>) \
  X(MAP_MODEL_LINEAR, 4, 2, 2, 0, ModelLinear<4 MS_COMMA 2 MS_COMMA 2>) \
  X(MAP_MODEL_LINEAR, 4, 2, 4, 0, ModelLinear<4 MS_COMMA 2 MS_COMMA 4>) \
  X(MAP_MODEL_LINEAR, 4, 4, 4, 0, ModelLinear<4 MS_COMMA 4 MS_COMMA 4>)
#define MS_COMMA ,

// General linear model for the (ny, nw) without an instantiation of their own:
// ny, nw <= nx padded to nx (ModelLinearPadded).
#define MS_PADDED_MODELS(X)                        \
  X(1, ModelLinearPadded<1>)                       \
  X(2, ModelLinearPadded<2>)                       \
  X(3, ModelLinearPadded<3>)                       \
  X(4, ModelLinearPadded<4>)                       \
  X(5, ModelLinearPadded<5>)                       \
  X(6, ModelLinearPadded<6>)                       \
  X(7, ModelLinearPadded<7>)                       \
  X(8, ModelLinearPadded<8>)

bool padded_linear(const map_problem& p) {
  return p.model == MAP_MODEL_LINEAR && p.nx >= 1 && p.nx <= 8 && p.ny >= 1 && p.ny <= p.nx &&
         p.nw >= 1 && p.nw <= p.nx;
}
// general linear model above nx = 4: flat schedules and the RTS form only
bool large_linear(const map_problem& p) { return p.model == MAP_MODEL_LINEAR && p.nx > 4; }

// Models built with sub-stepped blocks (Blocked<M>, n_sub > 1).
#define MS_BLOCKED_MODELS(X)                      \
  X(MAP_MODEL_CV, 4, 2, 2, 3, ModelCV<2>)         \
  X(MAP_MODEL_VDP, 2, 1, 2, 3, ModelVdP)

// Calls f.template run<T, M>() for the matching instantiation.
template <class Fn>
map_status dispatch(const map_problem& p, Fn&& f) {
  if (p.n_sub > 1) {
#define MS_BCASE(MODEL, NX, NY, NW, NTH, M)                                            \
  if (p.model == MODEL && p.nx == NX && p.ny == NY && p.nw == NW) {                   \
    if (p.dtype == MAP_F64) return f.template run<double, double, Blocked<M>>();      \
    if (p.dtype == MAP_F32) return f.template run<float, double, Blocked<M>>();       \
    return fail(MAP_E_UNSUPPORTED, "sub-stepped blocks need FP64 arithmetic (MAP_F64 or MAP_F32)"); \
  }
    MS_BLOCKED_MODELS(MS_BCASE)
#undef MS_BCASE
    return fail(MAP_E_UNSUPPORTED,
                "sub-stepped blocks (n_sub > 1) are built for the constant-velocity model with "
                "nx = 4 and for Van der Pol");
  }
#define MS_CASE(MODEL, NX, NY, NW, NTH, M)                                            \
  if (p.model == MODEL && p.nx == NX && p.ny == NY && p.nw == NW) {                   \
    if (p.dtype == MAP_F64) return f.template run<double, double, M>();               \
    if (p.dtype == MAP_F32) return f.template run<float, double, M>();                \
    return f.template run<float, float, M>();                                         \
  }
  MS_MODELS(MS_CASE)
#undef MS_CASE
  if (padded_linear(p)) {
#define MS_PCASE(NX, M)                                                      \
  if (p.nx == NX) {                                                          \
    if (p.dtype == MAP_F64) return f.template run<double, double, M>();      \
    if (p.dtype == MAP_F32) return f.template run<float, double, M>();       \
    if constexpr (NX <= 4) return f.template run<float, float, M>();         \
    return fail(MAP_E_UNSUPPORTED, "nx > 4 needs FP64 arithmetic (MAP_F64 or MAP_F32)"); \
  }
    MS_PADDED_MODELS(MS_PCASE)
#undef MS_PCASE
  }
  return fail(MAP_E_UNSUPPORTED, "model %d with (nx, ny, nw) = (%d, %d, %d) is not built", p.model,
              p.nx, p.ny, p.nw);
}

int model_ntheta(const map_problem& p) {
#define MS_NTH(MODEL, NX, NY, NW, NTH, M) \
  if (p.model == MODEL && p.nx == NX && p.ny == NY && p.nw == NW) return NTH;
  MS_MODELS(MS_NTH)
#undef MS_NTH
  if (padded_linear(p)) return 0;
  return -1;
}

bool model_nonlinear(int model) {
  return model == MAP_MODEL_VDP || model == MAP_MODEL_LORENZ63 || model == MAP_MODEL_CT;
}

map_status validate(const map_problem* pp, bool need_xbar = true) {
  if (pp == nullptr) return fail(MAP_E_ARG, "problem is NULL");
  const map_problem& p = *pp;
  if (p.dtype != MAP_F32 && p.dtype != MAP_F64 && p.dtype != MAP_F32_FAST)
    return fail(MAP_E_DTYPE, "unknown dtype %d", p.dtype);
  if (p.nx < 1 || p.nx > 8 || p.ny < 1 || p.ny > 8 || p.nw < 1 || p.nw > 8)
    return fail(MAP_E_DIM, "dimensions (nx, ny, nw) = (%d, %d, %d) outside [1, 8]", p.nx, p.ny, p.nw);
  if (p.model < MAP_MODEL_LINEAR || p.model > MAP_MODEL_CT)
    return fail(MAP_E_ARG, "unknown model %d", p.model);
  if (p.chunk != 0 && !valid_chunk(p.chunk))
    return fail(MAP_E_ARG,
                "chunk = %d; must be 0 (library's choice), 4, 8, 16, 32 or "
                "MAP_SCHED_SEGMENT_WAVE (-1)",
                p.chunk);
  if (p.flags & ~(MAP_CHECK_FINITE | MAP_OM_DIVERGENCE))
    return fail(MAP_E_ARG, "unknown flags 0x%x", unsigned(p.flags));
  if (p.n_sub < 0 || p.n_sub > 64) return fail(MAP_E_ARG, "n_sub = %d outside [0, 64]", p.n_sub);
  if (p.n_sub > 1 && (p.flags & MAP_OM_DIVERGENCE))
    return fail(MAP_E_UNSUPPORTED, "sub-stepped blocks do not take MAP_OM_DIVERGENCE");
  const int nth = model_ntheta(p);
  if (nth < 0)
    return fail(MAP_E_UNSUPPORTED, "model %d with (nx, ny, nw) = (%d, %d, %d) is not built", p.model,
                p.nx, p.ny, p.nw);
  if (p.n_theta != nth) return fail(MAP_E_DIM, "n_theta = %d, model needs %d", p.n_theta, nth);
  if (p.n_seg < 1) return fail(MAP_E_DIM, "n_seg = %lld < 1", (long long)p.n_seg);
  if (p.n_steps < 0) return fail(MAP_E_DIM, "n_steps < 0");
  if (p.n_steps + p.n_seg > (int64_t(1) << 31) * 64)
    return fail(MAP_E_DIM, "too many states");
  if (p.seg_off == nullptr) return fail(MAP_E_ARG, "seg_off is NULL");
  if (p.seg_off_host != nullptr) {
    if (p.seg_off_host[0] != 0) return fail(MAP_E_LAYOUT, "seg_off[0] != 0");
    for (int64_t s = 0; s < p.n_seg; ++s)
      if (p.seg_off_host[s + 1] < p.seg_off_host[s])
        return fail(MAP_E_LAYOUT, "seg_off decreases at segment %lld", (long long)s);
    if (p.seg_off_host[p.n_seg] != p.n_steps)
      return fail(MAP_E_LAYOUT, "seg_off[n_seg] = %lld != n_steps = %lld",
                  (long long)p.seg_off_host[p.n_seg], (long long)p.n_steps);
  }
  if (p.dt == nullptr) return fail(MAP_E_ARG, "dt is NULL");
  if (p.dt_stride != 0 && p.dt_stride != 1) return fail(MAP_E_ARG, "dt_stride must be 0 or 1");
  // y is indexed by state (a segment's first state holds an unused value), so
  // it is read even when there are no steps
  if (p.y == nullptr) return fail(MAP_E_ARG, "y is NULL");
  if (p.m0 == nullptr || p.P0 == nullptr) return fail(MAP_E_ARG, "m0/P0 is NULL");
  if (p.m0_stride < 0 || p.P0_stride < 0 || p.theta_stride < 0)
    return fail(MAP_E_ARG, "negative stride");
  if (nth > 0 && p.theta == nullptr) return fail(MAP_E_ARG, "theta is NULL");
  if (need_xbar && model_nonlinear(p.model) && p.xbar == nullptr)
    return fail(MAP_E_ARG, "nonlinear model needs xbar");
  if (p.model == MAP_MODEL_LINEAR) {
    const void* ptrs[7] = {p.F, p.c, p.L, p.W, p.H, p.r, p.R};
    const int64_t strides[7] = {p.F_stride, p.c_stride, p.L_stride, p.W_stride,
                                p.H_stride, p.r_stride, p.R_stride};
    for (int i = 0; i < 7; ++i) {
      if (ptrs[i] == nullptr) return fail(MAP_E_ARG, "linear model matrix %d is NULL", i);
      if (strides[i] < 0) return fail(MAP_E_ARG, "negative stride for matrix %d", i);
    }
  }
  return MAP_OK;
}

// MAP_OM_DIVERGENCE changes the minimised objective (eq. OM with its
// divergence term): the prediction-error likelihood and the gradients, which
// refer to the energy objective and the probabilistic model, are not defined
// with it, and the two-filter form's backward filter does not include it.
map_status check_divergence(const map_problem& p, bool wants_ll_or_grad, const char* what) {
  if ((p.flags & MAP_OM_DIVERGENCE) && wants_ll_or_grad)
    return fail(MAP_E_UNSUPPORTED, "%s: MAP_OM_DIVERGENCE gives x*, P^s and the objective only "
                                   "(no log-likelihood or gradients)", what);
  return MAP_OK;
}

// Sub-stepped blocks: a block's element is not one measurement step, so the
// prediction-error likelihood, the costate-form objective and the adjoint
// (all written per measurement step) are not defined for it.
map_status check_blocks(const map_problem& p, bool wants_ll_obj_or_grad, const char* what) {
  if (p.n_sub > 1 && wants_ll_obj_or_grad)
    return fail(MAP_E_UNSUPPORTED, "%s: sub-stepped blocks give the filter, x*, P^s and the "
                                   "dense output only", what);
  return MAP_OK;
}

size_t compute_bytes(int dtype) { return dtype == MAP_F32_FAST ? 4 : 8; }
size_t storage_bytes(int dtype) { return dtype == MAP_F64 ? 8 : 4; }

// ---------------------------------------------------------------- schedules
// The schedule is the number of states per lane (4, 8, 16 or 32, the last
// split: see later_chunk).  Choices made by map_autotune are kept per problem
// shape (model, dimensions, dtype, and the powers of two of the state and
// segment counts).  Otherwise: 32 when its filter up-sweep still gives every
// SIMD at least four wavefronts in turn (there the up-sweep's fixed cost per
// wavefront dominates: 4096 ragged segments, 1.6e7 steps, measured 1.96 ->
// 1.66 ms per fused step), else the largest of 16, 8 and 4 that gives at
// least one wavefront to every second SIMD (fewer states per lane shorten
// each lane's chain but add wavefront-scan levels per state: at 2^18 + 1
// states, 8 per lane on half the SIMDs measured faster than 4 per lane on all
// of them).
namespace sched {
static std::mutex g_mu;
static std::map<std::string, int> g_tuned;
static std::map<int, int> g_simds;  // device -> SIMD count

std::string key_of(const map_problem& p) {
  const int64_t ns = p.n_steps + p.n_seg;
  char buf[128];
  snprintf(buf, sizeof(buf), "m%d_x%d_y%d_w%d_d%d_s%d_g%d", p.model, p.nx, p.ny, p.nw, p.dtype,
           int(floor(log2(double(ns)))), int(floor(log2(double(p.n_seg)))));
  return buf;
}

int simds() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_simds.find(dev);
  if (it != g_simds.end()) return it->second;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  return g_simds[dev] = 4 * cus;
}

int heuristic(const map_problem& p) {
  const int64_t ns = p.n_steps + p.n_seg;
  if (work_tiles(ns, 32) >= 4 * int64_t(simds())) return 32;
  const int64_t want = simds() / 2;
  for (int c : {16, 8})
    if (work_tiles(ns, c) >= want) return c;
  return kMinChunk;
}

// The schedule of a call.  The segment-local schedule serves the fused step
// only (map_smooth, map_smooth_noalloc, and the iterations of
// map_iterated_nonlinear); the other entry points (allow_seg = false) use the
// flat heuristic where it was asked for or tuned.
int resolve(const map_problem& p, bool allow_seg) {
  int c = p.chunk;
  if (c == 0) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_tuned.find(key_of(p));
    if (it != g_tuned.end()) c = it->second;
  }
  if (c == 0) c = heuristic(p);
  if (c == kSchedSegWave && (!allow_seg || p.n_seg > int64_t(INT32_MAX) || large_linear(p)))
    c = heuristic(p);
  return c;
}

// workspace bytes of one schedule
size_t ws_need(const map_problem& p, int chunk) {
  if (chunk == kSchedSegWave) return seg_ws_bytes(p.n_seg);
  return ws_layout(p.nx, p.n_steps + p.n_seg, compute_bytes(p.dtype), chunk).total;
}

// workspace that fits the schedule `resolve` may pick for any entry point
// (every schedule when the choice is left to the library)
size_t ws_bytes_for(const map_problem& p) {
  size_t m = 0;
  if (p.chunk != 0) {
    m = ws_need(p, resolve(p, false));
    const size_t t = ws_need(p, resolve(p, true));
    return t > m ? t : m;
  }
  for (int c : kChunks) {
    const size_t t = ws_need(p, c);
    if (t > m) m = t;
  }
  const size_t t = ws_need(p, kSchedSegWave);
  return t > m ? t : m;
}
}  // namespace sched

// MAP_CHECK_FINITE: the kernels set the workspace's status word when they
// write a non-finite value.  After a successful launch sequence it is read
// back (one stream synchronisation), and cleared again when set.
map_status finish_check(const map_problem& p, void* ws, hipStream_t st, map_status s) {
  if (s != MAP_OK || !(p.flags & MAP_CHECK_FINITE)) return s;
  unsigned int* w = static_cast<unsigned int*>(ws) + kStatusWord;
  unsigned int word = 0;
  s = hip_status(hipMemcpyAsync(&word, w, sizeof(word), hipMemcpyDeviceToHost, st), "status read");
  if (s == MAP_OK) s = hip_status(hipStreamSynchronize(st), "status read");
  if (s != MAP_OK) return s;
  if (word != 0) {
    k_clear_words<<<1, 64, 0, st>>>(w, 1);
    s = hip_status(hipGetLastError(), "status clear");
    if (s != MAP_OK) return s;
    return fail(MAP_E_NUMERIC, "non-finite value in the results (non-finite inputs, or a "
                               "covariance that is not positive definite)");
  }
  return MAP_OK;
}

// ---------------------------------------------------------------- fixed scratch
// Workspace of map_smooth_noalloc: the file-scope device array `scratch`
// (below the includes) instead of a caller-owned buffer.  Host code never
// uses the array's name as an address (on the host it only names the
// symbol): the address on each device is looked up once, with that device
// current, and kept.
namespace scr {
static std::mutex g_mu;
static std::map<int, void*> g_ptr;  // device -> address of `scratch` there
}  // namespace scr

map_status scratch_address(void** out) {
  int dev = 0;
  map_status s = hip_status(hipGetDevice(&dev), "map_smooth_noalloc: hipGetDevice");
  if (s != MAP_OK) return s;
  std::lock_guard<std::mutex> lk(scr::g_mu);
  auto it = scr::g_ptr.find(dev);
  if (it == scr::g_ptr.end()) {
    void* ptr = nullptr;
    s = hip_status(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)),
                   "map_smooth_noalloc: hipGetSymbolAddress");
    if (s != MAP_OK) return s;
    if (ptr == nullptr) return fail(MAP_E_HIP, "map_smooth_noalloc: scratch has no address");
    it = scr::g_ptr.emplace(dev, ptr).first;
  }
  *out = it->second;
  return MAP_OK;
}

map_status check_ws(const map_problem& p, void* ws, size_t ws_bytes, bool allow_seg) {
  const size_t need = sched::ws_need(p, sched::resolve(p, allow_seg));
  if (ws == nullptr) return fail(MAP_E_WORKSPACE, "workspace is NULL");
  if (ws_bytes < need)
    return fail(MAP_E_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
  return MAP_OK;
}

// Bytes of a filter checkpoint at the flat schedule the adjoint resolves.
size_t ckpt_need(const map_problem& p) {
  return size_t(checkpoint_values(p.nx, p.n_steps + p.n_seg, sched::resolve(p, false))) *
         compute_bytes(p.dtype);
}

map_status check_ckpt(const map_problem& p, const void* ckpt, size_t ckpt_bytes, const void* ws,
                      size_t ws_bytes, const char* what) {
  if (p.model == MAP_MODEL_LINEAR)
    return fail(MAP_E_UNSUPPORTED, "%s: checkpoints serve map_backward, which needs a parametric "
                                   "model", what);
  if (p.n_sub > 1)
    return fail(MAP_E_UNSUPPORTED, "%s: no checkpoints for sub-stepped blocks", what);
  const size_t need = ckpt_need(p);
  if (ckpt_bytes < need)
    return fail(MAP_E_ARG, "%s: checkpoint has %zu bytes, needs %zu", what, ckpt_bytes, need);
  const char* c = static_cast<const char*>(ckpt);
  const char* w = static_cast<const char*>(ws);
  if (w != nullptr && c < w + ws_bytes && w < c + need)
    return fail(MAP_E_ARG, "%s: the checkpoint overlaps the workspace", what);
  return MAP_OK;
}

struct DoBuild {
  const map_problem& p;
  void* elems;
  hipStream_t st;
  template <typename TS, typename T, class M> map_status run() {
    return hip_status(Runner<TS, T, M>::build(p, elems, st), "map_build_elements");
  }
};
struct DoFilter {
  const map_problem& p;
  SmoothArgs a;
  template <typename TS, typename T, class M> map_status run() {
    return hip_status(Runner<TS, T, M>::filter(p, a), "map_filter_scan");
  }
};
struct DoSmoother {
  const map_problem& p;
  SmoothArgs a;
  bool grad;
  template <typename TS, typename T, class M> map_status run() {
    return hip_status(Runner<TS, T, M>::smoother(p, a, grad), grad ? "map_backward" : "map_smoother_scan");
  }
};
struct DoSmooth {
  const map_problem& p;
  SmoothArgs a;
  template <typename TS, typename T, class M> map_status run() {
    return hip_status(Runner<TS, T, M>::smooth(p, a), "map_smooth");
  }
};
struct DoTwoFilter {
  const map_problem& p;
  SmoothArgs a;
  template <typename TS, typename T, class M> map_status run() {
    return hip_status(Runner<TS, T, M>::two_filter(p, a), "map_two_filter_smooth");
  }
};
struct DoIft {
  const map_problem& p;
  SmoothArgs a;
  IftArgs b;
  template <typename TS, typename T, class M> map_status run() {
    return hip_status(Runner<TS, T, M>::ift(p, a, b), "map_backward (implicit-function VJP)");
  }
};
struct DoDense {
  const map_problem& p;
  const void *S, *v, *xs;
  void *xd, *Sd, *vd;
  hipStream_t st;
  template <typename TS, typename T, class M> map_status run() {
    return hip_status(Runner<TS, T, M>::dense(p, S, v, xs, xd, Sd, vd, st), "map_dense_output");
  }
};
struct DoInitX {
  const map_problem& p;
  void* xb;
  hipStream_t st;
  template <typename TS, typename T, class M> map_status run() {
    return hip_status(Runner<TS, T, M>::init_xbar(p, xb, st), "map_iterated_nonlinear");
  }
};

}  // namespace
}  // namespace ms

using namespace ms;

extern "C" {

size_t map_workspace_bytes(const map_problem* p) {
  if (validate(p, false) != MAP_OK) return 0;
  return sched::ws_bytes_for(*p);
}

map_status map_workspace_init(void* ws, size_t ws_bytes, void* stream) {
  if (ws == nullptr || ws_bytes < size_t(kCounterWords) * 4)
    return fail(MAP_E_WORKSPACE, "workspace too small");
  k_clear_words<<<1, 256, 0, static_cast<hipStream_t>(stream)>>>(static_cast<unsigned int*>(ws),
                                                                   kCounterWords);
  return hip_status(hipGetLastError(), "map_workspace_init");
}

map_status map_build_elements(const map_problem* p, void* elems, void* stream) {
  map_status s = validate(p);
  if (s != MAP_OK) return s;
  if (elems == nullptr) return fail(MAP_E_ARG, "elems is NULL");
  return dispatch(*p, DoBuild{*p, elems, static_cast<hipStream_t>(stream)});
}

map_status map_filter_scan(const map_problem* p, void* S, void* v, void* m, void* P, double* loglik,
                           void* ws, size_t ws_bytes, void* stream) {
  map_status s = validate(p);
  if (s != MAP_OK) return s;
  if (S == nullptr || v == nullptr) return fail(MAP_E_ARG, "S/v is NULL");
  if ((m == nullptr) != (P == nullptr)) return fail(MAP_E_ARG, "m and P must be given together");
  if ((s = check_divergence(*p, loglik != nullptr, "map_filter_scan")) != MAP_OK) return s;
  if ((s = check_blocks(*p, loglik != nullptr, "map_filter_scan")) != MAP_OK) return s;
  if ((s = check_ws(*p, ws, ws_bytes, false)) != MAP_OK) return s;
  SmoothArgs a{S, v, m, P, nullptr, nullptr, loglik, nullptr, nullptr, nullptr, ws,
               static_cast<hipStream_t>(stream), sched::resolve(*p, false)};
  return finish_check(*p, ws, a.stream, dispatch(*p, DoFilter{*p, a}));
}

map_status map_smoother_scan(const map_problem* p, const void* S, const void* v, void* xs, void* Ps,
                             double* obj, void* ws, size_t ws_bytes, void* stream) {
  map_status s = validate(p);
  if (s != MAP_OK) return s;
  if (S == nullptr || v == nullptr || xs == nullptr) return fail(MAP_E_ARG, "S/v/xs is NULL");
  if ((s = check_blocks(*p, obj != nullptr, "map_smoother_scan")) != MAP_OK) return s;
  if ((s = check_ws(*p, ws, ws_bytes, false)) != MAP_OK) return s;
  SmoothArgs a{const_cast<void*>(S), const_cast<void*>(v), nullptr, nullptr, xs, Ps, nullptr, obj,
               nullptr, nullptr, ws, static_cast<hipStream_t>(stream), sched::resolve(*p, false)};
  return finish_check(*p, ws, a.stream, dispatch(*p, DoSmoother{*p, a, false}));
}

map_status map_smooth(const map_problem* p, void* S, void* v, void* xs, void* Ps, double* loglik,
                      double* obj, double* g_loglik, double* g_obj, void* ws, size_t ws_bytes,
                      void* stream) {
  map_status s = validate(p);
  if (s != MAP_OK) return s;
  if (S == nullptr || v == nullptr || xs == nullptr) return fail(MAP_E_ARG, "S/v/xs is NULL");
  if ((g_loglik != nullptr || g_obj != nullptr) && p->model == MAP_MODEL_LINEAR)
    return fail(MAP_E_UNSUPPORTED, "gradients need a parametric model");
  if ((s = check_divergence(*p, loglik || g_loglik || g_obj, "map_smooth")) != MAP_OK) return s;
  if ((s = check_blocks(*p, loglik || obj || g_loglik || g_obj, "map_smooth")) != MAP_OK) return s;
  if ((s = check_ws(*p, ws, ws_bytes, true)) != MAP_OK) return s;
  SmoothArgs a{S, v, nullptr, nullptr, xs, Ps, loglik, obj, g_loglik, g_obj, ws,
               static_cast<hipStream_t>(stream), sched::resolve(*p, true)};
  return finish_check(*p, ws, a.stream, dispatch(*p, DoSmooth{*p, a}));
}

size_t map_checkpoint_bytes(const map_problem* p) {
  if (validate(p, false) != MAP_OK) return 0;
  return ckpt_need(*p);
}

map_status map_smooth_checkpointed(const map_problem* p, void* S, void* v, void* xs, void* Ps,
                                   double* loglik, double* obj, double* g_loglik, double* g_obj,
                                   void* ckpt, size_t ckpt_bytes, void* ws, size_t ws_bytes,
                                   void* stream) {
  map_status s = validate(p);
  if (s != MAP_OK) return s;
  if (S == nullptr || v == nullptr || xs == nullptr) return fail(MAP_E_ARG, "S/v/xs is NULL");
  if (ckpt == nullptr) return fail(MAP_E_ARG, "map_smooth_checkpointed: ckpt is NULL");
  {
    const void* others[8] = {S, v, xs, Ps, loglik, obj, g_loglik, g_obj};
    for (const void* o : others)
      if (o == ckpt) return fail(MAP_E_ARG, "map_smooth_checkpointed: ckpt aliases an output");
  }
  if ((s = check_ckpt(*p, ckpt, ckpt_bytes, ws, ws_bytes, "map_smooth_checkpointed")) != MAP_OK)
    return s;
  if ((s = check_divergence(*p, loglik || g_loglik || g_obj, "map_smooth_checkpointed")) != MAP_OK)
    return s;
  if ((s = check_ws(*p, ws, ws_bytes, false)) != MAP_OK) return s;
  SmoothArgs a{S, v, nullptr, nullptr, xs, Ps, loglik, obj, g_loglik, g_obj, ws,
               static_cast<hipStream_t>(stream), sched::resolve(*p, false)};
  a.ckpt = ckpt;
  return finish_check(*p, ws, a.stream, dispatch(*p, DoSmooth{*p, a}));
}

map_status map_smooth_noalloc(const map_problem* p, void* S, void* v, void* xs, void* Ps,
                              double* loglik, double* obj, double* g_loglik, double* g_obj,
                              void* stream) {
  map_status s = validate(p);
  if (s != MAP_OK) return s;
  if (S == nullptr || v == nullptr || xs == nullptr) return fail(MAP_E_ARG, "S/v/xs is NULL");
  if ((g_loglik != nullptr || g_obj != nullptr) && p->model == MAP_MODEL_LINEAR)
    return fail(MAP_E_UNSUPPORTED, "gradients need a parametric model");
  if ((s = check_divergence(*p, loglik || g_loglik || g_obj, "map_smooth_noalloc")) != MAP_OK)
    return s;
  if ((s = check_blocks(*p, loglik || obj || g_loglik || g_obj, "map_smooth_noalloc")) != MAP_OK)
    return s;
  const int chunk = sched::resolve(*p, true);
  const size_t need = sched::ws_need(*p, chunk);
  if (need > kScratchBytes)
    return fail(MAP_E_WORKSPACE,
                "map_smooth_noalloc: the problem needs %zu bytes of workspace, the fixed scratch "
                "holds %zu; use map_smooth with a caller-owned workspace",
                need, kScratchBytes);
  void* ws = nullptr;
  if ((s = scratch_address(&ws)) != MAP_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  // the control words must start at zero: cleared by a kernel (no memset)
  // before every call, also after a call that failed part-way
  k_clear_words<<<1, 256, 0, st>>>(static_cast<unsigned int*>(ws), kCounterWords);
  if ((s = hip_status(hipGetLastError(), "map_smooth_noalloc: clear")) != MAP_OK) return s;
  SmoothArgs a{S, v, nullptr, nullptr, xs, Ps, loglik, obj, g_loglik, g_obj, ws, st, chunk};
  return finish_check(*p, ws, st, dispatch(*p, DoSmooth{*p, a}));
}

map_status map_two_filter_smooth(const map_problem* p, void* S, void* v, void* xs, void* Ps,
                                 double* loglik, void* ws, size_t ws_bytes, void* stream) {
  map_status s = validate(p);
  if (s != MAP_OK) return s;
  if (S == nullptr || v == nullptr || xs == nullptr) return fail(MAP_E_ARG, "S/v/xs is NULL");
  if (p->flags & MAP_OM_DIVERGENCE)
    return fail(MAP_E_UNSUPPORTED, "map_two_filter_smooth: MAP_OM_DIVERGENCE is not supported");
  if ((s = check_blocks(*p, true, "map_two_filter_smooth")) != MAP_OK) return s;
  if (large_linear(*p))
    return fail(MAP_E_UNSUPPORTED, "map_two_filter_smooth: the general linear model is built up "
                                   "to nx = 4 for the two-filter form");
  if ((s = check_ws(*p, ws, ws_bytes, false)) != MAP_OK) return s;
  SmoothArgs a{S, v, nullptr, nullptr, xs, Ps, loglik, nullptr, nullptr, nullptr, ws,
               static_cast<hipStream_t>(stream), sched::resolve(*p, false)};
  return finish_check(*p, ws, a.stream, dispatch(*p, DoTwoFilter{*p, a}));
}

map_status map_dense_output(const map_problem* p, const void* S, const void* v, const void* xs,
                            void* xd, void* Sd, void* vd, void* stream) {
  map_status s = validate(p);
  if (s != MAP_OK) return s;
  if (p->n_sub < 2) return fail(MAP_E_ARG, "map_dense_output needs sub-stepped blocks (n_sub >= 2)");
  if (S == nullptr || v == nullptr || xs == nullptr || xd == nullptr || Sd == nullptr ||
      vd == nullptr)
    return fail(MAP_E_ARG, "S/v/xs/xd/Sd/vd is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  return dispatch(*p, DoDense{*p, S, v, xs, xd, Sd, vd, st});
}

map_status map_iterated_nonlinear(const map_problem* p, int32_t n_iter, const void* xbar0,
                                  void* xbar_buf, void* S, void* v, void* xs, void* Ps,
                                  double* loglik, double* obj, double* g_loglik, double* g_obj,
                                  void* ws, size_t ws_bytes, void* stream) {
  map_status s = validate(p, false);
  if (s != MAP_OK) return s;
  if (n_iter < 1) return fail(MAP_E_ARG, "n_iter must be >= 1");
  if (xbar_buf == nullptr || S == nullptr || v == nullptr || xs == nullptr)
    return fail(MAP_E_ARG, "xbar_buf/S/v/xs is NULL");
  if (xbar_buf == xs) return fail(MAP_E_ARG, "xbar_buf must not alias xs");
  if ((g_loglik != nullptr || g_obj != nullptr) && p->model == MAP_MODEL_LINEAR)
    return fail(MAP_E_UNSUPPORTED, "gradients need a parametric model");
  if ((s = check_divergence(*p, loglik || g_loglik || g_obj, "map_iterated_nonlinear")) != MAP_OK)
    return s;
  if ((s = check_blocks(*p, loglik || obj || g_loglik || g_obj, "map_iterated_nonlinear")) != MAP_OK)
    return s;
  if ((s = check_ws(*p, ws, ws_bytes, true)) != MAP_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t ns = p->n_steps + p->n_seg;
  const size_t tiles = size_t((ns + 1023) / 1024);
  const size_t bytes = size_t(p->nx) * tiles * 1024 * storage_bytes(p->dtype);
  // iteration i reads xbar from `src` and writes xs to the other buffer; the
  // last iteration must read xbar_buf and write xs
  void* bufs[2] = {xbar_buf, xs};
  int cur = ((n_iter - 1) % 2 == 0) ? 0 : 1;
  if (xbar0 != nullptr) {
    s = hip_status(hipMemcpyAsync(bufs[cur], xbar0, bytes, hipMemcpyDeviceToDevice, st),
                   "map_iterated_nonlinear");
    if (s != MAP_OK) return s;
  } else {
    s = dispatch(*p, DoInitX{*p, bufs[cur], st});
    if (s != MAP_OK) return s;
  }
  map_problem q = *p;
  for (int32_t it = 0; it < n_iter; ++it) {
    const bool last = it == n_iter - 1;
    q.xbar = bufs[cur];
    SmoothArgs a{S, v, nullptr, nullptr, bufs[1 - cur], last ? Ps : nullptr,
                 last ? loglik : nullptr, last ? obj : nullptr, last ? g_loglik : nullptr,
                 last ? g_obj : nullptr, ws, st, sched::resolve(q, true)};
    s = dispatch(q, DoSmooth{q, a});
    if (s != MAP_OK) return s;
    cur = 1 - cur;
  }
  return finish_check(*p, ws, st, MAP_OK);
}

map_status map_backward(const map_problem* p, void* S, void* v, void* xs, void* Ps,
                        double* obj, double* g_loglik, double* g_obj, const void* g_xs, void* mu,
                        void* vmu, double* g_xs_theta, double* g_elems, const void* ckpt,
                        size_t ckpt_bytes, void* ws, size_t ws_bytes, void* stream) {
  map_status s = validate(p);
  if (s != MAP_OK) return s;
  if (S == nullptr || v == nullptr || xs == nullptr) return fail(MAP_E_ARG, "S/v/xs is NULL");
  if (g_loglik == nullptr && g_obj == nullptr && g_xs == nullptr && g_elems == nullptr)
    return fail(MAP_E_ARG, "nothing to differentiate: g_loglik, g_obj, g_xs and g_elems are NULL");
  if (g_elems != nullptr) {
    const void* others[10] = {S, v, xs, Ps, obj, g_loglik, g_obj, g_xs, g_xs_theta, ckpt};
    for (const void* o : others)
      if (o == g_elems) return fail(MAP_E_ARG, "g_elems aliases another buffer");
  }
  if (ckpt != nullptr) {
    // S, v are rebuilt (written) here: distinct from each other, from the
    // other outputs and from the checkpoint
    const void* outs[7] = {S, v, xs, Ps, obj, g_loglik, g_obj};
    for (int a = 0; a < 2; ++a)
      for (int b = a + 1; b < 7; ++b)
        if (outs[a] == outs[b])
          return fail(MAP_E_ARG, "map_backward: with a checkpoint, S and v are outputs and must "
                                 "not alias each other or another output");
    const void* others[11] = {S, v, xs, Ps, obj, g_loglik, g_obj, g_xs, mu, vmu, g_xs_theta};
    for (const void* o : others)
      if (o == ckpt) return fail(MAP_E_ARG, "map_backward: the checkpoint aliases another buffer");
    if ((s = check_ckpt(*p, ckpt, ckpt_bytes, ws, ws_bytes, "map_backward")) != MAP_OK) return s;
  }
  if (g_xs != nullptr) {
    if (mu == nullptr || vmu == nullptr || g_xs_theta == nullptr)
      return fail(MAP_E_ARG, "g_xs needs mu, vmu and g_xs_theta");
    const void* outs[3] = {xs, mu, vmu};
    const void* ins[3] = {S, v, g_xs};
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        if (outs[a] == ins[b] || (a < b && outs[a] == outs[b]))
          return fail(MAP_E_ARG, "xs, mu and vmu must be distinct and not alias S, v or g_xs");
  }
  if (p->model == MAP_MODEL_LINEAR) return fail(MAP_E_UNSUPPORTED, "gradients need a parametric model");
  if ((s = check_divergence(*p, true, "map_backward")) != MAP_OK) return s;
  if ((s = check_blocks(*p, true, "map_backward")) != MAP_OK) return s;
  if ((s = check_ws(*p, ws, ws_bytes, false)) != MAP_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  SmoothArgs a{S, v, nullptr, nullptr, xs, Ps, nullptr, obj,
               g_loglik, g_obj, ws, st, sched::resolve(*p, false), g_elems};
  a.ckpt = const_cast<void*>(ckpt);
  s = dispatch(*p, DoSmoother{*p, a, g_loglik != nullptr || g_obj != nullptr || g_elems != nullptr});
  if (s == MAP_OK && g_xs != nullptr)
    s = dispatch(*p, DoIft{*p, a, IftArgs{g_xs, mu, vmu, g_xs_theta}});
  return finish_check(*p, ws, st, s);
}

map_status map_autotune(const map_problem* p, void* ws, size_t ws_bytes, const char* cache_path,
                        int32_t* chunk_out, void* stream) {
  map_status s = validate(p);
  if (s != MAP_OK) return s;
  if (chunk_out == nullptr) return fail(MAP_E_ARG, "chunk_out is NULL");
  map_problem q = *p;
  q.flags &= ~(MAP_CHECK_FINITE | MAP_OM_DIVERGENCE);  // timing runs: every output, nothing checked
  q.chunk = 0;
  if (ws == nullptr || ws_bytes < sched::ws_bytes_for(q))
    return fail(MAP_E_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes,
                sched::ws_bytes_for(q));
  const std::string key = sched::key_of(q);
  if (cache_path != nullptr) {
    if (FILE* fh = fopen(cache_path, "r")) {
      char k[128];
      int c = 0;
      double t = 0.0;
      std::lock_guard<std::mutex> lk(sched::g_mu);
      while (fscanf(fh, "%127s %d %lf", k, &c, &t) == 3)
        if (valid_chunk(c)) sched::g_tuned[k] = c;
      fclose(fh);
    }
  }
  {
    std::lock_guard<std::mutex> lk(sched::g_mu);
    auto it = sched::g_tuned.find(key);
    if (it != sched::g_tuned.end()) {
      *chunk_out = it->second;
      return MAP_OK;
    }
  }
  // temporary outputs for timing the fused step (the work map_smooth does
  // with every output requested)
  const int64_t ns = q.n_steps + q.n_seg;
  const size_t tiled = size_t((ns + 1023) / 1024) * 1024 * storage_bytes(q.dtype);
  const int nsym = q.nx * (q.nx + 1) / 2;
  const int nth = model_ntheta(q);
  const size_t sizes[8] = {tiled * nsym, tiled * q.nx, tiled * q.nx, tiled * nsym,
                           size_t(q.n_seg) * 8, size_t(q.n_seg) * 8,
                           nth > 0 ? size_t(q.n_seg) * nth * 8 : 0, nth > 0 ? size_t(q.n_seg) * nth * 8 : 0};
  void* buf[8] = {};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto cleanup = [&]() {
    for (void*& b : buf)
      if (b) { hipFree(b); b = nullptr; }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
  };
  for (int i = 0; i < 8; ++i)
    if (sizes[i] && hipMalloc(&buf[i], sizes[i]) != hipSuccess) {
      cleanup();
      return fail(MAP_E_HIP, "map_autotune: hipMalloc of %zu bytes failed", sizes[i]);
    }
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    return fail(MAP_E_HIP, "map_autotune: hipEventCreate failed");
  }
  constexpr int kReps = 3, kRounds = 2;
  // the flat schedules, and for batches of many segments the segment-local one
  std::vector<int> cands(std::begin(kChunks), std::end(kChunks));
  if (q.n_seg >= 64 && q.n_seg <= int64_t(INT32_MAX) && !large_linear(q))
    cands.push_back(kSchedSegWave);
  // every candidate timed in each of kRounds interleaved rounds (warm-up in
  // the first), its best round kept: schedules within ~10 % of each other
  // otherwise swap places from run to run
  std::vector<float> cand_ms(cands.size(), 0.f);
  for (int round = 0; round < kRounds; ++round)
    for (size_t ci = 0; ci < cands.size(); ++ci) {
      const int c = cands[ci];
      q.chunk = c;
      SmoothArgs a{buf[0], buf[1], nullptr, nullptr, buf[2], buf[3], static_cast<double*>(buf[4]),
                   static_cast<double*>(buf[5]), static_cast<double*>(buf[6]),
                   static_cast<double*>(buf[7]), ws, st, c};
      if (round == 0) s = dispatch(q, DoSmooth{q, a});  // warm-up
      if (s == MAP_OK) s = hip_status(hipEventRecord(e0, st), "map_autotune");
      for (int r = 0; r < kReps && s == MAP_OK; ++r) s = dispatch(q, DoSmooth{q, a});
      if (s == MAP_OK) s = hip_status(hipEventRecord(e1, st), "map_autotune");
      if (s == MAP_OK) s = hip_status(hipEventSynchronize(e1), "map_autotune");
      float ms = 0.f;
      if (s == MAP_OK) s = hip_status(hipEventElapsedTime(&ms, e0, e1), "map_autotune");
      if (s != MAP_OK) {
        cleanup();
        return s;
      }
      ms /= kReps;
      if (round == 0 || ms < cand_ms[ci]) cand_ms[ci] = ms;
    }
  int best = 0;
  float best_ms = 0.f;
  for (size_t ci = 0; ci < cands.size(); ++ci)
    if (best == 0 || cand_ms[ci] < best_ms) {
      best = cands[ci];
      best_ms = cand_ms[ci];
    }
  cleanup();
  {
    std::lock_guard<std::mutex> lk(sched::g_mu);
    sched::g_tuned[key] = best;
  }
  if (cache_path != nullptr) {
    if (FILE* fh = fopen(cache_path, "a")) {
      fprintf(fh, "%s %d %.6f\n", key.c_str(), best, double(best_ms));
      fclose(fh);
    }
  }
  *chunk_out = best;
  return MAP_OK;
}

// Finite tests on the stored bit pattern: the library is built with
// -ffinite-math-only, under which the compiler may fold std::isfinite (or any
// test of a double value) to true.  The bytes are read as integers.
static bool finite_at(const double* p) {
  uint64_t u;
  memcpy(&u, p, sizeof(u));
  return ((u >> 52) & 0x7ff) != 0x7ff;
}
static bool finite_value(double x) {
  volatile double v = x;
  const volatile unsigned char* b = reinterpret_cast<const volatile unsigned char*>(&v);
  uint64_t u = 0;
  for (int i = 0; i < 8; ++i) u |= uint64_t(b[i]) << (8 * i);
  return ((u >> 52) & 0x7ff) != 0x7ff;
}

map_status map_lti_exact_terms(int32_t nx, int32_t nw, const double* F, const double* c,
                               const double* L, const double* W, double dt, double* F_out,
                               double* c_out, double* L_out) {
  if (nx < 1 || nx > 8 || nw < 1 || nw > 8)
    return fail(MAP_E_DIM, "dimensions (nx, nw) = (%d, %d) outside [1, 8]", nx, nw);
  if (!finite_value(dt) || !(dt > 0.0)) return fail(MAP_E_ARG, "dt must be finite and > 0");
  if (F == nullptr || L == nullptr || W == nullptr || F_out == nullptr || c_out == nullptr ||
      L_out == nullptr)
    return fail(MAP_E_ARG, "F/L/W or an output is NULL");
  for (int i = 0; i < nx * nx; ++i)
    if (!finite_at(F + i)) return fail(MAP_E_NUMERIC, "F is not finite");
  for (int i = 0; i < nx * nw; ++i)
    if (!finite_at(L + i)) return fail(MAP_E_NUMERIC, "L is not finite");
  for (int i = 0; i < nw * nw; ++i)
    if (!finite_at(W + i)) return fail(MAP_E_NUMERIC, "W is not finite");
  if (c != nullptr)
    for (int i = 0; i < nx; ++i)
      if (!finite_at(c + i)) return fail(MAP_E_NUMERIC, "c is not finite");
  lti::exact_terms(nx, nw, F, c, L, W, dt, F_out, c_out, L_out);
  return MAP_OK;
}

map_status map_schedule(const map_problem* p, int32_t* chunk_out) {
  map_status s = validate(p, false);
  if (s != MAP_OK) return s;
  if (chunk_out == nullptr) return fail(MAP_E_ARG, "chunk_out is NULL");
  *chunk_out = sched::resolve(*p, true);
  return MAP_OK;
}

map_status map_profile_enable(int32_t capacity) {
  for (auto& r : prof::g_recs) {
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  prof::g_recs.clear();
  prof::g_used = 0;
  prof::g_on = capacity > 0;
  for (int32_t i = 0; i < capacity; ++i) {
    prof::Rec r;
    if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) {
      prof::g_on = false;
      return fail(MAP_E_HIP, "map_profile_enable: hipEventCreate failed");
    }
    r.kind = -1;
    prof::g_recs.push_back(r);
  }
  return MAP_OK;
}

map_status map_profile_read(int32_t kind, int64_t* count, double* total_ms) {
  if (count == nullptr || total_ms == nullptr) return fail(MAP_E_ARG, "count/total_ms is NULL");
  *count = 0;
  *total_ms = 0.0;
  for (size_t i = 0; i < prof::g_used; ++i) {
    const prof::Rec& r = prof::g_recs[i];
    if (r.kind != kind) continue;
    if (hipEventSynchronize(r.b) != hipSuccess) return fail(MAP_E_HIP, "hipEventSynchronize failed");
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
      return fail(MAP_E_HIP, "hipEventElapsedTime failed");
    *count += 1;
    *total_ms += ms;
  }
  return MAP_OK;
}

map_status map_profile_reset(void) {
  prof::g_used = 0;
  return MAP_OK;
}

const char* map_last_error(void) { return g_err.c_str(); }

int32_t map_abi_version(void) { return MAPSCAN_ABI_VERSION; }

}  // extern "C"
