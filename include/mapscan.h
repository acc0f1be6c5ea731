/*
 * mapscan: parallel-in-time MAP trajectory estimation for partially observed
 * SDEs on AMD Instinct MI355X (gfx950).
 *
 * The library solves, for every segment of a batch, the discretised
 * Onsager--Machlup MAP problem of the model (Sec. 2.1, eq. statespace and
 * eq. OM)
 *
 *     dx/dt = f(x) + L w,    y = h(x) + v,    w, v white noise with spectral
 *     densities W and R,     x(t0) ~ N(m0, P0),
 *
 * in its linear-affine form (Sec. 2.4, eq. linear-statespace) or, for a
 * nonlinear model, by iterated Taylor linearisation (Sec. 4.4).  One grid
 * step [t_{k-1}, t_k] of length dt_k contributes the element of Sec. 4.2
 * (eq. backwardLQT) obtained by one explicit-Euler step of its ODE from the
 * boundary value; the drift and measurement are evaluated at the step's right
 * end and y_k is the measurement of x_k.  The filter is the associative scan
 * of Sec. 3.4 (eq. valueparallel) with the linear combination rule of Sec. 4.1;
 * the trajectory is recovered by the affine scan of Sec. 4.3 (eq. 42), i.e. the
 * parallel Kalman--Bucy filter in information form and the parallel RTS
 * smoother (Sec. 2.5).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Real arrays have the dtype in map_problem.dtype (float or double);
 *    per-segment scalar outputs (log-likelihood, objective, gradients) are
 *    always double.
 *  - Every array pointer is a DEVICE pointer owned by the caller, except
 *    seg_off_host.  Nothing is allocated or freed by the library (except
 *    map_autotune's temporary outputs); the workspace is caller-owned too
 *    (map_workspace_bytes, map_workspace_init).
 *  - Work is enqueued asynchronously on `stream` (a hipStream_t passed as
 *    void*, NULL = the default stream).  A call returns after enqueueing.
 *  - Steps of all segments are concatenated: segment s owns steps
 *    seg_off[s] .. seg_off[s+1]-1 and states seg_off[s]+s .. seg_off[s+1]+s
 *    (T_s steps give T_s+1 states; state seg_off[s]+s is the prior time t0).
 *    n_states = n_steps + n_seg.  Step k of segment s ends at state k + s + 1.
 *  - State-indexed arrays use the TILED layout (MAPSCAN_TILE = 1024 states
 *    per tile: 16 rows of 64 states).  For an array with C components,
 *    component c of state i is at
 *        ((i / 1024) * C + c) * 1024 + (i % 16) * 64 + (i / 16) % 64,
 *    and the buffer holds ceil(n_states / 1024) * C * 1024 elements (the
 *    caller allocates the padding; padded entries are never read as data and
 *    may be written).  The kernels give each lane `chunk` consecutive states
 *    (a schedule: 4, 8, 16 or 32, see map_problem.chunk); up to 16, every
 *    access of a wavefront covers whole cache lines (at 32, every other value
 *    of a row, the rest 16 states later).  Measurements y and per-step lengths
 *    dt are given per state too:
 *    the value of the step that ends at state i (entries at a segment's first
 *    state are ignored).
 *  - Symmetric nx x nx matrices are nx(nx+1)/2 components, lower triangle in
 *    row order (0,0),(1,0),(1,1),(2,0)...
 *  - Errors: every entry returns a map_status; arguments are validated on the
 *    host before anything is launched, and a failing check launches nothing.
 *    map_last_error() gives a readable message for the calling thread.
 *  - One call at a time per workspace: calls that share a workspace must be
 *    ordered on one stream.
 */
#ifndef MAPSCAN_H
#define MAPSCAN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MAPSCAN_ABI_VERSION 9
#define MAPSCAN_TILE 1024
#define MAP_CHECK_FINITE 1
/* map_problem.flags: minimise the Onsager--Machlup objective with its
 * divergence term (Sec. 2.1, eq. OM: + 1/2 sum_k dt_k div f(x_k) in the
 * discretised objective) instead of the energy part alone.  Where div f
 * depends on the state (Van der Pol: mu (1 - x1^2)) each linearisation also
 * takes the term's second-order expansion about xbar (a Newton step on it;
 * the Gauss--Newton step of Sec. 4.4 drops it).  x*, P^s (the inverse
 * Hessian of the expanded objective) and the objective (with the term,
 * evaluated at x*) only: log-likelihood and gradients are rejected, as is
 * the two-filter form.  Valid while the combined information stays positive
 * definite (Van der Pol: 1/r > mu). */
#define MAP_OM_DIVERGENCE 2
/* map_problem.chunk: the segment-local schedule of map_smooth (see there) */
#define MAP_SCHED_SEGMENT_WAVE (-1)

typedef enum {
  MAP_OK = 0,
  MAP_E_ARG = -1,         /* null/invalid pointer or value */
  MAP_E_DIM = -2,         /* dimensions out of range or inconsistent */
  MAP_E_DTYPE = -3,       /* unknown dtype */
  MAP_E_LAYOUT = -4,      /* segment offsets not monotone / inconsistent */
  MAP_E_NUMERIC = -5,     /* with MAP_CHECK_FINITE: a non-finite value in the results */
  MAP_E_HIP = -6,         /* a HIP runtime call or kernel launch failed */
  MAP_E_WORKSPACE = -7,   /* workspace missing or too small */
  MAP_E_UNSUPPORTED = -8  /* model/dimension combination not built */
} map_status;

/* Storage and arithmetic precision.  On MI355X, FP64 and (non-packed) FP32
 * vector FMAs issue at the same rate, so MAP_F32 keeps the caller's arrays in
 * FP32 (half the HBM traffic) and computes in FP64: the information-form
 * recursion cancels large terms (v = S m for states far from the origin), and
 * FP64 arithmetic keeps the FP32 results at FP32 rounding level.  MAP_F32_FAST
 * also computes in FP32 (fewer registers, higher occupancy); its error grows
 * with |x| / (dt |dx/dt|) and can exceed 1e-4 relative on long trajectories.
 * The workspace is kept in the arithmetic type. */
typedef enum { MAP_F32 = 0, MAP_F64 = 1, MAP_F32_FAST = 2 } map_dtype;

/* Models.  Parameter vectors theta (per segment):
 *   MAP_MODEL_LINEAR    none; dense F, c, L, W, H, r, R given per step (forward only)
 *   MAP_MODEL_CV        (gamma, q, r): F = [[0, I], [0, -gamma I]], c = 0, L = [0; I],
 *                       W = q I, H = [I, 0], r = 0, R = r I; nx = 2d, ny = nw = d.
 *                       With gamma = 0 this is the Wiener velocity model (Sec. 5.1).
 *   MAP_MODEL_VDP       (mu, q, r): f = (x2, mu (1 - x1^2) x2 - x1), L = I, W = q I,
 *                       h = x1, R = r; nx = 2, ny = 1, nw = 2.
 *   MAP_MODEL_LORENZ63  (sigma, rho, beta, q, r): Lorenz-63 drift, L = I, W = q I,
 *                       h = x, R = r I; nx = ny = nw = 3.
 *   MAP_MODEL_CT        (sv, sw, r1, r2): coordinated turn (Sec. 5.2), state
 *                       (xi, zeta, dxi, dzeta, omega), f = (dxi, dzeta, -omega dzeta,
 *                       omega dxi, 0), L = [[0,0,0],[0,0,0],[sv,0,0],[0,sv,0],[0,0,sw]],
 *                       W = I, h = (sqrt(xi^2 + zeta^2), atan2(zeta, xi)),
 *                       R = diag(r1, r2); nx = 5, ny = 2, nw = 3.  Bearings are in
 *                       radians; the bearing residual is taken modulo 2 pi into
 *                       [-pi, pi), so measurements may be given on any branch.
 * Nonlinear models (VDP, LORENZ63, CT) are linearised about map_problem.xbar. */
typedef enum {
  MAP_MODEL_LINEAR = 0,
  MAP_MODEL_CV = 1,
  MAP_MODEL_VDP = 2,
  MAP_MODEL_LORENZ63 = 3,
  MAP_MODEL_CT = 4
} map_model;

typedef struct {
  int32_t nx, ny, nw;      /* state, measurement and driving-noise dimensions */
  int32_t dtype;           /* map_dtype: storage (and arithmetic) precision of the arrays */
  int32_t model;           /* map_model */
  int32_t n_theta;         /* must equal the model's parameter count (0 for LINEAR) */
  int64_t n_seg;           /* number of trajectories, >= 1 */
  int64_t n_steps;         /* total steps = seg_off[n_seg] */
  const int64_t* seg_off;       /* device [n_seg+1]: 0 = seg_off[0] <= seg_off[1] <= ... */
  const int64_t* seg_off_host;  /* optional host copy; when given it is validated */
  const void* dt;          /* device: one value (dt_stride 0) or tiled [1] per state, > 0 */
  int64_t dt_stride;       /* 0 (one shared value) or 1 (tiled per state) */
  const void* y;           /* device, tiled [ny] per state: measurement of that state
                            * (a segment's first state holds an unused value); never
                            * NULL, also when n_steps = 0 */
  const void* m0;          /* device [n_seg][nx] prior means (m0_stride = nx, or 0: shared) */
  int64_t m0_stride;
  const void* P0;          /* device [n_seg][nx*nx] row-major SPD prior covariances */
  int64_t P0_stride;       /* nx*nx, or 0: shared */
  const void* theta;       /* device [n_seg][n_theta] (theta_stride = n_theta, or 0: shared) */
  int64_t theta_stride;
  const void* xbar;        /* device, tiled [nx] per state: linearisation states (nonlinear) */
  /* MAP_MODEL_LINEAR only: row-major per-step matrices F [nx*nx], c [nx],
   * L [nx*nw], W [nw*nw] (SPD), H [ny*nx], r [ny], R [ny*ny] (SPD); matrix of
   * step k at base + k * stride (stride 0: one matrix for all steps). */
  const void *F, *c, *L, *W, *H, *r, *R;
  int64_t F_stride, c_stride, L_stride, W_stride, H_stride, r_stride, R_stride;
  /* Schedule.  Flat schedules cut the concatenated states of all segments
   * into lanes of `chunk` states (4, 8, 16 or 32; at 32 the filter up-sweep
   * runs 32 states per lane and the passes after it 16) joined by
   * cross-block scans.  MAP_SCHED_SEGMENT_WAVE (map_smooth and
   * map_smooth_noalloc only; the other entry points use the flat default
   * instead): one persistent wavefront per segment, segments taken longest
   * first, no cross-block step (for batches of many segments).  0 lets the
   * library choose: the choice map_autotune recorded for this problem's
   * shape, else 32 when the filter pass then still gives every SIMD of the
   * device four wavefronts, else the largest of 16, 8 and 4 that gives every
   * second SIMD a wavefront.
   * Results do not depend on it beyond rounding. */
  int32_t chunk;
  /* Flags: MAP_OM_DIVERGENCE (above), and
   * MAP_CHECK_FINITE: the kernels flag any non-finite value they write (S, v,
   * x*, P^s diagonals, log-likelihood, objective, gradients); the entry point
   * then waits for its stream, and returns MAP_E_NUMERIC if one was seen (a
   * non-finite input, or a covariance that is not positive definite).  The
   * flag lives in the workspace, which the entry point leaves clear again.
   * Costs one stream synchronisation per call; without it nothing is checked. */
  int32_t flags;
  /* Sub-stepped blocks (the paper's T blocks of n Euler substeps, Sec. 5.1):
   * 0 or 1: one grid step is one explicit-Euler step of the element ODE
   * (Sec. 4.2, eq. backwardLQT) from its boundary value, the element of every
   * other entry; n_sub in [2, 64]: each grid step is a block whose element is
   * that ODE integrated by n_sub explicit-Euler substeps of length dt / n_sub
   * (the A equation read as A' = -A (Q J + F)), the model's terms held over
   * the block (linearised at its last state), substep j using the
   * measurement at its end: y then holds ny * n_sub components per state,
   * component j * ny + c being measurement c at the end of substep j + 1 of
   * the block that ends at the state.  Built for the constant-velocity model
   * (nx = 4) and Van der Pol, MAP_F64 and MAP_F32.  Filter, smoother and
   * map_dense_output only: no log-likelihood, objective, gradients,
   * two-filter form or MAP_OM_DIVERGENCE. */
  int32_t n_sub;
} map_problem;

/* Size in bytes of the workspace every scan entry needs for this problem
 * (0 if the problem is invalid; see map_last_error).  With chunk = 0 it fits
 * every schedule the library may choose. */
size_t map_workspace_bytes(const map_problem* p);

/* Zero the workspace's control words.  Call once after allocating a
 * workspace; every entry point leaves them zero when its kernels finish. */
map_status map_workspace_init(void* ws, size_t ws_bytes, void* stream);

/* Element build (Sec. 4.2, eq. backwardLQT, one explicit-Euler step from the
 * boundary value; Sec. 3.4 for the prior element a_T = -log p(x(t0))):
 * writes, for every state i, the element of the step ending at i -- or the
 * prior element (A = 0, b = 0, C = 0, eta = P0^{-1} m0, J = P0^{-1}) at a
 * segment's first state -- as planes
 *   A (nx*nx, row-major), b (nx), C (sym), eta (nx), J (sym)
 * i.e. nx*nx + 2 nx + nx(nx+1) tiled components per state in `elems`. */
map_status map_build_elements(const map_problem* p, void* elems, void* stream);

/* Filter scan (Sec. 3.4 eq. valueparallel with the combination rule of
 * Sec. 4.1; information form of the Kalman--Bucy filter, Sec. 2.5):
 *   S     out tiled [nx(nx+1)/2] per state: information matrix S_k = P_k^{-1}
 *   v     out tiled [nx] per state:         information vector v_k = P_k^{-1} m_k
 *         with FP64 storage; with FP32 storage (MAP_F32, MAP_F32_FAST) the
 *         filter mean m_k itself (v rounded to FP32 loses the relative
 *         precision of small components of m: S^{-1} spreads its rounding
 *         over every component).  The smoother entry points read the plane
 *         the same way.
 *   m, P  optional out (NULL to skip) filter mean and covariance
 *   loglik optional out [n_seg] (double): log p(y_1..y_T) by the
 *         prediction-error decomposition of the same discrete model. */
map_status map_filter_scan(const map_problem* p, void* S, void* v, void* m, void* P,
                           double* loglik, void* ws, size_t ws_bytes, void* stream);

/* Trajectory scan (Sec. 4.3, eq. 42: x*_{k-1} = G_k x*_k + beta_k composed by an
 * associative affine scan in reverse time order) from the filter's S, v:
 *   xs    out tiled [nx] per state: MAP trajectory = smoothed means
 *   Ps    optional out tiled [nx(nx+1)/2] per state: smoothed covariances
 *   obj   optional out [n_seg] (double): the discretised OM objective (without
 *         the divergence term) at xs. */
map_status map_smoother_scan(const map_problem* p, const void* S, const void* v, void* xs, void* Ps,
                             double* obj, void* ws, size_t ws_bytes, void* stream);

/* Filter and trajectory scans fused (the filter fix-up and the trajectory
 * up-sweep share one pass), plus, when g_loglik / g_obj are given, the adjoint:
 * gradients with respect to theta of the log-likelihood (Fisher identity) and
 * of the objective's minimum (envelope theorem), [n_seg][n_theta] double.
 * Gradients need a parametric model (not LINEAR) and Ps != NULL. */
map_status map_smooth(const map_problem* p, void* S, void* v, void* xs, void* Ps, double* loglik,
                      double* obj, double* g_loglik, double* g_obj, void* ws, size_t ws_bytes,
                      void* stream);

/* map_smooth without a caller-owned workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and results as
 * map_smooth; the workspace is a fixed 64 MiB device array inside the library
 * (one per device, held until the process ends), so nothing is allocated or
 * freed.  Problems whose workspace (map_workspace_bytes at the schedule the
 * library resolves) exceeds 64 MiB are rejected with MAP_E_WORKSPACE before
 * anything is launched; a 2^20-step nx = 4 problem fits.  Every call on a
 * device shares that device's array: calls that overlap on one device (other
 * streams, other threads) race and must be serialised by the caller.  Each
 * call first clears the array's control words with a kernel on `stream`. */
map_status map_smooth_noalloc(const map_problem* p, void* S, void* v, void* xs, void* Ps,
                              double* loglik, double* obj, double* g_loglik, double* g_obj,
                              void* stream);

/* Filter checkpoints for the adjoint (activation checkpointing; not in the
 * paper).  The filter scan's state at the start of every block of the scan's
 * decomposition -- (S, v) before each run of 4 x 64 lanes x chunk states, the
 * carries of the block-level scan of Sec. 3.4 eq. valueparallel -- is all that
 * map_backward needs besides the inputs: from it, each block's lane and tile
 * prefixes and then S, v at every state are rebuilt locally, with no
 * cross-block step.  Between a forward call and its adjoint the caller then
 * keeps (nx(nx+1)/2 + nx) values per block instead of per state (at chunk 16,
 * one per 4096 states: 28 KB at nx = 4 and 2^20 steps, against 117 MB of
 * S, v planes).
 *
 * map_checkpoint_bytes: bytes of that checkpoint for this problem (0 if the
 * problem is invalid), at the flat schedule that map_backward resolves for it
 * (p->chunk, else map_autotune's record, else the heuristic).  The forward call
 * and the adjoint must resolve the same schedule: pin p->chunk (map_schedule)
 * if map_autotune may run in between.  Values have the arithmetic type
 * (double, float for MAP_F32_FAST). */
size_t map_checkpoint_bytes(const map_problem* p);

/* map_smooth on the flat schedule above that also writes the filter
 * checkpoint to ckpt (device, map_checkpoint_bytes bytes, distinct from every
 * other buffer and outside the workspace).  Same outputs, kernels and results
 * as map_smooth on that schedule; the block carries are written straight to
 * ckpt instead of the workspace.  S, v are still written (the trajectory pass
 * reads them) and may be scratch the caller drops afterwards.  Parametric
 * models only (the adjoint's domain); no sub-stepped blocks. */
map_status map_smooth_checkpointed(const map_problem* p, void* S, void* v, void* xs, void* Ps,
                                   double* loglik, double* obj, double* g_loglik, double* g_obj,
                                   void* ckpt, size_t ckpt_bytes, void* ws, size_t ws_bytes,
                                   void* stream);

/* Two-filter smoother (Sec. 4.3, eq. twofilter): the same MAP trajectory as
 * map_smooth, recovered the paper's second way.  The filter scan gives the
 * forward value function (S_k, v_k); a reverse segmented scan with the same
 * combination rule (Sec. 4.1) gives, for every state, the conditional value
 * function of the steps after it up to its segment's end (the backward
 * filter); each state then combines the two.  Eq. twofilter first minimises
 * the later run over the segment's last state, which needs the run's J to be
 * invertible; a single step observes only ny directions, so the library
 * minimises over both ends jointly instead, which equals the printed formula
 * wherever that J is invertible and stays defined where it is not.
 *   S, v   out, as map_filter_scan
 *   xs     out tiled [nx] per state: MAP trajectory = smoothed means
 *   Ps     optional out tiled [nx(nx+1)/2] per state: smoothed covariances
 *   loglik optional out [n_seg] (double), as map_filter_scan.
 * Costs more than map_smooth (one more element combination per state); no
 * objective or gradients here (map_smooth gives them). */
map_status map_two_filter_smooth(const map_problem* p, void* S, void* v, void* xs, void* Ps,
                                 double* loglik, void* ws, size_t ws_bytes, void* stream);

/* Dense output of sub-stepped blocks (n_sub >= 2): the filter and the MAP
 * state at the n_sub - 1 interior substep times of every block, from the
 * filter planes S, v and the block-boundary MAP states xs of map_smooth (or
 * map_filter_scan + map_smoother_scan) on the same problem.  The filter at
 * substep j is the filter at the block's start carried through the block's
 * partial element of its first j substeps (Sec. 4.1 rule); the MAP states
 * follow the paper's first recovery method (Sec. 3.5, Sec. 4.3): the closed-
 * loop ODE of the optimal trajectory, in original time
 * d/dt x* = (F + Q S) x* - Q v + c, integrated by explicit Euler backwards
 * from the block's end, each substep using the filter at its later end.
 *   xd  out, tiled [nx * (n_sub - 1)] per state: component (j - 1) * nx + a is
 *       x*_a at interior substep j of the block ending at the state
 *   Sd  out, tiled [nx(nx+1)/2 * (n_sub - 1)] per state: the filter's S there
 *   vd  out, tiled [nx * (n_sub - 1)] per state: the second filter plane there
 *       (v, or the mean with FP32 storage, as map_filter_scan)
 * Entries at a segment's first state are not written. */
map_status map_dense_output(const map_problem* p, const void* S, const void* v, const void* xs,
                            void* xd, void* Sd, void* vd, void* stream);

/* Iterated Taylor linearisation (Sec. 4.4): xbar^(0) = xbar0 (NULL: m0 of each
 * segment at every state), then n_iter times: linearise about xbar, solve
 * with map_smooth, xbar <- xs.  xbar_buf (tiled [nx] per state) is caller scratch that
 * holds the linearisation point of the last solve on return (p->xbar is
 * ignored).  loglik, obj and the gradients refer to that last linear problem
 * with its linearisation point held fixed. */
map_status map_iterated_nonlinear(const map_problem* p, int32_t n_iter, const void* xbar0,
                                  void* xbar_buf, void* S, void* v, void* xs, void* Ps,
                                  double* loglik, double* obj, double* g_loglik, double* g_obj,
                                  void* ws, size_t ws_bytes, void* stream);

/* Adjoint from saved filter moments.  Elements are recomputed from the
 * inputs (never stored).  With ckpt = NULL the filter's S and v planes
 * (map_filter_scan or map_smooth) are read.  With a filter checkpoint of
 * map_smooth_checkpointed on the same problem (ckpt, ckpt_bytes >=
 * map_checkpoint_bytes), S and v are OUTPUTS instead: the filter planes are
 * rebuilt from the checkpoint's block carries (one more filter up-sweep
 * without its cross-block step, and the filter fix-up fused with the
 * trajectory maps) and written there, distinct from each other and from every
 * other buffer.  The rebuilt planes equal the forward call's, and x*, P^s and
 * the gradients equal map_smooth's on the same schedule (the call with saved
 * planes agrees with them to rounding: with FP32 storage its trajectory maps
 * start from the rounded planes).  Reverse-scans the same elements to rebuild xs and
 * Ps (written to the caller's buffers) and accumulates, per segment
 * ([n_seg][n_theta] double, each optional):
 *   g_loglik, g_obj  d loglik / d theta (Fisher identity) and d obj / d theta
 *                    (envelope theorem), as map_smooth;
 *   g_xs_theta       with g_xs (tiled [nx] per state, the cotangent dl/dx* of
 *                    a scalar l of the trajectory): dl/dtheta by the implicit
 *                    function theorem.  x* is the stationary point of the
 *                    discretised objective (Sec. 2.1 eq. OM, Sec. 4.4), so
 *                    dl/dtheta = -mu^T d(grad_x M_d)/dtheta with mu = H^{-1} g
 *                    (H the objective's Hessian in x): mu solves the same
 *                    scan problem with every element's b set to 0 and eta to
 *                    g (three more passes), then the per-step cotangents of
 *                    A, b, C, R are reduced per segment.  mu (out, tiled [nx]
 *                    per state) receives mu, vmu (out, tiled [nx] per state)
 *                    the adjoint problem's second filter plane; both must be
 *                    distinct from xs, S, v and g_xs.
 *   g_elems          (debug output, or NULL) the per-step cotangents that
 *                    the two gradients above are reduced from: at the state
 *                    a step ends at (not at a segment's first state),
 *                    tiled [2 E] doubles per state, E = nx*nx + nx +
 *                    nx(nx+1)/2 + ny(ny+1)/2: d loglik / d(A, b, C, R) of
 *                    the step's element (A = I - dt F, b = -dt c, C = dt Q,
 *                    R the measurement density), then d obj / d(A, b, C, R);
 *                    A row-major, C and R as the lower triangle (row order)
 *                    of the gradient with respect to the full symmetric
 *                    matrix.  Distinct from every other buffer.
 * For nonlinear models every gradient holds the linearisation point
 * p->xbar fixed.  At least one of g_loglik, g_obj, g_xs, g_elems must be
 * given. */
map_status map_backward(const map_problem* p, void* S, void* v, void* xs, void* Ps,
                        double* obj, double* g_loglik, double* g_obj, const void* g_xs, void* mu,
                        void* vmu, double* g_xs_theta, double* g_elems, const void* ckpt,
                        size_t ckpt_bytes, void* ws, size_t ws_bytes, void* stream);

/* Schedule autotuner for the batched segmented scan.  Times the fused step
 * (map_smooth with every output, gradients for parametric models) at the
 * flat schedules chunk = 32, 16, 8 and 4 and, for 64 or more segments, the
 * segment-local MAP_SCHED_SEGMENT_WAVE, on the caller's inputs (p->chunk is ignored; p->xbar must be set for nonlinear
 * models) and records the fastest for this shape -- model, dimensions,
 * dtype, floor(log2 n_states), floor(log2 n_seg) -- so that later calls with
 * chunk = 0 use it.  ws: a workspace of map_workspace_bytes(p with chunk 0)
 * bytes, initialised.  cache_path (host string or NULL): a text file of
 * "key chunk ms" lines read first (a recorded shape is not timed again) and
 * appended to.  Allocates and frees its temporary outputs; synchronises
 * `stream`.  *chunk_out receives the chosen chunk. */
map_status map_autotune(const map_problem* p, void* ws, size_t ws_bytes, const char* cache_path,
                        int32_t* chunk_out, void* stream);

/* Exact element dynamics for a time-invariant linear-affine model (element
 * variant; only the element build changes).  For dx/dt = F x + c + L w
 * (w white with spectral density W) the exact transition over a step dt,
 * x_k = e^{F dt} x_{k-1} + u + N(0, Qd) (Van Loan), read backwards as
 * x_{k-1} = A x_k + b + N(0, C) with A = e^{-F dt}, b = -A u, C = A Qd A^T, is
 * returned as the terms of the library's one-step element (Sec. 4.2, one
 * explicit-Euler step of eq. backwardLQT: A = I - dt F~, b = -dt c~,
 * C = dt L~ W~ L~^T):
 *   F_out [nx*nx] = (I - A) / dt,  c_out [nx] = -b / dt,  L_out [nx*nx] with
 *   L_out L_out^T = C / dt and W~ = I.
 * A MAP_MODEL_LINEAR problem with F = F_out, c = c_out, L = L_out, W = I (nw = nx)
 * and the model's H, r, R then solves the exactly discretised dynamics (the
 * measurement term stays dt H^T R^{-1} H at the step's end).  Host arrays,
 * row-major doubles; c may be NULL (no offset).  Host-only; launches nothing.
 * Errors: dimensions outside [1, 8], dt <= 0, NULL or non-finite inputs. */
map_status map_lti_exact_terms(int32_t nx, int32_t nw, const double* F, const double* c,
                               const double* L, const double* W, double dt, double* F_out,
                               double* c_out, double* L_out);

/* The schedule (states per lane: 4, 8, 16 or 32) the scan entry points use for
 * this problem: p->chunk if set, else the choice map_autotune recorded for
 * its shape, else the library's heuristic.  Host-only; launches nothing. */
map_status map_schedule(const map_problem* p, int32_t* chunk_out);

/* Measurement hook (no effect on results).  map_profile_enable(n) creates n
 * pairs of HIP events (0 disables and releases them); while enabled, each
 * kernel the library launches is bracketed by one pair recorded on its
 * stream, until the n pairs are used up (map_profile_reset rewinds).
 * map_profile_read waits for the recorded events and returns, for one kernel
 * kind, the number of timed launches and their summed duration in ms.
 * Kinds: 0 filter up-sweep, 1 filter fix-up, 2 fused filter fix-up +
 * trajectory up-sweep, 3 trajectory up-sweep from stored S, v, 4 trajectory
 * fix-up, 5 trajectory fix-up with adjoint, 6 auxiliary (zeroing), 7 filter
 * fix-up + backward-filter up-sweep (two-filter), 8 two-filter combination,
 * 9 the adjoint problem's passes (implicit-function VJP), 10 its per-step
 * cotangent reduction, 11 the segment-local fused step, 12 dense output of
 * sub-stepped blocks. */
map_status map_profile_enable(int32_t capacity);
map_status map_profile_reset(void);
map_status map_profile_read(int32_t kind, int64_t* count, double* total_ms);

const char* map_last_error(void);
int32_t map_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MAPSCAN_H */
