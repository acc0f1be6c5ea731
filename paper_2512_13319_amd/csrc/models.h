// Model functors: the per-step terms of the linear-affine problem solved at
// one Gauss--Newton iteration (Sec. 2.4 eq. linear-statespace, linearised as
// in Sec. 4.4), and the parameter cotangents needed by the adjoint.
//
// A step k covers [t_{k-1}, t_k]; every term is evaluated at the right end,
// i.e. at the nominal state xbar_k of the state the step leads to.  From the
// terms the scan element of the step is one explicit-Euler step of the
// element ODE (Sec. 4.2, eq. backwardLQT, with the sign of the Q J term in
// the A equation read as +) from its boundary value (I, 0, 0, 0, 0):
//
//   A = I - dt F,  b = -dt c,  C = dt L W L^T = V V^T,
//   J = dt H^T R^{-1} H,  eta = dt H^T R^{-1} (y - r).
//
// Models hand out V = sqrt(dt) L chol(W) instead of C, so that every solve
// against a fresh element is a small SPD system.
#pragma once
#include "linalg.h"

namespace ms {

template <typename T, int NX, int NY, int NW>
struct Step {
  T dt;
  T F[NX][NX];
  T c[NX];
  T V[NX][NW];     // C = V V^T = dt L W L^T
  T H[NY][NX];
  T r[NY];
  T R[NY][NY];     // measurement spectral density
  T Rinv[NY][NY];
};

// Device-side view of the problem (all pointers device memory).
template <typename T>
struct Prob {
  int64_t n_seg, n_steps, n_states;
  const int64_t* seg_off;  // [n_seg+1] step offsets
  const T* dt;             // [n_steps] or one scalar (dt_stride 0)
  int64_t dt_stride;
  const T* y;              // [ny][n_steps]
  const T* m0;             // [n_seg][nx] (stride 0: shared)
  int64_t m0_stride;
  const T* P0;             // [n_seg][nx][nx] row-major (stride 0: shared)
  int64_t P0_stride;
  const T* theta;          // [n_seg][n_theta] (stride 0: shared)
  int64_t th_stride;
  const T* xbar;           // [nx][n_states] linearisation states (nonlinear models)
  const T* gx;             // [nx][n_states] cotangent of x* (the problem Ift<M> only)
  int om_div;              // MAP_OM_DIVERGENCE: the divergence term of eq. OM is included
  int n_sub;               // Euler substeps per grid step (Blocked<M> only; y holds ny * n_sub per state)
  int ny_in, nw_in;        // the problem's ny, nw (ModelLinearPadded pads them to NX)
  // general linear model: row-major per-step matrices, stride 0 = shared by all steps
  const T *F, *c, *L, *W, *H, *r, *R;
  int64_t sF, sc, sL, sW, sH, sr, sR;
};

// ------------------------------------------------------------------ constant velocity
// theta = (gamma, q, r): F = [[0, I], [0, -gamma I]], L = [0; I], W = q I,
// H = [I, 0], R = r I.  nx = 2D.  With gamma = 0 and D = 2 this is the
// Wiener velocity model of the paper's linear experiment (Sec. 5.1).
template <int D>
struct ModelCV {
  static constexpr int NX = 2 * D, NY = D, NW = D, NTH = 3;
  static constexpr bool kNonlinear = false;
  static constexpr bool kAdjoint = true;
  static constexpr bool kIft = false;  // see Ift below
  static constexpr bool kBlocked = false;  // see Blocked below
  static constexpr bool kPadded = false;   // see ModelLinearPadded below
  // wavefronts per SIMD asked of the compiler for the filter passes (2: fits
  // 256 registers a lane without spilling; see the kernels)
  static constexpr int kWaves = 2;
  static constexpr int kAngle = -1;  // no angular measurement component

  template <typename T>
  static MS_DEV void terms(const T* th, const T (&)[NX], T dt, Step<T, NX, NY, NW>& s) {
    const T g = th[0], q = th[1], rr = th[2];
    s.dt = dt;
    mzero(s.F);
    mzero(s.V);
    mzero(s.H);
    mzero(s.R);
    mzero(s.Rinv);
    const T sv = sqrt_(dt * q);
    const T ri = rcp(rr);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      s.F[i][D + i] = T(1);
      s.F[D + i][D + i] = -g;
      s.V[D + i][i] = sv;
      s.H[i][i] = T(1);
      s.R[i][i] = rr;
      s.Rinv[i][i] = ri;
      s.r[i] = T(0);
    }
#pragma unroll
    for (int i = 0; i < NX; ++i) s.c[i] = T(0);
  }

  // divergence of the drift (eq. OM): trace F = -D gamma, state independent
  static constexpr bool kDivNewton = false;
  template <typename T>
  static MS_DEV T divergence(const T* th, const T (&)[NX]) {
    return -T(D) * th[0];
  }

  // theta-cotangent of the element parameters: A = I - dt F(theta),
  // b = -dt c, C = dt q L L^T, R = r I.
  template <typename T>
  static MS_DEV void vjp(const T* th, const T (&)[NX], T dt, const T (&GA)[NX][NX],
                         const T (&)[NX], const T (&GC)[NX][NX], const T (&GR)[NY][NY],
                         double (&out)[NTH]) {
    (void)th;
    double a = 0.0, b = 0.0, c = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      a += double(GA[D + i][D + i]);
      b += double(GC[D + i][D + i]);
      c += double(GR[i][i]);
    }
    out[0] += double(dt) * a;  // dA/dgamma = dt on the velocity block
    out[1] += double(dt) * b;  // dC/dq = dt L L^T
    out[2] += c;               // dR/dr = I
  }
};

// ------------------------------------------------------------------ Van der Pol
// theta = (mu, q, r): f = (x2, mu (1 - x1^2) x2 - x1), L = I, W = q I, h = x1, R = r.
struct ModelVdP {
  static constexpr int NX = 2, NY = 1, NW = 2, NTH = 3;
  static constexpr bool kNonlinear = true;
  static constexpr bool kAdjoint = true;
  static constexpr bool kIft = false;  // see Ift below
  static constexpr bool kBlocked = false;  // see Blocked below
  static constexpr bool kPadded = false;   // see ModelLinearPadded below
  // wavefronts per SIMD asked of the compiler for the filter passes (2: fits
  // 256 registers a lane without spilling; see the kernels)
  static constexpr int kWaves = 2;
  static constexpr int kAngle = -1;

  template <typename T>
  static MS_DEV void terms(const T* th, const T (&x)[NX], T dt, Step<T, NX, NY, NW>& s) {
    const T mu = th[0], q = th[1], rr = th[2];
    const T x1 = x[0], x2 = x[1];
    s.dt = dt;
    s.F[0][0] = T(0);
    s.F[0][1] = T(1);
    s.F[1][0] = T(-2) * mu * x1 * x2 - T(1);
    s.F[1][1] = mu * (T(1) - x1 * x1);
    // c = f(x) - F x
    const T f1 = mu * (T(1) - x1 * x1) * x2 - x1;
    s.c[0] = x2 - x2;
    s.c[1] = f1 - (s.F[1][0] * x1 + s.F[1][1] * x2);
    const T sv = sqrt_(dt * q);
    s.V[0][0] = sv;
    s.V[0][1] = T(0);
    s.V[1][0] = T(0);
    s.V[1][1] = sv;
    s.H[0][0] = T(1);
    s.H[0][1] = T(0);
    s.r[0] = T(0);
    s.R[0][0] = rr;
    s.Rinv[0][0] = rcp(rr);
  }

  // divergence of the drift (eq. OM): d f2 / d x2 = mu (1 - x1^2), state
  // dependent.  Newton treatment of the term 1/2 dt div f(x_k) of the
  // discretised objective: its second-order expansion about xbar, added to
  // the step's element as J += 1/2 dt Hess, eta -= 1/2 dt (grad - Hess xbar)
  // with grad = (-2 mu x1, 0), Hess = diag(-2 mu, 0); the term is quadratic
  // in x, so the expansion is exact (eta is unchanged).
  static constexpr bool kDivNewton = true;
  template <typename T>
  static MS_DEV T divergence(const T* th, const T (&x)[NX]) {
    return th[0] * (T(1) - x[0] * x[0]);
  }
  template <typename T>
  static MS_DEV void div_newton(const T* th, const T (&)[NX], T dt, T (&J)[NX][NX], T (&)[NX]) {
    J[0][0] -= dt * th[0];
  }

  template <typename T>
  static MS_DEV void vjp(const T* th, const T (&x)[NX], T dt, const T (&GA)[NX][NX],
                         const T (&Gb)[NX], const T (&GC)[NX][NX], const T (&GR)[NY][NY],
                         double (&out)[NTH]) {
    (void)th;
    const double x1 = x[0], x2 = x[1], h = dt;
    // dF/dmu = [[0, 0], [-2 x1 x2, 1 - x1^2]]; dA = -dt dF
    // dc/dmu = df/dmu - dF/dmu x = (0, 2 x1^2 x2); db = -dt dc
    out[0] += -h * (double(GA[1][0]) * (-2.0 * x1 * x2) + double(GA[1][1]) * (1.0 - x1 * x1))
              - h * double(Gb[1]) * (2.0 * x1 * x1 * x2);
    out[1] += h * (double(GC[0][0]) + double(GC[1][1]));
    out[2] += double(GR[0][0]);
  }
};

// ------------------------------------------------------------------ Lorenz-63
// theta = (sigma, rho, beta, q, r): f = (sigma (x2 - x1), x1 (rho - x3) - x2,
// x1 x2 - beta x3), L = I, W = q I, h = x, R = r I.
struct ModelLorenz63 {
  static constexpr int NX = 3, NY = 3, NW = 3, NTH = 5;
  static constexpr bool kNonlinear = true;
  static constexpr bool kAdjoint = true;
  static constexpr bool kIft = false;  // see Ift below
  static constexpr bool kBlocked = false;  // see Blocked below
  static constexpr bool kPadded = false;   // see ModelLinearPadded below
  // wavefronts per SIMD asked of the compiler for the filter passes (2: fits
  // 256 registers a lane without spilling; see the kernels)
  static constexpr int kWaves = 1;
  static constexpr int kAngle = -1;

  template <typename T>
  static MS_DEV void terms(const T* th, const T (&x)[NX], T dt, Step<T, NX, NY, NW>& s) {
    const T sg = th[0], rho = th[1], be = th[2], q = th[3], rr = th[4];
    const T x1 = x[0], x2 = x[1], x3 = x[2];
    s.dt = dt;
    s.F[0][0] = -sg; s.F[0][1] = sg;   s.F[0][2] = T(0);
    s.F[1][0] = rho - x3; s.F[1][1] = T(-1); s.F[1][2] = -x1;
    s.F[2][0] = x2;  s.F[2][1] = x1;   s.F[2][2] = -be;
    // c = f(x) - F x: only the bilinear terms survive
    s.c[0] = T(0);
    s.c[1] = x1 * x3;   // x1 (rho - x3) - x2 - [(rho - x3) x1 - x2 - x1 x3]
    s.c[2] = -x1 * x2;  // x1 x2 - be x3 - [x2 x1 + x1 x2 - be x3]
    const T sv = sqrt_(dt * q);
    const T ri = rcp(rr);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        s.V[i][j] = i == j ? sv : T(0);
        s.H[i][j] = i == j ? T(1) : T(0);
        s.R[i][j] = i == j ? rr : T(0);
        s.Rinv[i][j] = i == j ? ri : T(0);
      }
      s.r[i] = T(0);
    }
  }

  // divergence of the drift (eq. OM): -(sigma + 1 + beta), state independent
  static constexpr bool kDivNewton = false;
  template <typename T>
  static MS_DEV T divergence(const T* th, const T (&)[NX]) {
    return -(th[0] + T(1) + th[2]);
  }

  template <typename T>
  static MS_DEV void vjp(const T* th, const T (&x)[NX], T dt, const T (&GA)[NX][NX],
                         const T (&)[NX], const T (&GC)[NX][NX], const T (&GR)[NY][NY],
                         double (&out)[NTH]) {
    (void)th;
    (void)x;
    const double h = dt;
    // dA = -dt dF; dF/dsigma = [[-1, 1, 0], 0, 0], dF/drho = e_1 e_0^T, dF/dbeta = -e_2 e_2^T.
    // c carries no theta dependence (f is linear in theta along the linear terms).
    out[0] += -h * (-double(GA[0][0]) + double(GA[0][1]));
    out[1] += -h * double(GA[1][0]);
    out[2] += h * double(GA[2][2]);
    out[3] += h * (double(GC[0][0]) + double(GC[1][1]) + double(GC[2][2]));
    out[4] += double(GR[0][0]) + double(GR[1][1]) + double(GR[2][2]);
  }
};

// ------------------------------------------------------------------ general linear
// Dense F, c, L, W, H, r, R read per step (or shared when the stride is 0).
// Forward path only (no parameter adjoint).
template <int NX_, int NY_, int NW_>
struct ModelLinear {
  static constexpr int NX = NX_, NY = NY_, NW = NW_, NTH = 0;
  static constexpr bool kNonlinear = false;
  static constexpr bool kAdjoint = false;
  static constexpr bool kIft = false;  // see Ift below
  static constexpr bool kBlocked = false;  // see Blocked below
  static constexpr bool kPadded = false;   // see ModelLinearPadded below
  // wavefronts per SIMD asked of the compiler for the filter passes (2: fits
  // 256 registers a lane without spilling; see the kernels)
  static constexpr int kWaves = 1;
  static constexpr int kAngle = -1;
  static constexpr bool kDivNewton = false;  // divergence trace F of the step (Cursor)
};

// General linear model of NX states whose measurement and noise dimensions
// (ny, nw <= NX, Prob::ny_in, nw_in) are padded to NX when the terms are read:
// H gets zero rows with r = 0 and R = I there, L zero columns with W = I
// there.  The padding adds nothing to J, eta, C or the objective; its constant
// in the prediction-error likelihood is removed (Cursor::loglik_pad).  One
// instantiation per NX serves every (ny, nw) without one of its own.
template <int NX_>
struct ModelLinearPadded : ModelLinear<NX_, NX_, NX_> {
  static constexpr bool kPadded = true;
};

// ------------------------------------------------------------------ coordinated turn
// The nonlinear model of Sec. 5.2: x = (xi, zeta, dxi, dzeta, omega),
// f = (dxi, dzeta, -omega dzeta, omega dxi, 0), L = [[0,0,0],[0,0,0],[sv,0,0],
// [0,sv,0],[0,0,sw]], W = I, h = (sqrt(xi^2 + zeta^2), atan2(zeta, xi)) (the
// paper's arctan(zeta / xi), continued to every direction), R = diag(r1, r2);
// theta = (sv, sw, r1, r2).  Taylor terms at xbar:
//   F rows 2, 3: (0, 0, 0, -omega, -dzeta), (0, 0, omega, 0, dxi);  c = (0, 0, omega dzeta, -omega dxi, 0)
//   H = [[xi/rho, zeta/rho, 0, 0, 0], [-zeta/rho^2, xi/rho^2, 0, 0, 0]],  r = (0, atan2(zeta, xi))
// (H xbar reproduces the range exactly and has no bearing part).  Measurement
// component kAngle is a bearing: its residual y - r is taken modulo 2 pi into
// [-pi, pi) (done where the step's measurement is read, see Cursor::terms).
// Q = L L^T is singular; C = dt Q keeps the factor V = sqrt(dt) L.
struct ModelCT {
  static constexpr int NX = 5, NY = 2, NW = 3, NTH = 4;
  static constexpr bool kNonlinear = true;
  static constexpr bool kAdjoint = true;
  static constexpr bool kIft = false;  // see Ift below
  static constexpr bool kBlocked = false;  // see Blocked below
  static constexpr bool kPadded = false;   // see ModelLinearPadded below
  // wavefronts per SIMD asked of the compiler for the filter passes (2: fits
  // 256 registers a lane without spilling; see the kernels)
  static constexpr int kWaves = 1;
  static constexpr int kAngle = 1;
  // divergence of the drift (eq. OM): zero (the turn rotates the velocity)
  static constexpr bool kDivNewton = false;
  template <typename T>
  static MS_DEV T divergence(const T*, const T (&)[NX]) {
    return T(0);
  }

  template <typename T>
  static MS_DEV void terms(const T* th, const T (&x)[NX], T dt, Step<T, NX, NY, NW>& s) {
    const T sv = th[0], sw = th[1], r1 = th[2], r2 = th[3];
    const T xi = x[0], ze = x[1], dxi = x[2], dze = x[3], om = x[4];
    s.dt = dt;
    mzero(s.F);
    s.F[0][2] = T(1);
    s.F[1][3] = T(1);
    s.F[2][3] = -om;
    s.F[2][4] = -dze;
    s.F[3][2] = om;
    s.F[3][4] = dxi;
    s.c[0] = T(0);
    s.c[1] = T(0);
    s.c[2] = om * dze;
    s.c[3] = -om * dxi;
    s.c[4] = T(0);
    const T sd = sqrt_(dt);
    mzero(s.V);
    s.V[2][0] = sd * sv;
    s.V[3][1] = sd * sv;
    s.V[4][2] = sd * sw;
    const T rho2 = xi * xi + ze * ze;
    T rho, rrho;
    sqrt_rsqrt(rho2, rho, rrho);
    const T irho2 = rrho * rrho;
    mzero(s.H);
    s.H[0][0] = xi * rrho;
    s.H[0][1] = ze * rrho;
    s.H[1][0] = -ze * irho2;
    s.H[1][1] = xi * irho2;
    s.r[0] = T(0);
    s.r[1] = atan2_(ze, xi);
    s.R[0][0] = r1;
    s.R[0][1] = T(0);
    s.R[1][0] = T(0);
    s.R[1][1] = r2;
    s.Rinv[0][0] = rcp(r1);
    s.Rinv[0][1] = T(0);
    s.Rinv[1][0] = T(0);
    s.Rinv[1][1] = rcp(r2);
  }

  // theta-cotangent: C = dt diag(0, 0, sv^2, sv^2, sw^2), R = diag(r1, r2); A, b
  // and the measurement terms do not depend on theta.
  template <typename T>
  static MS_DEV void vjp(const T* th, const T (&)[NX], T dt, const T (&)[NX][NX], const T (&)[NX],
                         const T (&GC)[NX][NX], const T (&GR)[NY][NY], double (&out)[NTH]) {
    const double h = dt;
    out[0] += h * 2.0 * double(th[0]) * (double(GC[2][2]) + double(GC[3][3]));
    out[1] += h * 2.0 * double(th[1]) * double(GC[4][4]);
    out[2] += double(GR[0][0]);
    out[3] += double(GR[1][1]);
  }
};

// ------------------------------------------------------------------ adjoint problem
// The problem whose minimiser is mu = H^{-1} g, H the Hessian of the discretised
// objective and g a cotangent of the trajectory x* (implicit-function VJP, see
// k_ift_grad): the quadratic part of the objective is unchanged (same A, C, J
// in every element) and its linear part is -g^T x, i.e. every fresh element has
// b = 0 and eta = g_k, and the prior element eta = g_0 (its J stays P0^{-1}).
// The scan kernels read g through Prob::gx when instantiated with Ift<M>.
template <class M>
struct Ift : M {
  static constexpr bool kIft = true;
  static constexpr int kWaves = 1;  // its passes carry more state (would spill)
};

// ------------------------------------------------------------------ sub-stepped blocks
// A grid step [t_{k-1}, t_k] taken as a block of n_sub explicit-Euler substeps
// of the element ODE (Sec. 4.2, eq. backwardLQT; the paper's T blocks of n
// Euler substeps, Sec. 5.1) instead of one: see Cursor::block_fresh.  The
// model's terms are held over the block (linearised at the block's right end
// for nonlinear models).  A block's C has full rank, so the wrapper's noise
// factor is NX wide (the base model's V, padded with zero columns, carries
// Q = V V^T / dt).  Filter, smoother and dense output only (no adjoint, no
// log-likelihood or objective).
template <class M>
struct Blocked : M {
  static constexpr int NW = M::NX;
  static constexpr bool kAdjoint = false;
  static constexpr bool kBlocked = true;
  static constexpr int kWaves = 1;  // the block state would spill at 256 registers

  template <typename T>
  static MS_DEV void terms(const T* th, const T (&x)[M::NX], T dt,
                           Step<T, M::NX, M::NY, M::NX>& s) {
    Step<T, M::NX, M::NY, M::NW> b;
    M::terms(th, x, dt, b);
    s.dt = b.dt;
#pragma unroll
    for (int a = 0; a < M::NX; ++a) {
      s.c[a] = b.c[a];
#pragma unroll
      for (int q = 0; q < M::NX; ++q) {
        s.F[a][q] = b.F[a][q];
        s.V[a][q] = q < M::NW ? b.V[a][q] : T(0);
      }
    }
#pragma unroll
    for (int a = 0; a < M::NY; ++a) {
      s.r[a] = b.r[a];
#pragma unroll
      for (int q = 0; q < M::NX; ++q) s.H[a][q] = b.H[a][q];
#pragma unroll
      for (int q = 0; q < M::NY; ++q) {
        s.R[a][q] = b.R[a][q];
        s.Rinv[a][q] = b.Rinv[a][q];
      }
    }
  }
};

}  // namespace ms
