/*
 * Sequential CPU oracle, plain C, FP64.  TEST INFRASTRUCTURE ONLY: it is used by
 * the tests, by the package's smoke check and by the benchmark's CPU-baseline
 * leg, never by the product path, and it shares no code with the GPU library.
 *
 * What it computes is the plain definition of the discretised MAP problem of
 * the linear-affine model (Sec. 2.4, eq. linear-statespace), written as the
 * textbook covariance-form Kalman filter plus the discrete Rauch--Tung--
 * Striebel smoother that the paper identifies its scans with (Sec. 2.5; the
 * parallel RTS smoother of Sec. 4.3).  The discretisation of one grid step
 * [t_{k-1}, t_k] is the one that makes a single explicit-Euler step of the
 * element ODE (Sec. 4.2, eq. backwardLQT, taken in reversed time) exact:
 *
 *   x_k - x_{k-1} = dt_k (F_k x_k + c_k) + w_k,   w_k ~ N(0, dt_k Q_k),  Q = L W L^T
 *   y_k = H_k x_k + r_k + v_k,                    v_k ~ N(0, R_k / dt_k)
 *   x_0 ~ N(m0, P0)
 *
 * i.e. an implicit-Euler step of the SDE (drift and measurement taken at the
 * step's right end, R a spectral density as in Sec. 2.1).  Written forward:
 * x_k = Phi_k (x_{k-1} + dt c + w) with Phi_k = (I - dt F_k)^{-1}.
 *
 * oracle_two_filter (at the end of this file) recomputes the smoothed moments
 * the second way the paper gives (Sec. 4.3, eq. twofilter) from the filter
 * moments and the conditional value functions of the later steps.
 *
 * Outputs per segment: filter moments m_k, P_k (k = 0..T, k = 0 is the prior),
 * smoothed moments xs_k, Ps_k, the log marginal likelihood by the prediction
 * error decomposition, and the discretised Onsager--Machlup objective (Sec. 2.1,
 * eq. OM, without the divergence term) evaluated at xs.  For singular Q the
 * transition cost is the driving-noise energy 1/2 u^T (dt W)^{-1} u with
 * u = L^+ D, D the step residual (the pseudo-inverse relaxation the paper
 * mentions below eq. OM); L must have full column rank.
 *
 * Layouts (this file's own): per-step model arrays are row-major matrices,
 * element (k, s) at base + k*stride_step + s*stride_seg (either may be 0);
 * y is [n_steps][ny]; outputs are [n_states][nx] and [n_states][nx*nx] with
 * segment s's states at seg_off[s] + s ... seg_off[s+1] + s.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MX 8

/* Running sum with Neumaier's compensation: the per-segment log-likelihood
 * and objective are sums of one term per step; over 2^20 steps a plain
 * running sum carries a rounding error of order sqrt(T) eps |sum|, which
 * changes erratically with the inputs.  The compensated sum stays within a
 * few eps of the exact sum of the computed terms. */
typedef struct { double s, c; } ksum;
static void ksum_add(ksum *k, double x) {
  const double t = k->s + x;
  if (fabs(k->s) >= fabs(x)) k->c += (k->s - t) + x;
  else k->c += (x - t) + k->s;
  k->s = t;
}
static double ksum_value(const ksum *k) { return k->s + k->c; }

/* ---------- small dense helpers (row-major, n <= 8) ---------- */

static void mm(int n, int m, int p, const double *a, const double *b, double *c) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < p; ++j) {
      double s = 0.0;
      for (int l = 0; l < m; ++l) s += a[i * m + l] * b[l * p + j];
      c[i * p + j] = s;
    }
}

/* c = a * b^T, a [n][m], b [p][m] */
static void mmt(int n, int m, int p, const double *a, const double *b, double *c) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < p; ++j) {
      double s = 0.0;
      for (int l = 0; l < m; ++l) s += a[i * m + l] * b[j * m + l];
      c[i * p + j] = s;
    }
}

static void mv(int n, int m, const double *a, const double *x, double *y) {
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int l = 0; l < m; ++l) s += a[i * m + l] * x[l];
    y[i] = s;
  }
}

static void symmetrize(int n, double *a) {
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      double s = 0.5 * (a[i * n + j] + a[j * n + i]);
      a[i * n + j] = s;
      a[j * n + i] = s;
    }
}

/* Gauss-Jordan inverse with partial pivoting; returns 0 if singular. */
static int inv(int n, const double *a, double *out) {
  double w[MX * 2 * MX];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < 2 * n; ++j)
      w[i * 2 * n + j] = j < n ? a[i * n + j] : (j - n == i ? 1.0 : 0.0);
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (fabs(w[i * 2 * n + k]) > fabs(w[p * 2 * n + k])) p = i;
    if (w[p * 2 * n + k] == 0.0) return 0;
    if (p != k)
      for (int j = 0; j < 2 * n; ++j) {
        double t = w[k * 2 * n + j];
        w[k * 2 * n + j] = w[p * 2 * n + j];
        w[p * 2 * n + j] = t;
      }
    double d = 1.0 / w[k * 2 * n + k];
    for (int j = 0; j < 2 * n; ++j) w[k * 2 * n + j] *= d;
    for (int i = 0; i < n; ++i)
      if (i != k) {
        double f = w[i * 2 * n + k];
        if (f != 0.0)
          for (int j = 0; j < 2 * n; ++j) w[i * 2 * n + j] -= f * w[k * 2 * n + j];
      }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) out[i * n + j] = w[i * 2 * n + n + j];
  return 1;
}

/* Cholesky a = l l^T (lower); returns 0 if not positive definite. */
static int chol(int n, const double *a, double *l) {
  memset(l, 0, sizeof(double) * n * n);
  for (int j = 0; j < n; ++j) {
    double s = a[j * n + j];
    for (int k = 0; k < j; ++k) s -= l[j * n + k] * l[j * n + k];
    if (!(s > 0.0)) return 0;
    double d = sqrt(s);
    l[j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double t = a[i * n + j];
      for (int k = 0; k < j; ++k) t -= l[i * n + k] * l[j * n + k];
      l[i * n + j] = t / d;
    }
  }
  return 1;
}

/* solve (l l^T) x = b in place, b has nrhs columns stored row-major [n][nrhs] */
static void chol_solve(int n, int nrhs, const double *l, double *b) {
  for (int c = 0; c < nrhs; ++c) {
    for (int i = 0; i < n; ++i) {
      double s = b[i * nrhs + c];
      for (int k = 0; k < i; ++k) s -= l[i * n + k] * b[k * nrhs + c];
      b[i * nrhs + c] = s / l[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = b[i * nrhs + c];
      for (int k = i + 1; k < n; ++k) s -= l[k * n + i] * b[k * nrhs + c];
      b[i * nrhs + c] = s / l[i * n + i];
    }
  }
}

typedef struct {
  const double *p;
  long step, seg;
} arr;

static const double *at(arr a, long k, long s) { return a.p + k * a.step + s * a.seg; }

/* Per-step model: F, c, L, W, H, r, R, dt (see header).  Returns number of
 * segments processed, or -(s+1) if segment s hit a non-positive-definite
 * covariance. */
long oracle_smooth(int nx, int ny, int nw, long n_seg, const long *seg_off,
                   const double *F, long F_step, long F_seg,
                   const double *c, long c_step, long c_seg,
                   const double *L, long L_step, long L_seg,
                   const double *W, long W_step, long W_seg,
                   const double *H, long H_step, long H_seg,
                   const double *r, long r_step, long r_seg,
                   const double *R, long R_step, long R_seg,
                   const double *dt, const double *y,
                   const double *m0, long m0_seg, const double *P0, long P0_seg,
                   double *m_out, double *P_out, double *xs_out, double *Ps_out,
                   double *loglik_out, double *mstar_out) {
  arr aF = {F, F_step, F_seg}, ac = {c, c_step, c_seg}, aL = {L, L_step, L_seg},
      aW = {W, W_step, W_seg}, aH = {H, H_step, H_seg}, ar = {r, r_step, r_seg},
      aR = {R, R_step, R_seg};
  const int n2 = nx * nx;
  long maxT = 0;
  for (long s = 0; s < n_seg; ++s)
    if (seg_off[s + 1] - seg_off[s] > maxT) maxT = seg_off[s + 1] - seg_off[s];
  double *mp = (double *)malloc(sizeof(double) * (maxT + 1) * nx);
  double *Pp = (double *)malloc(sizeof(double) * (maxT + 1) * n2);
  const double LOG2PI = log(2.0 * M_PI);

  for (long s = 0; s < n_seg; ++s) {
    const long k0 = seg_off[s], T = seg_off[s + 1] - seg_off[s];
    const long x0 = k0 + s; /* state offset */
    double *m = m_out + x0 * nx, *P = P_out + x0 * n2;
    double *xs = xs_out + x0 * nx, *Ps = Ps_out + x0 * n2;
    memcpy(m, m0 + s * m0_seg, sizeof(double) * nx);
    memcpy(P, P0 + s * P0_seg, sizeof(double) * n2);
    ksum ll = {0.0, 0.0};

    /* ---- forward: covariance-form Kalman filter ---- */
    for (long j = 1; j <= T; ++j) {
      const long k = k0 + j - 1; /* global step index */
      const double h = dt[k];
      double A[MX * MX], Phi[MX * MX], Q[MX * MX], LW[MX * MX], t1[MX * MX], t2[MX * MX];
      const double *Fk = at(aF, k, s), *ck = at(ac, k, s), *Lk = at(aL, k, s),
                   *Wk = at(aW, k, s), *Hk = at(aH, k, s), *rk = at(ar, k, s),
                   *Rk = at(aR, k, s);
      for (int i = 0; i < n2; ++i) A[i] = -h * Fk[i];
      for (int i = 0; i < nx; ++i) A[i * nx + i] += 1.0;
      if (!inv(nx, A, Phi)) { free(mp); free(Pp); return -(s + 1); }
      mm(nx, nw, nw, Lk, Wk, LW);
      mmt(nx, nw, nx, LW, Lk, Q);
      /* predict: m- = Phi (m + dt c), P- = Phi (P + dt Q) Phi^T */
      double u[MX];
      for (int i = 0; i < nx; ++i) u[i] = m[(j - 1) * nx + i] + h * ck[i];
      double *mpj = mp + j * nx, *Ppj = Pp + j * n2;
      mv(nx, nx, Phi, u, mpj);
      for (int i = 0; i < n2; ++i) t1[i] = P[(j - 1) * n2 + i] + h * Q[i];
      mm(nx, nx, nx, Phi, t1, t2);
      mmt(nx, nx, nx, t2, Phi, Ppj);
      symmetrize(nx, Ppj);
      /* update with y_k, covariance R/dt */
      double HP[MX * MX], Sg[MX * MX], Ls[MX * MX], e[MX], K[MX * MX];
      mm(ny, nx, nx, Hk, Ppj, HP);
      mmt(ny, nx, ny, HP, Hk, Sg);
      for (int i = 0; i < ny * ny; ++i) Sg[i] += Rk[i] / h;
      symmetrize(ny, Sg);
      double Hm[MX];
      mv(ny, nx, Hk, mpj, Hm);
      for (int i = 0; i < ny; ++i) e[i] = y[k * ny + i] - Hm[i] - rk[i];
      if (!chol(ny, Sg, Ls)) { free(mp); free(Pp); return -(s + 1); }
      double ld = 0.0, z[MX];
      for (int i = 0; i < ny; ++i) ld += 2.0 * log(Ls[i * ny + i]);
      memcpy(z, e, sizeof(double) * ny);
      chol_solve(ny, 1, Ls, z);
      double quad = 0.0;
      for (int i = 0; i < ny; ++i) quad += e[i] * z[i];
      ksum_add(&ll, -0.5 * (ny * LOG2PI + ld + quad));
      /* K^T = Sg^{-1} H P-  (Sg symmetric) */
      double KT[MX * MX];
      memcpy(KT, HP, sizeof(double) * ny * nx);
      chol_solve(ny, nx, Ls, KT);
      for (int i = 0; i < nx; ++i)
        for (int l = 0; l < ny; ++l) K[i * ny + l] = KT[l * nx + i];
      double *mj = m + j * nx, *Pj = P + j * n2;
      for (int i = 0; i < nx; ++i) {
        double acc = mpj[i];
        for (int l = 0; l < ny; ++l) acc += K[i * ny + l] * e[l];
        mj[i] = acc;
      }
      /* P = P- - K H P- */
      for (int i = 0; i < nx; ++i)
        for (int l = 0; l < nx; ++l) {
          double acc = Ppj[i * nx + l];
          for (int q = 0; q < ny; ++q) acc -= K[i * ny + q] * HP[q * nx + l];
          Pj[i * nx + l] = acc;
        }
      symmetrize(nx, Pj);
    }
    loglik_out[s] = ksum_value(&ll);

    /* ---- backward: discrete RTS smoother ---- */
    memcpy(xs + T * nx, m + T * nx, sizeof(double) * nx);
    memcpy(Ps + T * n2, P + T * n2, sizeof(double) * n2);
    for (long j = T; j >= 1; --j) {
      const long k = k0 + j - 1;
      const double h = dt[k];
      const double *Fk = at(aF, k, s);
      double A[MX * MX], Phi[MX * MX], Lp[MX * MX], GT[MX * MX], G[MX * MX], d[MX], t1[MX * MX],
          t2[MX * MX];
      for (int i = 0; i < n2; ++i) A[i] = -h * Fk[i];
      for (int i = 0; i < nx; ++i) A[i * nx + i] += 1.0;
      inv(nx, A, Phi);
      /* G = P_{j-1} Phi^T (P-_j)^{-1}  =>  G^T = (P-_j)^{-1} Phi P_{j-1} */
      if (!chol(nx, Pp + j * n2, Lp)) { free(mp); free(Pp); return -(s + 1); }
      mm(nx, nx, nx, Phi, P + (j - 1) * n2, GT);
      chol_solve(nx, nx, Lp, GT);
      for (int i = 0; i < nx; ++i)
        for (int l = 0; l < nx; ++l) G[i * nx + l] = GT[l * nx + i];
      for (int i = 0; i < nx; ++i) d[i] = xs[j * nx + i] - mp[j * nx + i];
      for (int i = 0; i < nx; ++i) {
        double acc = m[(j - 1) * nx + i];
        for (int l = 0; l < nx; ++l) acc += G[i * nx + l] * d[l];
        xs[(j - 1) * nx + i] = acc;
      }
      for (int i = 0; i < n2; ++i) t1[i] = Ps[j * n2 + i] - Pp[j * n2 + i];
      mm(nx, nx, nx, G, t1, t2);
      mmt(nx, nx, nx, t2, G, t1);
      for (int i = 0; i < n2; ++i) Ps[(j - 1) * n2 + i] = P[(j - 1) * n2 + i] + t1[i];
      symmetrize(nx, Ps + (j - 1) * n2);
    }

    /* ---- discretised OM objective at xs ---- */
    ksum M = {0.0, 0.0};
    {
      double Lq[MX * MX], dx[MX], z[MX];
      if (!chol(nx, P0 + s * P0_seg, Lq)) { free(mp); free(Pp); return -(s + 1); }
      for (int i = 0; i < nx; ++i) dx[i] = xs[i] - m0[s * m0_seg + i];
      memcpy(z, dx, sizeof(double) * nx);
      chol_solve(nx, 1, Lq, z);
      double m0t = 0.0;
      for (int i = 0; i < nx; ++i) m0t += 0.5 * dx[i] * z[i];
      ksum_add(&M, m0t);
    }
    for (long j = 1; j <= T; ++j) {
      const long k = k0 + j - 1;
      const double h = dt[k];
      const double *Fk = at(aF, k, s), *ck = at(ac, k, s), *Lk = at(aL, k, s),
                   *Wk = at(aW, k, s), *Hk = at(aH, k, s), *rk = at(ar, k, s),
                   *Rk = at(aR, k, s);
      const double *xj = xs + j * nx, *xm = xs + (j - 1) * nx;
      double D[MX], Fx[MX];
      mv(nx, nx, Fk, xj, Fx);
      for (int i = 0; i < nx; ++i) D[i] = xj[i] - xm[i] - h * (Fx[i] + ck[i]);
      /* u = (L^T L)^{-1} L^T D ; cost 1/2 u^T (h W)^{-1} u */
      double LtL[MX * MX], LtD[MX], Ll[MX * MX], Lw[MX * MX];
      for (int a = 0; a < nw; ++a) {
        double acc = 0.0;
        for (int i = 0; i < nx; ++i) acc += Lk[i * nw + a] * D[i];
        LtD[a] = acc;
        for (int b = 0; b < nw; ++b) {
          double t = 0.0;
          for (int i = 0; i < nx; ++i) t += Lk[i * nw + a] * Lk[i * nw + b];
          LtL[a * nw + b] = t;
        }
      }
      if (!chol(nw, LtL, Ll)) { free(mp); free(Pp); return -(s + 1); }
      chol_solve(nw, 1, Ll, LtD); /* LtD now holds u */
      double Wh[MX * MX], z[MX];
      for (int i = 0; i < nw * nw; ++i) Wh[i] = h * Wk[i];
      if (!chol(nw, Wh, Lw)) { free(mp); free(Pp); return -(s + 1); }
      memcpy(z, LtD, sizeof(double) * nw);
      chol_solve(nw, 1, Lw, z);
      double mk = 0.0;
      for (int a = 0; a < nw; ++a) mk += 0.5 * LtD[a] * z[a];
      /* measurement: (h/2) eps^T R^{-1} eps */
      double Hx[MX], eps[MX], LR[MX * MX];
      mv(ny, nx, Hk, xj, Hx);
      for (int i = 0; i < ny; ++i) eps[i] = y[k * ny + i] - Hx[i] - rk[i];
      if (!chol(ny, Rk, LR)) { free(mp); free(Pp); return -(s + 1); }
      memcpy(z, eps, sizeof(double) * ny);
      chol_solve(ny, 1, LR, z);
      for (int i = 0; i < ny; ++i) mk += 0.5 * h * eps[i] * z[i];
      ksum_add(&M, mk);
    }
    mstar_out[s] = ksum_value(&M);
  }
  free(mp);
  free(Pp);
  return n_seg;
}

/* ---------- two-filter smoother (Sec. 4.3, eq. twofilter) ----------
 *
 * For state j of a segment, the steps after it (j+1 .. T) form one
 * conditional value function of the segment's last state z = x_T and of x_j
 * (Sec. 4.1, eq. conditionalvalue_linear, later state carrying J and eta):
 *
 *   V_j(z, x) = 1/2 z^T J z - z^T eta + 1/2 |x - A z - b|^2_{C^{-1}},
 *
 * the combination (Sec. 4.1 rule, earlier run E, later run L) of the one-step
 * elements of Sec. 4.2 (A = I - dt F, b = -dt c, C = dt Q, eta = dt H^T R^{-1}
 * (y - r), J = dt H^T R^{-1} H), accumulated here from the segment's end with
 * the empty run (I, 0, 0, 0, 0).  Eq. twofilter minimises V_j over z first
 * (combination with the constant element e, kappa -> infinity), which leaves
 * the backward filter N(x; bbar, Cbar), Cbar = A J^{-1} A^T + C,
 * bbar = A J^{-1} eta + b, and then combines it with the forward value
 * function 1/2 x^T S x - x^T v.  Near a segment's end J is singular (one step
 * observes ny < nx directions), so here both minimisations are done at once:
 * with lambda = v - S x the stationarity conditions of
 * 1/2 x^T S x - x^T v + V_j(z, x) over (x, z) read
 *
 *   [ I + C S   -A ] [x]   [ b + C v     ]
 *   [ A^T S      J ] [z] = [ eta + A^T v ]
 *
 * (no C^{-1}, no J^{-1}); the same matrix with right-hand side [C; A^T] is
 * d(x, z)/dv, whose x-block is the smoothed covariance.  Where J is
 * invertible the x-part equals (I + Cbar S)^{-1} (bbar + Cbar v).
 *
 * Inputs as oracle_smooth plus the filter moments m, P it wrote; S = P^{-1},
 * v = S m (Sec. 2.5).  suf_out (optional, NULL to skip) receives per state the
 * run after it as A [nx*nx], b [nx], C [nx*nx], eta [nx], J [nx*nx].
 */
typedef struct {
  double A[MX * MX], b[MX], C[MX * MX], eta[MX], J[MX * MX];
} run_t;

/* out = E . L with E the earlier run (Sec. 4.1 combination rule):
 *   M = (I + C_L J_E)^{-1}
 *   A = A_E M A_L,  b = A_E M (b_L + C_L eta_E) + b_E,  C = A_E M C_L A_E^T + C_E,
 *   eta = A_L^T M^T (eta_E - J_E b_L) + eta_L,  J = A_L^T M^T J_E A_L + J_L. */
static int run_combine(int n, const run_t *E, const run_t *L, run_t *out) {
  double X[MX * MX], M[MX * MX], MT[MX * MX], t1[MX * MX], t2[MX * MX], u[MX], w[MX], t3[MX];
  mm(n, n, n, L->C, E->J, X);
  for (int i = 0; i < n; ++i) X[i * n + i] += 1.0;
  if (!inv(n, X, M)) return 0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) MT[i * n + j] = M[j * n + i];
  /* A */
  mm(n, n, n, M, L->A, t1);
  mm(n, n, n, E->A, t1, out->A);
  /* b */
  mv(n, n, L->C, E->eta, u);
  for (int i = 0; i < n; ++i) u[i] += L->b[i];
  mv(n, n, M, u, w);
  mv(n, n, E->A, w, t3);
  for (int i = 0; i < n; ++i) out->b[i] = t3[i] + E->b[i];
  /* C */
  mm(n, n, n, M, L->C, t1);
  mm(n, n, n, E->A, t1, t2);
  mmt(n, n, n, t2, E->A, t1);
  for (int i = 0; i < n * n; ++i) out->C[i] = t1[i] + E->C[i];
  symmetrize(n, out->C);
  /* eta */
  mv(n, n, E->J, L->b, u);
  for (int i = 0; i < n; ++i) u[i] = E->eta[i] - u[i];
  mv(n, n, MT, u, w);
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int l = 0; l < n; ++l) s += L->A[l * n + i] * w[l];
    out->eta[i] = s + L->eta[i];
  }
  /* J */
  mm(n, n, n, E->J, L->A, t1);
  mm(n, n, n, MT, t1, t2);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int l = 0; l < n; ++l) s += L->A[l * n + i] * t2[l * n + j];
      out->J[i * n + j] = s + L->J[i * n + j];
    }
  symmetrize(n, out->J);
  return 1;
}

/* Solve a x = b in place (a [n][n] destroyed, b [n][nrhs] overwritten) by
 * Gaussian elimination with partial pivoting; returns 0 if singular. */
static int lu_solve(int n, double *a, int nrhs, double *b) {
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (fabs(a[i * n + k]) > fabs(a[p * n + k])) p = i;
    if (a[p * n + k] == 0.0) return 0;
    if (p != k) {
      for (int j = 0; j < n; ++j) {
        double t = a[k * n + j]; a[k * n + j] = a[p * n + j]; a[p * n + j] = t;
      }
      for (int j = 0; j < nrhs; ++j) {
        double t = b[k * nrhs + j]; b[k * nrhs + j] = b[p * nrhs + j]; b[p * nrhs + j] = t;
      }
    }
    for (int i = k + 1; i < n; ++i) {
      const double f = a[i * n + k] / a[k * n + k];
      if (f == 0.0) continue;
      for (int j = k; j < n; ++j) a[i * n + j] -= f * a[k * n + j];
      for (int j = 0; j < nrhs; ++j) b[i * nrhs + j] -= f * b[k * nrhs + j];
    }
  }
  for (int i = n - 1; i >= 0; --i)
    for (int j = 0; j < nrhs; ++j) {
      double s = b[i * nrhs + j];
      for (int l = i + 1; l < n; ++l) s -= a[i * n + l] * b[l * nrhs + j];
      b[i * nrhs + j] = s / a[i * n + i];
    }
  return 1;
}

long oracle_two_filter(int nx, int ny, int nw, long n_seg, const long *seg_off,
                       const double *F, long F_step, long F_seg,
                       const double *c, long c_step, long c_seg,
                       const double *L, long L_step, long L_seg,
                       const double *W, long W_step, long W_seg,
                       const double *H, long H_step, long H_seg,
                       const double *r, long r_step, long r_seg,
                       const double *R, long R_step, long R_seg,
                       const double *dt, const double *y,
                       const double *m_in, const double *P_in,
                       double *xs_out, double *Ps_out, double *suf_out) {
  arr aF = {F, F_step, F_seg}, ac = {c, c_step, c_seg}, aL = {L, L_step, L_seg},
      aW = {W, W_step, W_seg}, aH = {H, H_step, H_seg}, ar = {r, r_step, r_seg},
      aR = {R, R_step, R_seg};
  const int n = nx, n2 = nx * nx, nn = 2 * nx, nr = 1 + nx;
  const int sufsz = 3 * n2 + 2 * nx;
  for (long s = 0; s < n_seg; ++s) {
    const long k0 = seg_off[s], T = seg_off[s + 1] - seg_off[s];
    const long x0 = k0 + s;
    run_t suf, tmp, e;
    memset(&suf, 0, sizeof(suf));
    for (int i = 0; i < n; ++i) suf.A[i * n + i] = 1.0;
    for (long j = T; j >= 0; --j) {
      if (j < T) {
        /* element of step j+1 (global step index k0 + j) in front of the run */
        const long k = k0 + j;
        const double h = dt[k];
        const double *Fk = at(aF, k, s), *ck = at(ac, k, s), *Lk = at(aL, k, s),
                     *Wk = at(aW, k, s), *Hk = at(aH, k, s), *rk = at(ar, k, s),
                     *Rk = at(aR, k, s);
        double LW[MX * MX], Q[MX * MX], Ri[MX * MX], RiH[MX * MX], d[MX], Rid[MX];
        for (int i = 0; i < n2; ++i) e.A[i] = -h * Fk[i];
        for (int i = 0; i < n; ++i) e.A[i * n + i] += 1.0;
        for (int i = 0; i < n; ++i) e.b[i] = -h * ck[i];
        mm(n, nw, nw, Lk, Wk, LW);
        mmt(n, nw, n, LW, Lk, Q);
        for (int i = 0; i < n2; ++i) e.C[i] = h * Q[i];
        if (!inv(ny, Rk, Ri)) return -(s + 1);
        mm(ny, ny, n, Ri, Hk, RiH);
        for (int i = 0; i < n; ++i)
          for (int l = 0; l < n; ++l) {
            double acc = 0.0;
            for (int q = 0; q < ny; ++q) acc += Hk[q * n + i] * RiH[q * n + l];
            e.J[i * n + l] = h * acc;
          }
        for (int q = 0; q < ny; ++q) d[q] = y[k * ny + q] - rk[q];
        mv(ny, ny, Ri, d, Rid);
        for (int i = 0; i < n; ++i) {
          double acc = 0.0;
          for (int q = 0; q < ny; ++q) acc += Hk[q * n + i] * Rid[q];
          e.eta[i] = h * acc;
        }
        if (!run_combine(n, &e, &suf, &tmp)) return -(s + 1);
        suf = tmp;
      }
      /* forward value function of state j: S = P^{-1}, v = S m */
      const double *mj = m_in + (x0 + j) * n, *Pj = P_in + (x0 + j) * n2;
      double S[MX * MX], v[MX];
      if (!inv(n, Pj, S)) return -(s + 1);
      symmetrize(n, S);
      mv(n, n, S, mj, v);
      /* joint stationarity system */
      double Mt[4 * MX * MX], B[2 * MX * (MX + 1)], CS[MX * MX], t[MX];
      mm(n, n, n, suf.C, S, CS);
      for (int i = 0; i < n; ++i)
        for (int l = 0; l < n; ++l) {
          double ats = 0.0;
          for (int q = 0; q < n; ++q) ats += suf.A[q * n + i] * S[q * n + l];
          Mt[i * nn + l] = CS[i * n + l] + (i == l ? 1.0 : 0.0);
          Mt[i * nn + n + l] = -suf.A[i * n + l];
          Mt[(n + i) * nn + l] = ats;
          Mt[(n + i) * nn + n + l] = suf.J[i * n + l];
        }
      mv(n, n, suf.C, v, t);
      for (int i = 0; i < n; ++i) {
        double atv = 0.0;
        for (int q = 0; q < n; ++q) atv += suf.A[q * n + i] * v[q];
        B[i * nr] = suf.b[i] + t[i];
        B[(n + i) * nr] = suf.eta[i] + atv;
        for (int l = 0; l < n; ++l) {
          B[i * nr + 1 + l] = suf.C[i * n + l];
          B[(n + i) * nr + 1 + l] = suf.A[l * n + i];
        }
      }
      if (!lu_solve(nn, Mt, nr, B)) return -(s + 1);
      double *xo = xs_out + (x0 + j) * n, *Po = Ps_out + (x0 + j) * n2;
      for (int i = 0; i < n; ++i) {
        xo[i] = B[i * nr];
        for (int l = 0; l < n; ++l) Po[i * n + l] = B[i * nr + 1 + l];
      }
      symmetrize(n, Po);
      if (suf_out) {
        double *o = suf_out + (x0 + j) * sufsz;
        memcpy(o, suf.A, sizeof(double) * n2);
        memcpy(o + n2, suf.b, sizeof(double) * n);
        memcpy(o + n2 + n, suf.C, sizeof(double) * n2);
        memcpy(o + 2 * n2 + n, suf.eta, sizeof(double) * n);
        memcpy(o + 2 * n2 + 2 * n, suf.J, sizeof(double) * n2);
      }
    }
  }
  return n_seg;
}
