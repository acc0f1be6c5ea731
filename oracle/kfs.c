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
    double ll = 0.0;

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
      ll += -0.5 * (ny * LOG2PI + ld + quad);
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
    loglik_out[s] = ll;

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
    double M = 0.0;
    {
      double Lq[MX * MX], dx[MX], z[MX];
      if (!chol(nx, P0 + s * P0_seg, Lq)) { free(mp); free(Pp); return -(s + 1); }
      for (int i = 0; i < nx; ++i) dx[i] = xs[i] - m0[s * m0_seg + i];
      memcpy(z, dx, sizeof(double) * nx);
      chol_solve(nx, 1, Lq, z);
      for (int i = 0; i < nx; ++i) M += 0.5 * dx[i] * z[i];
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
      for (int a = 0; a < nw; ++a) M += 0.5 * LtD[a] * z[a];
      /* measurement: (h/2) eps^T R^{-1} eps */
      double Hx[MX], eps[MX], LR[MX * MX];
      mv(ny, nx, Hk, xj, Hx);
      for (int i = 0; i < ny; ++i) eps[i] = y[k * ny + i] - Hx[i] - rk[i];
      if (!chol(ny, Rk, LR)) { free(mp); free(Pp); return -(s + 1); }
      memcpy(z, eps, sizeof(double) * ny);
      chol_solve(ny, 1, LR, z);
      for (int i = 0; i < ny; ++i) M += 0.5 * h * eps[i] * z[i];
    }
    mstar_out[s] = M;
  }
  free(mp);
  free(Pp);
  return n_seg;
}
