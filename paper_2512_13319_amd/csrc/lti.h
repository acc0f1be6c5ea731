// Exact discretisation of a time-invariant linear-affine model, host side.
//
// For dx/dt = F x + c + L w (w white with spectral density W, Q = L W L^T) the
// transition over a step dt is x_k = e^{F dt} x_{k-1} + u + w_k with
// u = int_0^dt e^{F s} ds c and w_k ~ N(0, Qd), Qd = int_0^dt e^{F s} Q e^{F^T s} ds.
// Van Loan's block exponential gives both integrals:
//   exp([[-F, Q], [0, F^T]] dt) = [[e^{-F dt}, X], [0, e^{F^T dt}]],  Qd = e^{F dt} X,
//   exp([[F, c], [0, 0]] dt)    = [[e^{F dt}, u], [0, 1]].
// Backwards, x_{k-1} = A x_k + b + noise with A = e^{-F dt}, b = -A u and
// covariance C = A Qd A^T = X A^T: the dynamics part of the exact one-step
// element.  The library's element build takes one implicit-Euler step of
// (F~, c~, L~, W~) (A = I - dt F~, b = -dt c~, C = dt L~ W~ L~^T), so the exact
// element is handed to it as F~ = (I - A) / dt, c~ = -b / dt, W~ = I and L~ a
// square root of C / dt (from a symmetric eigendecomposition).
//
// Matrix exponential: scaling and squaring of the Taylor polynomial of degree
// 18, with the argument scaled to 1-norm <= 1/2 (truncation below 1e-22
// relative); symmetric eigendecomposition by cyclic Jacobi rotations.
#pragma once
#include <cmath>
#include <cstring>

namespace ms {
namespace lti {

constexpr int kMax = 16;  // 2 nx <= 16

inline void matmul(int n, const double* a, const double* b, double* c) {
  double t[kMax * kMax];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int k = 0; k < n; ++k) s += a[i * n + k] * b[k * n + j];
      t[i * n + j] = s;
    }
  std::memcpy(c, t, sizeof(double) * n * n);
}

inline void expm(int n, const double* a, double* e) {
  double norm = 0.0;
  for (int j = 0; j < n; ++j) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += std::fabs(a[i * n + j]);
    norm = s > norm ? s : norm;
  }
  int sq = 0;
  while (norm > 0.5) {
    norm *= 0.5;
    ++sq;
  }
  const double scale = std::ldexp(1.0, -sq);
  double b[kMax * kMax], term[kMax * kMax];
  for (int i = 0; i < n * n; ++i) b[i] = a[i] * scale;
  for (int i = 0; i < n * n; ++i) e[i] = term[i] = (i % (n + 1) == 0) ? 1.0 : 0.0;
  for (int k = 1; k <= 18; ++k) {
    matmul(n, term, b, term);
    for (int i = 0; i < n * n; ++i) {
      term[i] /= k;
      e[i] += term[i];
    }
  }
  for (int s = 0; s < sq; ++s) matmul(n, e, e, e);
}

// a (symmetric, destroyed) = v diag(w) v^T
inline void sym_eig(int n, double* a, double* v, double* w) {
  for (int i = 0; i < n * n; ++i) v[i] = (i % (n + 1) == 0) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += a[i * n + j] * a[i * n + j];
        if (i != j) off += a[i * n + j] * a[i * n + j];
      }
    if (off <= 1e-32 * tot) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a[p * n + q];
        if (apq == 0.0) continue;
        const double theta = (a[q * n + q] - a[p * n + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = a[k * n + p], akq = a[k * n + q];
          a[k * n + p] = cs * akp - sn * akq;
          a[k * n + q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = a[p * n + k], aqk = a[q * n + k];
          a[p * n + k] = cs * apk - sn * aqk;
          a[q * n + k] = sn * apk + cs * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = v[k * n + p], vkq = v[k * n + q];
          v[k * n + p] = cs * vkp - sn * vkq;
          v[k * n + q] = sn * vkp + cs * vkq;
        }
      }
  }
  for (int i = 0; i < n; ++i) w[i] = a[i * n + i];
}

// F~, c~, L~ (W~ = I) for one step dt; c may be null (no drift offset).
inline void exact_terms(int nx, int nw, const double* F, const double* c, const double* L,
                        const double* W, double dt, double* Ft, double* ct, double* Lt) {
  const int n = nx, m = 2 * nx;
  double Q[kMax * kMax], LW[kMax * kMax];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < nw; ++j) {
      double s = 0.0;
      for (int k = 0; k < nw; ++k) s += L[i * nw + k] * W[k * nw + j];
      LW[i * nw + j] = s;
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int k = 0; k < nw; ++k) s += LW[i * nw + k] * L[j * nw + k];
      Q[i * n + j] = s;
    }
  double M[kMax * kMax], E[kMax * kMax];
  std::memset(M, 0, sizeof(M));
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      M[i * m + j] = -F[i * n + j] * dt;
      M[i * m + n + j] = Q[i * n + j] * dt;
      M[(n + i) * m + n + j] = F[j * n + i] * dt;
    }
  expm(m, M, E);
  double A[kMax * kMax], X[kMax * kMax], C[kMax * kMax];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      A[i * n + j] = E[i * m + j];
      X[i * n + j] = E[i * m + n + j];
    }
  // C = X A^T, symmetrised
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int k = 0; k < n; ++k) s += X[i * n + k] * A[j * n + k];
      C[i * n + j] = s;
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) C[i * n + j] = C[j * n + i] = 0.5 * (C[i * n + j] + C[j * n + i]);
  // u = int_0^dt e^{F s} ds c;  c~ = -b / dt = A u / dt
  double u[kMax];
  if (c != nullptr) {
    const int mu = n + 1;
    double Mu[kMax * kMax], Eu[kMax * kMax];
    std::memset(Mu, 0, sizeof(Mu));
    for (int i = 0; i < n; ++i) {
      for (int j = 0; j < n; ++j) Mu[i * mu + j] = F[i * n + j] * dt;
      Mu[i * mu + n] = c[i] * dt;
    }
    expm(mu, Mu, Eu);
    for (int i = 0; i < n; ++i) u[i] = Eu[i * mu + n];
  } else {
    for (int i = 0; i < n; ++i) u[i] = 0.0;
  }
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += A[i * n + k] * u[k];
    ct[i] = s / dt;
    for (int j = 0; j < n; ++j) Ft[i * n + j] = ((i == j ? 1.0 : 0.0) - A[i * n + j]) / dt;
  }
  // L~ = V diag(sqrt(max(w, 0))) with C / dt = V diag(w) V^T
  double Cs[kMax * kMax], V[kMax * kMax], w[kMax];
  for (int i = 0; i < n * n; ++i) Cs[i] = C[i] / dt;
  sym_eig(n, Cs, V, w);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Lt[i * n + j] = V[i * n + j] * std::sqrt(w[j] > 0.0 ? w[j] : 0.0);
}

}  // namespace lti
}  // namespace ms
