// Scan elements and their operators.
//
// Indexing is in original time.  A filter element e covers a run of grid
// steps ending at a "later" state x_l and starting from an "earlier" state
// x_e; it stores the conditional value function of the paper (Sec. 4.1,
// eq. conditionalvalue_linear) with phi = x_l and z = x_e:
//
//   V(x_l, x_e) = 1/2 x_l^T J x_l - x_l^T eta + 1/2 |x_e - A x_l - b|^2_{C^{-1}}.
//
// Reversing time (Sec. 2.2) turns the paper's prefix over sub-intervals into
// a prefix in t-order.  With E the earlier run and L the later one, the
// combination rule of Sec. 4.1 (the printed "I + J(s,gamma) C(gamma,t)" read
// as I + J_E C_L, the transpose of I + C_L J_E) gives
//
//   A = A_E M A_L,             M = (I + C_L J_E)^{-1}
//   b = A_E M (b_L + C_L eta_E) + b_E
//   C = A_E M C_L A_E^T + C_E
//   eta = A_L^T M^T (eta_E - J_E b_L) + eta_L
//   J = A_L^T M^T J_E A_L + J_L.
//
// The identity is (I, 0, 0, 0, 0) (the boundary value of Sec. 4.2); the prior
// is (0, 0, 0, P0^{-1} m0, P0^{-1}) (terminal cost of Sec. 2.4).  Any run that
// contains a prior has A = 0, and then its (J, eta) is the information form
// (S, v) of the filter at its last state (Sec. 2.5: P = S^{-1}, m = S^{-1} v).
// A fresh one-step element is kept with C in factored form C = V V^T.
//
// The trajectory pass (Sec. 4.3, eq. 42) is an affine scan in reverse
// t-order: x_{k-1} = G_k x_k + beta_k with G_k = (I + C_k S_{k-1})^{-1} A_k,
// beta_k = (I + C_k S_{k-1})^{-1} (b_k + C_k v_{k-1}).  Its covariance
// companion P_{k-1} = G_k P_k G_k^T + Lam_k, Lam_k = (I + C_k S_{k-1})^{-1} C_k,
// composes with the same maps.
#pragma once
#include "models.h"

namespace ms {

template <typename T, int N>
struct Elem {
  T A[N][N];
  T b[N];
  T C[N][N];
  T eta[N];
  T J[N][N];
};

template <typename T, int N>
MS_DEV void elem_identity(Elem<T, N>& e) {
  meye(e.A);
  mzero(e.C);
  mzero(e.J);
#pragma unroll
  for (int i = 0; i < N; ++i) e.b[i] = e.eta[i] = T(0);
}

// Fresh one-step element with C = V V^T.
template <typename T, int N, int NW>
struct Fresh {
  T A[N][N];
  T b[N];
  T V[N][NW];
  T eta[N];
  T J[N][N];
};

template <typename T, int N, int NY, int NW>
MS_DEV void fresh_from_step(const Step<T, N, NY, NW>& s, const T (&y)[NY], Fresh<T, N, NW>& f) {
  const T dt = s.dt;
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) f.A[i][j] = (i == j ? T(1) : T(0)) - dt * s.F[i][j];
    f.b[i] = -dt * s.c[i];
#pragma unroll
    for (int j = 0; j < NW; ++j) f.V[i][j] = s.V[i][j];
  }
  // RH = dt R^{-1} H  [NY][N]; J = H^T RH; eta = RH^T (y - r)... with R^{-1} symmetric
  T RH[NY][N];
  mm(s.Rinv, s.H, RH);
#pragma unroll
  for (int i = 0; i < NY; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) RH[i][j] *= dt;
  mtm_sym(s.H, RH, f.J);
  T e[NY];
#pragma unroll
  for (int i = 0; i < NY; ++i) e[i] = y[i] - s.r[i];
  mtv(RH, e, f.eta);
}

template <typename T, int N, int NW>
MS_DEV void fresh_to_elem(const Fresh<T, N, NW>& f, Elem<T, N>& e) {
  mcopy(f.A, e.A);
  mmt_sym(f.V, f.V, e.C);
  mcopy(f.J, e.J);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    e.b[i] = f.b[i];
    e.eta[i] = f.eta[i];
  }
}

// General combination E (earlier) . L (later); result may alias neither.
template <typename T, int N>
MS_DEV void combine(const Elem<T, N>& E, const Elem<T, N>& L, Elem<T, N>& out) {
  T X[N][N], M[N][N];
  mm(L.C, E.J, X);
#pragma unroll
  for (int i = 0; i < N; ++i) X[i][i] += T(1);
  inv(X, M);
  T MA[N][N];
  mm(M, L.A, MA);           // M A_L
  mm(E.A, MA, out.A);       // A_E M A_L
  T JMA[N][N];
  mm(E.J, MA, JMA);         // J_E M A_L  (= M^T J_E A_L)
  T Jn[N][N];
  mtm_sym(L.A, JMA, Jn);    // A_L^T M^T J_E A_L
  T MC[N][N], AMC[N][N];
  mm(M, L.C, MC);           // M C_L (symmetric)
  mm(E.A, MC, AMC);
  T Cn[N][N];
  mmt_sym(AMC, E.A, Cn);    // A_E M C_L A_E^T
  T u[N], Mu[N], t[N];
  mv(L.C, E.eta, u);
#pragma unroll
  for (int i = 0; i < N; ++i) u[i] += L.b[i];
  mv(M, u, Mu);
  mv(E.A, Mu, t);
  T w[N], Mw[N], s[N];
  mv(E.J, L.b, w);
#pragma unroll
  for (int i = 0; i < N; ++i) w[i] = E.eta[i] - w[i];
  mtv(M, w, Mw);
  mtv(L.A, Mw, s);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    out.b[i] = t[i] + E.b[i];
    out.eta[i] = s[i] + L.eta[i];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      out.C[i][j] = Cn[i][j] + E.C[i][j];
      out.J[i][j] = Jn[i][j] + L.J[i][j];
    }
  }
}

// agg <- agg . f  (fold a fresh element onto the right of a run).
// With Z = I + V^T J_E V (SPD), M = I - V Z^{-1} V^T J_E, M C_L = V Z^{-1} V^T.
template <typename T, int N, int NW>
MS_DEV void fold_fresh(Elem<T, N>& E, const Fresh<T, N, NW>& f) {
  T W[N][NW];
  mm(E.J, f.V, W);  // J_E V
  T Z[NW][NW];
  mtm_sym(f.V, W, Z);
#pragma unroll
  for (int i = 0; i < NW; ++i) Z[i][i] += T(1);
  T Lz[NW][NW], dz[NW];
  chol(Z, Lz, dz);
  // T3 = M A_L = A_L - V Z^{-1} (W^T A_L)
  T X[NW][N];
  mtm(W, f.A, X);
  trsm_lower(Lz, dz, X);
  trsm_upper_t(Lz, dz, X);
  T T3[N][N];
  mm(f.V, X, T3);
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) T3[i][j] = f.A[i][j] - T3[i][j];
  // vectors first (they read the old E)
  T u[N];  // b_L + V V^T eta_E
  {
    T vte[NW];
    mtv(f.V, E.eta, vte);
    mv(f.V, vte, u);
#pragma unroll
    for (int i = 0; i < N; ++i) u[i] += f.b[i];
  }
  T Mu[N];  // u - V Z^{-1} W^T u
  {
    T z[NW];
    mtv(W, u, z);
    trsv_lower(Lz, dz, z);
    trsv_upper_t(Lz, dz, z);
    T vz[N];
    mv(f.V, z, vz);
#pragma unroll
    for (int i = 0; i < N; ++i) Mu[i] = u[i] - vz[i];
  }
  T w[N];  // eta_E - J_E b_L
  mv(E.J, f.b, w);
#pragma unroll
  for (int i = 0; i < N; ++i) w[i] = E.eta[i] - w[i];
  T Mtw[N];  // w - W Z^{-1} V^T w
  {
    T z[NW];
    mtv(f.V, w, z);
    trsv_lower(Lz, dz, z);
    trsv_upper_t(Lz, dz, z);
    T wz[N];
    mv(W, z, wz);
#pragma unroll
    for (int i = 0; i < N; ++i) Mtw[i] = w[i] - wz[i];
  }
  T bn[N], en[N];
  mv(E.A, Mu, bn);
  mtv(f.A, Mtw, en);
  // J = A_L^T (J_E T3) + J_L
  T JT[N][N], Jn[N][N];
  mm(E.J, T3, JT);
  mtm_sym(f.A, JT, Jn);
  // C = (A_E V Lz^{-T}) (A_E V Lz^{-T})^T + C_E
  T AV[N][NW];
  mm(E.A, f.V, AV);
  T Yt[NW][N];
#pragma unroll
  for (int i = 0; i < NW; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) Yt[i][j] = AV[j][i];
  trsm_lower(Lz, dz, Yt);
  T Cn[N][N];
  mtm_sym(Yt, Yt, Cn);
  T An[N][N];
  mm(E.A, T3, An);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    E.b[i] += bn[i];
    E.eta[i] = en[i] + f.eta[i];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      E.A[i][j] = An[i][j];
      E.C[i][j] += Cn[i][j];
      E.J[i][j] = Jn[i][j] + f.J[i][j];
    }
  }
}

// Information step (S, v) . f -> (S', v'), and optionally the trajectory
// element (G, beta, Lam) of the state that (S, v) belongs to, which shares
// the factor Z = I + V^T S V:
//   (I + S C)^{-1} S = S - W Z^{-1} W^T,  (I + S C)^{-1} = I - W Z^{-1} V^T,
//   (I + C S)^{-1}   = I - V Z^{-1} W^T,  with W = S V.
template <typename T, int N, int NW, bool kTraj>
MS_DEV void info_step(const T (&S)[N][N], const T (&v)[N], const Fresh<T, N, NW>& f,
                      T (&Sn)[N][N], T (&vn)[N], T (&Sp)[N][N],
                      T (&G)[N][N], T (&beta)[N], T (&Lam)[N][N]) {
  T W[N][NW];
  mm(S, f.V, W);
  T Z[NW][NW];
  mtm_sym(f.V, W, Z);
#pragma unroll
  for (int i = 0; i < NW; ++i) Z[i][i] += T(1);
  T Lz[NW][NW], dz[NW];
  chol(Z, Lz, dz);
  // Nm = S - (Lz^{-1} W^T)^T (Lz^{-1} W^T)
  T Yw[NW][N];
#pragma unroll
  for (int i = 0; i < NW; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) Yw[i][j] = W[j][i];
  trsm_lower(Lz, dz, Yw);
  T Nm[N][N];
  mtm_sym(Yw, Yw, Nm);
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) Nm[i][j] = S[i][j] - Nm[i][j];
  T NA[N][N];
  mm(Nm, f.A, NA);
  mtm_sym(f.A, NA, Sp);  // predicted information A^T (S^{-1} + C)^{-1} A
  // u = v - S b;  u' = u - W Z^{-1} V^T u;  v' = A^T u' + eta
  T u[N];
  mv(S, f.b, u);
#pragma unroll
  for (int i = 0; i < N; ++i) u[i] = v[i] - u[i];
  {
    T z[NW];
    mtv(f.V, u, z);
    trsv_lower(Lz, dz, z);
    trsv_upper_t(Lz, dz, z);
    T wz[N];
    mv(W, z, wz);
#pragma unroll
    for (int i = 0; i < N; ++i) u[i] -= wz[i];
  }
  T an[N];
  mtv(f.A, u, an);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    vn[i] = an[i] + f.eta[i];
#pragma unroll
    for (int j = 0; j < N; ++j) Sn[i][j] = Sp[i][j] + f.J[i][j];
  }
  if constexpr (kTraj) {
    // G = A - V Z^{-1} (W^T A)
    T X[NW][N];
    mtm(W, f.A, X);
    trsm_lower(Lz, dz, X);
    trsm_upper_t(Lz, dz, X);
    T VX[N][N];
    mm(f.V, X, VX);
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) G[i][j] = f.A[i][j] - VX[i][j];
    // beta = (b + V V^T v) - V Z^{-1} W^T (b + V V^T v)
    T bc[N];
    {
      T z[NW];
      mtv(f.V, v, z);
      mv(f.V, z, bc);
#pragma unroll
      for (int i = 0; i < N; ++i) bc[i] += f.b[i];
    }
    {
      T z[NW];
      mtv(W, bc, z);
      trsv_lower(Lz, dz, z);
      trsv_upper_t(Lz, dz, z);
      T vz[N];
      mv(f.V, z, vz);
#pragma unroll
      for (int i = 0; i < N; ++i) beta[i] = bc[i] - vz[i];
    }
    // Lam = V Z^{-1} V^T = (Lz^{-1} V^T)^T (Lz^{-1} V^T)
    T Yv[NW][N];
#pragma unroll
    for (int i = 0; i < NW; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) Yv[i][j] = f.V[j][i];
    trsm_lower(Lz, dz, Yv);
    mtm_sym(Yv, Yv, Lam);
  }
}

// Carry application (S, v) . agg for a general run agg: only (J, eta) of the
// result are needed.  S = 0 (no information yet) is allowed.
template <typename T, int N>
MS_DEV void carry_apply(T (&S)[N][N], T (&v)[N], const Elem<T, N>& L) {
  T X[N][N], M[N][N];
  mm(S, L.C, X);  // I + S C_L  (= I + J_E C_L with E the carry)
#pragma unroll
  for (int i = 0; i < N; ++i) X[i][i] += T(1);
  inv(X, M);
  T MS_[N][N];
  mm(M, S, MS_);  // (I + S C)^{-1} S, symmetric
  T MSA[N][N];
  mm(MS_, L.A, MSA);
  T Sn[N][N];
  mtm_sym(L.A, MSA, Sn);
  T u[N];
  mv(S, L.b, u);
#pragma unroll
  for (int i = 0; i < N; ++i) u[i] = v[i] - u[i];
  T Mu[N], an[N];
  mv(M, u, Mu);
  mtv(L.A, Mu, an);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    v[i] = an[i] + L.eta[i];
#pragma unroll
    for (int j = 0; j < N; ++j) S[i][j] = Sn[i][j] + L.J[i][j];
  }
}

// ------------------------------------------------------------------ trajectory maps
// x_first = Phi x_after + bt;  P_first = Phi P_after Phi^T + Om
template <typename T, int N>
struct Aff {
  T Phi[N][N];
  T bt[N];
  T Om[N][N];
};

template <typename T, int N>
MS_DEV void aff_identity(Aff<T, N>& a) {
  meye(a.Phi);
  mzero(a.Om);
#pragma unroll
  for (int i = 0; i < N; ++i) a.bt[i] = T(0);
}

// a <- a o (G, beta, Lam): append a later map on the right.
template <typename T, int N>
MS_DEV void aff_append(Aff<T, N>& a, const T (&G)[N][N], const T (&beta)[N], const T (&Lam)[N][N]) {
  T PG[N][N], Pb[N], PL[N][N], PLP[N][N];
  mm(a.Phi, G, PG);
  mv(a.Phi, beta, Pb);
  mm(a.Phi, Lam, PL);
  mmt_sym(PL, a.Phi, PLP);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    a.bt[i] += Pb[i];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      a.Phi[i][j] = PG[i][j];
      a.Om[i][j] += PLP[i][j];
    }
  }
}

template <typename T, int N>
MS_DEV void aff_append(Aff<T, N>& a, const Aff<T, N>& o) { aff_append(a, o.Phi, o.bt, o.Om); }

// (x, P) <- map applied to the value after it
template <typename T, int N>
MS_DEV void aff_apply(const Aff<T, N>& a, T (&x)[N], T (&P)[N][N]) {
  T nx_[N], PP[N][N], PPP[N][N];
  mv(a.Phi, x, nx_);
  mm(a.Phi, P, PP);
  mmt_sym(PP, a.Phi, PPP);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    x[i] = nx_[i] + a.bt[i];
#pragma unroll
    for (int j = 0; j < N; ++j) P[i][j] = PPP[i][j] + a.Om[i][j];
  }
}

template <typename T, int N>
MS_DEV void traj_step(const T (&G)[N][N], const T (&beta)[N], const T (&Lam)[N][N], T (&x)[N],
                      T (&P)[N][N]) {
  T nx_[N], GP[N][N], GPG[N][N];
  mv(G, x, nx_);
  mm(G, P, GP);
  mmt_sym(GP, G, GPG);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    x[i] = nx_[i] + beta[i];
#pragma unroll
    for (int j = 0; j < N; ++j) P[i][j] = GPG[i][j] + Lam[i][j];
  }
}

}  // namespace ms
