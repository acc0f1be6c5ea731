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
  mtm_symavg(L.A, JMA, Jn);  // A_L^T M^T J_E A_L
  T MC[N][N], AMC[N][N];
  mm(M, L.C, MC);           // M C_L (symmetric)
  mm(E.A, MC, AMC);
  T Cn[N][N];
  mmt_symavg(AMC, E.A, Cn);  // A_E M C_L A_E^T
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

// L <- E . L in place: the same arithmetic as combine(E, L, out), with the
// earlier element E read field by field through `src` (get_J, get_eta,
// get_A, get_b, get_C) when each is first needed, instead of being held whole.
// Every field of E is read before the same field of L is overwritten, so E
// may be another lane's L seen through a shuffle, in lockstep.  Live at the
// peak: L, E's J, M, M A_L and M C_L (against E, L and the output for
// combine).
template <typename T, int N, class Src>
MS_DEV void combine_into(const Src& src, Elem<T, N>& L) {
  T JE[N][N], eE[N];
  src.get_J(JE);
  src.get_eta(eE);
  T X[N][N], M[N][N];
  mm(L.C, JE, X);
#pragma unroll
  for (int i = 0; i < N; ++i) X[i][i] += T(1);
  inv(X, M);
  T MA[N][N], MC[N][N];
  mm(M, L.A, MA);  // M A_L
  mm(M, L.C, MC);  // M C_L (symmetric in exact arithmetic)
  T u[N], Mu[N];
  mv(L.C, eE, u);
#pragma unroll
  for (int i = 0; i < N; ++i) u[i] += L.b[i];
  mv(M, u, Mu);
  T w[N], Mw[N], s[N];
  mv(JE, L.b, w);
#pragma unroll
  for (int i = 0; i < N; ++i) w[i] = eE[i] - w[i];
  mtv(M, w, Mw);
  mtv(L.A, Mw, s);
  {
    T JMA[N][N], Jn[N][N];
    mm(JE, MA, JMA);
    mtm_symavg(L.A, JMA, Jn);  // A_L^T M^T J_E A_L
#pragma unroll
    for (int i = 0; i < N; ++i) {
      L.eta[i] = s[i] + L.eta[i];
#pragma unroll
      for (int j = 0; j < N; ++j) L.J[i][j] = Jn[i][j] + L.J[i][j];
    }
  }
  T EA[N][N], eb[N];
  src.get_A(EA);
  src.get_b(eb);
  T t[N];
  mv(EA, Mu, t);
  T EC[N][N];
  src.get_C(EC);
  T AMC[N][N], Cn[N][N];
  mm(EA, MC, AMC);
  mmt_symavg(AMC, EA, Cn);  // A_E M C_L A_E^T
  mm(EA, MA, L.A);          // A_E M A_L
#pragma unroll
  for (int i = 0; i < N; ++i) {
    L.b[i] = t[i] + eb[i];
#pragma unroll
    for (int j = 0; j < N; ++j) L.C[i][j] = Cn[i][j] + EC[i][j];
  }
}

// agg <- agg . f  (fold a fresh element onto the right of a run).
// With W = J_E V, Z = I + V^T W (SPD), M = I - V Z^{-1} W^T, M C_L = V Z^{-1} V^T,
// and X = Z^{-1} W^T A_L: M A_L = A_L - V X, A_L^T M^T J_E A_L = (M A_L)^T J_E (M A_L) + X^T X.
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
  // J = A_L^T M^T J_E A_L + J_L in Joseph form, T3^T J_E T3 + X^T X + J_L
  // (as in info_step: the difference J_E - W Z^{-1} W^T cancels where J_E is
  // ill-conditioned)
  T JT[N][N], Jn[N][N], XX[N][N];
  mm(E.J, T3, JT);
  mtm_sym(T3, JT, Jn);
  mtm_sym(X, X, XX);
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) Jn[i][j] += XX[i][j];
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
// the factor Z = I + V^T S V.  With W = S V and X = Z^{-1} W^T A:
//   (I + C S)^{-1} A = A - V X = G,   (I + S C)^{-1} = I - W Z^{-1} V^T,
//   A^T (I + S C)^{-1} S A = G^T S G + X^T X.
// The last line is the Joseph form of A^T (S - W Z^{-1} W^T) A: a sum of two
// PSD terms instead of a difference.  Where S is ill-conditioned (strongly
// observed directions next to weakly observed ones) the difference loses
// everything below eps |S|, and the recursion then amplifies that loss
// through A = I - dt F step after step; the Joseph form keeps the small
// eigenvalues to the accuracy of their own scale.
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
  // X = Z^{-1} W^T A,  G = A - V X
  T X[NW][N];
  mtm(W, f.A, X);
  trsm_lower(Lz, dz, X);
  trsm_upper_t(Lz, dz, X);
  T Gm[N][N];
  mm(f.V, X, Gm);
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) Gm[i][j] = f.A[i][j] - Gm[i][j];
  // predicted information A^T (S^{-1} + C)^{-1} A = G^T S G + X^T X
  {
    T SG[N][N], XX[N][N];
    mm(S, Gm, SG);
    mtm_sym(Gm, SG, Sp);
    mtm_sym(X, X, XX);
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) Sp[i][j] += XX[i][j];
  }
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
    mcopy(Gm, G);
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

// Trajectory element (G, beta, Lam) of a state with filter (S, v) from the
// fresh element f of the step after it: the trajectory half of info_step,
// with its own factor Z = I + V^T S V.
template <typename T, int N, int NW>
MS_DEV void traj_map(const T (&S)[N][N], const T (&v)[N], const Fresh<T, N, NW>& f,
                     T (&G)[N][N], T (&beta)[N], T (&Lam)[N][N]) {
  T W[N][NW];
  mm(S, f.V, W);
  T Z[NW][NW];
  mtm_sym(f.V, W, Z);
#pragma unroll
  for (int i = 0; i < NW; ++i) Z[i][i] += T(1);
  T Lz[NW][NW], dz[NW];
  chol(Z, Lz, dz);
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
  T Yv[NW][N];
#pragma unroll
  for (int i = 0; i < NW; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) Yv[i][j] = f.V[j][i];
  trsm_lower(Lz, dz, Yv);
  mtm_sym(Yv, Yv, Lam);
}

// An element held whole (in registers), as a source for combine_into and
// carry_apply.
template <typename T, int N>
struct RegSrc {
  const Elem<T, N>& e;
  MS_DEV void get_A(T (&a)[N][N]) const { mcopy(e.A, a); }
  MS_DEV void get_b(T (&b)[N]) const {
#pragma unroll
    for (int r = 0; r < N; ++r) b[r] = e.b[r];
  }
  MS_DEV void get_eta(T (&b)[N]) const {
#pragma unroll
    for (int r = 0; r < N; ++r) b[r] = e.eta[r];
  }
  MS_DEV void get_C(T (&a)[N][N]) const { mcopy(e.C, a); }
  MS_DEV void get_J(T (&a)[N][N]) const { mcopy(e.J, a); }
};

// Carry application (S, v) . agg for a general run agg: only (J, eta) of the
// result are needed.  S = 0 (no information yet) is allowed.  The run is read
// field by field through `src` (see combine_into).
template <typename T, int N, class Src>
MS_DEV void carry_apply_src(T (&S)[N][N], T (&v)[N], const Src& src) {
  T X[N][N], M[N][N];
  {
    T LC[N][N];
    src.get_C(LC);
    mm(S, LC, X);  // I + S C_L  (= I + J_E C_L with E the carry)
  }
#pragma unroll
  for (int i = 0; i < N; ++i) X[i][i] += T(1);
  inv(X, M);
  T MS_[N][N];
  mm(M, S, MS_);  // (I + S C)^{-1} S, symmetric in exact arithmetic
  T LA[N][N];
  src.get_A(LA);
  T Sn[N][N];
  {
    T MSA[N][N];
    mm(MS_, LA, MSA);
    mtm_symavg(LA, MSA, Sn);
  }
  T Lb[N], u[N];
  src.get_b(Lb);
  mv(S, Lb, u);
#pragma unroll
  for (int i = 0; i < N; ++i) u[i] = v[i] - u[i];
  T Mu[N], an[N];
  mv(M, u, Mu);
  mtv(LA, Mu, an);
  T Le[N], LJ[N][N];
  src.get_eta(Le);
  src.get_J(LJ);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    v[i] = an[i] + Le[i];
#pragma unroll
    for (int j = 0; j < N; ++j) S[i][j] = Sn[i][j] + LJ[i][j];
  }
}
template <typename T, int N>
MS_DEV void carry_apply(T (&S)[N][N], T (&v)[N], const Elem<T, N>& L) {
  carry_apply_src(S, v, RegSrc<T, N>{L});
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

// ------------------------------------------------------------------ two-filter smoother
// The steps after a state form one run s whose later state is the segment's
// last state z; the two-filter smoother (Sec. 4.3, eq. twofilter) combines it
// with the forward value function of the state.

// s <- f . s: the element of one step in front of a later run s (the Sec. 4.1
// rule with E = f).  Writing the step's measurement terms as J_f = H^T D H,
// eta_f = H^T D e (D = dt R^{-1}, e = y - r), the factor M = (I + C_s J_f)^{-1}
// only needs the NY x NY matrix Y = R / dt + H C_s H^T (push-through identity):
//   M = I - K Y^{-1} H,  K = C_s H^T;   M^T J_f = H^T Y^{-1} H;   M^T H^T D = H^T Y^{-1}
// hence, with A_f = I - dt F, b_f = -dt c, C_f = V V^T,
//   A   = A_f (A_s - K Y^{-1} H A_s)
//   b   = A_f (u - K Y^{-1} H u) + b_f,      u = b_s + K D e
//   C   = A_f (C_s - K Y^{-1} K^T) A_f^T + V V^T   (the bracket in Joseph form)
//   eta = (H A_s)^T Y^{-1} (e - H b_s) + eta_s
//   J   = (H A_s)^T Y^{-1} (H A_s) + J_s.
template <typename T, int N, int NY, int NW>
MS_DEV void prepend_step(const Step<T, N, NY, NW>& st, const T (&y)[NY], Elem<T, N>& s) {
  const T dt = st.dt;
  T K[N][NY];
  mmt(s.C, st.H, K);  // C_s H^T
  T Y[NY][NY];
  mm(st.H, K, Y);
  const T rdt = rcp(dt);
#pragma unroll
  for (int a = 0; a < NY; ++a)
#pragma unroll
    for (int b = 0; b < NY; ++b) Y[a][b] = fma_(st.R[a][b], rdt, Y[a][b]);
  T Ly[NY][NY], dy[NY];
  chol(Y, Ly, dy);
  // Yh = Ly^{-1} H A_s; J and the A update share it
  T Yh[NY][N];
  mm(st.H, s.A, Yh);
  trsm_lower(Ly, dy, Yh);
  T Jn[N][N];
  mtm_sym(Yh, Yh, Jn);
  // eta: Yh^T Ly^{-1} (e - H b_s)
  T e[NY], w[NY], Hb[NY];
  mv(st.H, s.b, Hb);
#pragma unroll
  for (int a = 0; a < NY; ++a) {
    e[a] = y[a] - st.r[a];
    w[a] = e[a] - Hb[a];
  }
  trsv_lower(Ly, dy, w);
  T en[N];
  mtv(Yh, w, en);
  // b: u = b_s + K D e,  M u = u - K Y^{-1} H u
  T De[NY], u[N];
  mv(st.Rinv, e, De);
#pragma unroll
  for (int a = 0; a < NY; ++a) De[a] *= dt;
  mv(K, De, u);
#pragma unroll
  for (int i = 0; i < N; ++i) u[i] += s.b[i];
  T zu[NY], Ku[N];
  mv(st.H, u, zu);
  trsv_lower(Ly, dy, zu);
  trsv_upper_t(Ly, dy, zu);
  mv(K, zu, Ku);
  T Mu[N];
#pragma unroll
  for (int i = 0; i < N; ++i) Mu[i] = u[i] - Ku[i];
  // A: A_s - K Ly^{-T} Yh
  trsm_upper_t(Ly, dy, Yh);  // Yh <- Y^{-1} H A_s
  T KX[N][N], MA[N][N];
  mm(K, Yh, KX);
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) MA[i][j] = s.A[i][j] - KX[i][j];
  // C: M C_s = C_s - K Y^{-1} K^T in Joseph form Pi C_s Pi^T + Kg (R/dt) Kg^T
  // with Kg = K Y^{-1}, Pi = I - Kg H (a sum of PSD terms: no cancellation
  // where C_s is ill-conditioned)
  T Kgt[NY][N];  // Kg^T = Y^{-1} K^T
#pragma unroll
  for (int a = 0; a < NY; ++a)
#pragma unroll
    for (int i = 0; i < N; ++i) Kgt[a][i] = K[i][a];
  trsm_lower(Ly, dy, Kgt);
  trsm_upper_t(Ly, dy, Kgt);
  T Pi[N][N], MC[N][N];
  mtm(Kgt, st.H, Pi);
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) Pi[i][j] = (i == j ? T(1) : T(0)) - Pi[i][j];
  {
    T PC[N][N], RK[NY][N], KRK[N][N];
    mm(Pi, s.C, PC);
    mmt_sym(PC, Pi, MC);
    mm(st.R, Kgt, RK);
    mtm_sym(Kgt, RK, KRK);
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) MC[i][j] = fma_(KRK[i][j], rdt, MC[i][j]);
  }
  // outer factor A_f = I - dt F:  A_f X = X - dt F X
  T FX[N][N], FMC[N][N], Fm[N];
  mm(st.F, MA, FX);
  mm(st.F, MC, FMC);
  mv(st.F, Mu, Fm);
  T AMC[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    s.b[i] = fma_(-dt, Fm[i] + st.c[i], Mu[i]);
    s.eta[i] = en[i] + s.eta[i];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      s.A[i][j] = fma_(-dt, FX[i][j], MA[i][j]);
      AMC[i][j] = fma_(-dt, FMC[i][j], MC[i][j]);
      s.J[i][j] = Jn[i][j] + s.J[i][j];
    }
  }
  // C = AMC A_f^T + V V^T = AMC - dt AMC F^T + V V^T
  T AMCF[N][N], VV[N][N];
  mmt(AMC, st.F, AMCF);
  mmt_sym(st.V, st.V, VV);
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      const T c = fma_(-dt, AMCF[i][j], AMC[i][j]) + VV[i][j];
      s.C[i][j] = c;
      s.C[j][i] = c;
    }
}

// Two-filter estimate of one state from its forward value function (S, v)
// and the run s of the steps after it.  Eq. twofilter minimises s over the
// far end z first, x = (I + Cbar S)^{-1} (bbar + Cbar v) with
// Cbar = A J^{-1} A^T + C and bbar = A J^{-1} eta + b; J is singular near a
// segment's end, so the joint minimum over (x, z) of
// 1/2 x^T S x - x^T v + V_s(z, x) is taken instead, eliminating x first:
//   x = beta + G z,  G = (I + C S)^{-1} A,  beta = (I + C S)^{-1} (b + C v)
//   Shat z = vhat,   Shat = J + A^T S (I + C S)^{-1} A,  vhat = eta + A^T (v - S beta)
// ((Shat, vhat) is (S, v) carried through s: the filter at the segment's
// last state).  The same elimination applied to d(x, z)/dv gives the
// smoothed covariance P = Lam + G Shat^{-1} G^T, Lam = (I + C S)^{-1} C.
// Where J is invertible this equals eq. twofilter exactly.
template <typename T, int N, bool kCov>
MS_DEV void two_filter_point(const T (&S)[N][N], const T (&v)[N], const Elem<T, N>& s, T (&x)[N],
                             T (&P)[N][N]) {
  T X[N][N], Mi[N][N];
  mm(s.C, S, X);
#pragma unroll
  for (int i = 0; i < N; ++i) X[i][i] += T(1);
  inv(X, Mi);  // det(I + C S) >= 1
  T G[N][N];
  mm(Mi, s.A, G);
  T u[N], beta[N];
  mv(s.C, v, u);
#pragma unroll
  for (int i = 0; i < N; ++i) u[i] += s.b[i];
  mv(Mi, u, beta);
  T SG[N][N], Sh[N][N];
  mm(S, G, SG);
  mtm_symavg(s.A, SG, Sh);
  T Sb[N], w[N], vh[N];
  mv(S, beta, Sb);
#pragma unroll
  for (int i = 0; i < N; ++i) w[i] = v[i] - Sb[i];
  mtv(s.A, w, vh);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    vh[i] += s.eta[i];
#pragma unroll
    for (int j = 0; j < N; ++j) Sh[i][j] += s.J[i][j];
  }
  T Ls[N][N], ds[N];
  chol(Sh, Ls, ds);
  trsv_lower(Ls, ds, vh);
  trsv_upper_t(Ls, ds, vh);  // vh <- z
  T Gz[N];
  mv(G, vh, Gz);
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] = beta[i] + Gz[i];
  if constexpr (kCov) {
    T Lam[N][N];
    mmt_symavg(Mi, s.C, Lam);  // (I + C S)^{-1} C, symmetric in exact arithmetic
    T Yg[N][N];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) Yg[i][j] = G[j][i];
    trsm_lower(Ls, ds, Yg);
    T GG[N][N];
    mtm_sym(Yg, Yg, GG);
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) P[i][j] = Lam[i][j] + GG[i][j];
  }
}

// Segmented product for a reverse scan whose runs must stop at segment
// starts: (P, f) is the run from a position up to the first segment start
// at or after it (exclusive) and f whether one occurred.  (P, f) of a range X
// followed by a range Y: f = f_X | f_Y, P = f_X ? P_X : P_X . P_Y.
template <typename T, int N>
MS_DEV void seg_append(Elem<T, N>& P, T& f, const Elem<T, N>& Py, T fy) {
  if (f == T(0)) {
    Elem<T, N> t;
    combine(P, Py, t);
    P = t;
  }
  f = f > fy ? f : fy;
}

}  // namespace ms
