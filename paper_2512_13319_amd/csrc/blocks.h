// Dense output of sub-stepped blocks (Blocked<M>): the filter and the MAP
// state at the interior substep times of every block.
//
// A block [t_{k-1}, t_k] of n substeps has the partial elements E_j of its
// first j substeps (the Euler integration of Cursor::Block stopped after j
// substeps).  The filter at substep j is the filter at the block's start
// carried through E_j (the scan's combination rule, Sec. 4.1, applied to the
// information form).  The MAP state inside the block follows the paper's
// first recovery method (Sec. 3.5 and Sec. 4.3): the closed-loop ODE of the
// optimal trajectory, whose control law uses the value function (the filter)
// at the same time, here in original time dx*/dt = (F + Q S) x* - Q v + c,
// integrated by explicit Euler backwards from x*_k at the block's end, each
// substep using the filter at its later end.
#pragma once
#include "kernels.h"

namespace ms {

struct DenseIO {
  const void* S;   // filter planes of the problem (block boundaries)
  const void* v;
  const void* xs;  // MAP states at the block boundaries
  void* xd;        // out, tiled [nx * (n_sub - 1)] per state
  void* Sd;        // out, tiled [sym * (n_sub - 1)] per state
  void* vd;        // out, tiled [nx * (n_sub - 1)] per state (the second filter plane)
};

template <typename TS, typename T, class M>
__global__ void __launch_bounds__(kBlock) k_dense(Prob<TS> p, DenseIO io) {
  constexpr int N = M::NX, NY = M::NY, NW = M::NW, NS = Sym<N>::n;
  using Cur = Cursor<TS, T, M>;
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= p.n_states) return;
  Cur cur;
  cur.init(p, i);
  if (cur.is_head(i)) return;
  const TS* Si = static_cast<const TS*>(io.S);
  const TS* vi = static_cast<const TS*>(io.v);
  const TS* xi = static_cast<const TS*>(io.xs);
  TS* xdo = static_cast<TS*>(io.xd);
  TS* Sdo = static_cast<TS*>(io.Sd);
  TS* vdo = static_cast<TS*>(io.vd);
  const int n = p.n_sub;
  const int CS = NS * (n - 1), CV = N * (n - 1);
  typename Cur::Raw r;
  cur.fetch(p, i, r);
  Step<T, N, NY, NW> st;
  cur.terms(p, i, r, st);
  T S0[N][N], v0[N];
  tload_sym(Si, NS, i - 1, S0);
  tload_vec(vi, N, i - 1, v0);
  filter_plane_in<TS>(S0, v0);
  typename Cur::Block blk;
  blk.begin(st, n);
  // filter at the interior substeps
  for (int j = 0; j + 1 < n; ++j) {
    T y[NY];
    cur.block_meas(p, i, j, y);
    blk.substep(st, y);
    Elem<T, N> e;
    mcopy(blk.A, e.A);
    mcopy(blk.C, e.C);
    mcopy(blk.J, e.J);
#pragma unroll
    for (int a = 0; a < N; ++a) {
      e.b[a] = blk.b[a];
      e.eta[a] = blk.eta[a];
    }
    T S[N][N], v[N];
    mcopy(S0, S);
#pragma unroll
    for (int a = 0; a < N; ++a) v[a] = v0[a];
    carry_apply(S, v, e);
    T vs[N];
    filter_plane_out<TS>(S, v, vs);
    tstore_sym(Sdo, CS, i, S, j * NS);
    tstore_vec(vdo, CV, i, vs, j * N);
  }
  // MAP state at the interior substeps, backwards from the block's end
  T x[N], S[N][N], v[N];
  tload_vec(xi, N, i, x);
  tload_sym(Si, NS, i, S);
  tload_vec(vi, N, i, v);
  filter_plane_in<TS>(S, v);
  for (int j = n - 1; j >= 1; --j) {
    // substep j ends at interior point j (component j - 1); (S, v) is the
    // filter at the later point j + 1
    T QS[N][N], d[N], Fx[N], QSx[N], Qv[N];
    mm(blk.Q, S, QS);
    mv(st.F, x, Fx);
    mv(QS, x, QSx);
    mv(blk.Q, v, Qv);
#pragma unroll
    for (int a = 0; a < N; ++a) {
      d[a] = Fx[a] + QSx[a] - Qv[a] + st.c[a];
      x[a] = fma_(-blk.h, d[a], x[a]);
    }
    tstore_vec(xdo, CV, i, x, (j - 1) * N);
    if (j > 1) {
      tload_sym(Sdo, CS, i, S, (j - 1) * NS);
      tload_vec(vdo, CV, i, v, (j - 1) * N);
      filter_plane_in<TS>(S, v);
    }
  }
}

}  // namespace ms
