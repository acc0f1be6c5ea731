// Segment-local schedule of the fused step: one wavefront per segment.
//
// For a batch of many independent segments the flat schedule's cross-block
// machinery (lane prefixes in the workspace, block trees, last-block scans,
// three launches) is not needed: a wavefront can take a whole segment.  It
// walks the segment in rounds of 64 lanes x kRow consecutive states (one
// storage row of every lane per iteration, as in the flat schedule, so every
// access of the wavefront is one or two contiguous runs whatever the
// segment's alignment):
//
//   forward, round by round   each lane folds its states' elements (Sec. 4.1
//       rule), a wavefront scan gives its exclusive in-round prefix, the
//       filter (S, v) at the end of the previous round is carried through it
//       (Sec. 3.4 scan, information form of Sec. 2.5), and the lane runs the
//       information step through its states writing S_k, v_k and the
//       prediction-error likelihood terms;
//   backward, round by round from the last   each lane folds the trajectory
//       maps (G, beta, Lam) of its states (Sec. 4.3, eq. 42), a reverse
//       wavefront scan composes the maps after it, the value at the first
//       state of the following round is carried through them, and the lane
//       walks its states backwards writing x*_k, P^s_k and accumulating the
//       objective and the adjoint (traj_walk_state, as the flat trajectory
//       pass).
//
// Per-segment sums are reduced over the wavefront and stored by lane 0: no
// atomics, no zeroing, and the results do not depend on which wavefront took
// the segment.  The wavefronts are persistent: each takes the next segment
// from a queue ordered by decreasing length (k_seg_order, longest first, so
// that the longest segments do not start last) until the queue is empty;
// nothing waits on another wavefront.
#pragma once
#include "kernels.h"

namespace ms {

constexpr int kLenBuckets = 32;

// floor(log2(len + 1)), clamped to the bucket range
MS_DEVONLY int len_bucket(int64_t len) {
  const int b = 63 - __clzll(static_cast<unsigned long long>(len) + 1ull);
  return b < kLenBuckets ? b : kLenBuckets - 1;
}

// Queue of segments for k_seg_wave: order[0..n_seg) holds the segment ids by
// decreasing length bucket (within a bucket in any order); the queue counter
// is reset.  One block.
static __global__ void __launch_bounds__(kBlock) k_seg_order(const int64_t* seg_off, int64_t n_seg,
                                                      int* order, unsigned int* queue) {
  __shared__ unsigned int cnt[kLenBuckets], pos[kLenBuckets];
  if (threadIdx.x < kLenBuckets) cnt[threadIdx.x] = 0u;
  __syncthreads();
  for (int64_t s = threadIdx.x; s < n_seg; s += kBlock)
    atomicAdd(&cnt[len_bucket(seg_off[s + 1] - seg_off[s])], 1u);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned int acc = 0u;
    for (int b = kLenBuckets - 1; b >= 0; --b) {
      pos[b] = acc;
      acc += cnt[b];
    }
    *queue = 0u;
  }
  __syncthreads();
  for (int64_t s = threadIdx.x; s < n_seg; s += kBlock) {
    const unsigned int at = atomicAdd(&pos[len_bucket(seg_off[s + 1] - seg_off[s])], 1u);
    order[at] = int(s);
  }
}

struct SegOut {
  void* S;  // [Sym][n_states] tiled
  void* v;  // [N][n_states] tiled (the second filter plane)
  void* xs;
  void* Ps;  // optional
  double* loglik;
  double* obj;
  double* g_loglik;  // [n_seg][NTH]
  double* g_obj;
  const int* order;
  unsigned int* queue;
  unsigned int* status;  // MAP_CHECK_FINITE word, or null
};

MS_DEVONLY double wave_sum(double x) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) x += shfl(x, (threadIdx.x & (kWave - 1)) ^ d);
  return x;
}

template <typename TS, typename T, class M, bool kGrad, bool kCov>
__global__ void __launch_bounds__(kBlock) k_seg_wave(Prob<TS> p, SegOut o) {
  constexpr int N = M::NX, NY = M::NY, NW = M::NW;
  constexpr int NTH = M::NTH > 0 ? M::NTH : 1;
  constexpr int KV = 1 + 2 * NTH;
  using Cur = Cursor<TS, T, M>;
  using Raw = typename Cur::Raw;
  __shared__ __align__(16) T s_step[SharedStep<T, M>::n];
  const T* sstep = shared_step<TS, T, M>(p, s_step);
  const int lane = threadIdx.x & (kWave - 1);
  TS* So = static_cast<TS*>(o.S);
  TS* vo = static_cast<TS*>(o.v);
  TS* xo = static_cast<TS*>(o.xs);
  TS* Po = static_cast<TS*>(o.Ps);
  const bool want_ll = o.loglik != nullptr;
  const bool want_obj = o.obj != nullptr;
  bool bad = false;
  for (;;) {
    int idx = 0;
    if (lane == 0) idx = int(atomicAdd(o.queue, 1u));
    idx = shfl(idx, 0);
    if (int64_t(idx) >= p.n_seg) break;
    Cur cur;
    cur.sstep = sstep;
    cur.s = o.order[idx];
    cur.load_seg(p);
    const int64_t head = cur.head, end = cur.next_head;
    const int64_t rounds = (end - head + kTile - 1) / kTile;

    // ---------------------------------------------------------------- forward
    T Sr[N][N], vr[N];
    mzero(Sr);
#pragma unroll
    for (int a = 0; a < N; ++a) vr[a] = T(0);
    double ll = 0.0;
    for (int64_t r = 0; r < rounds; ++r) {
      const int64_t j0 = head + r * kTile + int64_t(kRow) * lane;
      const int64_t j1 = j0 + kRow < end ? j0 + kRow : end;
      Elem<T, N> agg;
      elem_identity(agg);
      if (j0 < j1) {
        Raw rn;
        cur.fetch(p, j0, rn);
        drain_vmem();
        for (int64_t i = j0; i < j1; ++i) {
          const Raw rc = rn;
          cur.fetch(p, i + 1 < j1 ? i + 1 : i, rn);
          if (i == head) {
            T m0[N], P0i[N][N];
            cur.prior(p, agg.J, agg.eta, m0, P0i);
            cur.ift_prior(rc, agg.eta);
            mzero(agg.A);
            mzero(agg.C);
#pragma unroll
            for (int a = 0; a < N; ++a) agg.b[a] = T(0);
          } else {
            Step<T, N, NY, NW> st;
            cur.terms(p, i, rc, st);
            T y[NY];
            rc.meas(y);
            Fresh<T, N, NW> f;
            fresh_from_step(st, y, f);
            cur.adjust_fresh(p, i, rc, st, f);
            fold_fresh(agg, f);
          }
        }
      }
      // exclusive in-round prefix of the lane
      Elem<T, N> pre, tmp;
#pragma unroll 1  // one copy of the level body: keeps the kernel inside the instruction cache
      for (int d = 1; d < kWave; d <<= 1) {
        shfl_elem(pre, agg, lane >= d ? lane - d : lane);
        if (lane >= d) {
          combine(pre, agg, tmp);
          agg = tmp;
        }
      }
      shfl_elem(pre, agg, lane > 0 ? lane - 1 : 0);
      if (lane == 0) elem_identity(pre);
      T S[N][N], v[N];
      mcopy(Sr, S);
#pragma unroll
      for (int a = 0; a < N; ++a) v[a] = vr[a];
      carry_apply(S, v, pre);
      if (j0 < j1) {
        Raw rn;
        cur.fetch(p, j0, rn);
        drain_vmem();
        for (int64_t i = j0; i < j1; ++i) {
          const Raw rc = rn;
          cur.fetch(p, i + 1 < j1 ? i + 1 : i, rn);
          if (i == head) {
            T m0[N], P0i[N][N];
            cur.prior(p, S, v, m0, P0i);
            cur.ift_prior(rc, v);
          } else {
            Step<T, N, NY, NW> st;
            T y[NY];
            rc.meas(y);
            cur.terms(p, i, rc, st);
            Fresh<T, N, NW> f;
            fresh_from_step(st, y, f);
            cur.adjust_fresh(p, i, rc, st, f);
            T Sn[N][N], vn[N], Sp[N][N], G[N][N], beta[N], Lam[N][N];
            info_step<T, N, NW, false>(S, v, f, Sn, vn, Sp, G, beta, Lam);
            if (want_ll) {
              T vp[N];
#pragma unroll
              for (int a = 0; a < N; ++a) vp[a] = vn[a] - f.eta[a];
              ll += pred_loglik(Sp, vp, st, y) + cur.loglik_pad(st, p);
            }
            mcopy(Sn, S);
#pragma unroll
            for (int a = 0; a < N; ++a) v[a] = vn[a];
          }
          tstore_sym<TS, T, N>(So, Sym<N>::n, i, S);
          T vs[N];
          filter_plane_out<TS>(S, v, vs);
          tstore_vec<TS, T, N>(vo, N, i, vs);
          if (o.status) bad = bad | nonfinite_vd(vs, S);
        }
      }
      // the filter at the round's last state carries into the next round
      // (a round followed by another is full: its last state is lane 63's)
      if (r + 1 < rounds) {
        shfl_sym(Sr, S, kWave - 1);
        shfl_vec(vr, v, kWave - 1);
      }
    }

    // ---------------------------------------------------------------- backward
    struct Ahead {
      TS S[Sym<N>::n];
      TS v[N];
      Raw r;
    };
    // filter moments of state k and inputs of state k + 1 (clamped into the segment)
    auto load = [&](int64_t k, Ahead& q) {
      tload_raw(So, Sym<N>::n, k, q.S);
      tload_raw(vo, N, k, q.v);
      cur.fetch(p, k + 1 < end ? k + 1 : k, q.r);
    };
    double val[KV];
#pragma unroll
    for (int t = 0; t < KV; ++t) val[t] = 0.0;
    T xr[N], Pr[N][N];
#pragma unroll
    for (int a = 0; a < N; ++a) xr[a] = T(0);
    mzero(Pr);
    for (int64_t r = rounds - 1; r >= 0; --r) {
      const int64_t j0 = head + r * kTile + int64_t(kRow) * lane;
      const int64_t j1 = j0 + kRow < end ? j0 + kRow : end;
      Aff<T, N> sagg;
      aff_identity(sagg);
      if (j0 < j1) {
        Ahead qn;
        load(j0, qn);
        drain_vmem();
        for (int64_t i = j0; i < j1; ++i) {
          const Ahead q = qn;
          load(i + 1 < j1 ? i + 1 : i, qn);
          T S[N][N], v[N];
          sym_from_raw<TS, T, N>(q.S, S);
          vec_from_raw(q.v, v);
          filter_plane_in<TS>(S, v);
          T G[N][N], beta[N], Lam[N][N];
          if (i + 1 == end) {
            // the segment's last state: constant map (0, S^{-1} v, S^{-1})
            mzero(G);
            spd_inv(S, Lam);
            mv(Lam, v, beta);
          } else {
            Step<T, N, NY, NW> st;
            T y[NY];
            q.r.meas(y);
            cur.terms(p, i + 1, q.r, st);
            Fresh<T, N, NW> f;
            fresh_from_step(st, y, f);
            cur.adjust_fresh(p, i + 1, q.r, st, f);
            traj_map(S, v, f, G, beta, Lam);
          }
          aff_append(sagg, G, beta, Lam);
        }
      }
      // maps after the lane's states to the end of the round
      Aff<T, N> suf;
#pragma unroll 1  // one copy of the level body: keeps the kernel inside the instruction cache
      for (int d = 1; d < kWave; d <<= 1) {
        shfl_aff(suf, sagg, lane + d < kWave ? lane + d : lane);
        if (lane + d < kWave) aff_append(sagg, suf);
      }
      shfl_aff(suf, sagg, lane + 1 < kWave ? lane + 1 : lane);
      if (lane == kWave - 1) aff_identity(suf);
      T x[N], P[N][N];
#pragma unroll
      for (int a = 0; a < N; ++a) x[a] = xr[a];
      mcopy(Pr, P);
      aff_apply(suf, x, P);
      if (j0 < j1) {
        Ahead qn;
        load(j1 - 1, qn);
        drain_vmem();
        for (int64_t i = j1 - 1; i >= j0; --i) {
          const Ahead q = qn;
          load(i - 1 >= j0 ? i - 1 : i, qn);
          T S[N][N], v[N];
          sym_from_raw<TS, T, N>(q.S, S);
          vec_from_raw(q.v, v);
          filter_plane_in<TS>(S, v);
          traj_walk_state<TS, T, M, kGrad>(p, cur, i, S, v, q.r, want_obj, x, P, val);
          tstore_vec(xo, N, i, x);
          if constexpr (kCov) tstore_sym(Po, Sym<N>::n, i, P);
          if (o.status) bad = bad | (kCov ? nonfinite_vd(x, P) : nonfinite_v(x));
          if (i == head && want_obj) val[0] += prior_objective(p, cur, x);
        }
      }
      // the value at the round's first state (lane 0's) carries into the round before
      if (r > 0) {
        shfl_vec(xr, x, 0);
        shfl_sym(Pr, P, 0);
      }
    }
    // per-segment sums
    ll = wave_sum(ll);
#pragma unroll
    for (int t = 0; t < KV; ++t) val[t] = wave_sum(val[t]);
    if (lane == 0) {
      const int64_t s = cur.s;
      if (want_ll) o.loglik[s] = ll;
      if (want_obj) o.obj[s] = val[0];
      if constexpr (kGrad && M::NTH > 0) {
#pragma unroll
        for (int t = 0; t < NTH; ++t) {
          if (o.g_loglik) o.g_loglik[s * NTH + t] = val[1 + t];
          if (o.g_obj) o.g_obj[s * NTH + t] = val[1 + NTH + t];
        }
      }
    }
    if (o.status) bad = bad | nonfinite(ll) | nonfinite(val[0]);
  }
  if (o.status) report_nonfinite(o.status, bad);
}

}  // namespace ms
