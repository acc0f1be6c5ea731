// Scan kernels for gfx950.
//
// Work decomposition (all passes): the flat sequence of states of all
// segments (segment s owns states seg_off[s]+s .. seg_off[s+1]+s) is cut into
// chunks of L consecutive states, one chunk per lane; a 64-lane wavefront is a
// tile; a 256-thread block holds four independent tiles.
//
//   pass A  (filter up-sweep)     each lane folds its chunk's elements into one
//           element; a Hillis-Steele scan over the wavefront gives every lane
//           its exclusive in-tile prefix (stored); lane 63's inclusive value is
//           the tile aggregate (stored).  The block that finishes last scans
//           the tile aggregates and stores one (S, v) carry per tile.
//   pass B  (filter fix-up, fused with the trajectory up-sweep)  each lane
//           applies tile carry and in-tile prefix to get (S, v) before its
//           chunk, runs the information step through its chunk writing S_k,
//           v_k (and on request m_k, P_k and the prediction-error terms of the
//           log-likelihood), and with the same factorisation builds the
//           trajectory maps (G, beta, Lam) of its states and folds them.  A
//           reverse Hillis-Steele scan and a last-block reverse tile scan give
//           the value (x, P) after every tile.
//   pass C  (trajectory fix-up)   each lane gets (x, P) after its chunk and
//           walks backwards writing x*_k and P^s_k; the adjoint terms of the
//           log-likelihood and of the objective are accumulated on the way.
//
// Segment boundaries need no flags: a segment's first state carries the prior
// element (A = 0, C = 0), which cuts every run that contains it, and a
// segment's last state carries the constant trajectory map (0, S^{-1} v,
// S^{-1}), which cuts the reverse scan.
#pragma once
#include "counters.h"
#include "elements.h"

namespace ms {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kRow = 16;                     // storage: states per row of a tile
constexpr int64_t kTile = kWave * kRow;      // storage: states per tile

// Tiled storage layout of every state-indexed array with C components: tile
// (i / 1024) holds C blocks of 1024 values; inside a block, value of state i
// sits at (i % 16) * 64 + (i / 16) % 64.
//
// Work decomposition: lane g runs `chunk` consecutive states (chunk = 4, 8 or
// 16, a schedule parameter); 64 lanes form a work tile of 64 * chunk states.
// Iteration t of a wavefront then touches, per component, 64 / (16 / chunk)
// consecutive values in each of 16 / chunk rows: whole 128-byte lines (FP64)
// in every case, one 512-byte run at chunk 16.
MS_DEV int64_t tix(int64_t i, int64_t c, int64_t C) {
  return ((i >> 10) * C + c) * kTile + ((i & (kRow - 1)) << 6) + ((i >> 4) & (kWave - 1));
}

// One past the last state of lane g, whose states start at chunk * g: lane g
// runs chunk states, the sequence's last work lane also runs whatever follows
// (a short final work tile merged into the one before it; n_lanes counts work
// lanes), and a lane past the work lanes runs none (its range is empty even
// where chunk * g < n_states, i.e. in a merged final tile).
MS_DEV int64_t lane_end(int64_t g, int64_t n_lanes, int64_t n_states, int64_t chunk) {
  const int64_t j0 = g * chunk;
  if (g >= n_lanes || j0 >= n_states) return j0;
  if (g == n_lanes - 1) return n_states;
  return j0 + chunk < n_states ? j0 + chunk : n_states;
}

// Logical block of this workgroup.  Workgroups are dispatched to the eight
// XCDs round robin (workgroup b runs on XCD b % 8); the logical order gives
// each XCD one contiguous range of tiles, so that every XCD streams through
// contiguous memory instead of every eighth group of tiles of each array (a
// fixed stride that loaded some XCDs' memory traffic much more than others').
// A bijection of [0, gridDim.x).
MS_DEVONLY int64_t logical_block() {
  constexpr int64_t kXcd = 8;
  const int64_t b = blockIdx.x, nb = gridDim.x;
  const int64_t x = b % kXcd, k = b / kXcd, q = nb / kXcd, r = nb % kXcd;
  return x * q + (x < r ? x : r) + k;
}

// Wait for every outstanding vector memory operation.  Used once before each
// state loop: the compiler's waits inside a loop must hold for every path into
// the loop header, and loads still in flight from before the loop would
// otherwise make the wait of every iteration stricter than the loop itself
// needs (down to waiting for the previous state's stores).
MS_DEVONLY void drain_vmem() { __builtin_amdgcn_s_waitcnt(0); }

// Device-coherent (write-through) store: a relaxed agent-scope atomic store,
// which bypasses keeping the line dirty in the XCD's L2.  Used for everything a
// pass with a last-block tile scan writes before its blocks arrive: the
// agent-scope release fence of the arrival writes back every dirty line of the
// XCD's L2, and bulk outputs left dirty there made the last arrivals wait for
// megabytes of write-back.
template <typename P>
MS_DEVONLY void wt_store(P* p, P v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// store: plain or write-through
template <bool kWT, typename P>
MS_DEVONLY void put(P* p, P v) {
  if constexpr (kWT) wt_store(p, v); else *p = v;
}

template <int N> struct Sym { static constexpr int n = N * (N + 1) / 2; };
template <int N> struct ElemSz { static constexpr int n = N * N + 2 * N + 2 * Sym<N>::n; };
// Per-step cotangents of (A, b, C, R): N * N + N + Sym<N> + Sym<NY> values.
template <int N, int NY> struct ElemGradSz {
  static constexpr int n = N * N + N + Sym<N>::n + Sym<NY>::n;
};
template <int N> struct AffSz { static constexpr int n = N * N + N + Sym<N>::n; };

// --------------------------------------------------------------------------- SoA I/O
// A "plane set" stores component c of item i at base[c * ld + i].
template <typename T, int N, bool kWT = false>
MS_DEVONLY void store_sym(T* base, int64_t ld, int64_t i, const T (&a)[N][N], int c0 = 0) {
  int c = c0;
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int q = 0; q <= r; ++q) put<kWT>(&base[(c++) * ld + i], a[r][q]);
}
template <typename T, int N>
MS_DEVONLY void load_sym(const T* base, int64_t ld, int64_t i, T (&a)[N][N], int c0 = 0) {
  int c = c0;
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int q = 0; q <= r; ++q) {
      a[r][q] = base[(c++) * ld + i];
      a[q][r] = a[r][q];
    }
}
template <typename T, int N, bool kWT = false>
MS_DEVONLY void store_vec(T* base, int64_t ld, int64_t i, const T (&a)[N], int c0 = 0) {
#pragma unroll
  for (int r = 0; r < N; ++r) put<kWT>(&base[(c0 + r) * ld + i], a[r]);
}
template <typename T, int N>
MS_DEVONLY void load_vec(const T* base, int64_t ld, int64_t i, T (&a)[N], int c0 = 0) {
#pragma unroll
  for (int r = 0; r < N; ++r) a[r] = base[(c0 + r) * ld + i];
}
template <typename T, int N, int M, bool kWT = false>
MS_DEVONLY void store_mat(T* base, int64_t ld, int64_t i, const T (&a)[N][M], int c0 = 0) {
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int q = 0; q < M; ++q) put<kWT>(&base[(c0 + r * M + q) * ld + i], a[r][q]);
}
template <typename T, int N, int M>
MS_DEVONLY void load_mat(const T* base, int64_t ld, int64_t i, T (&a)[N][M], int c0 = 0) {
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int q = 0; q < M; ++q) a[r][q] = base[(c0 + r * M + q) * ld + i];
}

// tiled state-indexed I/O (C = components of the buffer, c0 = first one written)
// (P = storage type of the buffer, T = compute type of the registers)
template <typename P, typename T, int N, bool kWT = false>
MS_DEVONLY void tstore_sym(P* base, int C, int64_t i, const T (&a)[N][N], int c0 = 0) {
  int c = c0;
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int q = 0; q <= r; ++q) put<kWT>(&base[tix(i, c++, C)], P(a[r][q]));
}
template <typename P, typename T, int N>
MS_DEVONLY void tload_sym(const P* base, int C, int64_t i, T (&a)[N][N], int c0 = 0) {
  int c = c0;
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int q = 0; q <= r; ++q) {
      a[r][q] = T(base[tix(i, c++, C)]);
      a[q][r] = a[r][q];
    }
}
template <typename P, typename T, int N, bool kWT = false>
MS_DEVONLY void tstore_vec(P* base, int C, int64_t i, const T (&a)[N], int c0 = 0) {
#pragma unroll
  for (int r = 0; r < N; ++r) put<kWT>(&base[tix(i, c0 + r, C)], P(a[r]));
}
template <typename P, typename T, int N>
MS_DEVONLY void tload_vec(const P* base, int C, int64_t i, T (&a)[N], int c0 = 0) {
#pragma unroll
  for (int r = 0; r < N; ++r) a[r] = T(base[tix(i, c0 + r, C)]);
}
// raw components in the storage type (prefetch buffers), converted where used
template <typename P, int K>
MS_DEVONLY void tload_raw(const P* base, int C, int64_t i, P (&a)[K], int c0 = 0) {
#pragma unroll
  for (int r = 0; r < K; ++r) a[r] = base[tix(i, c0 + r, C)];
}
template <typename P, typename T, int N>
MS_DEVONLY void sym_from_raw(const P (&a)[Sym<N>::n], T (&m)[N][N]) {
  int c = 0;
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int q = 0; q <= r; ++q) {
      m[r][q] = T(a[c++]);
      m[q][r] = m[r][q];
    }
}
template <typename P, typename T, int K>
MS_DEVONLY void vec_from_raw(const P (&a)[K], T (&o)[K]) {
#pragma unroll
  for (int r = 0; r < K; ++r) o[r] = T(a[r]);
}
template <typename P, typename T, int N, int M>
MS_DEVONLY void tstore_mat(P* base, int C, int64_t i, const T (&a)[N][M], int c0 = 0) {
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int q = 0; q < M; ++q) base[tix(i, c0 + r * M + q, C)] = P(a[r][q]);
}

// The filter's second output plane.  FP64 storage keeps the information
// vector v = S m.  FP32 storage keeps the filter mean m instead: rounding v to
// FP32 perturbs it by about eps32 |S| |m|, and S^{-1} spreads that over every
// component of the mean, so a small component (a velocity near zero beside
// positions far from the origin) loses its relative precision; the rounded
// mean keeps each component's own.  Readers rebuild v = S m from the rounded
// S and m in the arithmetic type (then S^{-1} v is the stored mean up to
// arithmetic rounding).
template <typename TS>
constexpr bool kStoreMean = sizeof(TS) < sizeof(double);

// value to store in the plane for the state with information form (S, v)
template <typename TS, typename T, int N>
MS_DEVONLY void filter_plane_out(const T (&S)[N][N], const T (&v)[N], T (&o)[N]) {
#pragma unroll
  for (int r = 0; r < N; ++r) o[r] = v[r];
  if constexpr (kStoreMean<TS>) {
    T Ls[N][N], ds[N];
    chol(S, Ls, ds);
    trsv_lower(Ls, ds, o);
    trsv_upper_t(Ls, ds, o);
  }
}
// v from the stored plane value (in place) and the state's S
template <typename TS, typename T, int N>
MS_DEVONLY void filter_plane_in(const T (&S)[N][N], T (&v)[N]) {
  if constexpr (kStoreMean<TS>) {
    T m[N];
#pragma unroll
    for (int r = 0; r < N; ++r) m[r] = v[r];
    mv(S, m, v);
  }
}

// Per-lane workspace (the in-tile prefixes) is blocked by tile like the state
// arrays: component c of lane g sits at ((g / 64) * C + c) * 64 + g % 64, so a
// wavefront writes its own contiguous C * 512 bytes, one full 512-byte run per
// component.  (Component-major planes over all lanes made every wavefront
// write the same plane at the same moment.)
struct LaneTiled {
  int64_t C;  // components per lane
  MS_DEV int64_t at(int64_t g, int64_t c) const { return ((g >> 6) * C + c) * kWave + (g & (kWave - 1)); }
};
// kFlag: one more component after the element (the segment flag of the
// reverse scan of the two-filter smoother).
template <typename T, int N, bool kFlag = false>
MS_DEVONLY void lt_store_elem(T* base, int64_t g, const Elem<T, N>& e, T flag = T(0)) {
  const LaneTiled L{ElemSz<N>::n + (kFlag ? 1 : 0)};
  int c = 0;
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int q = 0; q < N; ++q) wt_store(&base[L.at(g, c++)], e.A[r][q]);
#pragma unroll
  for (int r = 0; r < N; ++r) wt_store(&base[L.at(g, c++)], e.b[r]);
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int q = 0; q <= r; ++q) wt_store(&base[L.at(g, c++)], e.C[r][q]);
#pragma unroll
  for (int r = 0; r < N; ++r) wt_store(&base[L.at(g, c++)], e.eta[r]);
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int q = 0; q <= r; ++q) wt_store(&base[L.at(g, c++)], e.J[r][q]);
  if constexpr (kFlag) wt_store(&base[L.at(g, c)], flag);
}
template <typename T, int N, bool kFlag = false>
MS_DEVONLY void lt_load_elem(const T* base, int64_t g, Elem<T, N>& e, T* flag = nullptr) {
  const LaneTiled L{ElemSz<N>::n + (kFlag ? 1 : 0)};
  int c = 0;
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int q = 0; q < N; ++q) e.A[r][q] = base[L.at(g, c++)];
#pragma unroll
  for (int r = 0; r < N; ++r) e.b[r] = base[L.at(g, c++)];
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int q = 0; q <= r; ++q) { e.C[r][q] = base[L.at(g, c++)]; e.C[q][r] = e.C[r][q]; }
#pragma unroll
  for (int r = 0; r < N; ++r) e.eta[r] = base[L.at(g, c++)];
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int q = 0; q <= r; ++q) { e.J[r][q] = base[L.at(g, c++)]; e.J[q][r] = e.J[r][q]; }
  if constexpr (kFlag) *flag = base[L.at(g, c)];
}
template <typename T, int N>
MS_DEVONLY void lt_store_aff(T* base, int64_t g, const Aff<T, N>& a) {
  const LaneTiled L{AffSz<N>::n};
  int c = 0;
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int q = 0; q < N; ++q) wt_store(&base[L.at(g, c++)], a.Phi[r][q]);
#pragma unroll
  for (int r = 0; r < N; ++r) wt_store(&base[L.at(g, c++)], a.bt[r]);
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int q = 0; q <= r; ++q) wt_store(&base[L.at(g, c++)], a.Om[r][q]);
}
template <typename T, int N>
MS_DEVONLY void lt_load_aff(const T* base, int64_t g, Aff<T, N>& a) {
  const LaneTiled L{AffSz<N>::n};
  int c = 0;
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int q = 0; q < N; ++q) a.Phi[r][q] = base[L.at(g, c++)];
#pragma unroll
  for (int r = 0; r < N; ++r) a.bt[r] = base[L.at(g, c++)];
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int q = 0; q <= r; ++q) { a.Om[r][q] = base[L.at(g, c++)]; a.Om[q][r] = a.Om[r][q]; }
}

// element planes: A (N*N), b (N), C (sym), eta (N), J (sym)
template <typename T, int N, bool kWT = false>
MS_DEVONLY void store_elem(T* base, int64_t ld, int64_t i, const Elem<T, N>& e) {
  store_mat<T, N, N, kWT>(base, ld, i, e.A, 0);
  store_vec<T, N, kWT>(base, ld, i, e.b, N * N);
  store_sym<T, N, kWT>(base, ld, i, e.C, N * N + N);
  store_vec<T, N, kWT>(base, ld, i, e.eta, N * N + N + Sym<N>::n);
  store_sym<T, N, kWT>(base, ld, i, e.J, N * N + 2 * N + Sym<N>::n);
}
template <typename T, int N>
MS_DEVONLY void load_elem(const T* base, int64_t ld, int64_t i, Elem<T, N>& e) {
  load_mat(base, ld, i, e.A, 0);
  load_vec(base, ld, i, e.b, N * N);
  load_sym(base, ld, i, e.C, N * N + N);
  load_vec(base, ld, i, e.eta, N * N + N + Sym<N>::n);
  load_sym(base, ld, i, e.J, N * N + 2 * N + Sym<N>::n);
}
template <typename T, int N, bool kWT = false>
MS_DEVONLY void store_aff(T* base, int64_t ld, int64_t i, const Aff<T, N>& a) {
  store_mat<T, N, N, kWT>(base, ld, i, a.Phi, 0);
  store_vec<T, N, kWT>(base, ld, i, a.bt, N * N);
  store_sym<T, N, kWT>(base, ld, i, a.Om, N * N + N);
}
template <typename T, int N>
MS_DEVONLY void load_aff(const T* base, int64_t ld, int64_t i, Aff<T, N>& a) {
  load_mat(base, ld, i, a.Phi, 0);
  load_vec(base, ld, i, a.bt, N * N);
  load_sym(base, ld, i, a.Om, N * N + N);
}

template <typename T, int N>
MS_DEVONLY void shfl_elem(Elem<T, N>& o, const Elem<T, N>& e, int src) {
  shfl_mat(o.A, e.A, src);
  shfl_vec(o.b, e.b, src);
  shfl_sym(o.C, e.C, src);
  shfl_vec(o.eta, e.eta, src);
  shfl_sym(o.J, e.J, src);
}
// Sources of the earlier element for combine_into.
// ShflSrc: lane `src`'s element e through shuffles, or the identity element
// where !act (combining with the identity changes nothing, exactly).  Every
// lane of the wavefront must run the combination, as each shuffle reads all
// lanes.
template <typename T, int N>
struct ShflSrc {
  const Elem<T, N>& e;
  int src;
  bool act;
  MS_DEVONLY void get_A(T (&a)[N][N]) const {
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
      for (int q = 0; q < N; ++q) {
        const T x = shfl(e.A[r][q], src);
        a[r][q] = act ? x : (r == q ? T(1) : T(0));
      }
  }
  MS_DEVONLY void get_b(T (&b)[N]) const {
#pragma unroll
    for (int r = 0; r < N; ++r) {
      const T x = shfl(e.b[r], src);
      b[r] = act ? x : T(0);
    }
  }
  MS_DEVONLY void get_eta(T (&b)[N]) const {
#pragma unroll
    for (int r = 0; r < N; ++r) {
      const T x = shfl(e.eta[r], src);
      b[r] = act ? x : T(0);
    }
  }
  MS_DEVONLY void sym(const T (&m)[N][N], T (&a)[N][N]) const {
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
      for (int q = 0; q <= r; ++q) {
        const T x = shfl(m[r][q], src);
        a[r][q] = act ? x : T(0);
        a[q][r] = a[r][q];
      }
  }
  MS_DEVONLY void get_C(T (&a)[N][N]) const { sym(e.C, a); }
  MS_DEVONLY void get_J(T (&a)[N][N]) const { sym(e.J, a); }
};
// BulkSrc: lane `src`'s element shuffled whole, in one burst, into registers
// (the identity where !act); for kernels with registers to spare, where the
// field-by-field shuffles of ShflSrc would only add latency.
template <typename T, int N>
struct BulkSrc {
  Elem<T, N> e;
  MS_DEVONLY BulkSrc(const Elem<T, N>& from, int src, bool act) {
    shfl_elem(e, from, src);
    if (!act) elem_identity(e);
  }
  MS_DEVONLY void get_A(T (&a)[N][N]) const { mcopy(e.A, a); }
  MS_DEVONLY void get_b(T (&b)[N]) const {
#pragma unroll
    for (int r = 0; r < N; ++r) b[r] = e.b[r];
  }
  MS_DEVONLY void get_eta(T (&b)[N]) const {
#pragma unroll
    for (int r = 0; r < N; ++r) b[r] = e.eta[r];
  }
  MS_DEVONLY void get_C(T (&a)[N][N]) const { mcopy(e.C, a); }
  MS_DEVONLY void get_J(T (&a)[N][N]) const { mcopy(e.J, a); }
};
// The source of a wavefront-scan partner: bulk where registers allow it.
template <typename T, int N, bool kBulk>
MS_DEVONLY void scan_step(Elem<T, N>& agg, int src, bool act) {
  if constexpr (kBulk) {
    combine_into(BulkSrc<T, N>(agg, src, act), agg);
  } else {
    combine_into(ShflSrc<T, N>{agg, src, act}, agg);
  }
}

// PackedSrc: an element in the packed layout of pack_elem (LDS).
template <typename T, int N>
struct PackedSrc {
  const T* w;
  MS_DEVONLY void get_A(T (&a)[N][N]) const {
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
      for (int q = 0; q < N; ++q) a[r][q] = w[r * N + q];
  }
  MS_DEVONLY void get_b(T (&b)[N]) const {
#pragma unroll
    for (int r = 0; r < N; ++r) b[r] = w[N * N + r];
  }
  MS_DEVONLY void sym(int o, T (&a)[N][N]) const {
    int c = o;
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
      for (int q = 0; q <= r; ++q) {
        a[r][q] = w[c++];
        a[q][r] = a[r][q];
      }
  }
  MS_DEVONLY void get_C(T (&a)[N][N]) const { sym(N * N + N, a); }
  MS_DEVONLY void get_eta(T (&b)[N]) const {
#pragma unroll
    for (int r = 0; r < N; ++r) b[r] = w[N * N + N + Sym<N>::n + r];
  }
  MS_DEVONLY void get_J(T (&a)[N][N]) const { sym(N * N + 2 * N + Sym<N>::n, a); }
};

// element <-> ElemSz contiguous values (LDS staging)
template <typename T, int N>
MS_DEVONLY void pack_elem(T* w, const Elem<T, N>& e) {
  int c = 0;
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int q = 0; q < N; ++q) w[c++] = e.A[r][q];
#pragma unroll
  for (int r = 0; r < N; ++r) w[c++] = e.b[r];
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int q = 0; q <= r; ++q) w[c++] = e.C[r][q];
#pragma unroll
  for (int r = 0; r < N; ++r) w[c++] = e.eta[r];
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int q = 0; q <= r; ++q) w[c++] = e.J[r][q];
}
template <typename T, int N>
MS_DEVONLY void unpack_elem(const T* w, Elem<T, N>& e) {
  int c = 0;
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int q = 0; q < N; ++q) e.A[r][q] = w[c++];
#pragma unroll
  for (int r = 0; r < N; ++r) e.b[r] = w[c++];
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int q = 0; q <= r; ++q) { e.C[r][q] = w[c++]; e.C[q][r] = e.C[r][q]; }
#pragma unroll
  for (int r = 0; r < N; ++r) e.eta[r] = w[c++];
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int q = 0; q <= r; ++q) { e.J[r][q] = w[c++]; e.J[q][r] = e.J[r][q]; }
}
template <typename T, int N>
MS_DEVONLY void pack_aff(T* w, const Aff<T, N>& a) {
  int c = 0;
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int q = 0; q < N; ++q) w[c++] = a.Phi[r][q];
#pragma unroll
  for (int r = 0; r < N; ++r) w[c++] = a.bt[r];
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int q = 0; q <= r; ++q) w[c++] = a.Om[r][q];
}
template <typename T, int N>
MS_DEVONLY void unpack_aff(const T* w, Aff<T, N>& a) {
  int c = 0;
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int q = 0; q < N; ++q) a.Phi[r][q] = w[c++];
#pragma unroll
  for (int r = 0; r < N; ++r) a.bt[r] = w[c++];
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int q = 0; q <= r; ++q) { a.Om[r][q] = w[c++]; a.Om[q][r] = a.Om[r][q]; }
}
template <typename T, int N>
MS_DEVONLY void shfl_aff(Aff<T, N>& o, const Aff<T, N>& a, int src) {
  shfl_mat(o.Phi, a.Phi, src);
  shfl_vec(o.bt, a.bt, src);
  shfl_sym(o.Om, a.Om, src);
}

// --------------------------------------------------------------------------- workspace
// Pointers into the caller's workspace; sizes fixed by (n_states, L, N).
template <typename T>
struct Ws {
  unsigned int* counters;  // two sets of arrival counters (filter, trajectory), zero between launches
  T* lane_pre;             // lane-tiled [ElemSz] per lane: exclusive in-tile filter prefix
  T* tile_agg;             // [ElemSz][n_blocks]  block aggregates
  T* tile_carry;           // [Sym + N][n_blocks]  (S, v) before each block of four tiles
  T* tile_pre;             // [ElemSz][n_tiles]  exclusive prefix of each tile inside its block
  T* stile_suf;            // [AffSz][n_tiles]  trajectory map from after each tile to the end of its block
  T* slane_pre;            // lane-tiled [AffSz] per lane: trajectory map from after the lane's chunk to tile end
  T* stile_agg;            // [AffSz][n_tiles]
  T* stile_carry;          // [N + Sym][n_tiles]  (x, P) after each tile
  T* lane_half;            // split schedule: lane-tiled [ElemSz] per filter up-sweep lane, fold of its first half
  int64_t n_lanes, n_tiles;
  int64_t chunk;           // states per lane
  // the filter up-sweep's decomposition (the same unless the schedule is
  // split, see later_chunk): its lane g1 holds the start of lane g >> k1_shift
  int64_t n_lanes1, n_tiles1, chunk1;
  int k1_shift;
  // 1: the filter up-sweep's last block scans the block aggregates into
  // tile_carry; 0: tile_carry already holds those carries (a checkpoint of an
  // earlier forward pass on the same problem and schedule), and the up-sweep
  // only rebuilds the lane and tile prefixes inside each block
  int up_tail;
  unsigned int* status;    // MAP_CHECK_FINITE: set to 1 when a non-finite value is written; else null
};

// Non-finite test on the bits.  The library is built with -ffinite-math-only,
// under which a floating-point test (and the same exponent test on the bits,
// which the compiler recognises) may be folded to false; the empty asm hides
// where the bits came from.
MS_DEVONLY bool nonfinite(double x) {
  uint64_t u = __builtin_bit_cast(uint64_t, x);
  asm volatile("" : "+v"(u));
  return (u & 0x7ff0000000000000ull) == 0x7ff0000000000000ull;
}
MS_DEVONLY bool nonfinite(float x) {
  uint32_t u = __builtin_bit_cast(uint32_t, x);
  asm volatile("" : "+v"(u));
  return (u & 0x7f800000u) == 0x7f800000u;
}
// a vector and the diagonal of a matrix (a non-finite entry anywhere in a
// state's moments reaches these within a step)
template <typename T, int N>
MS_DEVONLY bool nonfinite_vd(const T (&v)[N], const T (&m)[N][N]) {
  bool b = false;
#pragma unroll
  for (int r = 0; r < N; ++r) b = b | nonfinite(v[r]) | nonfinite(m[r][r]);
  return b;
}
template <typename T, int N>
MS_DEVONLY bool nonfinite_v(const T (&v)[N]) {
  bool b = false;
#pragma unroll
  for (int r = 0; r < N; ++r) b = b | nonfinite(v[r]);
  return b;
}
MS_DEVONLY void report_nonfinite(unsigned int* status, bool bad) {
  if (status != nullptr && bad) atomicOr(status, 1u);
}

// Per-segment accumulators (double): loglik [n_seg], obj [n_seg],
// g_loglik [n_seg][NTH], g_obj [n_seg][NTH].
struct Acc {
  double* loglik;
  double* obj;
  double* g_loglik;
  double* g_obj;
};

// --------------------------------------------------------------------------- model access
// TS: storage type of the problem's arrays; T: compute type.
template <typename TS, typename T, class M>
struct Cursor {
  static constexpr int NX = M::NX, NY = M::NY, NW = M::NW;
  static constexpr int NTH_ = M::NTH > 0 ? M::NTH : 1;
  int64_t s;          // current segment
  int64_t head;       // its first state
  int64_t next_head;  // first state of the next segment (n_states after the last)
  T th[NTH_];
  const T* sstep = nullptr;  // general linear model, every term shared: the step's terms in LDS

  MS_DEVONLY void load_seg(const Prob<TS>& p) {
    head = p.seg_off[s] + s;
    next_head = p.seg_off[s + 1] + s + 1;
    if constexpr (M::NTH > 0) {
#pragma unroll
      for (int t = 0; t < M::NTH; ++t) th[t] = T(p.theta[s * p.th_stride + t]);
    }
    // Every later state uses these values.  Loaded in a branch that runs only
    // when the segment changes, they would count as possibly outstanding at
    // every iteration of the state loops, and the compiler would then wait for
    // all vector memory operations (the prefetched inputs and the stores of
    // the previous state included) before each state.  Waiting here, once per
    // segment, keeps that wait out of the loops.
    __builtin_amdgcn_s_waitcnt(0);
  }
  // segment containing state i (0 <= i < n_states)
  MS_DEVONLY void init(const Prob<TS>& p, int64_t i) {
    int64_t lo = 0, hi = p.n_seg - 1;
    while (lo < hi) {
      int64_t mid = (lo + hi + 1) >> 1;
      if (p.seg_off[mid] + mid <= i) lo = mid; else hi = mid - 1;
    }
    s = lo;
    load_seg(p);
  }
  MS_DEVONLY void next(const Prob<TS>& p) { ++s; load_seg(p); }
  MS_DEVONLY void prev(const Prob<TS>& p) { --s; load_seg(p); }
  MS_DEVONLY bool is_head(int64_t i) const { return i == head; }
  MS_DEVONLY bool is_last(int64_t i) const { return i + 1 == next_head; }

  // The per-state inputs of the step that ends at state i (measurement, step
  // length, linearisation state).  Loads only, so that a loop can issue them
  // ahead of their use; valid for any i < n_states (the values of a segment's
  // first state are simply not used).  They stay in the storage type until
  // used: a conversion on arrival would make the loop wait for the load there,
  // and would double the registers of FP32 storage.
  struct Raw {
    TS dt;
    TS y[NY];
    TS xb[M::kNonlinear ? NX : 1];
    TS g[M::kIft ? NX : 1];  // cotangent of x* at the state (adjoint problem)
    MS_DEVONLY void meas(T (&o)[NY]) const {
#pragma unroll
      for (int c = 0; c < NY; ++c) o[c] = T(y[c]);
    }
  };
  MS_DEVONLY void fetch(const Prob<TS>& p, int64_t i, Raw& r) const {
    r.dt = p.dt_stride ? p.dt[tix(i, 0, 1)] : p.dt[0];
    if constexpr (M::kPadded) {
      // measurements beyond the problem's ny are padding (zero)
#pragma unroll
      for (int c = 0; c < NY; ++c) r.y[c] = c < p.ny_in ? p.y[tix(i, c, p.ny_in)] : TS(0);
    } else {
#pragma unroll
      for (int c = 0; c < NY; ++c) r.y[c] = p.y[tix(i, c, NY)];
    }
    if constexpr (M::kNonlinear) {
#pragma unroll
      for (int c = 0; c < NX; ++c) r.xb[c] = p.xbar[tix(i, c, NX)];
    }
    if constexpr (M::kIft) {
#pragma unroll
      for (int c = 0; c < NX; ++c) r.g[c] = p.gx[tix(i, c, NX)];
    }
  }

  // Changes to the fresh element of the step that ends at state i (its
  // fetched inputs r, terms st):
  //  - sub-stepped blocks (Blocked<M>, n_sub > 1): the element of the block
  //    integrated over its substeps (block_fresh) replaces the one-step one;
  //  - MAP_OM_DIVERGENCE with a state-dependent divergence: the Newton
  //    expansion of 1/2 dt div f about xbar (M::div_newton);
  //  - adjoint problem (Ift<M>): b = 0 and eta = g there (the prior's eta is g
  //    at the segment's first state, ift_prior).
  // No-ops otherwise.
  template <int NW_>
  MS_DEVONLY void adjust_fresh(const Prob<TS>& p, int64_t i, const Raw& r,
                               const Step<T, NX, NY, NW_>& st, Fresh<T, NX, NW_>& f) const {
    if constexpr (M::kBlocked) {
      if (p.n_sub > 1) block_fresh(p, i, st, f);
    }
    if constexpr (M::kDivNewton) {
      if (p.om_div) {
        T xb[NX];
#pragma unroll
        for (int c = 0; c < NX; ++c) xb[c] = T(r.xb[c]);
        M::div_newton(th, xb, T(r.dt), f.J, f.eta);
      }
    }
    if constexpr (M::kIft) {
#pragma unroll
      for (int c = 0; c < NX; ++c) {
        f.b[c] = T(0);
        f.eta[c] = T(r.g[c]);
      }
    }
  }

  // Element of a block of n_sub explicit-Euler substeps of length h = dt /
  // n_sub of the element ODE (Sec. 4.2, eq. backwardLQT, written in original
  // time, with the A equation read as A' = -A (Q J + F)), from the boundary
  // value (I, 0, 0, 0, 0); substep j uses the measurement at its end
  // (component j * NY + c of y at the block's last state):
  //   A' = -A (Q J + F)               b' = A (Q eta - c)      C' = A Q A^T
  //   eta' = -F^T eta - J Q eta + J c + H^T R^{-1} (y_j - r)
  //   J' = -F^T J - J F - J Q J + H^T R^{-1} H.
  // One substep reproduces the one-step element.  Substeps 1..k give the
  // block's partial element up to its k-th substep (Euler, the dense output).
  struct Block {
    T A[NX][NX], b[NX], C[NX][NX], eta[NX], J[NX][NX];
    T Q[NX][NX], HRH[NX][NX], RH[NY][NX], h;
    template <int NW_>
    MS_DEVONLY void begin(const Step<T, NX, NY, NW_>& st, int n) {
      h = st.dt * rcp(T(n));
      const T rdt = rcp(st.dt);
      mmt_sym(st.V, st.V, Q);
#pragma unroll
      for (int a = 0; a < NX; ++a)
#pragma unroll
        for (int q = 0; q < NX; ++q) Q[a][q] *= rdt;
      mm(st.Rinv, st.H, RH);
      mtm_sym(st.H, RH, HRH);
      meye(A);
      mzero(C);
      mzero(J);
#pragma unroll
      for (int a = 0; a < NX; ++a) b[a] = eta[a] = T(0);
    }
    template <int NW_>
    MS_DEVONLY void substep(const Step<T, NX, NY, NW_>& st, const T (&y)[NY]) {
      T e[NY], g[NX];
#pragma unroll
      for (int c = 0; c < NY; ++c) e[c] = y[c] - st.r[c];
      mtv(RH, e, g);  // H^T R^{-1} (y - r)
      T QJ[NX][NX], QJF[NX][NX], dA[NX][NX], AQ[NX][NX], dC[NX][NX];
      mm(Q, J, QJ);
#pragma unroll
      for (int a = 0; a < NX; ++a)
#pragma unroll
        for (int q = 0; q < NX; ++q) QJF[a][q] = QJ[a][q] + st.F[a][q];
      mm(A, QJF, dA);
      mm(A, Q, AQ);
      mmt_sym(AQ, A, dC);
      T Qe[NX], db[NX];
      mv(Q, eta, Qe);
#pragma unroll
      for (int a = 0; a < NX; ++a) Qe[a] -= st.c[a];
      mv(A, Qe, db);
      T Fe[NX], JQe[NX], Jc[NX], JQ[NX][NX], JQJ[NX][NX], FJ[NX][NX];
      mtv(st.F, eta, Fe);
      mtv(QJ, eta, JQe);  // (Q J)^T eta = J Q eta
      mv(J, st.c, Jc);
      mtm(QJ, J, JQJ);    // J Q J
      mtm(st.F, J, FJ);   // F^T J
#pragma unroll
      for (int a = 0; a < NX; ++a) {
        b[a] = fma_(h, db[a], b[a]);
        eta[a] += h * (g[a] + Jc[a] - Fe[a] - JQe[a]);
      }
      T Jn[NX][NX];
#pragma unroll
      for (int a = 0; a < NX; ++a)
#pragma unroll
        for (int q = 0; q < NX; ++q) {
          A[a][q] = fma_(-h, dA[a][q], A[a][q]);
          C[a][q] = fma_(h, dC[a][q], C[a][q]);
          // -F^T J - J F = -(F^T J) - (F^T J)^T
          Jn[a][q] = J[a][q] + h * (HRH[a][q] - FJ[a][q] - FJ[q][a] - JQJ[a][q]);
        }
      mcopy(Jn, J);
      (void)JQ;
    }
  };
  MS_DEVONLY void block_meas(const Prob<TS>& p, int64_t i, int j, T (&y)[NY]) const {
    const int C = NY * p.n_sub;
#pragma unroll
    for (int c = 0; c < NY; ++c) y[c] = T(p.y[tix(i, j * NY + c, C)]);
  }
  template <int NW_>
  MS_DEVONLY void block_fresh(const Prob<TS>& p, int64_t i, const Step<T, NX, NY, NW_>& st,
                              Fresh<T, NX, NW_>& f) const {
    static_assert(NW_ == NX, "a block's noise factor is NX wide");
    Block blk;
    blk.begin(st, p.n_sub);
    for (int j = 0; j < p.n_sub; ++j) {
      T y[NY];
      block_meas(p, i, j, y);
      blk.substep(st, y);
    }
    mcopy(blk.A, f.A);
    mcopy(blk.J, f.J);
#pragma unroll
    for (int a = 0; a < NX; ++a) {
      f.b[a] = blk.b[a];
      f.eta[a] = blk.eta[a];
    }
    psd_factor(blk.C, f.V);
  }
  // ModelLinearPadded: each padded measurement component adds
  // -1/2 (log 2 pi - log dt) to the prediction-error log-likelihood of a step
  // (innovation 0, variance 1/dt, uncorrelated with the rest); this removes it
  MS_DEVONLY double loglik_pad(const Step<T, NX, NY, NW>& st, const Prob<TS>& p) const {
    if constexpr (M::kPadded) {
      return 0.5 * double(NY - p.ny_in) * (1.8378770664093453 - ::log(double(st.dt)));
    } else {
      return 0.0;
    }
  }
  // divergence of the drift of a step (its terms st) at x, for the objective
  MS_DEVONLY T divergence(const Step<T, NX, NY, NW>& st, const T (&x)[NX]) const {
    if constexpr (M::NTH > 0) {
      return M::divergence(th, x);
    } else {
      T tr = T(0);
#pragma unroll
      for (int c = 0; c < NX; ++c) tr += st.F[c][c];
      return tr;
    }
  }
  MS_DEVONLY void ift_prior(const Raw& r, T (&v0)[NX]) const {
    if constexpr (M::kIft) {
#pragma unroll
      for (int c = 0; c < NX; ++c) v0[c] = T(r.g[c]);
    }
  }

  // Model terms of the step that ends at (non-head) state i from its fetched inputs.
  MS_DEVONLY void terms(const Prob<TS>& p, int64_t i, const Raw& r, Step<T, NX, NY, NW>& st) const {
    const int64_t k = i - s - 1;  // step index
    const T dt = T(r.dt);
    if constexpr (M::NTH > 0) {
      T xb[NX];
      if constexpr (M::kNonlinear) {
#pragma unroll
        for (int c = 0; c < NX; ++c) xb[c] = T(r.xb[c]);
      } else {
#pragma unroll
        for (int c = 0; c < NX; ++c) xb[c] = T(0);
      }
      M::terms(th, xb, dt, st);
      if constexpr (M::kAngle >= 0) {
        // angular component: the residual y - r modulo 2 pi into [-pi, pi),
        // i.e. the measurement taken on the branch nearest the prediction
        constexpr int a = M::kAngle;
        const T ya = T(r.y[a]);
        st.r[a] = ya - wrap_angle(ya - st.r[a]);
      }
    } else {
      if (sstep != nullptr) {
        T* d = reinterpret_cast<T*>(&st);
#pragma unroll
        for (int q = 0; q < int(sizeof(st) / sizeof(T)); ++q) d[q] = sstep[q];
        return;
      }
      st.dt = dt;
      const TS* F = p.F + k * p.sF;
      const TS* c = p.c + k * p.sc;
      const TS* L = p.L + k * p.sL;
      const TS* W = p.W + k * p.sW;
      const TS* H = p.H + k * p.sH;
      const TS* r = p.r + k * p.sr;
      const TS* R = p.R + k * p.sR;
#pragma unroll
      for (int a = 0; a < NX; ++a) {
#pragma unroll
        for (int b = 0; b < NX; ++b) st.F[a][b] = F[a * NX + b];
        st.c[a] = c[a];
      }
      T Wm[NW][NW], Lw[NW][NW], dw[NW], Lm[NX][NW];
      // the problem's noise dimension (ModelLinearPadded: padded to NW with
      // zero columns of L and W = I there)
      const int nw = M::kPadded ? p.nw_in : NW;
#pragma unroll
      for (int a = 0; a < NW; ++a)
#pragma unroll
        for (int b = 0; b < NW; ++b)
          Wm[a][b] = (a < nw && b < nw) ? T(W[a * nw + b]) : (a == b ? T(1) : T(0));
      chol(Wm, Lw, dw);
#pragma unroll
      for (int a = 0; a < NX; ++a)
#pragma unroll
        for (int b = 0; b < NW; ++b) Lm[a][b] = b < nw ? T(L[a * nw + b]) : T(0);
      mm(Lm, Lw, st.V);
      const T sd = sqrt_(dt);
#pragma unroll
      for (int a = 0; a < NX; ++a)
#pragma unroll
        for (int b = 0; b < NW; ++b) st.V[a][b] *= sd;
      // the problem's measurement dimension (ModelLinearPadded: padded to NY
      // with zero rows of H, r = 0 and R = I there)
      const int ny = M::kPadded ? p.ny_in : NY;
#pragma unroll
      for (int a = 0; a < NY; ++a) {
#pragma unroll
        for (int b = 0; b < NX; ++b) st.H[a][b] = a < ny ? T(H[a * NX + b]) : T(0);
        st.r[a] = a < ny ? T(r[a]) : T(0);
#pragma unroll
        for (int b = 0; b < NY; ++b)
          st.R[a][b] = (a < ny && b < ny) ? T(R[a * ny + b]) : (a == b ? T(1) : T(0));
      }
      spd_inv(st.R, st.Rinv);
    }
  }

  MS_DEVONLY void step(const Prob<TS>& p, int64_t i, Step<T, NX, NY, NW>& st, T (&y)[NY]) const {
    Raw r;
    fetch(p, i, r);
    terms(p, i, r, st);
    r.meas(y);
  }

  MS_DEVONLY void xbar(const Prob<TS>& p, int64_t i, T (&xb)[NX]) const {
    if constexpr (M::kNonlinear) {
#pragma unroll
      for (int c = 0; c < NX; ++c) xb[c] = T(p.xbar[tix(i, c, NX)]);
    } else {
#pragma unroll
      for (int c = 0; c < NX; ++c) xb[c] = T(0);
    }
  }

  // prior of the current segment: S0 = P0^{-1}, v0 = P0^{-1} m0
  MS_DEVONLY void prior(const Prob<TS>& p, T (&S0)[NX][NX], T (&v0)[NX], T (&m0)[NX],
                        T (&P0i)[NX][NX]) const {
    T P0[NX][NX];
#pragma unroll
    for (int a = 0; a < NX; ++a) {
      m0[a] = T(p.m0[s * p.m0_stride + a]);
#pragma unroll
      for (int b = 0; b < NX; ++b) P0[a][b] = T(p.P0[s * p.P0_stride + a * NX + b]);
    }
    spd_inv(P0, P0i);
    mcopy(P0i, S0);
    mv(P0i, m0, v0);
  }
};

// General linear model with every matrix and the step length shared by all
// steps: every step has the same terms.  One thread of the block builds them
// into LDS at the start (through the general path), and the cursors read them
// from there instead of loading 66 values and repeating a Cholesky
// factorisation, a product and an inverse at every step.  Every thread of the
// block calls it, before any thread leaves.
template <typename T, class M>
struct SharedStep {
  static constexpr int n =
      M::NTH == 0 ? int(sizeof(Step<T, M::NX, M::NY, M::NW>) / sizeof(T)) : 1;
};
template <typename TS, typename T, class M>
MS_DEVONLY const T* shared_step(const Prob<TS>& p, T* lds) {
  if constexpr (M::NTH == 0) {
    if (p.sF != 0 || p.sc != 0 || p.sL != 0 || p.sW != 0 || p.sH != 0 || p.sr != 0 ||
        p.sR != 0 || p.dt_stride != 0)
      return nullptr;
    if (threadIdx.x == 0) {
      Cursor<TS, T, M> c;
      c.s = 0;
      typename Cursor<TS, T, M>::Raw r;
      r.dt = p.dt[0];
      Step<T, M::NX, M::NY, M::NW> st;
      c.terms(p, 1, r, st);  // step index 0; every index reads the same matrices
      const T* src = reinterpret_cast<const T*>(&st);
      for (int q = 0; q < SharedStep<T, M>::n; ++q) lds[q] = src[q];
    }
    __syncthreads();
    return lds;
  } else {
    return nullptr;
  }
}

// --------------------------------------------------------------------------- reductions
// Segmented sum over the lanes of a block (segment ids non-decreasing with the
// thread index; seg < 0 marks no data), added atomically into dst[t][seg *
// stride[t]].  Each wavefront sums its runs; a run that starts inside a
// wavefront is added by its first lane, and the run that starts at lane 0 goes
// through LDS, where one thread joins those of consecutive wavefronts in the
// same segment before adding them.  Atomics on one address are serialised at
// the memory side: with long segments, one atomic per wavefront on each
// accumulator kept the trajectory fix-up waiting for ~30 us after its last
// state; one per block cost ~1.5 us.  Every thread of the block calls it.
template <int K>
MS_DEVONLY void flush_block(int64_t seg, double (&val)[K], double* const (&dst)[K],
                            const int64_t (&stride)[K]) {
  __shared__ double s_val[kBlock / kWave][K];
  __shared__ int s_seg[kBlock / kWave];
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x >> 6;
  const int sg = int(seg);
#pragma unroll 1  // one copy of the level body: keeps the kernel inside the instruction cache
  for (int d = 1; d < kWave; d <<= 1) {
    const int src = lane + d < kWave ? lane + d : lane;
    const int so = shfl(sg, src);
#pragma unroll
    for (int t = 0; t < K; ++t) {
      double o = shfl(val[t], src);
      if (lane + d < kWave && so == sg) val[t] += o;
    }
  }
  const int sp = shfl(sg, lane > 0 ? lane - 1 : 0);
  if (lane == 0) {
    s_seg[wv] = sg;
#pragma unroll
    for (int t = 0; t < K; ++t) s_val[wv][t] = sg >= 0 ? val[t] : 0.0;
  } else if (sg >= 0 && sp != sg) {
#pragma unroll
    for (int t = 0; t < K; ++t)
      if (dst[t]) unsafeAtomicAdd(dst[t] + sg * stride[t], val[t]);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int t = 0; t < K; ++t) {
      if (!dst[t]) continue;
      int cur = -1;
      double a = 0.0;
      for (int w = 0; w < kBlock / kWave; ++w) {
        if (s_seg[w] != cur) {
          if (cur >= 0) unsafeAtomicAdd(dst[t] + cur * stride[t], a);
          cur = s_seg[w];
          a = 0.0;
        }
        a += s_val[w][t];
      }
      if (cur >= 0) unsafeAtomicAdd(dst[t] + cur * stride[t], a);
    }
  }
}

template <int K>
MS_DEVONLY void flush_lane(int64_t seg, double (&val)[K], double* const (&dst)[K],
                           const int64_t (&stride)[K]) {
  if (seg < 0) return;
#pragma unroll
  for (int t = 0; t < K; ++t) {
    if (dst[t]) unsafeAtomicAdd(dst[t] + seg * stride[t], val[t]);
    val[t] = 0.0;
  }
}

// --------------------------------------------------------------------------- last block
// Two-level arrival: a block first increments the counter of its group
// (workgroup id mod 8, i.e. its XCD), and the last block of each group then
// increments the top counter; the last of those is the last block overall.
// Each device-scope atomic on one address is serialised at the memory side,
// so 256 blocks on a single counter put ~20 us of queueing in front of the
// last arrival; groups of 32 contend in parallel and only 8 reach the top.
// Counter layout: counters.h (each counter on a cache line of its own).
//
// Ordering.  Everything the last block reads (the tile aggregates) is written
// with device-coherent stores (wt_store: past the XCD's non-coherent L2), so a
// block only has to wait for its own stores to complete before it counts
// itself in; the last block then invalidates its L2 (agent-scope acquire)
// before reading.  This is the protocol the compiler emits for agent-scope
// release/acquire of atomic data; an agent-scope release fence would add an
// L2 write-back (buffer_wbl2) per wavefront, which measured 10-30 us each here
// and is only needed for ordinary (write-back) stores, of which the data read
// across blocks has none.

MS_DEVONLY bool arrive_last(unsigned int* counters) {
  __shared__ unsigned int s_last;
  drain_vmem();  // this wavefront's device-coherent stores have completed
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned nb = gridDim.x, grp = blockIdx.x % kArriveGroups;
    const unsigned gsize = nb / kArriveGroups + (grp < nb % kArriveGroups ? 1u : 0u);
    const unsigned ngroups = nb < unsigned(kArriveGroups) ? nb : unsigned(kArriveGroups);
    unsigned last = 0;
    const unsigned t = __hip_atomic_fetch_add(counters + grp * kArriveStride, 1u, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
    if (t == gsize - 1) {
      const unsigned u = __hip_atomic_fetch_add(counters + kArriveGroups * kArriveStride, 1u, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
      last = (u == ngroups - 1) ? 1u : 0u;
    }
    s_last = last;
  }
  __syncthreads();
  const bool last = s_last != 0;
  if (last) {
    drain_vmem();  // the counter increment has returned
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  return last;
}

// Reset by the last block once every block has arrived.
MS_DEVONLY void release_counter(unsigned int* counters) {
  if (threadIdx.x < kArriveWords)
    __hip_atomic_store(counters + threadIdx.x * kArriveStride, 0u, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// Filter block scan, run by the last block: (S, v) before every block of
// four tiles, from the block aggregates (plane sets of nt items).
template <typename T, int N, bool kBulk>
MS_DEVONLY void filter_tile_scan(const T* tile_agg, T* tile_carry, int64_t nt) {
  // The run of one block only, but its registers size the whole kernel:
  // elements are read field by field (combine_into, carry_apply_src) and no
  // whole element is prefetched.
  __shared__ T s_w[4][ElemSz<N>::n];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid >> 6;
  const int64_t K = (nt + kBlock - 1) / kBlock;
  const int64_t t0 = min<int64_t>(tid * K, nt), t1 = min<int64_t>(t0 + K, nt);
  Elem<T, N> acc;
  if (t0 < t1) {
    load_elem(tile_agg, nt, t0, acc);
    for (int64_t t = t0 + 1; t < t1; ++t) {
      Elem<T, N> o;
      load_elem(tile_agg, nt, t, o);
      combine_into(RegSrc<T, N>{acc}, o);
      acc = o;
    }
  } else {
    elem_identity(acc);
  }
#pragma unroll 1  // one copy of the level body: keeps the kernel inside the instruction cache
  for (int d = 1; d < kWave; d <<= 1) scan_step<T, N, kBulk>(acc, lane >= d ? lane - d : lane, lane >= d);
  if (lane == kWave - 1) pack_elem(s_w[wv], acc);
  __syncthreads();
  // exclusive prefix of the lane: waves before, then lanes before (lane 0:
  // the identity)
  T S[N][N], v[N];
  mzero(S);
#pragma unroll
  for (int r = 0; r < N; ++r) v[r] = T(0);
  // applying a run to S = 0 gives its (J, eta) exactly: wave 0's total is
  // taken as it is, the later ones applied
  if (wv > 0) {
    const PackedSrc<T, N> w0{s_w[0]};
    w0.get_J(S);
    w0.get_eta(v);
  }
  for (int w = 1; w < wv; ++w) {
    if constexpr (kBulk) {
      Elem<T, N> e;
      unpack_elem(s_w[w], e);
      carry_apply(S, v, e);
    } else {
      carry_apply_src(S, v, PackedSrc<T, N>{s_w[w]});
    }
  }
  if constexpr (kBulk)
    carry_apply_src(S, v, BulkSrc<T, N>(acc, lane > 0 ? lane - 1 : 0, lane > 0));
  else
    carry_apply_src(S, v, ShflSrc<T, N>{acc, lane > 0 ? lane - 1 : 0, lane > 0});
  // carries before this thread's tiles (the one after its last tile is not needed)
  for (int64_t t = t0; t < t1; ++t) {
    store_sym(tile_carry, nt, t, S, 0);
    store_vec(tile_carry, nt, t, v, Sym<N>::n);
    if (t + 1 < t1) {
      Elem<T, N> o;
      load_elem(tile_agg, nt, t, o);
      carry_apply(S, v, o);
    }
  }
}

// Trajectory block scan, run by the last block: (x, P) after every block of
// four tiles, from the block maps (plane sets of nt items).
template <typename T, int N>
MS_DEVONLY void traj_tile_scan(const Ws<T>& ws, int64_t nt) {
  __shared__ T s_w[4][AffSz<N>::n];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid >> 6;
  const int64_t K = (nt + kBlock - 1) / kBlock;
  const int64_t t0 = min<int64_t>(tid * K, nt), t1 = min<int64_t>(t0 + K, nt);
  // (run by one block, but its registers size the whole kernel: no map is
  // prefetched)
  Aff<T, N> acc, o;
  if (t0 < t1) {
    load_aff(ws.stile_agg, nt, t0, acc);
    for (int64_t t = t0 + 1; t < t1; ++t) {
      load_aff(ws.stile_agg, nt, t, o);
      aff_append(acc, o);
    }
  } else {
    aff_identity(acc);
  }
  // reverse inclusive scan: acc <- acc o (lanes to the right)
#pragma unroll 1  // one copy of the level body: keeps the kernel inside the instruction cache
  for (int d = 1; d < kWave; d <<= 1) {
    shfl_aff(o, acc, lane + d < kWave ? lane + d : lane);
    if (lane + d < kWave) aff_append(acc, o);
  }
  if (lane == 0) {
    T* w = s_w[wv];
    int c = 0;
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
      for (int q = 0; q < N; ++q) w[c++] = acc.Phi[r][q];
#pragma unroll
    for (int r = 0; r < N; ++r) w[c++] = acc.bt[r];
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
      for (int q = 0; q <= r; ++q) w[c++] = acc.Om[r][q];
  }
  __syncthreads();
  Aff<T, N> ex;  // lanes to the right within the wave, then waves to the right
  shfl_aff(ex, acc, lane + 1 < kWave ? lane + 1 : lane);
  if (lane == kWave - 1) aff_identity(ex);
  for (int w = wv + 1; w < 4; ++w) {
    const T* s = s_w[w];
    int c = 0;
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
      for (int q = 0; q < N; ++q) o.Phi[r][q] = s[c++];
#pragma unroll
    for (int r = 0; r < N; ++r) o.bt[r] = s[c++];
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
      for (int q = 0; q <= r; ++q) { o.Om[r][q] = s[c++]; o.Om[q][r] = o.Om[r][q]; }
    aff_append(ex, o);
  }
  // the composition to the end of the sequence is a constant map (it contains
  // the last state), so its offset is the value after this thread's tiles
  T x[N], P[N][N];
#pragma unroll
  for (int r = 0; r < N; ++r) x[r] = ex.bt[r];
  mcopy(ex.Om, P);
  // values after this thread's tiles (the one before its first tile is not needed)
  for (int64_t t = t1 - 1; t >= t0; --t) {
    store_vec(ws.stile_carry, nt, t, x, 0);
    store_sym(ws.stile_carry, nt, t, P, N);
    if (t > t0) {
      load_aff(ws.stile_agg, nt, t, o);
      aff_apply(o, x, P);
    }
  }
}

// A flagged run (element plus segment-start flag): the flag is component
// ElemSz of the plane set.
template <typename T, int N>
MS_DEVONLY void load_selem(const T* base, int64_t ld, int64_t i, Elem<T, N>& e, T& f) {
  load_elem(base, ld, i, e);
  f = base[ElemSz<N>::n * ld + i];
}

// Backward-filter block scan of the two-filter smoother, run by the last
// block: for every block of four tiles, the run after it up to the next
// segment start (segmented reverse scan, see seg_append), from the block runs
// (plane sets of nt flagged items).
template <typename T, int N>
MS_DEVONLY void suffix_tile_scan(const T* agg, T* carry, int64_t nt) {
  constexpr int E = ElemSz<N>::n;
  __shared__ T s_w[4][E + 1];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid >> 6;
  const int64_t K = (nt + kBlock - 1) / kBlock;
  const int64_t t0 = min<int64_t>(tid * K, nt), t1 = min<int64_t>(t0 + K, nt);
  Elem<T, N> acc, o, nx_;
  T af = T(0), of = T(0), nf = T(0);
  if (t0 < t1) {
    load_selem(agg, nt, t0, acc, af);
    if (t0 + 1 < t1) load_selem(agg, nt, t0 + 1, nx_, nf);
    for (int64_t t = t0 + 1; t < t1; ++t) {
      o = nx_;
      of = nf;
      if (t + 1 < t1) load_selem(agg, nt, t + 1, nx_, nf);  // one tile ahead
      seg_append(acc, af, o, of);
    }
  } else {
    elem_identity(acc);
  }
  // reverse inclusive scan over the lanes: acc <- acc (+) lanes to the right
#pragma unroll 1  // one copy of the level body: keeps the kernel inside the instruction cache
  for (int d = 1; d < kWave; d <<= 1) {
    const int src = lane + d < kWave ? lane + d : lane;
    shfl_elem(o, acc, src);
    of = shfl(af, src);
    if (lane + d < kWave) seg_append(acc, af, o, of);
  }
  if (lane == 0) {
    T* w = s_w[wv];
    int c = 0;
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
      for (int q = 0; q < N; ++q) w[c++] = acc.A[r][q];
#pragma unroll
    for (int r = 0; r < N; ++r) w[c++] = acc.b[r];
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
      for (int q = 0; q <= r; ++q) w[c++] = acc.C[r][q];
#pragma unroll
    for (int r = 0; r < N; ++r) w[c++] = acc.eta[r];
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
      for (int q = 0; q <= r; ++q) w[c++] = acc.J[r][q];
    w[c] = af;
  }
  __syncthreads();
  // run after this thread's tiles: lanes to the right, then waves to the right
  Elem<T, N> ex;
  T exf;
  shfl_elem(ex, acc, lane + 1 < kWave ? lane + 1 : lane);
  exf = shfl(af, lane + 1 < kWave ? lane + 1 : lane);
  if (lane == kWave - 1) {
    elem_identity(ex);
    exf = T(0);
  }
  for (int w = wv + 1; w < 4; ++w) {
    const T* sw = s_w[w];
    int c = 0;
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
      for (int q = 0; q < N; ++q) o.A[r][q] = sw[c++];
#pragma unroll
    for (int r = 0; r < N; ++r) o.b[r] = sw[c++];
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
      for (int q = 0; q <= r; ++q) { o.C[r][q] = sw[c++]; o.C[q][r] = o.C[r][q]; }
#pragma unroll
    for (int r = 0; r < N; ++r) o.eta[r] = sw[c++];
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
      for (int q = 0; q <= r; ++q) { o.J[r][q] = sw[c++]; o.J[q][r] = o.J[r][q]; }
    seg_append(ex, exf, o, sw[c]);
  }
  // runs after each of this thread's tiles, right to left (the one before
  // its first tile is not needed)
  if (t1 - 1 > t0) load_selem(agg, nt, t1 - 1, nx_, nf);
  for (int64_t t = t1 - 1; t >= t0; --t) {
    store_elem(carry, nt, t, ex);
    if (t > t0) {
      o = nx_;
      of = nf;
      if (t - 1 > t0) load_selem(agg, nt, t - 1, nx_, nf);
      // ex <- tile t (+) ex
      T f2 = of;
      seg_append(o, f2, ex, exf);
      ex = o;
      exf = f2;
    }
  }
}

// --------------------------------------------------------------------------- pass A
// Zero the per-segment accumulators over the whole grid.  The filter
// up-sweep does this for the passes that follow it (it runs before any of
// them adds to the accumulators), which saves a launch.
MS_DEVONLY void zero_acc_grid(const Acc& a, int64_t n_seg, int64_t nth) {
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  const int64_t t0 = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  for (int64_t i = t0; i < n_seg; i += stride) {
    if (a.loglik) a.loglik[i] = 0.0;
    if (a.obj) a.obj[i] = 0.0;
  }
  for (int64_t i = t0; i < n_seg * nth; i += stride) {
    if (a.g_loglik) a.g_loglik[i] = 0.0;
    if (a.g_obj) a.g_obj[i] = 0.0;
  }
}

// Two variants: kW = 2 asks the compiler for two wavefronts per SIMD (at
// nx = 4 a spill of ~130 B a lane), kW = 1 for none (one wavefront, no
// spill).  The launch takes the first when the grid has more wavefronts than
// the chip has SIMDs, so that two can share one and hide each other's
// latency; the second when every SIMD runs at most one.
template <class M, int kW>
struct UpWaves {
  static constexpr int n = kW == 2 ? M::kWaves : 1;
};
template <typename TS, typename T, class M, int kW>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(UpWaves<M, kW>::n)))
k_filter_up(Prob<TS> p, Ws<T> ws, Acc zacc) {
  constexpr int N = M::NX;
  // one wavefront per SIMD of a model that fits two elsewhere: registers to
  // spare for whole-element shuffles in the scans
  constexpr bool kBulkUp = M::kWaves == 2 && kW == 1;
  __shared__ __align__(16) T s_step[SharedStep<T, M>::n];
  const T* sstep = shared_step<TS, T, M>(p, s_step);
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t g = logical_block() * kBlock + threadIdx.x;
  zero_acc_grid(zacc, p.n_seg, M::NTH > 0 ? M::NTH : 1);
  const int64_t tile = g >> 6;
  const int64_t j0 = g * ws.chunk;
  const int64_t j1 = lane_end(g, ws.n_lanes, p.n_states, ws.chunk);
  Elem<T, N> agg;
  elem_identity(agg);
  if (j0 < j1) {
    Cursor<TS, T, M> cur;
    cur.sstep = sstep;
    cur.init(p, j0);
    typename Cursor<TS, T, M>::Raw rn;
    cur.fetch(p, j0, rn);
    drain_vmem();
    // split schedule: the fold of the first half of the chunk is stored too
    // (the passes after this one start a lane there)
    const int64_t jm = ws.lane_half ? min<int64_t>(j0 + (ws.chunk >> 1), j1) : j1;
    int64_t i = j0;
    for (int h = 0; h < 2; ++h) {
      const int64_t je = h == 0 ? jm : j1;
      for (; i < je; ++i) {
        const typename Cursor<TS, T, M>::Raw rc = rn;
        // one state ahead, always issued (a repeat of state i on the last
        // one): the same number of loads on every path keeps the compiler's
        // waits for them exact
        cur.fetch(p, i + 1 < j1 ? i + 1 : i, rn);
        if (cur.is_head(i)) {
          T m0[N], P0i[N][N];
          cur.prior(p, agg.J, agg.eta, m0, P0i);
          cur.ift_prior(rc, agg.eta);
          mzero(agg.A);
          mzero(agg.C);
#pragma unroll
          for (int r = 0; r < N; ++r) agg.b[r] = T(0);
        } else {
          Step<T, N, M::NY, M::NW> st;
          cur.terms(p, i, rc, st);
          T y[M::NY];
          rc.meas(y);
          Fresh<T, N, M::NW> f;
          fresh_from_step(st, y, f);
          cur.adjust_fresh(p, i, rc, st, f);
          fold_fresh(agg, f);
        }
        if (cur.is_last(i) && i + 1 < p.n_states) cur.next(p);
      }
      if (h == 0 && jm < j1) lt_store_elem(ws.lane_half, g, agg);
    }
  }
  // in-tile inclusive scan (every lane combines; lanes below d with the
  // identity, which leaves them unchanged)
  Elem<T, N> o;
#pragma unroll 1  // one copy of the level body: keeps the kernel inside the instruction cache
  for (int d = 1; d < kWave; d <<= 1) scan_step<T, N, kBulkUp>(agg, lane >= d ? lane - d : lane, lane >= d);
  shfl_elem(o, agg, lane > 0 ? lane - 1 : 0);
  if (lane == 0) elem_identity(o);
  // Lane prefixes are read only by the next kernel; written here, they drain
  // while the block combines its tiles (measured: faster than holding them
  // in LDS and storing them after the arrival).
  if (g < ws.n_lanes) lt_store_elem(ws.lane_pre, g, o);
  // The block's four tiles (a0..a3, identities past the last tile) are
  // combined in a two-level tree: x01 = a0 a1 and x23 = a2 a3, then the block
  // aggregate x01 x23 (scanned by the last block) and the exclusive prefixes
  // of the tiles inside the block: 0, a0, x01, x01 a2.
  __shared__ T s_blk[6][ElemSz<N>::n];
  const int wv = threadIdx.x >> 6;
  if (lane == kWave - 1) pack_elem(s_blk[wv], agg);
  __syncthreads();
  Elem<T, N> pre;
  elem_identity(pre);
  // E . L with E from the packed LDS copy: read whole where registers allow
  auto lds_step = [&](const T* w, Elem<T, N>& l) {
    if constexpr (kBulkUp) {
      Elem<T, N> e;
      unpack_elem(w, e);
      combine_into(RegSrc<T, N>{e}, l);
    } else {
      combine_into(PackedSrc<T, N>{w}, l);
    }
  };
  if (wv == 1 || wv == 3) {
    unpack_elem(s_blk[wv], agg);
    lds_step(s_blk[wv - 1], agg);  // x01 (wave 1), x23 (wave 3)
    if (lane == 0) pack_elem(s_blk[4 + (wv >> 1)], agg);
  }
  __syncthreads();
  if (wv == 0) {
    unpack_elem(s_blk[5], agg);
    lds_step(s_blk[4], agg);
    if (lane == 0) store_elem<T, N, true>(ws.tile_agg, gridDim.x, tile >> 2, agg);
  } else if (wv == 1) {
    unpack_elem(s_blk[0], pre);
  } else if (wv == 2) {
    unpack_elem(s_blk[4], pre);
  } else {
    unpack_elem(s_blk[2], pre);
    lds_step(s_blk[4], pre);
  }
  // (the carries of a checkpoint need no arrival: up_tail is the same for the whole grid)
  const bool last = ws.up_tail && arrive_last(ws.counters + kCountersFilter);
  // tile prefixes: read only by the next kernel, written after the arrival
  if (lane == 0 && wv > 0 && tile < ws.n_tiles) store_elem(ws.tile_pre, ws.n_tiles, tile, pre);
  if (last) {
    filter_tile_scan<T, N, kBulkUp>(ws.tile_agg, ws.tile_carry, int64_t(gridDim.x));
    release_counter(ws.counters + kCountersFilter);
  }
}

// --------------------------------------------------------------------------- pass B
// kModeTwoFilter: the filter fix-up plus the up-sweep of the backward filter
// of the two-filter smoother (the runs of later steps, Sec. 4.3).
enum : int { kModeFilter = 0, kModeFused = 1, kModeTrajOnly = 2, kModeTwoFilter = 3 };

struct FilterOut {
  void* S;    // [Sym][n_states]
  void* v;    // [N][n_states]
  void* m;    // optional [N][n_states]
  void* P;    // optional [Sym][n_states]
  int want_loglik;
};

// log N(y; H m^- + r, H P^- H^T + R/dt) with P^- = Sp^{-1}, m^- = Sp^{-1} vp
template <typename T, int N, int NY, int NW>
MS_DEVONLY double pred_loglik(const T (&Sp)[N][N], const T (&vp)[N], const Step<T, N, NY, NW>& st,
                              const T (&y)[NY]) {
  T Ls[N][N], ds[N];
  chol(Sp, Ls, ds);
  T mp[N];
#pragma unroll
  for (int i = 0; i < N; ++i) mp[i] = vp[i];
  trsv_lower(Ls, ds, mp);
  trsv_upper_t(Ls, ds, mp);
  T X[N][NY];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < NY; ++j) X[i][j] = st.H[j][i];
  trsm_lower(Ls, ds, X);
  T Sg[NY][NY];
  mtm_sym(X, X, Sg);
  const T idt = rcp(st.dt);
#pragma unroll
  for (int i = 0; i < NY; ++i)
#pragma unroll
    for (int j = 0; j < NY; ++j) Sg[i][j] += st.R[i][j] * idt;
  T Hm[NY], e[NY];
  mv(st.H, mp, Hm);
#pragma unroll
  for (int i = 0; i < NY; ++i) e[i] = y[i] - st.r[i] - Hm[i];
  T Lg[NY][NY], dg[NY];
  chol(Sg, Lg, dg);
  trsv_lower(Lg, dg, e);
  double q = 0.0, det = 1.0;
#pragma unroll
  for (int i = 0; i < NY; ++i) {
    q += double(e[i]) * double(e[i]);
    det *= double(Lg[i][i]);
  }
  return -0.5 * (double(NY) * 1.8378770664093453 + 2.0 * ::log(det) + q);
}

// Two wavefronts per SIMD asked of the compiler (256 registers a lane) for
// the models that fit without spilling (M::kWaves): the filter fix-up modes;
// the two-filter mode would spill about 1 KB a lane and keeps one.
template <class M, int kMode>
struct DownWaves {
  static constexpr int n = kMode != 3 ? M::kWaves : 1;
};
template <typename TS, typename T, class M, int kMode>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(DownWaves<M, kMode>::n)))
k_filter_down(Prob<TS> p, Ws<T> ws, FilterOut fo, Acc acc) {
  constexpr int N = M::NX, NY = M::NY, NW = M::NW;
  constexpr bool kFilter = kMode != kModeTrajOnly;
  constexpr bool kTraj = kMode == kModeFused || kMode == kModeTrajOnly;
  constexpr bool kSuf = kMode == kModeTwoFilter;
  __shared__ __align__(16) T s_step[SharedStep<T, M>::n];
  const T* sstep = shared_step<TS, T, M>(p, s_step);
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t g = logical_block() * kBlock + threadIdx.x;
  const int64_t tile = g >> 6;
  const int64_t j0 = g * ws.chunk;
  const int64_t ns = p.n_states;
  const int64_t j1 = lane_end(g, ws.n_lanes, ns, ws.chunk);
  TS* So = static_cast<TS*>(fo.S);
  TS* vo = static_cast<TS*>(fo.v);
  TS* mo = static_cast<TS*>(fo.m);
  TS* Po = static_cast<TS*>(fo.P);
  T S[N][N], v[N];
  if constexpr (kFilter) {
    if (tile < ws.n_tiles) {
      // block carry, then the tile's prefix inside its block, then the lane's
      // (all in the filter up-sweep's decomposition), then, for the second
      // half of a split lane, the fold of its first half
      const int64_t g1 = g >> ws.k1_shift, tile1 = g1 >> 6;
      const int64_t nb = (ws.n_tiles1 + 3) >> 2;
      load_sym(ws.tile_carry, nb, tile1 >> 2, S, 0);
      load_vec(ws.tile_carry, nb, tile1 >> 2, v, Sym<N>::n);
      Elem<T, N> lp;
      if (tile1 & 3) {
        load_elem(ws.tile_pre, ws.n_tiles1, tile1, lp);
        carry_apply(S, v, lp);
      }
      lt_load_elem(ws.lane_pre, g1, lp);
      carry_apply(S, v, lp);
      if (ws.k1_shift && (g & 1) && j0 < j1) {
        lt_load_elem(ws.lane_half, g1, lp);
        carry_apply(S, v, lp);
      }
    }
  }
  Aff<T, N> sagg;
  aff_identity(sagg);
  // backward filter: the run from the chunk's first state up to the first
  // segment start in the chunk (exclusive), and whether there is one
  Elem<T, N> pagg;
  T pf = T(0);
  if constexpr (kSuf) elem_identity(pagg);
  double ll = 0.0;
  bool bad = false;  // a non-finite S, v (MAP_CHECK_FINITE)
  int64_t seg_acc = -1;
  if (j0 < j1) {
    Cursor<TS, T, M> cur;
    cur.sstep = sstep;
    cur.init(p, j0);
    seg_acc = cur.s;
    typename Cursor<TS, T, M>::Raw rn;
    cur.fetch(p, kFilter ? j0 : min<int64_t>(j0 + 1, ns - 1), rn);
    drain_vmem();
    for (int64_t i = j0; i < j1; ++i) {
      const bool first = i == j0;
      // inputs of state i (filter) or of state i + 1 (trajectory maps only),
      // with the next ones requested one state ahead
      const typename Cursor<TS, T, M>::Raw rc = rn;
      {
        // always issued, clamped into the sequence (see the filter up-sweep)
        const int64_t nxt = kFilter ? i + 1 : i + 2;
        const int64_t lim = j1 < ns ? j1 : ns - 1;
        cur.fetch(p, nxt <= lim ? nxt : lim, rn);
      }
      if constexpr (kFilter) {
        if (cur.is_head(i)) {
          if (kTraj && !first) {
            // previous state ends its segment: constant trajectory map
            T G[N][N], beta[N], Lam[N][N];
            mzero(G);
            spd_inv(S, Lam);
            mv(Lam, v, beta);
            aff_append(sagg, G, beta, Lam);
          }
          if (fo.want_loglik && seg_acc != cur.s) {
            double* d[1] = {acc.loglik};
            const int64_t sd[1] = {1};
            double val[1] = {ll};
            flush_lane<1>(seg_acc, val, d, sd);
            ll = 0.0;
            seg_acc = cur.s;
          }
          T m0[N], P0i[N][N];
          cur.prior(p, S, v, m0, P0i);
          cur.ift_prior(rc, v);
          if constexpr (kSuf) pf = T(1);
        } else {
          Step<T, N, NY, NW> st;
          T y[NY];
          rc.meas(y);
          cur.terms(p, i, rc, st);
          Fresh<T, N, NW> f;
          fresh_from_step(st, y, f);
          cur.adjust_fresh(p, i, rc, st, f);
          T Sn[N][N], vn[N], Sp[N][N], G[N][N], beta[N], Lam[N][N];
          if (kTraj && !first) {
            info_step<T, N, NW, true>(S, v, f, Sn, vn, Sp, G, beta, Lam);
            aff_append(sagg, G, beta, Lam);
          } else {
            info_step<T, N, NW, false>(S, v, f, Sn, vn, Sp, G, beta, Lam);
          }
          if constexpr (kSuf) {
            if (pf == T(0)) fold_fresh(pagg, f);
          }
          if (fo.want_loglik) {
            T vp[N];
#pragma unroll
            for (int r = 0; r < N; ++r) vp[r] = vn[r] - f.eta[r];
            ll += pred_loglik(Sp, vp, st, y) + cur.loglik_pad(st, p);
          }
          mcopy(Sn, S);
#pragma unroll
          for (int r = 0; r < N; ++r) v[r] = vn[r];
        }
        // the adjoint problem's S is the original problem's (stored by its pass)
        if constexpr (!M::kIft) tstore_sym<TS, T, N, kTraj || kSuf>(So, Sym<N>::n, i, S);
        {
          T vs[N];
          filter_plane_out<TS>(S, v, vs);
          tstore_vec<TS, T, N, kTraj || kSuf>(vo, N, i, vs);
          if (ws.status) bad = bad | nonfinite_vd(vs, S);
        }
        if (kMode == kModeFilter && mo != nullptr) {
          T Pm[N][N], mm_[N];
          spd_inv(S, Pm);
          mv(Pm, v, mm_);
          tstore_vec(mo, N, i, mm_);
          tstore_sym(Po, Sym<N>::n, i, Pm);
        }
      } else {
        // trajectory maps from stored filter moments
        tload_sym(So, Sym<N>::n, i, S);
        tload_vec(vo, N, i, v);
        filter_plane_in<TS>(S, v);
      }
      if constexpr (!kFilter) {
        // map of state i needs the element of state i+1
        if (cur.is_last(i)) {
          T G[N][N], beta[N], Lam[N][N];
          mzero(G);
          spd_inv(S, Lam);
          mv(Lam, v, beta);
          aff_append(sagg, G, beta, Lam);
        } else {
          Step<T, N, NY, NW> st;
          cur.terms(p, i + 1, rc, st);
          T y[NY];
          rc.meas(y);
          Fresh<T, N, NW> f;
          fresh_from_step(st, y, f);
          cur.adjust_fresh(p, i + 1, rc, st, f);
          T Sn[N][N], vn[N], Sp[N][N], G[N][N], beta[N], Lam[N][N];
          info_step<T, N, NW, true>(S, v, f, Sn, vn, Sp, G, beta, Lam);
          aff_append(sagg, G, beta, Lam);
        }
      }
      if (cur.is_last(i) && i + 1 < ns) cur.next(p);
    }
    if constexpr (kFilter && kTraj) {
      // trajectory map of the chunk's last state
      const int64_t il = j1 - 1;
      if (il + 1 >= ns || il + 1 == cur.head) {
        T G[N][N], beta[N], Lam[N][N];
        mzero(G);
        spd_inv(S, Lam);
        mv(Lam, v, beta);
        aff_append(sagg, G, beta, Lam);
      } else {
        // il + 1 = j1 < ns here, and its inputs were fetched in the last
        // iteration
        Step<T, N, NY, NW> st;
        cur.terms(p, il + 1, rn, st);
        T y[NY];
        rn.meas(y);
        Fresh<T, N, NW> f;
        fresh_from_step(st, y, f);
        cur.adjust_fresh(p, il + 1, rn, st, f);
        T Sn[N][N], vn[N], Sp[N][N], G[N][N], beta[N], Lam[N][N];
        info_step<T, N, NW, true>(S, v, f, Sn, vn, Sp, G, beta, Lam);
        aff_append(sagg, G, beta, Lam);
      }
    }
  }
  if constexpr (kFilter) {
    if (ws.status) report_nonfinite(ws.status, bad | nonfinite(ll));
    if (fo.want_loglik) {
      double* d[1] = {acc.loglik};
      const int64_t sd[1] = {1};
      double val[1] = {ll};
      flush_block<1>(seg_acc, val, d, sd);
    }
  }
  if constexpr (kTraj) {
    // reverse in-tile scan of the trajectory maps
    Aff<T, N> o;
#pragma unroll 1  // one copy of the level body: keeps the kernel inside the instruction cache
    for (int d = 1; d < kWave; d <<= 1) {
      shfl_aff(o, sagg, lane + d < kWave ? lane + d : lane);
      if (lane + d < kWave) aff_append(sagg, o);
    }
    shfl_aff(o, sagg, lane + 1 < kWave ? lane + 1 : lane);
    if (lane == kWave - 1) aff_identity(o);
    // read only by the next kernel; written here, they drain while the block
    // combines its tiles
    if (g < ws.n_lanes) lt_store_aff(ws.slane_pre, g, o);
    // The block's four tile maps (a0..a3, identities past the last tile) are
    // composed in a two-level tree: x01 = a0 a1 and x23 = a2 a3, then the
    // block map x01 x23 (scanned by the last block) and the maps from after
    // each tile to the end of the block: a1 x23, x23, a3, identity.
    __shared__ T s_tb[6][AffSz<N>::n];
    const int wv = threadIdx.x >> 6;
    if (lane == 0) pack_aff(s_tb[wv], sagg);
    __syncthreads();
    if (wv == 0 || wv == 2) {
      unpack_aff(s_tb[wv], sagg);
      unpack_aff(s_tb[wv + 1], o);
      aff_append(sagg, o);  // x01 (wave 0), x23 (wave 2)
      if (lane == 0) pack_aff(s_tb[4 + (wv >> 1)], sagg);
    }
    __syncthreads();
    Aff<T, N> suf;
    int64_t suf_tile = tile;
    if (wv == 0) {
      unpack_aff(s_tb[4], sagg);
      unpack_aff(s_tb[5], o);
      aff_append(sagg, o);
      if (lane == 0) store_aff<T, N, true>(ws.stile_agg, gridDim.x, tile >> 2, sagg);
    } else if (wv == 1) {
      unpack_aff(s_tb[5], suf);
    } else if (wv == 2) {
      unpack_aff(s_tb[3], suf);
    } else {
      unpack_aff(s_tb[1], suf);  // tile 0 of the block: a1 x23
      unpack_aff(s_tb[5], o);
      aff_append(suf, o);
      suf_tile = tile - 3;
    }
    const bool last = arrive_last(ws.counters + kCountersTraj);
    // read only by the next kernel: written after the arrival
    if (lane == 0 && wv > 0 && suf_tile < ws.n_tiles) store_aff(ws.stile_suf, ws.n_tiles, suf_tile, suf);
    if (last) {
      traj_tile_scan<T, N>(ws, int64_t(gridDim.x));
      release_counter(ws.counters + kCountersTraj);
    }
  }
  if constexpr (kSuf) {
    // reverse in-tile segmented scan of the backward-filter runs
    Elem<T, N> o;
    T of;
#pragma unroll 1  // one copy of the level body: keeps the kernel inside the instruction cache
    for (int d = 1; d < kWave; d <<= 1) {
      const int src = lane + d < kWave ? lane + d : lane;
      shfl_elem(o, pagg, src);
      of = shfl(pf, src);
      if (lane + d < kWave) seg_append(pagg, pf, o, of);
    }
    shfl_elem(o, pagg, lane + 1 < kWave ? lane + 1 : lane);
    of = shfl(pf, lane + 1 < kWave ? lane + 1 : lane);
    if (lane == kWave - 1) {
      elem_identity(o);
      of = T(0);
    }
    // The lane runs are read only by the next kernel; written here, they
    // drain while the block joins its tiles.
    constexpr int E = ElemSz<N>::n;
    if (g < ws.n_lanes) lt_store_elem<T, N, true>(ws.slane_pre, g, o, of);
    // The block's four tile runs (a0..a3 with their flags; identities with
    // no segment start past the last tile) are joined in a two-level tree:
    // x01 = a0 (+) a1 and x23 = a2 (+) a3, then the block run x01 (+) x23
    // (scanned by the last block) and the runs from after each tile to the
    // end of the block: a1 (+) x23, x23, a3, empty.
    __shared__ T s_tb[6][E + 1];
    const int wv = threadIdx.x >> 6;
    if (lane == 0) {
      pack_elem(s_tb[wv], pagg);
      s_tb[wv][E] = pf;
    }
    __syncthreads();
    if (wv == 0 || wv == 2) {
      unpack_elem(s_tb[wv + 1], o);
      seg_append(pagg, pf, o, s_tb[wv + 1][E]);  // x01 (wave 0), x23 (wave 2)
      if (lane == 0) {
        pack_elem(s_tb[4 + (wv >> 1)], pagg);
        s_tb[4 + (wv >> 1)][E] = pf;
      }
    }
    __syncthreads();
    Elem<T, N> suf;
    T sf = T(0);
    int64_t suf_tile = tile;
    if (wv == 0) {
      unpack_elem(s_tb[5], o);
      seg_append(pagg, pf, o, s_tb[5][E]);
      if (lane == 0) {
        const int64_t nb = gridDim.x;
        store_elem<T, N, true>(ws.stile_agg, nb, tile >> 2, pagg);
        wt_store(&ws.stile_agg[E * nb + (tile >> 2)], pf);
      }
    } else if (wv == 1) {
      unpack_elem(s_tb[5], suf);
      sf = s_tb[5][E];
    } else if (wv == 2) {
      unpack_elem(s_tb[3], suf);
      sf = s_tb[3][E];
    } else {
      unpack_elem(s_tb[1], suf);  // tile 0 of the block: a1 (+) x23
      sf = s_tb[1][E];
      unpack_elem(s_tb[5], o);
      seg_append(suf, sf, o, s_tb[5][E]);
      suf_tile = tile - 3;
    }
    const bool last = arrive_last(ws.counters + kCountersTraj);
    // in-block runs: read only by the next kernel, written after the arrival
    if (lane == 0 && wv > 0 && suf_tile < ws.n_tiles) {
      store_elem(ws.stile_suf, ws.n_tiles, suf_tile, suf);
      ws.stile_suf[E * ws.n_tiles + suf_tile] = sf;
    }
    if (last) {
      suffix_tile_scan<T, N>(ws.stile_agg, ws.stile_carry, int64_t(gridDim.x));
      release_counter(ws.counters + kCountersTraj);
    }
  }
}

// --------------------------------------------------------------------------- pass C
// One state of the trajectory walk (Sec. 4.3, eq. 42), shared by the flat and
// the segment-local schedules.  (S, v) is the filter at state i, rc the
// fetched inputs of state i + 1; (x, P) hold the value at state i + 1 (not
// read when i ends its segment) and receive the value at state i.  With
// want_obj / kGrad, the objective term of the step ending at i + 1
// (costate form) and its Fisher-identity and envelope cotangents are added
// to val = (objective, d loglik / d theta, d obj / d theta).
template <typename TS, typename T, class M, bool kGrad>
MS_DEVONLY void traj_walk_state(const Prob<TS>& p, const Cursor<TS, T, M>& cur, int64_t i,
                                const T (&S)[M::NX][M::NX], const T (&v)[M::NX],
                                const typename Cursor<TS, T, M>::Raw& rc, bool want_obj,
                                T (&x)[M::NX], T (&P)[M::NX][M::NX],
                                double (&val)[1 + 2 * (M::NTH > 0 ? M::NTH : 1)],
                                double* ge = nullptr) {
  constexpr int N = M::NX, NY = M::NY, NW = M::NW;
  constexpr int NTH = M::NTH > 0 ? M::NTH : 1;
  (void)NTH;
  if (cur.is_last(i)) {
    spd_inv(S, P);
    mv(P, v, x);
  } else {
    Step<T, N, NY, NW> st;
    T y[NY];
    rc.meas(y);
    cur.terms(p, i + 1, rc, st);
    Fresh<T, N, NW> f;
    fresh_from_step(st, y, f);
    cur.adjust_fresh(p, i + 1, rc, st, f);
    // trajectory map of state i (shares Z with the information step)
    T W[N][NW];
    mm(S, f.V, W);
    T Z[NW][NW];
    mtm_sym(f.V, W, Z);
#pragma unroll
    for (int a = 0; a < NW; ++a) Z[a][a] += T(1);
    T Lz[NW][NW], dz[NW];
    chol(Z, Lz, dz);
    T X[NW][N];
    mtm(W, f.A, X);
    trsm_lower(Lz, dz, X);
    trsm_upper_t(Lz, dz, X);
    T G[N][N], VX[N][N];
    mm(f.V, X, VX);
#pragma unroll
    for (int a = 0; a < N; ++a)
#pragma unroll
      for (int b = 0; b < N; ++b) G[a][b] = f.A[a][b] - VX[a][b];
    T bc[N], beta[N];
    {
      T z[NW];
      mtv(f.V, v, z);
      mv(f.V, z, bc);
#pragma unroll
      for (int a = 0; a < N; ++a) bc[a] += f.b[a];
      mtv(W, bc, z);
      trsv_lower(Lz, dz, z);
      trsv_upper_t(Lz, dz, z);
      T vz[N];
      mv(f.V, z, vz);
#pragma unroll
      for (int a = 0; a < N; ++a) beta[a] = bc[a] - vz[a];
    }
    T Yv[NW][N], Lam[N][N];
#pragma unroll
    for (int a = 0; a < NW; ++a)
#pragma unroll
      for (int b = 0; b < N; ++b) Yv[a][b] = f.V[b][a];
    trsm_lower(Lz, dz, Yv);
    mtm_sym(Yv, Yv, Lam);
    // x, P currently hold state i+1
    T xn[N], Pn[N][N];
#pragma unroll
    for (int a = 0; a < N; ++a) xn[a] = x[a];
    mcopy(P, Pn);
    traj_step(G, beta, Lam, x, P);
    if (want_obj || kGrad) {
      // costate lambda = v_i - S_i x*_i
      T Sx[N], lam[N];
      mv(S, x, Sx);
#pragma unroll
      for (int a = 0; a < N; ++a) lam[a] = v[a] - Sx[a];
      T vl[NW];
      mtv(f.V, lam, vl);
      double ob = 0.0;
#pragma unroll
      for (int a = 0; a < NW; ++a) ob += 0.5 * double(vl[a]) * double(vl[a]);
      // measurement of state i+1
      T Hx[NY], eps[NY];
      mv(st.H, xn, Hx);
#pragma unroll
      for (int a = 0; a < NY; ++a) eps[a] = y[a] - st.r[a] - Hx[a];
      T Re[NY];
      mv(st.Rinv, eps, Re);
#pragma unroll
      for (int a = 0; a < NY; ++a) ob += 0.5 * double(st.dt) * double(eps[a]) * double(Re[a]);
      // MAP_OM_DIVERGENCE: the divergence term 1/2 dt div f(x*) of eq. OM
      if (p.om_div) ob += 0.5 * double(st.dt) * double(cur.divergence(st, xn));
      val[0] += ob;
      if constexpr (kGrad && M::NTH > 0) {
        // Nm = (I + S C)^{-1} S = S - W Z^{-1} W^T, in Joseph form
        // Pi S Pi^T + K K^T with K = W Z^{-1}, Pi^T = I - V K^T (no
        // cancellation where S is ill-conditioned)
        T Kt[NW][N], Pt[N][N], Nm[N][N];
#pragma unroll
        for (int a = 0; a < NW; ++a)
#pragma unroll
          for (int b = 0; b < N; ++b) Kt[a][b] = W[b][a];
        trsm_lower(Lz, dz, Kt);
        trsm_upper_t(Lz, dz, Kt);
        mm(f.V, Kt, Pt);
#pragma unroll
        for (int a = 0; a < N; ++a)
#pragma unroll
          for (int b = 0; b < N; ++b) Pt[a][b] = (a == b ? T(1) : T(0)) - Pt[a][b];
        {
          T SPt[N][N], KK[N][N];
          mm(S, Pt, SPt);
          mtm_sym(Pt, SPt, Nm);
          mtm_sym(Kt, Kt, KK);
#pragma unroll
          for (int a = 0; a < N; ++a)
#pragma unroll
            for (int b = 0; b < N; ++b) Nm[a][b] += KK[a][b];
        }
        T NA[N][N], NAP[N][N], E2[N][N];
        mm(Nm, f.A, NA);
        mm(NA, Pn, NAP);
        mmt_sym(NAP, NA, E2);  // Nm A P^s A^T Nm
        T Ainv[N][N];
        inv(f.A, Ainv);
        T GAl[N][N], GAm[N][N], GCl[N][N], GCm[N][N], Gbl[N], Gbm[N];
#pragma unroll
        for (int a = 0; a < N; ++a) {
          Gbl[a] = lam[a];
          Gbm[a] = -lam[a];
#pragma unroll
          for (int b = 0; b < N; ++b) {
            const T lx = lam[a] * xn[b];
            GAl[a][b] = lx - NAP[a][b] + Ainv[b][a];
            GAm[a][b] = -lx;
            const T ll_ = lam[a] * lam[b];
            GCl[a][b] = T(0.5) * (ll_ + E2[a][b] - Nm[a][b]);
            GCm[a][b] = T(-0.5) * ll_;
          }
        }
        // measurement: R-cotangents
        T HP[NY][N], HPH[NY][NY];
        mm(st.H, Pn, HP);
        mmt_sym(HP, st.H, HPH);
        T GRl[NY][NY], GRm[NY][NY];
#pragma unroll
        for (int a = 0; a < NY; ++a)
#pragma unroll
          for (int b = 0; b < NY; ++b) {
            T sRe = Re[a] * Re[b];
            T t2[1];
            t2[0] = T(0);
#pragma unroll
            for (int c = 0; c < NY; ++c)
#pragma unroll
              for (int d = 0; d < NY; ++d) t2[0] += st.Rinv[a][c] * HPH[c][d] * st.Rinv[d][b];
            GRl[a][b] = T(-0.5) * st.Rinv[a][b] + T(0.5) * st.dt * (sRe + t2[0]);
            GRm[a][b] = T(-0.5) * st.dt * sRe;
          }
        T xb[N];
        if constexpr (M::kNonlinear) {
#pragma unroll
          for (int a = 0; a < N; ++a) xb[a] = T(rc.xb[a]);
        } else {
#pragma unroll
          for (int a = 0; a < N; ++a) xb[a] = T(0);
        }
        if (ge != nullptr) {
          // the step's element cotangents, at the state it ends at: those of
          // loglik, then those of the objective, each A (row-major), b, C
          // (lower triangle, row order), R (lower triangle); C and R as the
          // gradient with respect to the full symmetric matrix
          constexpr int EG = ElemGradSz<N, NY>::n;
          const int64_t j = i + 1;
          int c = 0;
          auto put2 = [&](T vl, T vm) {
            ge[tix(j, c, 2 * EG)] = double(vl);
            ge[tix(j, EG + c, 2 * EG)] = double(vm);
            ++c;
          };
#pragma unroll
          for (int a = 0; a < N; ++a)
#pragma unroll
            for (int b = 0; b < N; ++b) put2(GAl[a][b], GAm[a][b]);
#pragma unroll
          for (int a = 0; a < N; ++a) put2(Gbl[a], Gbm[a]);
#pragma unroll
          for (int a = 0; a < N; ++a)
#pragma unroll
            for (int b = 0; b <= a; ++b) put2(GCl[a][b], GCm[a][b]);
#pragma unroll
          for (int a = 0; a < NY; ++a)
#pragma unroll
            for (int b = 0; b <= a; ++b) put2(GRl[a][b], GRm[a][b]);
        }
        double gl[NTH], gm[NTH];
#pragma unroll
        for (int t = 0; t < NTH; ++t) gl[t] = gm[t] = 0.0;
        M::vjp(cur.th, xb, st.dt, GAl, Gbl, GCl, GRl, gl);
        M::vjp(cur.th, xb, st.dt, GAm, Gbm, GCm, GRm, gm);
#pragma unroll
        for (int t = 0; t < NTH; ++t) {
          val[1 + t] += gl[t];
          val[1 + NTH + t] += gm[t];
        }
      }
    }
  }
}

// Prior term 1/2 |x_0 - m0|^2_{P0^{-1}} of the objective at a segment's first state.
template <typename TS, typename T, class M>
MS_DEVONLY double prior_objective(const Prob<TS>& p, const Cursor<TS, T, M>& cur,
                                  const T (&x)[M::NX]) {
  constexpr int N = M::NX;
  T S0[N][N], v0[N], m0[N], P0i[N][N];
  cur.prior(p, S0, v0, m0, P0i);
  T dlt[N], Pd[N];
#pragma unroll
  for (int a = 0; a < N; ++a) dlt[a] = x[a] - m0[a];
  mv(P0i, dlt, Pd);
  double ob = 0.0;
#pragma unroll
  for (int a = 0; a < N; ++a) ob += 0.5 * double(dlt[a]) * double(Pd[a]);
  return ob;
}

struct TrajOut {
  const void* S;
  const void* v;
  void* xs;   // [N][n_states]
  void* Ps;   // optional [Sym][n_states]
  int want_obj;
  int want_grad;
  double* g_elems;  // optional [2 ElemGradSz][n_states] (see traj_walk_state)
};

// kDepth: states prefetched ahead (rotating buffers); three keep the
// registers within two wavefronts per SIMD.
template <typename TS, typename T, class M, bool kGrad, bool kCov, int kDepth>
__global__ void __launch_bounds__(kBlock) k_traj_down(Prob<TS> p, Ws<T> ws, TrajOut to, Acc acc) {
  constexpr int N = M::NX, NY = M::NY, NW = M::NW;
  constexpr int NTH = M::NTH > 0 ? M::NTH : 1;
  constexpr int KV = 1 + 2 * NTH;
  __shared__ __align__(16) T s_step[SharedStep<T, M>::n];
  const T* sstep = shared_step<TS, T, M>(p, s_step);
  const int64_t g = logical_block() * kBlock + threadIdx.x;
  const int64_t tile = g >> 6;
  const int64_t j0 = g * ws.chunk;
  const int64_t ns = p.n_states;
  const TS* Si = static_cast<const TS*>(to.S);
  const TS* vi = static_cast<const TS*>(to.v);
  TS* xo = static_cast<TS*>(to.xs);
  TS* Po = static_cast<TS*>(to.Ps);
  T x[N], P[N][N];
  if (tile < ws.n_tiles) {
    // value after the tile's block, through the tiles after it in the block,
    // then through the lanes after this one in the tile
    const int64_t nb = (ws.n_tiles + 3) >> 2;
    load_vec(ws.stile_carry, nb, tile >> 2, x, 0);
    load_sym(ws.stile_carry, nb, tile >> 2, P, N);
    Aff<T, N> lp;
    if ((tile & 3) != 3) {
      load_aff(ws.stile_suf, ws.n_tiles, tile, lp);
      aff_apply(lp, x, P);
    }
    lt_load_aff(ws.slane_pre, g, lp);
    aff_apply(lp, x, P);
  }
  double val[KV];
#pragma unroll
  for (int t = 0; t < KV; ++t) val[t] = 0.0;
  double* dst[KV];
  int64_t dstr[KV];
  dst[0] = to.want_obj ? acc.obj : nullptr;
  dstr[0] = 1;
#pragma unroll
  for (int t = 0; t < NTH; ++t) {
    dst[1 + t] = (kGrad && M::NTH > 0 && acc.g_loglik) ? acc.g_loglik + t : nullptr;
    dst[1 + NTH + t] = (kGrad && M::NTH > 0 && acc.g_obj) ? acc.g_obj + t : nullptr;
    dstr[1 + t] = dstr[1 + NTH + t] = NTH;
  }
  int64_t seg_acc = -1;
  bool bad = false;  // a non-finite x*, P^s (MAP_CHECK_FINITE)
  const int64_t j1 = lane_end(g, ws.n_lanes, ns, ws.chunk);
  if (j0 < j1) {
    const int64_t il = j1 - 1;
    Cursor<TS, T, M> cur;
    cur.sstep = sstep;
    cur.init(p, il);
    seg_acc = cur.s;
    // Filter moments of a state and inputs of the state after it, in kDepth
    // rotating buffers: this pass streams the most data, so each buffer is
    // refilled (always issued, clamped into the lane) at the end of the state
    // that used it, for the state kDepth steps further down, and its loads have
    // kDepth - 1 whole states to arrive.  Each buffer is read in place and
    // refilled only after its last use, so the loop carries it in the same
    // registers (a register copy of a buffer would make its loads wait early).
    constexpr int K = kDepth;
    struct Ahead {
      TS S[Sym<N>::n];
      TS v[N];
      typename Cursor<TS, T, M>::Raw r;
    } q[K];
    auto refill = [&](int64_t k, Ahead& qq) {
      const int64_t ia = k >= j0 ? k : j0;
      tload_raw(Si, Sym<N>::n, ia, qq.S);
      tload_raw(vi, N, ia, qq.v);
      cur.fetch(p, ia + 1 < ns ? ia + 1 : ia, qq.r);
    };
#pragma unroll
    for (int k = 0; k < K; ++k) refill(il - k, q[k]);
    // one state of the backward walk; qq holds state i
    auto body = [&](int64_t i, Ahead& qq) {
      T S[N][N], v[N];
      sym_from_raw<TS, T, N>(qq.S, S);
      vec_from_raw(qq.v, v);
      filter_plane_in<TS>(S, v);
      const typename Cursor<TS, T, M>::Raw rc = qq.r;
      traj_walk_state<TS, T, M, kGrad>(p, cur, i, S, v, rc, to.want_obj != 0, x, P, val,
                                       to.g_elems);
      tstore_vec(xo, N, i, x);
      if constexpr (kCov) tstore_sym(Po, Sym<N>::n, i, P);
      if (ws.status) bad = bad | (kCov ? nonfinite_vd(x, P) : nonfinite_v(x));
      if (cur.is_head(i)) {
        if (to.want_obj) val[0] += prior_objective(p, cur, x);
        if (i > j0) {
          flush_lane<KV>(seg_acc, val, dst, dstr);
          cur.prev(p);
          seg_acc = cur.s;
        }
      }
      refill(i - K, qq);
    };
    drain_vmem();
    int64_t i = il;
    for (; i - (K - 1) >= j0; i -= K) {
#pragma unroll
      for (int k = 0; k < K; ++k) body(i - k, q[k]);
    }
    // the last K - 1 states at most (the rotation continues with q[0], q[1], ...)
#pragma unroll
    for (int k = 0; k < K - 1; ++k)
      if (i - k >= j0) body(i - k, q[k]);
  }
  if (ws.status) {
#pragma unroll
    for (int t = 0; t < KV; ++t) bad = bad | nonfinite(val[t]);
    report_nonfinite(ws.status, bad);
  }
  if (to.want_obj || kGrad) flush_block<KV>(seg_acc, val, dst, dstr);
}

// --------------------------------------------------------------------------- pass C'
// Two-filter combination (Sec. 4.3, eq. twofilter).  Each lane gets the run
// of the steps after its chunk (its in-tile run and the tile's run, both from
// the backward-filter up-sweep) and walks its chunk backwards: the state's
// forward value function (S, v) and the run after it give x*_k and P^s_k;
// then the step that ends at the state is put in front of the run.
template <typename TS, typename T, class M, bool kCov>
__global__ void __launch_bounds__(kBlock) k_two_filter_down(Prob<TS> p, Ws<T> ws, TrajOut to) {
  constexpr int N = M::NX, NY = M::NY, NW = M::NW;
  __shared__ __align__(16) T s_step[SharedStep<T, M>::n];
  const T* sstep = shared_step<TS, T, M>(p, s_step);
  const int64_t g = logical_block() * kBlock + threadIdx.x;
  const int64_t tile = g >> 6;
  const int64_t j0 = g * ws.chunk;
  const int64_t ns = p.n_states;
  const TS* Si = static_cast<const TS*>(to.S);
  const TS* vi = static_cast<const TS*>(to.v);
  TS* xo = static_cast<TS*>(to.xs);
  TS* Po = static_cast<TS*>(to.Ps);
  const int64_t j1 = lane_end(g, ws.n_lanes, ns, ws.chunk);
  if (j0 >= j1) return;
  // the run after the chunk: in-tile part, then (each unless the run so far
  // reached a segment start) the rest of the block's, then the block's
  Elem<T, N> s;
  {
    T f;
    lt_load_elem<T, N, true>(ws.slane_pre, g, s, &f);
    Elem<T, N> c, t;
    if (f == T(0) && (tile & 3) != 3) {
      // the rest of the block after this tile (the last tile of a block has none)
      load_selem(ws.stile_suf, ws.n_tiles, tile, c, f);
      combine(s, c, t);
      s = t;
    }
    if (f == T(0)) {
      load_elem(ws.stile_carry, (ws.n_tiles + 3) >> 2, tile >> 2, c);
      combine(s, c, t);
      s = t;
    }
  }
  const int64_t il = j1 - 1;
  Cursor<TS, T, M> cur;
  cur.sstep = sstep;
  cur.init(p, il);
  // filter moments and step inputs of a state, in three rotating buffers
  // refilled three states ahead (as in the trajectory fix-up)
  struct Ahead {
    TS S[Sym<N>::n];
    TS v[N];
    typename Cursor<TS, T, M>::Raw r;
  } q0, q1, q2;
  auto refill = [&](int64_t k, Ahead& q) {
    const int64_t ia = k >= j0 ? k : j0;
    tload_raw(Si, Sym<N>::n, ia, q.S);
    tload_raw(vi, N, ia, q.v);
    cur.fetch(p, ia, q.r);
  };
  refill(il, q0);
  refill(il - 1, q1);
  refill(il - 2, q2);
  bool bad = false;  // a non-finite x*, P^s (MAP_CHECK_FINITE)
  auto body = [&](int64_t i, Ahead& q) {
    T x[N], P[N][N];
    T S[N][N], v[N];
    sym_from_raw<TS, T, N>(q.S, S);
    vec_from_raw(q.v, v);
    filter_plane_in<TS>(S, v);
    two_filter_point<T, N, kCov>(S, v, s, x, P);
    tstore_vec(xo, N, i, x);
    if constexpr (kCov) tstore_sym(Po, Sym<N>::n, i, P);
    if (ws.status) bad = bad | (kCov ? nonfinite_vd(x, P) : nonfinite_v(x));
    if (i > j0) {
      if (cur.is_head(i)) {
        // state i - 1 ends the previous segment: nothing comes after it
        elem_identity(s);
        cur.prev(p);
      } else {
        Step<T, N, NY, NW> st;
        const typename Cursor<TS, T, M>::Raw rc = q.r;
        cur.terms(p, i, rc, st);
        T y[NY];
        rc.meas(y);
        prepend_step(st, y, s);
      }
    }
    refill(i - 3, q);
  };
  drain_vmem();
  int64_t i = il;
  for (; i - 2 >= j0; i -= 3) {
    body(i, q0);
    body(i - 1, q1);
    body(i - 2, q2);
  }
  for (; i >= j0; --i) {
    body(i, q0);
    q0 = q1;
  }
  report_nonfinite(ws.status, bad);
}

// --------------------------------------------------------------------------- IFT
// Implicit-function VJP: the gradient with respect to theta of a scalar
// l(x*) of the trajectory, given its cotangent g = dl/dx* at every state.
// x* is the stationary point of the discretised objective M_d(x; theta), so
// dx*/dtheta = -H^{-1} d(grad_x M_d)/dtheta with H the (symmetric) Hessian
// of M_d in x, and
//   dl/dtheta = -d/dtheta [mu^T grad_x M_d(x*; theta)],   mu = H^{-1} g,
// with x* and mu held fixed.  mu minimises 1/2 mu^T H mu - g^T mu: the
// problem Ift<M> (same elements with b = 0 and eta = g), solved by the
// smoother's kernels.  Differentiating the element terms
// 1/2 x_k^T J x_k - x_k^T eta + 1/2 |x_{k-1} - A x_k - b|^2_{C^{-1}} of
// mu^T grad_x M_d gives, per step k, the cotangents of the element
//   A: lam mu_k^T + nu x*_k^T,   b: nu,   C: (nu lam^T + lam nu^T) / 2,
//   R (through J = dt H^T R^{-1} H and eta = dt H^T R^{-1} (y - r)):
//      -dt (R^{-1} eps (R^{-1} H mu_k)^T + its transpose) / 2,
// with lam = C^{-1}(x*_{k-1} - A x*_k - b) = v_{k-1} - S_{k-1} x*_{k-1}, the
// costate of the problem, nu = v'_{k-1} - S_{k-1} mu_{k-1} that of the adjoint
// problem (v' its filter vector) and eps = y_k - r_k - H x*_k; no C^{-1} is
// formed, so Q may be singular.  The model's vjp maps them to theta (the
// prior has no theta).  One lane per run of kRow consecutive states, per-
// segment sums reduced over the block.
struct IftIn {
  const void* S;    // filter information matrices of the problem
  const void* v;    // its second filter plane (v, or m with FP32 storage)
  const void* vmu;  // the adjoint problem's second filter plane
  const void* xs;   // x*
  const void* mu;   // mu = H^{-1} g
};

template <typename TS, typename T, class M>
__global__ void __launch_bounds__(kBlock) k_ift_grad(Prob<TS> p, IftIn in, double* gout) {
  constexpr int N = M::NX, NY = M::NY, NW = M::NW, NTH = M::NTH;
  const TS* Si = static_cast<const TS*>(in.S);
  const TS* vi = static_cast<const TS*>(in.v);
  const TS* gi = static_cast<const TS*>(in.vmu);
  const TS* xi = static_cast<const TS*>(in.xs);
  const TS* mi = static_cast<const TS*>(in.mu);
  const int64_t g = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t ns = p.n_states;
  const int64_t j0 = g * kRow, j1 = j0 + kRow < ns ? j0 + kRow : ns;
  double val[NTH];
#pragma unroll
  for (int t = 0; t < NTH; ++t) val[t] = 0.0;
  double* dst[NTH];
  int64_t dstr[NTH];
#pragma unroll
  for (int t = 0; t < NTH; ++t) {
    dst[t] = gout + t;
    dstr[t] = NTH;
  }
  int64_t seg_acc = -1;
  if (j0 < j1) {
    Cursor<TS, T, M> cur;
    cur.init(p, j0);
    seg_acc = cur.s;
    for (int64_t i = j0; i < j1; ++i) {
      if (cur.s != seg_acc) {
        flush_lane<NTH>(seg_acc, val, dst, dstr);
        seg_acc = cur.s;
      }
      if (!cur.is_head(i)) {
        typename Cursor<TS, T, M>::Raw r;
        cur.fetch(p, i, r);
        Step<T, N, NY, NW> st;
        cur.terms(p, i, r, st);
        T y[NY];
        r.meas(y);
        T S[N][N], v[N], vg[N], xp[N], xk[N], mp[N], mk[N];
        tload_sym(Si, Sym<N>::n, i - 1, S);
        tload_vec(vi, N, i - 1, v);
        filter_plane_in<TS>(S, v);
        tload_vec(gi, N, i - 1, vg);
        filter_plane_in<TS>(S, vg);
        tload_vec(xi, N, i - 1, xp);
        tload_vec(xi, N, i, xk);
        tload_vec(mi, N, i - 1, mp);
        tload_vec(mi, N, i, mk);
        T Sx[N], Sm[N], lam[N], nu[N];
        mv(S, xp, Sx);
        mv(S, mp, Sm);
#pragma unroll
        for (int a = 0; a < N; ++a) {
          lam[a] = v[a] - Sx[a];
          nu[a] = vg[a] - Sm[a];
        }
        T GA[N][N], Gb[N], GC[N][N];
#pragma unroll
        for (int a = 0; a < N; ++a) {
          Gb[a] = nu[a];
#pragma unroll
          for (int b = 0; b < N; ++b) {
            GA[a][b] = lam[a] * mk[b] + nu[a] * xk[b];
            GC[a][b] = T(0.5) * (nu[a] * lam[b] + lam[a] * nu[b]);
          }
        }
        T Hx[NY], Hm[NY], eps[NY], Re[NY], Rm[NY];
        mv(st.H, xk, Hx);
        mv(st.H, mk, Hm);
#pragma unroll
        for (int a = 0; a < NY; ++a) eps[a] = y[a] - st.r[a] - Hx[a];
        mv(st.Rinv, eps, Re);
        mv(st.Rinv, Hm, Rm);
        T GR[NY][NY];
#pragma unroll
        for (int a = 0; a < NY; ++a)
#pragma unroll
          for (int b = 0; b < NY; ++b) GR[a][b] = T(-0.5) * st.dt * (Re[a] * Rm[b] + Rm[a] * Re[b]);
        T xb[N];
        cur.xbar(p, i, xb);
        M::vjp(cur.th, xb, st.dt, GA, Gb, GC, GR, val);
      }
      if (cur.is_last(i) && i + 1 < ns) cur.next(p);
    }
  }
  flush_block<NTH>(seg_acc, val, dst, dstr);
}

// --------------------------------------------------------------------------- misc
template <typename TS, typename T, class M>
__global__ void __launch_bounds__(kBlock) k_build_elements(Prob<TS> p, TS* out) {
  constexpr int N = M::NX;
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= p.n_states) return;
  Cursor<TS, T, M> cur;
  cur.init(p, i);
  Elem<T, N> e;
  if (cur.is_head(i)) {
    T m0[N], P0i[N][N];
    cur.prior(p, e.J, e.eta, m0, P0i);
    mzero(e.A);
    mzero(e.C);
#pragma unroll
    for (int r = 0; r < N; ++r) e.b[r] = T(0);
  } else {
    Step<T, N, M::NY, M::NW> st;
    typename Cursor<TS, T, M>::Raw r;
    cur.fetch(p, i, r);
    cur.terms(p, i, r, st);
    T y[M::NY];
    r.meas(y);
    Fresh<T, N, M::NW> f;
    fresh_from_step(st, y, f);
    cur.adjust_fresh(p, i, r, st, f);
    fresh_to_elem(f, e);
  }
  constexpr int C = ElemSz<N>::n;
  tstore_mat(out, C, i, e.A, 0);
  tstore_vec(out, C, i, e.b, N * N);
  tstore_sym(out, C, i, e.C, N * N + N);
  tstore_vec(out, C, i, e.eta, N * N + N + Sym<N>::n);
  tstore_sym(out, C, i, e.J, N * N + 2 * N + Sym<N>::n);
}

// Zero the per-segment accumulators that a pass adds into atomically.
static __global__ void __launch_bounds__(kBlock) k_zero_acc(Acc a, int64_t n_seg, int64_t nth) {
  zero_acc_grid(a, n_seg, nth);
}

}  // namespace ms
