// Register-resident small dense linear algebra for gfx950 (n <= 8).
//
// All matrices are fixed-size arrays that the compiler keeps in VGPRs after
// full unrolling.  Symmetric results are computed on the lower triangle and
// mirrored, so the mirrored entries alias the same registers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define MS_DEV __host__ __device__ __forceinline__
#define MS_DEVONLY __device__ __forceinline__

namespace ms {

// Type-exact helpers (a bare __builtin_fma on float would promote to double).
template <typename T> MS_DEV T fma_(T a, T b, T c);
template <> MS_DEV double fma_<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <> MS_DEV float fma_<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <typename T> MS_DEV T fabs_(T x);
template <> MS_DEV double fabs_<double>(double x) { return __builtin_fabs(x); }
template <> MS_DEV float fabs_<float>(float x) { return __builtin_fabsf(x); }
template <typename T> MS_DEV T sqrt_(T x);
template <> MS_DEV double sqrt_<double>(double x) { return __builtin_sqrt(x); }
template <> MS_DEV float sqrt_<float>(float x) { return __builtin_sqrtf(x); }

// Reciprocal and square root on the device: the hardware estimates (v_rcp,
// v_rsq) refined by iteration rather than the correctly rounded sequences,
// which are about twice as long on a dependent chain.  Results are within a
// few ulp, far inside the tolerances the solvers need.
//   rcp(x):          Newton-Raphson  e = 1 - x y,  y <- y + y e  (the relative
//                    error squares at each step; two steps in FP64, one in FP32).
//   sqrt_rsqrt(x):   Goldschmidt's coupled iteration from y ~ x^{-1/2}:
//                    g = x y, h = y / 2;  r = 1/2 - g h,  g <- g + g r,
//                    h <- h + h r;  g -> sqrt(x) and 2 h -> 1 / sqrt(x).
template <typename T> MS_DEV T rcp(T x);
template <> MS_DEV double rcp<double>(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double y = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, y, 1.0);
  y = __builtin_fma(y, e, y);
  e = __builtin_fma(-x, y, 1.0);
  return __builtin_fma(y, e, y);
#else
  return 1.0 / x;
#endif
}
template <> MS_DEV float rcp<float>(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  float y = __builtin_amdgcn_rcpf(x);
  float e = __builtin_fmaf(-x, y, 1.0f);
  return __builtin_fmaf(y, e, y);
#else
  return 1.0f / x;
#endif
}
// (d, di) = (sqrt(x), 1 / sqrt(x)) for x > 0
template <typename T> MS_DEV void sqrt_rsqrt(T x, T& d, T& di);
template <> MS_DEV void sqrt_rsqrt<double>(double x, double& d, double& di) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  double r = __builtin_fma(-g, h, 0.5);
  g = __builtin_fma(g, r, g);
  h = __builtin_fma(h, r, h);
  r = __builtin_fma(-g, h, 0.5);
  d = __builtin_fma(g, r, g);
  di = 2.0 * __builtin_fma(h, r, h);
#else
  d = __builtin_sqrt(x);
  di = 1.0 / d;
#endif
}
template <> MS_DEV void sqrt_rsqrt<float>(float x, float& d, float& di) {
#if defined(__HIP_DEVICE_COMPILE__)
  const float y = __builtin_amdgcn_rsqf(x);
  const float g = x * y, h = 0.5f * y;
  const float r = __builtin_fmaf(-g, h, 0.5f);
  d = __builtin_fmaf(g, r, g);
  di = 2.0f * __builtin_fmaf(h, r, h);
#else
  d = __builtin_sqrtf(x);
  di = 1.0f / d;
#endif
}
template <typename T> MS_DEV T atan2_(T y, T x);
template <> MS_DEV double atan2_<double>(double y, double x) { return ::atan2(y, x); }
template <> MS_DEV float atan2_<float>(float y, float x) { return ::atan2f(y, x); }
template <typename T> MS_DEV T floor_(T x);
template <> MS_DEV double floor_<double>(double x) { return __builtin_floor(x); }
template <> MS_DEV float floor_<float>(float x) { return __builtin_floorf(x); }

// e modulo 2 pi into [-pi, pi): e - 2 pi floor(e / (2 pi) + 1/2)
template <typename T>
MS_DEV T wrap_angle(T e) {
  constexpr double kTwoPi = 6.283185307179586476925286766559;
  constexpr double kInvTwoPi = 0.15915494309189533576888376337251;
  return e - T(kTwoPi) * floor_(e * T(kInvTwoPi) + T(0.5));
}

template <typename T> MS_DEV T log_(T x);
template <> MS_DEV double log_<double>(double x) { return ::log(x); }
template <> MS_DEV float log_<float>(float x) { return ::logf(x); }

// c = a b, a [N][K], b [K][M]
template <typename T, int N, int K, int M>
MS_DEV void mm(const T (&a)[N][K], const T (&b)[K][M], T (&c)[N][M]) {
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < M; ++j) {
      T s = a[i][0] * b[0][j];
#pragma unroll
      for (int l = 1; l < K; ++l) s = fma_(a[i][l], b[l][j], s);
      c[i][j] = s;
    }
}

// c = a^T b, a [K][N], b [K][M]
template <typename T, int N, int K, int M>
MS_DEV void mtm(const T (&a)[K][N], const T (&b)[K][M], T (&c)[N][M]) {
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < M; ++j) {
      T s = a[0][i] * b[0][j];
#pragma unroll
      for (int l = 1; l < K; ++l) s = fma_(a[l][i], b[l][j], s);
      c[i][j] = s;
    }
}

// c = a b^T, a [N][K], b [M][K]
template <typename T, int N, int K, int M>
MS_DEV void mmt(const T (&a)[N][K], const T (&b)[M][K], T (&c)[N][M]) {
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < M; ++j) {
      T s = a[i][0] * b[j][0];
#pragma unroll
      for (int l = 1; l < K; ++l) s = fma_(a[i][l], b[j][l], s);
      c[i][j] = s;
    }
}

// symmetric c = a b^T where the product is known to be symmetric (lower computed, mirrored)
template <typename T, int N, int K>
MS_DEV void mmt_sym(const T (&a)[N][K], const T (&b)[N][K], T (&c)[N][N]) {
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      T s = a[i][0] * b[j][0];
#pragma unroll
      for (int l = 1; l < K; ++l) s = fma_(a[i][l], b[j][l], s);
      c[i][j] = s;
      c[j][i] = s;
    }
}

// symmetric c = a^T b (known symmetric), a [K][N], b [K][N]
template <typename T, int N, int K>
MS_DEV void mtm_sym(const T (&a)[K][N], const T (&b)[K][N], T (&c)[N][N]) {
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      T s = a[0][i] * b[0][j];
#pragma unroll
      for (int l = 1; l < K; ++l) s = fma_(a[l][i], b[l][j], s);
      c[i][j] = s;
      c[j][i] = s;
    }
}

// c = (a b^T + b a^T) / 2 and c = (a^T b + b^T a) / 2: products that are
// symmetric only in exact arithmetic because one factor holds an inverse
// (A_E (I + C J)^{-1} C A_E^T and the like).  The inverse's rounding has an
// antisymmetric part that can exceed the product itself where the inverted
// matrix is ill-conditioned; one triangle alone keeps it, the average drops
// it.  Cost: the full N x N product.
template <typename T, int N, int K>
MS_DEV void mmt_symavg(const T (&a)[N][K], const T (&b)[N][K], T (&c)[N][N]) {
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      T s = a[i][0] * b[j][0];
#pragma unroll
      for (int l = 1; l < K; ++l) s = fma_(a[i][l], b[j][l], s);
      if (j < i) {
        T t = a[j][0] * b[i][0];
#pragma unroll
        for (int l = 1; l < K; ++l) t = fma_(a[j][l], b[i][l], t);
        s = T(0.5) * (s + t);
      }
      c[i][j] = s;
      c[j][i] = s;
    }
}
template <typename T, int N, int K>
MS_DEV void mtm_symavg(const T (&a)[K][N], const T (&b)[K][N], T (&c)[N][N]) {
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      T s = a[0][i] * b[0][j];
#pragma unroll
      for (int l = 1; l < K; ++l) s = fma_(a[l][i], b[l][j], s);
      if (j < i) {
        T t = a[0][j] * b[0][i];
#pragma unroll
        for (int l = 1; l < K; ++l) t = fma_(a[l][j], b[l][i], t);
        s = T(0.5) * (s + t);
      }
      c[i][j] = s;
      c[j][i] = s;
    }
}

// y = a x
template <typename T, int N, int K>
MS_DEV void mv(const T (&a)[N][K], const T (&x)[K], T (&y)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T s = a[i][0] * x[0];
#pragma unroll
    for (int l = 1; l < K; ++l) s = fma_(a[i][l], x[l], s);
    y[i] = s;
  }
}

// y = a^T x, a [K][N]
template <typename T, int N, int K>
MS_DEV void mtv(const T (&a)[K][N], const T (&x)[K], T (&y)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T s = a[0][i] * x[0];
#pragma unroll
    for (int l = 1; l < K; ++l) s = fma_(a[l][i], x[l], s);
    y[i] = s;
  }
}

template <typename T, int N, int M>
MS_DEV void mcopy(const T (&a)[N][M], T (&b)[N][M]) {
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < M; ++j) b[i][j] = a[i][j];
}

template <typename T, int N, int M>
MS_DEV void mzero(T (&a)[N][M]) {
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < M; ++j) a[i][j] = T(0);
}

template <typename T, int N>
MS_DEV void meye(T (&a)[N][N]) {
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) a[i][j] = i == j ? T(1) : T(0);
}

// Cholesky a = l l^T of an SPD matrix (lower triangle read).  Also returns
// the reciprocals of the diagonal, used by the triangular solves.
template <typename T, int N>
MS_DEV void chol(const T (&a)[N][N], T (&l)[N][N], T (&dinv)[N]) {
#pragma unroll
  for (int j = 0; j < N; ++j) {
    T s = a[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) s = fma_(-l[j][k], l[j][k], s);
    T d, di;
    sqrt_rsqrt(s, d, di);
    l[j][j] = d;
    dinv[j] = di;
#pragma unroll
    for (int i = j + 1; i < N; ++i) {
      T t = a[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) t = fma_(-l[i][k], l[j][k], t);
      l[i][j] = t * di;
    }
#pragma unroll
    for (int i = 0; i < j; ++i) l[i][j] = T(0);
  }
}

// Solve l z = b (forward substitution) for M right-hand sides, b [N][M] in place.
template <typename T, int N, int M>
MS_DEV void trsm_lower(const T (&l)[N][N], const T (&dinv)[N], T (&b)[N][M]) {
#pragma unroll
  for (int c = 0; c < M; ++c)
#pragma unroll
    for (int i = 0; i < N; ++i) {
      T s = b[i][c];
#pragma unroll
      for (int k = 0; k < i; ++k) s = fma_(-l[i][k], b[k][c], s);
      b[i][c] = s * dinv[i];
    }
}

// Solve l^T z = b (back substitution), b [N][M] in place.
template <typename T, int N, int M>
MS_DEV void trsm_upper_t(const T (&l)[N][N], const T (&dinv)[N], T (&b)[N][M]) {
#pragma unroll
  for (int c = 0; c < M; ++c)
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {
      T s = b[i][c];
#pragma unroll
      for (int k = i + 1; k < N; ++k) s = fma_(-l[k][i], b[k][c], s);
      b[i][c] = s * dinv[i];
    }
}

template <typename T, int N>
MS_DEV void trsv_lower(const T (&l)[N][N], const T (&dinv)[N], T (&b)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T s = b[i];
#pragma unroll
    for (int k = 0; k < i; ++k) s = fma_(-l[i][k], b[k], s);
    b[i] = s * dinv[i];
  }
}

template <typename T, int N>
MS_DEV void trsv_upper_t(const T (&l)[N][N], const T (&dinv)[N], T (&b)[N]) {
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
    T s = b[i];
#pragma unroll
    for (int k = i + 1; k < N; ++k) s = fma_(-l[k][i], b[k], s);
    b[i] = s * dinv[i];
  }
}

// Inverse of an SPD matrix through its Cholesky factor (symmetric result).
// Lower-triangular l with l l^T = a for positive semidefinite a: Cholesky
// that leaves a zero column where the pivot vanishes (at most a few ulp of the
// diagonal), as for a covariance of less than full rank.
template <typename T, int N>
MS_DEV void psd_factor(const T (&a)[N][N], T (&l)[N][N]) {
  constexpr T kRel = sizeof(T) == 8 ? T(1e-13) : T(1e-6);
#pragma unroll
  for (int j = 0; j < N; ++j) {
    T s = a[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) s = fma_(-l[j][k], l[j][k], s);
    const bool pos = s > kRel * a[j][j];
    T d, di;
    sqrt_rsqrt(pos ? s : T(1), d, di);
    l[j][j] = pos ? d : T(0);
#pragma unroll
    for (int i = j + 1; i < N; ++i) {
      T t = a[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) t = fma_(-l[i][k], l[j][k], t);
      l[i][j] = pos ? t * di : T(0);
    }
#pragma unroll
    for (int i = 0; i < j; ++i) l[i][j] = T(0);
  }
}

template <typename T, int N>
MS_DEV void spd_inv(const T (&a)[N][N], T (&out)[N][N]) {
  T l[N][N], dinv[N], li[N][N];
  chol(a, l, dinv);
  meye(li);
  trsm_lower(l, dinv, li);  // li = l^{-1}
  mtm_sym(li, li, out);     // a^{-1} = l^{-T} l^{-1}
}

// General inverse.  For n <= 4 the adjugate formula (no pivoting needed; the
// callers only invert matrices of the form I + C J with C, J positive
// semi-definite, whose determinant is at least 1).  Larger n use Gauss-Jordan
// elimination with partial pivoting.
template <typename T, int N> struct Inverse;

template <typename T> struct Inverse<T, 1> {
  static MS_DEV void run(const T (&a)[1][1], T (&o)[1][1]) { o[0][0] = rcp(a[0][0]); }
};

template <typename T> struct Inverse<T, 2> {
  static MS_DEV void run(const T (&a)[2][2], T (&o)[2][2]) {
    T det = fma_(a[0][0], a[1][1], -a[0][1] * a[1][0]);
    T di = rcp(det);
    o[0][0] = a[1][1] * di;
    o[0][1] = -a[0][1] * di;
    o[1][0] = -a[1][0] * di;
    o[1][1] = a[0][0] * di;
  }
};

template <typename T> struct Inverse<T, 3> {
  static MS_DEV void run(const T (&a)[3][3], T (&o)[3][3]) {
    T c00 = fma_(a[1][1], a[2][2], -a[1][2] * a[2][1]);
    T c01 = fma_(a[1][2], a[2][0], -a[1][0] * a[2][2]);
    T c02 = fma_(a[1][0], a[2][1], -a[1][1] * a[2][0]);
    T det = fma_(a[0][0], c00, fma_(a[0][1], c01, a[0][2] * c02));
    T di = rcp(det);
    o[0][0] = c00 * di;
    o[1][0] = c01 * di;
    o[2][0] = c02 * di;
    o[0][1] = fma_(a[0][2], a[2][1], -a[0][1] * a[2][2]) * di;
    o[1][1] = fma_(a[0][0], a[2][2], -a[0][2] * a[2][0]) * di;
    o[2][1] = fma_(a[0][1], a[2][0], -a[0][0] * a[2][1]) * di;
    o[0][2] = fma_(a[0][1], a[1][2], -a[0][2] * a[1][1]) * di;
    o[1][2] = fma_(a[0][2], a[1][0], -a[0][0] * a[1][2]) * di;
    o[2][2] = fma_(a[0][0], a[1][1], -a[0][1] * a[1][0]) * di;
  }
};

template <typename T> struct Inverse<T, 4> {
  // Laplace expansion along the first two rows: 2x2 minors s (rows 0,1) and
  // c (rows 2,3), then the 16 cofactors.
  static MS_DEV void run(const T (&m)[4][4], T (&o)[4][4]) {
    T s0 = fma_(m[0][0], m[1][1], -m[1][0] * m[0][1]);
    T s1 = fma_(m[0][0], m[1][2], -m[1][0] * m[0][2]);
    T s2 = fma_(m[0][0], m[1][3], -m[1][0] * m[0][3]);
    T s3 = fma_(m[0][1], m[1][2], -m[1][1] * m[0][2]);
    T s4 = fma_(m[0][1], m[1][3], -m[1][1] * m[0][3]);
    T s5 = fma_(m[0][2], m[1][3], -m[1][2] * m[0][3]);
    T c5 = fma_(m[2][2], m[3][3], -m[3][2] * m[2][3]);
    T c4 = fma_(m[2][1], m[3][3], -m[3][1] * m[2][3]);
    T c3 = fma_(m[2][1], m[3][2], -m[3][1] * m[2][2]);
    T c2 = fma_(m[2][0], m[3][3], -m[3][0] * m[2][3]);
    T c1 = fma_(m[2][0], m[3][2], -m[3][0] * m[2][2]);
    T c0 = fma_(m[2][0], m[3][1], -m[3][0] * m[2][1]);
    T det = s0 * c5 - s1 * c4 + s2 * c3 + s3 * c2 - s4 * c1 + s5 * c0;
    T di = rcp(det);
    o[0][0] = (m[1][1] * c5 - m[1][2] * c4 + m[1][3] * c3) * di;
    o[0][1] = (-m[0][1] * c5 + m[0][2] * c4 - m[0][3] * c3) * di;
    o[0][2] = (m[3][1] * s5 - m[3][2] * s4 + m[3][3] * s3) * di;
    o[0][3] = (-m[2][1] * s5 + m[2][2] * s4 - m[2][3] * s3) * di;
    o[1][0] = (-m[1][0] * c5 + m[1][2] * c2 - m[1][3] * c1) * di;
    o[1][1] = (m[0][0] * c5 - m[0][2] * c2 + m[0][3] * c1) * di;
    o[1][2] = (-m[3][0] * s5 + m[3][2] * s2 - m[3][3] * s1) * di;
    o[1][3] = (m[2][0] * s5 - m[2][2] * s2 + m[2][3] * s1) * di;
    o[2][0] = (m[1][0] * c4 - m[1][1] * c2 + m[1][3] * c0) * di;
    o[2][1] = (-m[0][0] * c4 + m[0][1] * c2 - m[0][3] * c0) * di;
    o[2][2] = (m[3][0] * s4 - m[3][1] * s2 + m[3][3] * s0) * di;
    o[2][3] = (-m[2][0] * s4 + m[2][1] * s2 - m[2][3] * s0) * di;
    o[3][0] = (-m[1][0] * c3 + m[1][1] * c1 - m[1][2] * c0) * di;
    o[3][1] = (m[0][0] * c3 - m[0][1] * c1 + m[0][2] * c0) * di;
    o[3][2] = (-m[3][0] * s3 + m[3][1] * s1 - m[3][2] * s0) * di;
    o[3][3] = (m[2][0] * s3 - m[2][1] * s1 + m[2][2] * s0) * di;
  }
};

template <typename T, int N> struct Inverse {
  static MS_DEV void run(const T (&a)[N][N], T (&o)[N][N]) {
    // Gauss-Jordan with partial pivoting on [a | I]; row exchanges done with
    // selects so that everything stays in registers.
    T w[N][2 * N];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < 2 * N; ++j) w[i][j] = j < N ? a[i][j] : (j - N == i ? T(1) : T(0));
#pragma unroll
    for (int k = 0; k < N; ++k) {
      T best = fabs_(w[k][k]);
      int p = k;
#pragma unroll
      for (int i = k + 1; i < N; ++i) {
        T v = fabs_(w[i][k]);
        bool gt = v > best;
        best = gt ? v : best;
        p = gt ? i : p;
      }
#pragma unroll
      for (int i = k + 1; i < N; ++i) {
        bool sw = p == i;
#pragma unroll
        for (int j = 0; j < 2 * N; ++j) {
          T t = w[k][j];
          w[k][j] = sw ? w[i][j] : t;
          w[i][j] = sw ? t : w[i][j];
        }
      }
      T d = rcp(w[k][k]);
#pragma unroll
      for (int j = 0; j < 2 * N; ++j) w[k][j] *= d;
#pragma unroll
      for (int i = 0; i < N; ++i)
        if (i != k) {
          T f = w[i][k];
#pragma unroll
          for (int j = 0; j < 2 * N; ++j) w[i][j] = fma_(-f, w[k][j], w[i][j]);
        }
    }
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) o[i][j] = w[i][N + j];
  }
};

template <typename T, int N>
MS_DEV void inv(const T (&a)[N][N], T (&o)[N][N]) { Inverse<T, N>::run(a, o); }

// ---------------------------------------------------------------- wave shuffles
// 64-bit values move as two 32-bit halves through ds_bpermute.
MS_DEVONLY double shfl(double v, int src) {
  int2 p = *reinterpret_cast<int2*>(&v);
  p.x = __builtin_amdgcn_ds_bpermute(src << 2, p.x);
  p.y = __builtin_amdgcn_ds_bpermute(src << 2, p.y);
  return *reinterpret_cast<double*>(&p);
}
MS_DEVONLY float shfl(float v, int src) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}
MS_DEVONLY int shfl(int v, int src) { return __builtin_amdgcn_ds_bpermute(src << 2, v); }

template <typename T, int N, int M>
MS_DEVONLY void shfl_mat(T (&a)[N][M], const T (&src)[N][M], int lane) {
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < M; ++j) a[i][j] = shfl(src[i][j], lane);
}

template <typename T, int N>
MS_DEVONLY void shfl_sym(T (&a)[N][N], const T (&src)[N][N], int lane) {
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      a[i][j] = shfl(src[i][j], lane);
      a[j][i] = a[i][j];
    }
}

template <typename T, int N>
MS_DEVONLY void shfl_vec(T (&a)[N], const T (&src)[N], int lane) {
#pragma unroll
  for (int i = 0; i < N; ++i) a[i] = shfl(src[i], lane);
}

}  // namespace ms
