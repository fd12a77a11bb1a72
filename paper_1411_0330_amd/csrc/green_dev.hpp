// Device evaluation of the discrete Green operators applied to one
// wave-vector's c-vector of polarisation spectra.
//
// Gamma0_hat(xi) = xi xi^T / (xi^T A0 xi) (Section 2.2.1; zero at xi = 0).
// Truncated (eqs. 14/15): xi = centred index; if any axis of even length sits
// at N/2 the operator is A0^{-1} (Nyquist rule of Section 3.2.1).
// Filtered (Section 3.2.2): sum over the 2^d aliases k_a and k_a - N_a with
// weights prod cos^2(pi k_a/(2N_a)) / sin^2(pi k_a/(2N_a)), k_a in [0, N_a).
// Physical frequencies are used (alias k + nN); Gamma0_hat has degree 0.
//
// Elasticity with an isotropic reference (lambda0, mu0): for a unit direction
// n, Gamma0_hat tau = (n (x) tau n + tau n (x) n)/(2 mu0)
//                    - kappa (n.tau.n) n (x) n,  kappa = (lambda0+mu0)/(mu0 (lambda0+2 mu0)),
// which follows from the acoustic tensor mu0 |xi|^2 I + (lambda0+mu0) xi xi^T.
// A sum of such terms with weights w is carried by B = sum w n n^T and the
// fully symmetric D = sum w n n n n:  out = (B tau + tau B)/(2 mu0) - kappa D:tau.
#pragma once

#include "fft_dev.hpp"

namespace lsh {

enum : int { kGreenTruncated = 0, kGreenFiltered = 1, kGreenConsistent = 2, kGreenFD = 3 };

// Parameters shared by all wave-vectors (kernel argument, by value).
struct GreenParams {
  int variant;
  int n[3];          // grid along x, y, z (n[2] = 1 in 2D)
  double a0[9];      // scalar reference, row-major 3x3 (2D uses the top-left 2x2)
  double a0inv[9];
  double mu0, kappa; // elastic reference
  double s0_diag;    // Mandel compliance: 1/(2 mu0) on the diagonal ...
  double s0_vol;     // ... plus s0_vol on the 3x3 normal block
};

// Device tables of the Green operators:
//  w      per-axis filter weights, w[a*wstride + k] = (cos^2, sin^2)(pi k/(2 N_a));
//  tw[a]  per-axis twiddles exp(-2 pi i m / N_a) (finite differences);
//  tab    stored operator (consistent): the upper triangle (row-major, c(c+1)/2
//         entries) of the real symmetric c x c matrix at every stored
//         wave-vector, main spectrum order then the Nyquist plane.
template <typename T>
struct GreenTabs {
  const cpx<T>* w;
  int wstride;
  const cpx<T>* tw[3];
  const T* tab;
  const T* st;   // stored operator of the z pass (layout below), or nullptr
};

// ----------------------------------------------------------------------------
// Stored operator of the z pass.  The matrix of one wave-vector (the upper
// triangle of green_matrix, padded with zeros to NG groups of four entries)
// is formed once per reference medium, in FP64, and kept in the field type.
// Group g of wave-vector (kx, ky, kz) sits at
//   main spectrum  ((kz ny + ky) NG + g) mx + kx
//   Nyquist plane  nz ny mx NG + (kz NG + g) ny + ky
// (in units of four entries), so the TX pencils of a z tile read each group
// as one contiguous run of TX quads.
// ----------------------------------------------------------------------------
template <typename T>
struct alignas(4 * sizeof(T)) Quad {
  T a, b, c, d;
};

template <int C>
constexpr int store_groups() {
  return (C * (C + 1) / 2 + 3) / 4;
}

// The NE = C(C+1)/2 entries of the wave-vector whose group 0 is at q, groups
// `gstride` quads apart.
template <typename T, int C>
__device__ __forceinline__ void stored_matrix(const Quad<T>* __restrict__ q, const long long gstride,
                                              T (&G)[C * (C + 1) / 2]) {
  constexpr int NE = C * (C + 1) / 2, NG = store_groups<C>();
  T e[4 * NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    const Quad<T> v = q[g * gstride];
    e[4 * g] = v.a;
    e[4 * g + 1] = v.b;
    e[4 * g + 2] = v.c;
    e[4 * g + 3] = v.d;
  }
#pragma unroll
  for (int i = 0; i < NE; ++i) G[i] = e[i];
}

// Stored symmetric table applied to a c-vector
template <typename T, int D>
__device__ __forceinline__ void green_table_apply(const T* e, cpx<T> (&v)[D]) {
  T M[D][D];
  int q = 0;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i; j < D; ++j) {
      M[i][j] = M[j][i] = e[q];
      ++q;
    }
  cpx<T> o[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    o[i] = cpx<T>{0, 0};
#pragma unroll
    for (int j = 0; j < D; ++j) {
      o[i].x += M[i][j] * v[j].x;
      o[i].y += M[i][j] * v[j].y;
    }
  }
#pragma unroll
  for (int i = 0; i < D; ++i) v[i] = o[i];
}

// Finite-difference operator of Section 3.2.3 (scalar problems):
// V V^H / (V^H A0 V) with V_a = (exp(2 i pi k_a/N_a) - 1) N_a, zero at k = 0.
template <typename T, int D>
__device__ __forceinline__ void green_fd(const GreenParams& gp, const GreenTabs<T>& tb, const int (&k)[3],
                                         cpx<T> (&v)[D]) {
  cpx<T> V[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const cpx<T> wv = tb.tw[a][k[a]];                       // exp(-2 pi i k/N)
    const T n = static_cast<T>(gp.n[a]);
    V[a] = cpx<T>{(wv.x - T(1)) * n, -wv.y * n};            // (exp(+2 pi i k/N) - 1) N
  }
  T den = 0;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const T a = static_cast<T>(gp.a0[3 * i + j]);
      den += a * (V[i].x * V[j].x + V[i].y * V[j].y);       // Re(conj(V_i) A_ij V_j)
    }
  if (!(den > T(0))) {
#pragma unroll
    for (int i = 0; i < D; ++i) v[i] = cpx<T>{0, 0};
    return;
  }
  cpx<T> s{0, 0};                                           // V^H v
#pragma unroll
  for (int i = 0; i < D; ++i) s = cadd(s, cmulc(v[i], V[i]));
  const T inv = T(1) / den;
#pragma unroll
  for (int i = 0; i < D; ++i) v[i] = cscale(cmul(V[i], s), inv);
}

// reciprocal: the FP32 path uses the hardware reciprocal (1 ulp), FP64 divides
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// ----------------------------------------------------------------------------
// scalar conduction, D = 2 or 3 components, general symmetric A0
// ----------------------------------------------------------------------------
template <typename T, int D>
__device__ __forceinline__ void green_scalar(const GreenParams& gp, const GreenTabs<T>& tb, const int (&k)[3],
                                             cpx<T> (&v)[D]) {
  T A[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) A[i][j] = static_cast<T>(gp.a0[3 * i + j]);

  if (gp.variant == kGreenTruncated) {
    bool nyq = false, zero = true;
    T xi[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int n = gp.n[a];
      const int kc = (k[a] <= n / 2) ? k[a] : k[a] - n;
      xi[a] = static_cast<T>(kc);
      nyq |= ((n & 1) == 0) && (k[a] == n / 2);
      zero &= (k[a] == 0);
    }
    if (nyq) {
      cpx<T> o[D];
#pragma unroll
      for (int i = 0; i < D; ++i) {
        o[i] = cpx<T>{0, 0};
#pragma unroll
        for (int j = 0; j < D; ++j) {
          const T m = static_cast<T>(gp.a0inv[3 * i + j]);
          o[i].x += m * v[j].x;
          o[i].y += m * v[j].y;
        }
      }
#pragma unroll
      for (int i = 0; i < D; ++i) v[i] = o[i];
      return;
    }
    if (zero) {
#pragma unroll
      for (int i = 0; i < D; ++i) v[i] = cpx<T>{0, 0};
      return;
    }
    T den = 0;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) den += xi[i] * A[i][j] * xi[j];
    cpx<T> s{0, 0};
#pragma unroll
    for (int i = 0; i < D; ++i) {
      s.x += xi[i] * v[i].x;
      s.y += xi[i] * v[i].y;
    }
    const T inv = T(1) / den;
#pragma unroll
    for (int i = 0; i < D; ++i) v[i] = cpx<T>{xi[i] * s.x * inv, xi[i] * s.y * inv};
    return;
  }

  // filtered: M = sum_aliases w xi xi^T / (xi^T A0 xi)
  T M[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) M[i][j] = 0;
  cpx<T> wa[D];
#pragma unroll
  for (int a = 0; a < D; ++a) wa[a] = tb.w[a * tb.wstride + k[a]];
#pragma unroll
  for (int alias = 0; alias < (1 << D); ++alias) {
    T w = 1;
    T xi[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const bool lo = (alias >> a) & 1;  // alias k_a - N_a
      w *= lo ? wa[a].y : wa[a].x;
      xi[a] = static_cast<T>(lo ? k[a] - gp.n[a] : k[a]);
    }
    T den = 0;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) den += xi[i] * A[i][j] * xi[j];
    if (w != T(0) && den > T(0)) {
      const T f = w * recip(den);
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) M[i][j] += f * xi[i] * xi[j];
    }
  }
  cpx<T> o[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    o[i] = cpx<T>{0, 0};
#pragma unroll
    for (int j = 0; j < D; ++j) {
      o[i].x += M[i][j] * v[j].x;
      o[i].y += M[i][j] * v[j].y;
    }
  }
#pragma unroll
  for (int i = 0; i < D; ++i) v[i] = o[i];
}

// ----------------------------------------------------------------------------
// isotropic elasticity, Mandel 6-vectors
// ----------------------------------------------------------------------------
template <typename T>
struct BD {
  T b11, b22, b33, b23, b13, b12;
  T d1111, d2222, d3333, d1122, d1133, d2233;
  T d1112, d1113, d2221, d2223, d3331, d3332, d1123, d2213, d3312;
};

template <typename T>
__device__ __forceinline__ void bd_zero(BD<T>& s) {
  s.b11 = s.b22 = s.b33 = s.b23 = s.b13 = s.b12 = 0;
  s.d1111 = s.d2222 = s.d3333 = s.d1122 = s.d1133 = s.d2233 = 0;
  s.d1112 = s.d1113 = s.d2221 = s.d2223 = s.d3331 = s.d3332 = s.d1123 = s.d2213 = s.d3312 = 0;
}

// accumulate weight w along frequency xi (any length; normalised here)
template <typename T>
__device__ __forceinline__ void bd_add(BD<T>& s, T w, T a, T b, T c) {
  const T aa = a * a, bb = b * b, cc = c * c;
  const T n2 = aa + bb + cc;
  // no branch: a zero wave-vector (or weight) adds zeros
  const T inv = (n2 > T(0)) ? recip(n2) : T(0);
  const T q = w * inv;      // w / |xi|^2
  const T u = q * inv;      // w / |xi|^4
  const T ab = a * b, ac = a * c, bc = b * c;
  s.b11 += q * aa; s.b22 += q * bb; s.b33 += q * cc;
  s.b23 += q * bc; s.b13 += q * ac; s.b12 += q * ab;
  const T ua = u * aa, ub = u * bb, uc = u * cc;
  s.d1111 += ua * aa; s.d2222 += ub * bb; s.d3333 += uc * cc;
  s.d1122 += ua * bb; s.d1133 += ua * cc; s.d2233 += ub * cc;
  s.d1112 += ua * ab; s.d1113 += ua * ac;
  s.d2221 += ub * ab; s.d2223 += ub * bc;
  s.d3331 += uc * ac; s.d3332 += uc * bc;
  s.d1123 += ua * bc; s.d2213 += ub * ac; s.d3312 += uc * ab;
}

// out = (B t + t B)/(2 mu0) - kappa D:t on one real symmetric tensor (Mandel in/out)
template <typename T>
__device__ __forceinline__ void bd_apply_real(const BD<T>& s, T inv2mu, T kappa, const T (&m)[6], T (&o)[6]) {
  constexpr T r2 = T(1.4142135623730950488);
  constexpr T ir2 = T(0.70710678118654752440);
  const T t11 = m[0], t22 = m[1], t33 = m[2], t23 = m[3] * ir2, t13 = m[4] * ir2, t12 = m[5] * ir2;
  // symmetric part of B t (doubled)
  const T s11 = 2 * (s.b11 * t11 + s.b12 * t12 + s.b13 * t13);
  const T s22 = 2 * (s.b12 * t12 + s.b22 * t22 + s.b23 * t23);
  const T s33 = 2 * (s.b13 * t13 + s.b23 * t23 + s.b33 * t33);
  const T s23 = s.b12 * t13 + s.b22 * t23 + s.b23 * t33 + s.b13 * t12 + s.b23 * t22 + s.b33 * t23;
  const T s13 = s.b11 * t13 + s.b12 * t23 + s.b13 * t33 + s.b13 * t11 + s.b23 * t12 + s.b33 * t13;
  const T s12 = s.b11 * t12 + s.b12 * t22 + s.b13 * t23 + s.b12 * t11 + s.b22 * t12 + s.b23 * t13;
  // D : t
  const T e23 = 2 * t23, e13 = 2 * t13, e12 = 2 * t12;
  const T d11 = s.d1111 * t11 + s.d1122 * t22 + s.d1133 * t33 + s.d1123 * e23 + s.d1113 * e13 + s.d1112 * e12;
  const T d22 = s.d1122 * t11 + s.d2222 * t22 + s.d2233 * t33 + s.d2223 * e23 + s.d2213 * e13 + s.d2221 * e12;
  const T d33 = s.d1133 * t11 + s.d2233 * t22 + s.d3333 * t33 + s.d3332 * e23 + s.d3331 * e13 + s.d3312 * e12;
  const T d23 = s.d1123 * t11 + s.d2223 * t22 + s.d3332 * t33 + s.d2233 * e23 + s.d3312 * e13 + s.d2213 * e12;
  const T d13 = s.d1113 * t11 + s.d2213 * t22 + s.d3331 * t33 + s.d3312 * e23 + s.d1133 * e13 + s.d1123 * e12;
  const T d12 = s.d1112 * t11 + s.d2221 * t22 + s.d3312 * t33 + s.d2213 * e23 + s.d1123 * e13 + s.d1122 * e12;
  o[0] = s11 * inv2mu - kappa * d11;
  o[1] = s22 * inv2mu - kappa * d22;
  o[2] = s33 * inv2mu - kappa * d33;
  o[3] = r2 * (s23 * inv2mu - kappa * d23);
  o[4] = r2 * (s13 * inv2mu - kappa * d13);
  o[5] = r2 * (s12 * inv2mu - kappa * d12);
}

// ----------------------------------------------------------------------------
// The operator at one wave-vector as a real symmetric c x c matrix (upper
// triangle, row-major, c(c+1)/2 entries): truncated, filtered and consistent
// operators (the finite-difference one is complex Hermitian and stays with
// green_apply).  Used where one matrix serves several loads.
// ----------------------------------------------------------------------------
// Mandel matrix of (B t + t B)/(2 mu0) - kappa D:t.  With the tensor
// (d_ik B_jl + d_il B_jk + d_jk B_il + d_jl B_ik)/(4 mu0) - kappa D_ijkl and
// weights 1 (normal) and sqrt 2 (shear) per Mandel index.
template <typename T>
__device__ __forceinline__ void bd_matrix(const BD<T>& s, T inv2mu, T kappa, T (&G)[21]) {
  constexpr T r2 = T(1.4142135623730950488);
  const T im = T(2) * inv2mu, h = inv2mu, k2 = T(2) * kappa;
  // row 0: (11, .)
  G[0] = s.b11 * im - kappa * s.d1111;
  G[1] = -kappa * s.d1122;
  G[2] = -kappa * s.d1133;
  G[3] = -r2 * kappa * s.d1123;
  G[4] = r2 * (s.b13 * h - kappa * s.d1113);
  G[5] = r2 * (s.b12 * h - kappa * s.d1112);
  // row 1: (22, .)
  G[6] = s.b22 * im - kappa * s.d2222;
  G[7] = -kappa * s.d2233;
  G[8] = r2 * (s.b23 * h - kappa * s.d2223);
  G[9] = -r2 * kappa * s.d2213;
  G[10] = r2 * (s.b12 * h - kappa * s.d2221);
  // row 2: (33, .)
  G[11] = s.b33 * im - kappa * s.d3333;
  G[12] = r2 * (s.b23 * h - kappa * s.d3332);
  G[13] = r2 * (s.b13 * h - kappa * s.d3331);
  G[14] = -r2 * kappa * s.d3312;
  // rows 3..5: shear-shear
  G[15] = (s.b22 + s.b33) * h - k2 * s.d2233;
  G[16] = s.b12 * h - k2 * s.d3312;
  G[17] = s.b13 * h - k2 * s.d2213;
  G[18] = (s.b11 + s.b33) * h - k2 * s.d1133;
  G[19] = s.b23 * h - k2 * s.d1123;
  G[20] = (s.b11 + s.b22) * h - k2 * s.d1122;
}

template <typename T, int C>
__device__ __forceinline__ void green_matrix(const GreenParams& gp, const GreenTabs<T>& tb, const int (&k)[3],
                                             long long tidx, T (&G)[C * (C + 1) / 2]) {
  constexpr int NE = C * (C + 1) / 2;
  if (gp.variant == kGreenConsistent) {
    const T* e = tb.tab + tidx * NE;
#pragma unroll
    for (int q = 0; q < NE; ++q) G[q] = e[q];
    return;
  }
  bool nyq = false, zero = true;
  T xi[3] = {T(0), T(0), T(0)};
  constexpr int D = (C == 6) ? 3 : C;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const int n = gp.n[a];
    const int kc = (k[a] <= n / 2) ? k[a] : k[a] - n;
    xi[a] = static_cast<T>(kc);
    nyq |= ((n & 1) == 0) && (k[a] == n / 2);
    zero &= (k[a] == 0);
  }
  if (gp.variant == kGreenTruncated && (nyq || zero)) {
    // A0^{-1} at the Nyquist frequencies, zero at k = 0
    int q = 0;
#pragma unroll
    for (int i = 0; i < C; ++i)
#pragma unroll
      for (int j = i; j < C; ++j) {
        T v = T(0);
        if (nyq) {
          if constexpr (C == 6) v = (i == j ? static_cast<T>(gp.s0_diag) : T(0)) + ((i < 3 && j < 3) ? static_cast<T>(gp.s0_vol) : T(0));
          else v = static_cast<T>(gp.a0inv[3 * i + j]);
        }
        G[q++] = v;
      }
    return;
  }
  if constexpr (C == 6) {
    BD<T> s;
    bd_zero(s);
    if (gp.variant == kGreenTruncated) {
      bd_add(s, T(1), xi[0], xi[1], xi[2]);
    } else {
      cpx<T> wa[3];
      T x0[3], x1[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        wa[a] = tb.w[a * tb.wstride + k[a]];
        x0[a] = static_cast<T>(k[a]);
        x1[a] = static_cast<T>(k[a] - gp.n[a]);
      }
      const T wxy[4] = {wa[0].x * wa[1].x, wa[0].y * wa[1].x, wa[0].x * wa[1].y, wa[0].y * wa[1].y};
#pragma unroll
      for (int alias = 0; alias < 8; ++alias) {
        const T w = wxy[alias & 3] * ((alias & 4) ? wa[2].y : wa[2].x);
        bd_add(s, w, (alias & 1) ? x1[0] : x0[0], (alias & 2) ? x1[1] : x0[1], (alias & 4) ? x1[2] : x0[2]);
      }
    }
    bd_matrix(s, static_cast<T>(0.5 / gp.mu0), static_cast<T>(gp.kappa), G);
  } else {
    T A[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) A[i][j] = static_cast<T>(gp.a0[3 * i + j]);
    T M[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) M[i][j] = 0;
    if (gp.variant == kGreenTruncated) {
      T den = 0;
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) den += xi[i] * A[i][j] * xi[j];
      const T inv = T(1) / den;
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) M[i][j] = xi[i] * xi[j] * inv;
    } else {
      cpx<T> wa[D];
#pragma unroll
      for (int a = 0; a < D; ++a) wa[a] = tb.w[a * tb.wstride + k[a]];
#pragma unroll
      for (int alias = 0; alias < (1 << D); ++alias) {
        T w = 1;
        T x[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
          const bool lo = (alias >> a) & 1;
          w *= lo ? wa[a].y : wa[a].x;
          x[a] = static_cast<T>(lo ? k[a] - gp.n[a] : k[a]);
        }
        T den = 0;
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
          for (int j = 0; j < D; ++j) den += x[i] * A[i][j] * x[j];
        if (w != T(0) && den > T(0)) {
          const T f = w * recip(den);
#pragma unroll
          for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) M[i][j] += f * x[i] * x[j];
        }
      }
    }
    int q = 0;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = i; j < D; ++j) G[q++] = M[i][j];
  }
}

// Symmetric matrix (upper triangle, row-major) applied to a complex c-vector.
template <typename T, int C>
__device__ __forceinline__ void sym_apply(const T (&G)[C * (C + 1) / 2], cpx<T> (&v)[C]) {
  cpx<T> o[C];
#pragma unroll
  for (int i = 0; i < C; ++i) o[i] = cpx<T>{0, 0};
  int q = 0;
#pragma unroll
  for (int i = 0; i < C; ++i)
#pragma unroll
    for (int j = i; j < C; ++j) {
      const T g = G[q++];
      o[i].x += g * v[j].x;
      o[i].y += g * v[j].y;
      if (j != i) {
        o[j].x += g * v[i].x;
        o[j].y += g * v[i].y;
      }
    }
#pragma unroll
  for (int i = 0; i < C; ++i) v[i] = o[i];
}

template <typename T>
__device__ __forceinline__ void green_elastic(const GreenParams& gp, const GreenTabs<T>& tb, const int (&k)[3],
                                              cpx<T> (&v)[6]) {
  const T inv2mu = static_cast<T>(0.5 / gp.mu0);
  const T kappa = static_cast<T>(gp.kappa);
  BD<T> s;
  bd_zero(s);
  if (gp.variant == kGreenTruncated) {
    bool nyq = false, zero = true;
    T xi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int n = gp.n[a];
      const int kc = (k[a] <= n / 2) ? k[a] : k[a] - n;
      xi[a] = static_cast<T>(kc);
      nyq |= ((n & 1) == 0) && (k[a] == n / 2);
      zero &= (k[a] == 0);
    }
    if (nyq) {
      const T dg = static_cast<T>(gp.s0_diag), vol = static_cast<T>(gp.s0_vol);
      const cpx<T> tr{v[0].x + v[1].x + v[2].x, v[0].y + v[1].y + v[2].y};
#pragma unroll
      for (int i = 0; i < 6; ++i) v[i] = cpx<T>{dg * v[i].x, dg * v[i].y};
#pragma unroll
      for (int i = 0; i < 3; ++i) v[i] = cpx<T>{v[i].x + vol * tr.x, v[i].y + vol * tr.y};
      return;
    }
    if (zero) {
#pragma unroll
      for (int i = 0; i < 6; ++i) v[i] = cpx<T>{0, 0};
      return;
    }
    bd_add(s, T(1), xi[0], xi[1], xi[2]);
  } else {
    cpx<T> wa[3];
    T x0[3], x1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      wa[a] = tb.w[a * tb.wstride + k[a]];
      x0[a] = static_cast<T>(k[a]);
      x1[a] = static_cast<T>(k[a] - gp.n[a]);
    }
    const T wxy[4] = {wa[0].x * wa[1].x, wa[0].y * wa[1].x, wa[0].x * wa[1].y, wa[0].y * wa[1].y};
#pragma unroll
    for (int alias = 0; alias < 8; ++alias) {
      const T w = wxy[alias & 3] * ((alias & 4) ? wa[2].y : wa[2].x);
      bd_add(s, w, (alias & 1) ? x1[0] : x0[0], (alias & 2) ? x1[1] : x0[1], (alias & 4) ? x1[2] : x0[2]);
    }
  }
  // the Mandel matrix once, applied to the real and imaginary parts together
  T G[21];
  bd_matrix(s, inv2mu, kappa, G);
  sym_apply<T, 6>(G, v);
}

// Dispatch on the operator; `tidx` is the wave-vector's position in the
// stored table (consistent operator only).
template <typename T, int C>
__device__ __forceinline__ void green_apply(const GreenParams& gp, const GreenTabs<T>& tb, const int (&k)[3],
                                            long long tidx, cpx<T> (&v)[C]) {
  if (gp.variant == kGreenConsistent) {
    green_table_apply<T, C>(tb.tab + tidx * (C * (C + 1) / 2), v);
    return;
  }
  if constexpr (C == 6) {
    green_elastic<T>(gp, tb, k, v);
  } else {
    if (gp.variant == kGreenFD) {
      green_fd<T, C>(gp, tb, k, v);
      return;
    }
    green_scalar<T, C>(gp, tb, k, v);
  }
}

}  // namespace lsh
