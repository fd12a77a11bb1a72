// Device building blocks: complex arithmetic, compile-time loops, in-register
// DFTs and the pencil FFT used by every transform pass.
//
// The transform is the unnormalised DFT of Section 3.1 (sign -1 forward, +1
// inverse; the 1/N^d of DFT^{-1} is applied once by the last pass).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <utility>

#include "twiddle_consts.hpp"

namespace lsh {

template <typename T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };
template <typename T> using cpx = typename Vec2<T>::type;

template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return V{a.x + b.x, a.y + b.y}; }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return V{a.x - b.x, a.y - b.y}; }
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
  return V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename V> __device__ __forceinline__ V cmulc(V a, V b) {
  return V{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename V> __device__ __forceinline__ V cconj(V a) { return V{a.x, -a.y}; }
template <typename V, typename S> __device__ __forceinline__ V cscale(V a, S s) { return V{a.x * s, a.y * s}; }
template <typename V> __device__ __forceinline__ V mul_i(V a) { return V{-a.y, a.x}; }      // i a
template <typename V> __device__ __forceinline__ V mul_neg_i(V a) { return V{a.y, -a.x}; }  // -i a

// ---------------------------------------------------------------------------
// compile-time loops
// ---------------------------------------------------------------------------
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(std::forward<F>(f));
  }
}

template <int N> struct ILog2 { static constexpr int value = 1 + ILog2<N / 2>::value; };
template <> struct ILog2<1> { static constexpr int value = 0; };

template <int K, int BITS> struct BitRev {
  static constexpr int value = ((K & 1) << (BITS - 1)) | BitRev<(K >> 1), BITS - 1>::value;
};
template <int K> struct BitRev<K, 0> { static constexpr int value = 0; };

// v * exp(DIR * 2 pi i M / 64), DIR = -1 (forward) or +1 (inverse).
template <int M, int DIR, typename V>
__device__ __forceinline__ V twc(V v) {
  constexpr int m = M & 63;
  if constexpr (m == 0) {
    return v;
  } else if constexpr (m == 16) {
    return DIR < 0 ? mul_neg_i(v) : mul_i(v);
  } else if constexpr (m == 32) {
    return V{-v.x, -v.y};
  } else if constexpr (m == 48) {
    return DIR < 0 ? mul_i(v) : mul_neg_i(v);
  } else {
    using T = decltype(v.x);
    const T c = static_cast<T>(kCos64[m]);
    const T s = static_cast<T>(DIR * kSin64[m]);
    return V{v.x * c - v.y * s, v.x * s + v.y * c};
  }
}

// In-place R-point DFT of a register array (R a power of two <= 64):
// radix-2 decimation in frequency, then a compile-time bit reversal.
template <int R, int DIR, typename V>
__device__ __forceinline__ void dft(V* a) {
  if constexpr (R == 2) {
    const V u = a[0], w = a[1];
    a[0] = cadd(u, w);
    a[1] = csub(u, w);
  } else if constexpr (R > 2) {
    constexpr int LG = ILog2<R>::value;
    static_for<0, LG>([&](auto s_) {
      constexpr int s = decltype(s_)::value;
      constexpr int h = R >> (s + 1);
      static_for<0, R / (2 * h)>([&](auto g_) {
        constexpr int g = decltype(g_)::value * 2 * h;
        static_for<0, h>([&](auto j_) {
          constexpr int j = decltype(j_)::value;
          const V u = a[g + j], w = a[g + j + h];
          a[g + j] = cadd(u, w);
          a[g + j + h] = twc<j * (64 / (2 * h)), DIR>(csub(u, w));
        });
      });
    });
    V t[R];
    static_for<0, R>([&](auto k_) {
      constexpr int k = decltype(k_)::value;
      t[k] = a[BitRev<k, LG>::value];
    });
    static_for<0, R>([&](auto k_) {
      constexpr int k = decltype(k_)::value;
      a[k] = t[k];
    });
  }
}

// ---------------------------------------------------------------------------
// Pencil FFT (Stockham autosort, radix P with a smaller last radix).
//
// An N-point pencil is spread over TT = N/P threads; thread t holds
// v[j] = x[t + TT*j] on entry and X[t + TT*j] on exit.  Stages exchange data
// through `lds` (element e at lds[e*es]); the stage of span NS and radix R
// multiplies its inputs by W_{NS R}^{r k} read from `tw`, which holds
// W_L^m = exp(-2 pi i m / L) at tw[m] for a table length L = N * tstride.
// Every thread of the workgroup must call this the same number of times
// (it contains barriers).
// ---------------------------------------------------------------------------
template <int N, int P, int NS, int DIR, typename T>
__device__ __forceinline__ void fft_stages(cpx<T> (&v)[P], int t, cpx<T>* lds, int es, const cpx<T>* __restrict__ tw,
                                           int tstride) {
  if constexpr (NS < N) {
    constexpr int R = (N / NS < P) ? N / NS : P;
    constexpr int TT = N / P;
    constexpr bool last = (NS * R == N);
    static_for<0, P / R>([&](auto i_) {
      constexpr int i = decltype(i_)::value;
      cpx<T> u[R];
      static_for<0, R>([&](auto r_) {
        constexpr int r = decltype(r_)::value;
        u[r] = v[i + r * (P / R)];
      });
      const int b = t + TT * i;
      const int k = b & (NS - 1);
      if constexpr (NS > 1) {
        static_for<1, R>([&](auto r_) {
          constexpr int r = decltype(r_)::value;
          cpx<T> w = tw[(r * k * (N / (NS * R))) * tstride];
          if constexpr (DIR > 0) w.y = -w.y;
          u[r] = cmul(u[r], w);
        });
      }
      dft<R, DIR>(u);
      if constexpr (last) {
        static_for<0, R>([&](auto r_) {
          constexpr int r = decltype(r_)::value;
          v[i + r * (P / R)] = u[r];
        });
      } else {
        const int base = (b / NS) * NS * R + k;
        static_for<0, R>([&](auto r_) {
          constexpr int r = decltype(r_)::value;
          lds[(base + r * NS) * es] = u[r];
        });
      }
    });
    if constexpr (!last) {
      __syncthreads();
      static_for<0, P>([&](auto j_) {
        constexpr int j = decltype(j_)::value;
        v[j] = lds[(t + TT * j) * es];
      });
      __syncthreads();
      fft_stages<N, P, NS * R, DIR, T>(v, t, lds, es, tw, tstride);
    }
  }
}

template <int N, int P, int DIR, typename T>
__device__ __forceinline__ void fft_pencil(cpx<T> (&v)[P], int t, cpx<T>* lds, int es, const cpx<T>* __restrict__ tw,
                                           int tstride) {
  static_assert(P <= N || N == 1, "points per thread exceed the pencil length");
  fft_stages<N, P, 1, DIR, T>(v, t, lds, es, tw, tstride);
}

}  // namespace lsh
