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

// Streaming (non-temporal) global access of one complex value: fields and
// spectra are touched once per pass and come back from HBM in the next one.
template <typename V>
__device__ __forceinline__ V ld_stream(const V* p) {
  using T = std::remove_cv_t<std::remove_reference_t<decltype(V{}.x)>>;
  typedef T N __attribute__((ext_vector_type(2)));
  const N v = __builtin_nontemporal_load(reinterpret_cast<const N*>(p));
  return V{v.x, v.y};
}
template <typename V>
__device__ __forceinline__ void st_stream(V* p, const V& v) {
  using T = std::remove_cv_t<std::remove_reference_t<decltype(V{}.x)>>;
  typedef T N __attribute__((ext_vector_type(2)));
  const N w = {v.x, v.y};
  __builtin_nontemporal_store(w, reinterpret_cast<N*>(p));
}

// 16-byte (four-float) forms, for component pairs of the paired spectrum layout
__device__ __forceinline__ float4 ld_stream4(const float4* p) {
  typedef float N __attribute__((ext_vector_type(4)));
  const N v = __builtin_nontemporal_load(reinterpret_cast<const N*>(p));
  return float4{v.x, v.y, v.z, v.w};
}
__device__ __forceinline__ void st_stream4(float4* p, const float4& v) {
  typedef float N __attribute__((ext_vector_type(4)));
  const N w = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(w, reinterpret_cast<N*>(p));
}

// Streaming access only where one access instruction covers whole 128-byte
// lines (W contiguous bytes per row segment).  Narrower segments read each
// line in two halves by consecutive instructions, and a streaming hint lets
// the line go between them (measured: the 160-point x pass with 64-byte
// segments ran 25% slower with the hint).
template <int W, typename V>
__device__ __forceinline__ V ld_seg(const V* p) {
  if constexpr (W >= 128) return ld_stream(p);
  else return *p;
}
template <int W, typename V>
__device__ __forceinline__ void st_seg(V* p, const V& v) {
  if constexpr (W >= 128) st_stream(p, v);
  else *p = v;
}

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

constexpr int pow2_part(int n) {
  int r = 1;
  while (n > 0 && n % 2 == 0) {
    n /= 2;
    r *= 2;
  }
  return r;
}
constexpr int odd_part(int n) { return n / pow2_part(n); }

// v * exp(DIR * 2 pi i M / L) for a period L dividing 64 or 960.
template <int M, int L, int DIR, typename V>
__device__ __forceinline__ V twl(V v) {
  if constexpr (64 % L == 0) {
    return twc<(M % L) * (64 / L), DIR>(v);
  } else {
    static_assert(960 % L == 0, "twiddle period must divide 960");
    constexpr int m = (M % L) * (960 / L);
    if constexpr (m == 0) {
      return v;
    } else if constexpr (4 * m == 960) {
      return DIR < 0 ? mul_neg_i(v) : mul_i(v);
    } else if constexpr (2 * m == 960) {
      return V{-v.x, -v.y};
    } else if constexpr (4 * m == 3 * 960) {
      return DIR < 0 ? mul_i(v) : mul_neg_i(v);
    } else {
      using T = decltype(v.x);
      const T c = static_cast<T>(kCos960[m]);
      const T s = static_cast<T>(DIR * kSin960[m]);
      return V{v.x * c - v.y * s, v.x * s + v.y * c};
    }
  }
}

// In-place DFT of odd prime length F (3 or 5) by pairing x_n with x_{F-n}:
// with b_n = x_n + x_{F-n} and d_n = x_n - x_{F-n},
//   X_k = x_0 + sum_n cos(2 pi n k / F) b_n + i DIR sum_n sin(2 pi n k / F) d_n,
// and X_{F-k} is the same with the sine sum negated.
template <int F, int DIR, typename V>
__device__ __forceinline__ void dft_odd(V* a) {
  using T = decltype(a[0].x);
  constexpr int H = (F - 1) / 2;
  V b[H + 1], d[H + 1];
  V x0 = a[0];
  static_for<1, H + 1>([&](auto n_) {
    constexpr int n = decltype(n_)::value;
    b[n] = cadd(a[n], a[F - n]);
    d[n] = csub(a[n], a[F - n]);
    x0 = cadd(x0, b[n]);
  });
  static_for<1, H + 1>([&](auto k_) {
    constexpr int k = decltype(k_)::value;
    V A = a[0], B = V{0, 0};
    static_for<1, H + 1>([&](auto n_) {
      constexpr int n = decltype(n_)::value;
      constexpr int m = ((n * k) % F) * (960 / F);
      const T c = static_cast<T>(kCos960[m]);
      const T s = static_cast<T>(kSin960[m]);
      A = V{A.x + c * b[n].x, A.y + c * b[n].y};
      B = V{B.x + s * d[n].x, B.y + s * d[n].y};
    });
    const V iB = DIR < 0 ? mul_neg_i(B) : mul_i(B);
    a[k] = cadd(A, iB);
    a[F - k] = csub(A, iB);
  });
  a[0] = x0;
}

// In-place R-point DFT of a register array.  R a power of two <= 64:
// radix-2 decimation in frequency, then a compile-time bit reversal.
// R = F Q with F in {3, 5} and Q a power of two: with n = n1 + Q n2 and
// k = k2 + F k1, F-point DFTs over n2, twiddles W_R^{n1 k2}, then Q-point
// DFTs over n1.
template <int R, int DIR, typename V>
__device__ __forceinline__ void dft(V* a) {
  if constexpr (odd_part(R) != 1) {
    constexpr int F = odd_part(R), Q = R / F;
    static_assert(F == 3 || F == 5, "odd radix must be 3 or 5");
    if constexpr (Q == 1) {
      dft_odd<F, DIR>(a);
    } else {
      V y[Q][F];
      static_for<0, Q>([&](auto n1_) {
        constexpr int n1 = decltype(n1_)::value;
        V u[F];
        static_for<0, F>([&](auto n2_) { u[decltype(n2_)::value] = a[n1 + Q * decltype(n2_)::value]; });
        dft_odd<F, DIR>(u);
        static_for<0, F>([&](auto k2_) {
          constexpr int k2 = decltype(k2_)::value;
          y[n1][k2] = twl<n1 * k2, R, DIR>(u[k2]);
        });
      });
      static_for<0, F>([&](auto k2_) {
        constexpr int k2 = decltype(k2_)::value;
        V w[Q];
        static_for<0, Q>([&](auto n1_) { w[decltype(n1_)::value] = y[decltype(n1_)::value][k2]; });
        dft<Q, DIR>(w);
        static_for<0, Q>([&](auto k1_) { a[k2 + F * decltype(k1_)::value] = w[decltype(k1_)::value]; });
      });
    }
  } else if constexpr (R == 2) {
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
// N = F 2^m with F in {1, 3, 5}; P = F 2^a must divide N.  The first stage
// has radix P (the odd factor included), every later stage the power-of-two
// part of P (the last one possibly smaller).
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
    constexpr int P2 = pow2_part(P);
    constexpr int R = (NS == 1) ? P : ((N / NS < P2) ? N / NS : P2);
    static_assert(N % (NS * R) == 0, "pencil length must be a multiple of the stage spans");
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
      const int k = b % NS;
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

// The same transform on C pencils held by the same threads (v[j] = pencil j):
// each stage reads its twiddles once for all pencils; the exchanges run pencil
// by pencil through the one exchange buffer.
template <int N, int P, int NS, int DIR, typename T, int C, int CG = 1>
__device__ __forceinline__ void fft_stages_multi(cpx<T> (&v)[C][P], int t, cpx<T>* lds, int es,
                                                 const cpx<T>* __restrict__ tw, int tstride, int cs = 0) {
  static_assert(C % CG == 0, "components per exchange must divide the component count");
  if constexpr (NS < N) {
    constexpr int P2 = pow2_part(P);
    constexpr int R = (NS == 1) ? P : ((N / NS < P2) ? N / NS : P2);
    static_assert(N % (NS * R) == 0, "pencil length must be a multiple of the stage spans");
    constexpr int TT = N / P;
    constexpr int G = P / R;  // butterflies per thread
    constexpr bool last = (NS * R == N);
    cpx<T> w[G][R];
    if constexpr (NS > 1) {
      static_for<0, G>([&](auto i_) {
        constexpr int i = decltype(i_)::value;
        const int k = (t + TT * i) % NS;
        static_for<1, R>([&](auto r_) {
          constexpr int r = decltype(r_)::value;
          cpx<T> x = tw[(r * k * (N / (NS * R))) * tstride];
          if constexpr (DIR > 0) x.y = -x.y;
          w[i][r] = x;
        });
      });
    }
    // CG components per exchange: component jj of a group uses lds + jj cs
    static_for<0, C / CG>([&](auto g_) {
      constexpr int g0 = decltype(g_)::value * CG;
      static_for<0, CG>([&](auto jj_) {
        constexpr int jj = decltype(jj_)::value;
        constexpr int j = g0 + jj;
        static_for<0, G>([&](auto i_) {
          constexpr int i = decltype(i_)::value;
          cpx<T> u[R];
          static_for<0, R>([&](auto r_) {
            constexpr int r = decltype(r_)::value;
            u[r] = v[j][i + r * G];
          });
          if constexpr (NS > 1) {
            static_for<1, R>([&](auto r_) {
              constexpr int r = decltype(r_)::value;
              u[r] = cmul(u[r], w[i][r]);
            });
          }
          dft<R, DIR>(u);
          if constexpr (last) {
            static_for<0, R>([&](auto r_) {
              constexpr int r = decltype(r_)::value;
              v[j][i + r * G] = u[r];
            });
          } else {
            const int b = t + TT * i;
            const int base = (b / NS) * NS * R + b % NS;
            static_for<0, R>([&](auto r_) {
              constexpr int r = decltype(r_)::value;
              lds[jj * cs + (base + r * NS) * es] = u[r];
            });
          }
        });
      });
      if constexpr (!last) {
        __syncthreads();
        static_for<0, CG>([&](auto jj_) {
          constexpr int jj = decltype(jj_)::value;
          static_for<0, P>([&](auto q_) {
            constexpr int q = decltype(q_)::value;
            v[g0 + jj][q] = lds[jj * cs + (t + TT * q) * es];
          });
        });
        __syncthreads();
      }
    });
    if constexpr (!last) fft_stages_multi<N, P, NS * R, DIR, T, C, CG>(v, t, lds, es, tw, tstride, cs);
  }
}

// CG > 1: CG components share each exchange (one barrier pair per group),
// component jj of a group in lds + jj cs.
template <int N, int P, int DIR, typename T, int C, int CG = 1>
__device__ __forceinline__ void fft_pencil_multi(cpx<T> (&v)[C][P], int t, cpx<T>* lds, int es,
                                                 const cpx<T>* __restrict__ tw, int tstride, int cs = 0) {
  static_assert(N == 1 || (P <= N && N % P == 0 && odd_part(N) == odd_part(P)),
                "points per thread must divide the pencil length and carry its odd factor");
  fft_stages_multi<N, P, 1, DIR, T, C, CG>(v, t, lds, es, tw, tstride, cs);
}

template <int N, int P, int DIR, typename T>
__device__ __forceinline__ void fft_pencil(cpx<T> (&v)[P], int t, cpx<T>* lds, int es, const cpx<T>* __restrict__ tw,
                                           int tstride) {
  static_assert(N == 1 || (P <= N && N % P == 0 && odd_part(N) == odd_part(P)),
                "points per thread must divide the pencil length and carry its odd factor");
  fft_stages<N, P, 1, DIR, T>(v, t, lds, es, tw, tstride);
}

}  // namespace lsh
