// Kernel templates of the Lippmann--Schwinger operator and its solvers.
//
// Data layout (all HBM-resident, one load after another):
//   real field      T     [load][c][nz][ny][nx]              (x fastest)
//   main spectrum   cpx<T>[load][c][nz][ny][mx], mx = nx/2    kx = 0..mx-1
//   Nyquist plane   cpx<T>[load][c][nz][ny]                   kx = nx/2
// The main spectrum of one load occupies exactly the bytes of its real field,
// so the last pass writes its real output over the spectrum it has read.
//
// One application of eq. (13) is five passes:
//   xfwd  real rows -> half spectrum (R2C through an nx/2-point complex FFT),
//         optionally fused with the CG updates x += alpha p (of the previous
//         step) and p = r + beta p;
//   y     strided y-pencils (and contiguous rows of the Nyquist plane);
//   zg    strided z-pencils: forward z FFT, Gamma_hat on the c components of
//         every wave-vector, inverse z FFT (the Nyquist plane too);
//   y     inverse;
//   xinv  C2R, 1/N^d, and the local term (A - A0)^{-1} tau with the solver's
//         epilogue (CG q and p.q, basic-scheme update, FP64 residual, ...).
#pragma once

#include "green_dev.hpp"

namespace lsh {

// Per-load solver state, updated on the device between passes.
struct LoadState {
  double rr;     // r.r of the current residual
  double pq;     // p.Lp
  double alpha;  // CG step (of the newest step whose x update is pending)
  double beta;   // CG direction update
  double bb;     // ||b||^2
  double res2;   // last residual norm^2 (basic scheme, refinement)
  double tol2;   // tol^2 ||b||^2
  double alpha2; // fused CG: step of the older of two pending steps
  int active;    // 1 while the load iterates
  int iters;     // operator applications spent
  int status;    // lsh_status of the load
  int first;     // next CG direction is p = r
  int pending;   // CG steps whose x += alpha p is still to be applied (fused step: 0, 1 or 2)
  int pbuf;      // fused step: direction buffer (0/1) holding the newest pending direction
};

// Residual history: per load a ring of kHistCap entries, each the squared
// relative residual ||r||^2 / ||b||^2 of the iterated state after one
// iteration and its level (0: FP64 solve or the FP64 refinement residual of a
// mixed solve, 1: the FP32 inner CG of a mixed solve, relative to its own
// right-hand side, the FP64 residual it started from), and per load the
// number of entries written since the solve began.  One writer per load at a
// time (thread 0 of the load's scalar workgroup).
constexpr int kHistCap = 4096;
struct HistRef {
  double* ring;                 // [load][kHistCap][2], null: no history
  unsigned long long* count;    // [load]
  int level;
};
__device__ __forceinline__ void hist_push(const HistRef& h, const int load, const double rel2) {
  if (h.ring == nullptr) return;
  const unsigned long long i = h.count[load];
  h.count[load] = i + 1;
  double* e = h.ring + ((long long)load * kHistCap + (long long)(i % kHistCap)) * 2;
  e[0] = rel2;
  e[1] = (double)h.level;
}

// The FP64 refinement x pass of a mixed solve (XF_IRX, x += d) also applies
// the x updates that the FP32 inner CG left pending (one or two steps, from
// the direction buffers its load states name: pa, or pa and pb for the fused
// step's alternating buffers), so that no separate flush pass reads and
// writes d; with xzero it writes x = d (the first refinement of a solve that
// starts at zero, which then needs no zeroing pass).
struct IrxFold {
  const float* pa;
  const float* pb;
  const LoadState* sti;   // inner states (null: nothing pending)
  int xzero;
};

struct Geo {
  int nx, ny, nz, mx, c, pad;
  long long nvox;  // nx*ny*nz
};

// 16-byte vector of the field type
template <typename T> struct Vec16;
template <> struct Vec16<float> { using type = float4; static constexpr int n = 4; };
template <> struct Vec16<double> { using type = double2; static constexpr int n = 2; };

__host__ __device__ inline long long field_elems(const Geo& g) { return (long long)g.c * g.nvox; }
__host__ __device__ inline long long main_cpx(const Geo& g) { return (long long)g.c * g.nz * g.ny * g.mx; }
__host__ __device__ inline long long nyq_cpx(const Geo& g) { return (long long)g.c * g.nz * g.ny; }

enum : int { XF_PLAIN = 0, XF_CG = 1, XF_IRX = 2 };
enum : int { XI_APPLY = 0, XI_CG = 1, XI_BASIC = 2, XI_IRRES = 3, XI_RESNORM = 4, XI_STRAIN = 5, XI_EM = 6,
              XI_CGR = 7 };
enum : int { Z_GAMMA = 0, Z_FWD = 1 };
enum : int { SC_INIT = 0, SC_ALPHA = 1, SC_BETA = 2, SC_BASIC = 3, SC_OUTER = 4, SC_SUM = 5, SC_INITG = 6 };

constexpr int kMaxPhases = 32;
constexpr int kStatusOk = 0, kStatusBreakdown = -5, kStatusNumeric = -6;

// ----------------------------------------------------------------------------
// workgroup reduction of one double (wave64 shuffles, then LDS), fixed order
// ----------------------------------------------------------------------------
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  constexpr int NW = (NT + 63) / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < NW; ++i) s += red[i];
  }
  return s;
}

// ----------------------------------------------------------------------------
// XCD-aware tile order for strided passes.  Workgroups are dealt round-robin
// to the 8 XCDs, each with its own L2, so consecutive ids land on different
// XCDs.  Where a tile of TX pencils spans less than a 128-byte line, S = 128 /
// (TX * element) adjacent x tiles share every line; within each run of 8 S
// ids, ids r, r + 8, ..., r + 8 (S - 1) (one XCD, dispatched one after
// another) take x tiles r S, ..., r S + S - 1.  Ids past the last whole run
// keep their order.
// ----------------------------------------------------------------------------
template <int S>
__device__ __forceinline__ int xcd_tile(const int b, const int n) {
  if constexpr (S <= 1) {
    return b;
  } else {
    constexpr int RUN = 8 * S;
    const int b0 = b - b % RUN;
    if (b0 + RUN > n) return b;
    const int r = b % RUN;
    return b0 + (r % 8) * S + r / 8;
  }
}

template <typename T, int TX>
constexpr int line_share() {
  return (TX * 2 * (int)sizeof(T) < 128) ? 128 / (TX * 2 * (int)sizeof(T)) : 1;
}

// Requested waves per SIMD of the fused x pass: the FP32 six-component
// 128-point instance (the mixed elastic 256^3 path) fits 5 waves in 93 VGPRs
// without spilling, against 4 at the allocator's own 100 (2.64 -> 2.58 ms);
// 1 leaves every other instance unconstrained.  (The matching C2R instance
// spills at 4 waves and measured slower, so it keeps its allocation.)
template <typename T, int MX, int P, int C>
constexpr int xfwdc_waves() {
  return (sizeof(T) == 4 && C == 6 && MX == 128 && P == 4) ? 5 : 1;
}

// ----------------------------------------------------------------------------
// x forward: R2C along rows
// ----------------------------------------------------------------------------
template <typename T, int MX, int P>
__global__ __launch_bounds__(256) void k_xfwd(const Geo g, const int mode, const T* __restrict__ src,
                                              T* __restrict__ pdir, T* __restrict__ xacc,
                                              const float* __restrict__ dsrc, cpx<T>* __restrict__ smain,
                                              cpx<T>* __restrict__ snyq, const cpx<T>* __restrict__ twx,
                                              const LoadState* __restrict__ st, const IrxFold fold) {
  constexpr int TR = MX / P;
  constexpr int RPW = 256 / TR;
  constexpr int SEG = TR * (int)sizeof(cpx<T>);   // contiguous bytes per access instruction
  __shared__ cpx<T> lds[RPW * MX];
  __shared__ cpx<T> twl[2 * MX];
  const int l = blockIdx.y;
  const int tid = threadIdx.x;
  const int slot = tid / TR, t = tid % TR;
  const long long rows = (long long)g.c * g.nz * g.ny;
  const long long row = (long long)blockIdx.x * RPW + slot;
  const bool valid = row < rows;
  const long long roff = (long long)l * field_elems(g) + row * (2 * MX);
  if (st != nullptr && !st[l].active) {
    // a load that is not refined still gets its zero start written (x was not zeroed)
    if (mode == XF_IRX && fold.xzero && valid) {
      cpx<T>* x2 = reinterpret_cast<cpx<T>*>(pdir + roff);
#pragma unroll
      for (int i = 0; i < P; ++i) x2[t + TR * i] = cpx<T>{0, 0};
    }
    return;
  }
  for (int i = tid; i < 2 * MX; i += 256) twl[i] = twx[i];   // twiddles of the row length, staged in LDS

  cpx<T> v[P];
  if (mode == XF_CG) {
    // x += alpha p (the previous step, when pending), then p = r + beta p
    const cpx<T>* r2 = reinterpret_cast<const cpx<T>*>(src + roff);
    cpx<T>* p2 = reinterpret_cast<cpx<T>*>(pdir + roff);
    cpx<T>* x2 = reinterpret_cast<cpx<T>*>(xacc + roff);
    const bool first = st[l].first != 0;
    const bool pend = st[l].pending != 0;
    const T beta = static_cast<T>(st[l].beta);
    const T alpha = static_cast<T>(st[l].alpha);
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int n = t + TR * i;
      cpx<T> pv{0, 0};
      if (valid) {
        const cpx<T> rv = ld_seg<SEG>(r2 + n);
        if (first) {
          pv = rv;
        } else {
          const cpx<T> po = ld_seg<SEG>(p2 + n);
          if (pend) {
            const cpx<T> xo = ld_seg<SEG>(x2 + n);
            st_seg<SEG>(x2 + n, cpx<T>{xo.x + alpha * po.x, xo.y + alpha * po.y});
          }
          pv = cpx<T>{rv.x + beta * po.x, rv.y + beta * po.y};
        }
        st_seg<SEG>(p2 + n, pv);
      }
      v[i] = pv;
    }
  } else if (mode == XF_IRX) {
    cpx<T>* x2 = reinterpret_cast<cpx<T>*>(pdir + roff);
    const float2* d2 = reinterpret_cast<const float2*>(dsrc + roff);
    // pending inner steps of this load: d + alpha p_newest (+ alpha2 p_older), in FP32
    const int np = fold.sti != nullptr ? fold.sti[l].pending : 0;
    const float al = np > 0 ? static_cast<float>(fold.sti[l].alpha) : 0.0f;
    const float al2 = np == 2 ? static_cast<float>(fold.sti[l].alpha2) : 0.0f;
    const bool nb1 = np > 0 && fold.pb != nullptr && fold.sti[l].pbuf != 0;
    const float2* pn2 = np > 0 ? reinterpret_cast<const float2*>((nb1 ? fold.pb : fold.pa) + roff) : nullptr;
    const float2* po2 = np == 2 ? reinterpret_cast<const float2*>((nb1 ? fold.pa : fold.pb) + roff) : nullptr;
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int n = t + TR * i;
      cpx<T> xv{0, 0};
      if (valid) {
        const cpx<T> xo = fold.xzero ? cpx<T>{0, 0} : x2[n];
        float2 dv = d2[n];
        if (np > 0) {
          const float2 q = pn2[n];
          dv = float2{dv.x + al * q.x, dv.y + al * q.y};
          if (np == 2) {
            const float2 q2 = po2[n];
            dv = float2{dv.x + al2 * q2.x, dv.y + al2 * q2.y};
          }
        }
        xv = cpx<T>{xo.x + static_cast<T>(dv.x), xo.y + static_cast<T>(dv.y)};
        x2[n] = xv;
      }
      v[i] = xv;
    }
  } else {
    const cpx<T>* s2 = reinterpret_cast<const cpx<T>*>(src + roff);
#pragma unroll
    for (int i = 0; i < P; ++i) v[i] = valid ? ld_seg<SEG>(s2 + t + TR * i) : cpx<T>{0, 0};
  }

  cpx<T>* lrow = lds + slot * MX;
  __syncthreads();
  fft_pencil<MX, P, -1, T>(v, t, lrow, 1, twl, 2);

  // unpack the half-length transform: X[k] = E[k] + W_nx^k O[k]
#pragma unroll
  for (int i = 0; i < P; ++i) lrow[t + TR * i] = v[i];
  __syncthreads();
  const long long so = (long long)l * main_cpx(g) + row * MX;
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const int k = t + TR * i;
    const cpx<T> z = v[i];
    if (k == 0) {
      if (valid) {
        st_seg<SEG>(smain + so, cpx<T>{z.x + z.y, T(0)});
        snyq[(long long)l * nyq_cpx(g) + row] = cpx<T>{z.x - z.y, T(0)};
      }
    } else {
      const cpx<T> zm = lrow[MX - k];
      const cpx<T> a = cpx<T>{z.x + zm.x, z.y - zm.y};   // Z + conj(Zm)
      const cpx<T> b = cpx<T>{z.x - zm.x, z.y + zm.y};   // Z - conj(Zm)
      const cpx<T> wo = cmul(twl[k], mul_neg_i(b));
      if (valid) st_seg<SEG>(smain + so + k, cpx<T>{T(0.5) * (a.x + wo.x), T(0.5) * (a.y + wo.y)});
    }
  }
}

// Row j of a per-phase c x c matrix applied to v.  Table row layout:
// [(A-A0)^{-1} (c*c) | (A-A0) (c*c) | in-I0 flag | a_inv b_inv a_dir b_dir]
// where, when every phase is "isotropic", each matrix is a Id + b m m^T with
// m the indicator of the three normal Mandel components (b = 0 for scalar
// problems), and the short form is used.
template <typename T, int C>
__device__ __forceinline__ T phase_row(const T* tb, int which, bool iso, int j, const T (&v)[C]) {
  if (iso) {
    const T a = tb[2 * C * C + 1 + 2 * which], b = tb[2 * C * C + 2 + 2 * which];
    T r = a * v[j];
    if (C == 6 && j < 3) r += b * (v[0] + v[1] + v[2]);
    return r;
  }
  const T* M = tb + which * C * C + j * C;
  T r = 0;
#pragma unroll
  for (int m = 0; m < C; ++m) r += M[m] * v[m];
  return r;
}

// Local operator of one voxel: a row of the phase table, or (per-voxel mode)
// the short form a_inv Id + b_inv m m^T of (A_beta - A0)^{-1} with its
// inverse a_dir = 1/a_inv, b_dir = -b_inv / (a_inv (a_inv + 3 b_inv)).
// a_inv = 0 marks a voxel outside I0.
template <typename T>
struct Loc {
  const T* tb;
  T in, ai, bi;
};

// which = 0: (A - A0)^{-1}; 1: the table's second matrix, i.e. (A - A0) for
// the basic scheme or (A - A0)(A + A0)^{-1} for Eyre--Milton; per-voxel mode
// forms the first (which 1) or the second (which 2, from 2 A0 = (ea, eb)) in place.
// (A - A0)(A + A0)^{-1} = (Id + 2 A0 (A - A0)^{-1})^{-1}, with
// 2 A0 (a_inv Id + b_inv m m^T) = 4 mu0 a_inv Id + (4 mu0 b_inv + 2 lambda0 (a_inv + 3 b_inv)) m m^T.
template <typename T>
__device__ __forceinline__ void iso_inverse(T& a, T& b, bool six) {
  const bool z = a == T(0);
  const T ad = z ? T(0) : T(1) / a;
  b = (six && !z) ? -b / (a * (a + T(3) * b)) : T(0);
  a = ad;
}

// v . (A - A0)^{-1} v at one voxel (the local quadratic form)
template <typename T, int C>
__device__ __forceinline__ T loc_quad(const Loc<T>& L, bool vm, bool iso, const T (&v)[C]) {
  if (vm || iso) {
    const T a = vm ? L.ai : L.tb[2 * C * C + 1];
    const T b = vm ? L.bi : L.tb[2 * C * C + 2];
    T s = 0;
#pragma unroll
    for (int j = 0; j < C; ++j) s += v[j] * v[j];
    T q = a * s;
    if (C == 6) {
      const T tr = v[0] + v[1] + v[2];
      q += b * tr * tr;
    }
    return q;
  }
  T q = 0;
#pragma unroll
  for (int j = 0; j < C; ++j) {
    T r = 0;
#pragma unroll
    for (int k = 0; k < C; ++k) r += L.tb[j * C + k] * v[k];
    q += v[j] * r;
  }
  return q;
}

template <typename T, int C>
__device__ __forceinline__ T loc_row(const Loc<T>& L, bool vm, int which, bool iso, int j, const T (&v)[C],
                                     T ea = T(0), T eb = T(0)) {
  if (!vm) return phase_row<T, C>(L.tb, which, iso, j, v);
  T a = L.ai, b = L.bi;
  if (which == 1) {
    iso_inverse(a, b, C == 6);
  } else if (which == 2) {
    if (C == 6) {
      T al = T(1) + ea * a;
      T be = ea * b + eb * (a + T(3) * b);
      iso_inverse(al, be, true);
      a = al;
      b = be;
    } else {
      a = T(1) / (T(1) + ea * a);
      b = T(0);
    }
  }
  T r = a * v[j];
  if (C == 6 && j < 3) r += b * (v[0] + v[1] + v[2]);
  return r;
}

// ----------------------------------------------------------------------------
// x forward for conjugate gradients with all c components of a voxel row in one
// thread group: p_k = r + beta p_{k-1}, the R2C transforms of every component,
// and the local quadratic form p . (A - A0)^{-1} p (one FP64 partial per
// workgroup).  With the spectral form of the z pass this gives p . Lp before
// the inverse passes run.  The directions alternate between two buffers (pin
// holds p_{k-1}, pout p_{k-2} on entry and p_k on exit), and the solution
// updates of the steps are applied in pairs: when two are pending, x += alpha2
// p_{k-2} + alpha p_{k-1} before p_{k-2} is overwritten; with one pending (its
// direction in pin, which survives this pass) x is not touched.  On average
// x is read and written every second iteration.
// ----------------------------------------------------------------------------
template <typename T>
struct XfwdcArgs {
  Geo g;
  const T* r;
  const T* pin;   // p_{k-1}
  T* pout;        // p_k (holds p_{k-2} on entry)
  T* x;
  cpx<T>* smain;
  cpx<T>* snyq;
  const cpx<T>* twx;
  const LoadState* st;
  int nphase, iso;
  const T* ptab;
  const uint8_t* phase;
  const T* vcoef;
  double* partials;
  int pstride;
  int paired;     // write the main spectrum in the component-paired layout (FP32, even c)
};

template <typename T, int MX, int P, int C>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(xfwdc_waves<T, MX, P, C>()))) void k_xfwdc(const XfwdcArgs<T> a) {
  constexpr int TR = MX / P;
  constexpr int RPW = 256 / TR;
  constexpr int SEG = TR * (int)sizeof(cpx<T>);   // contiguous bytes per access instruction
  constexpr int TABW = 2 * C * C + 5;   // phase table row, see phase_row
  // FP32 six components: two components share each FFT exchange (the LDS of
  // five workgroups per CU still fits)
  constexpr int CG = (sizeof(T) == 4 && C == 6) ? 2 : 1;
  __shared__ cpx<T> lds[CG * RPW * MX];
  __shared__ cpx<T> twl[2 * MX];
  __shared__ T tab[kMaxPhases * TABW];
  __shared__ double red[4];
  const Geo& g = a.g;
  const int l = blockIdx.y;
  if (!a.st[l].active) return;
  const int tid = threadIdx.x;
  const int slot = tid / TR, t = tid % TR;
  const long long vrows = (long long)g.nz * g.ny;
  const long long vr = (long long)blockIdx.x * RPW + slot;
  const bool valid = vr < vrows;
  const long long vrc = valid ? vr : 0;
  const long long fo = (long long)l * field_elems(g);
  const bool first = a.st[l].first != 0;
  const bool pair = a.st[l].pending == 2;
  const T beta = static_cast<T>(a.st[l].beta);
  const T alpha = static_cast<T>(a.st[l].alpha);
  const T alpha2 = static_cast<T>(a.st[l].alpha2);
  cpx<T> v[C][P];
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const long long roff = fo + (long long)j * g.nvox + vrc * (2 * MX);
    const cpx<T>* r2 = reinterpret_cast<const cpx<T>*>(a.r + roff);
    const cpx<T>* pi2 = reinterpret_cast<const cpx<T>*>(a.pin + roff);
    cpx<T>* po2 = reinterpret_cast<cpx<T>*>(a.pout + roff);
    cpx<T>* x2 = reinterpret_cast<cpx<T>*>(a.x + roff);
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int n = t + TR * i;
      cpx<T> pv{0, 0};
      if (valid) {
        const cpx<T> rv = ld_seg<SEG>(r2 + n);
        if (first) {
          pv = rv;
        } else {
          const cpx<T> po = ld_seg<SEG>(pi2 + n);
          if (pair) {
            const cpx<T> pp = ld_seg<SEG>(po2 + n);
            const cpx<T> xo = ld_seg<SEG>(x2 + n);
            st_seg<SEG>(x2 + n, cpx<T>{xo.x + alpha2 * pp.x + alpha * po.x, xo.y + alpha2 * pp.y + alpha * po.y});
          }
          pv = cpx<T>{rv.x + beta * po.x, rv.y + beta * po.y};
        }
        st_seg<SEG>(po2 + n, pv);
      }
      v[j][i] = pv;
    }
    // one component's rows at a time: bounds the registers the loads occupy
    __builtin_amdgcn_sched_barrier(0);
  }
  // material table and twiddles, staged after the row reads (a wait on them
  // first would hold the reads back)
  for (int i = tid; i < a.nphase * TABW; i += 256) tab[i] = a.ptab[i];
  for (int i = tid; i < 2 * MX; i += 256) twl[i] = a.twx[i];
  __syncthreads();
  // local quadratic form on the voxel pairs this thread holds
  double part = 0.0;
  const bool iso = a.iso != 0;
  const bool vm = a.vcoef != nullptr;
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const int n = t + TR * i;
    const long long vox = vrc * (2 * MX) + 2 * n;
    Loc<T> L0, L1;
    if (vm) {
      const cpx<T> ai = *reinterpret_cast<const cpx<T>*>(a.vcoef + vox);
      const cpx<T> bi = *reinterpret_cast<const cpx<T>*>(a.vcoef + g.nvox + vox);
      L0 = Loc<T>{nullptr, ai.x != T(0) ? T(1) : T(0), ai.x, bi.x};
      L1 = Loc<T>{nullptr, ai.y != T(0) ? T(1) : T(0), ai.y, bi.y};
    } else {
      const uint16_t ph2 = *reinterpret_cast<const uint16_t*>(a.phase + vox);
      const T* tb0 = tab + (ph2 & 0xff) * TABW;
      const T* tb1 = tab + (ph2 >> 8) * TABW;
      L0 = Loc<T>{tb0, tb0[2 * C * C], T(0), T(0)};
      L1 = Loc<T>{tb1, tb1[2 * C * C], T(0), T(0)};
    }
    T p0[C], p1[C];
#pragma unroll
    for (int j = 0; j < C; ++j) {
      p0[j] = v[j][i].x;
      p1[j] = v[j][i].y;
    }
    part += (double)(L0.in * loc_quad<T, C>(L0, vm, iso, p0)) + (double)(L1.in * loc_quad<T, C>(L1, vm, iso, p1));
    __builtin_amdgcn_sched_barrier(0);
  }
  if (!valid) part = 0.0;
  // R2C of every component: half-length transforms, then the unpacking (CG
  // components per exchange, in the exchange buffers of the transforms)
  cpx<T>* lrow = lds + slot * MX;
  fft_pencil_multi<MX, P, -1, T, C, CG>(v, t, lrow, 1, twl, 2, RPW * MX);
#pragma unroll
  for (int j0 = 0; j0 < C; j0 += CG) {
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < CG; ++jj)
#pragma unroll
      for (int i = 0; i < P; ++i) lrow[jj * RPW * MX + t + TR * i] = v[j0 + jj][i];
    __syncthreads();
    // X[k] = (Z[k] + conj Z[M-k]) / 2 - i W^k (Z[k] - conj Z[M-k]) / 2 for k > 0;
    // X[0] = Re Z[0] + Im Z[0] and the Nyquist value Re Z[0] - Im Z[0]
    auto unpack = [&](const int jj, const int i) -> cpx<T> {
      const int k = t + TR * i;
      const cpx<T> z = v[j0 + jj][i];
      if (k == 0) return cpx<T>{z.x + z.y, T(0)};
      const cpx<T> zm = lrow[jj * RPW * MX + MX - k];
      const cpx<T> s1 = cpx<T>{z.x + zm.x, z.y - zm.y};   // Z + conj(Zm)
      const cpx<T> d1 = cpx<T>{z.x - zm.x, z.y + zm.y};   // Z - conj(Zm)
      const cpx<T> wo = cmul(twl[k], mul_neg_i(d1));
      return cpx<T>{T(0.5) * (s1.x + wo.x), T(0.5) * (s1.y + wo.y)};
    };
#pragma unroll
    for (int jj = 0; jj < CG; ++jj) {
      const long long row = (long long)(j0 + jj) * vrows + vrc;
      if (t == 0 && valid) {
        const cpx<T> z = v[j0 + jj][0];
        a.snyq[(long long)l * nyq_cpx(g) + row] = cpx<T>{z.x - z.y, T(0)};
      }
    }
    bool done = false;
    if constexpr (CG == 2 && sizeof(T) == 4) {
      if (a.paired) {
        // components j0 and j0 + 1 of each wave-vector side by side (16 bytes)
        float4* pr = reinterpret_cast<float4*>(a.smain + (long long)l * main_cpx(g) +
                                               ((long long)(j0 / 2) * vrows + vrc) * 2 * MX);
#pragma unroll
        for (int i = 0; i < P; ++i) {
          const cpx<T> e0 = unpack(0, i), e1 = unpack(1, i);
          if (valid) st_stream4(pr + t + TR * i, float4{e0.x, e0.y, e1.x, e1.y});
        }
        done = true;
      }
    }
    if (!done) {
#pragma unroll
      for (int jj = 0; jj < CG; ++jj) {
        const long long so = (long long)l * main_cpx(g) + ((long long)(j0 + jj) * vrows + vrc) * MX;
#pragma unroll
        for (int i = 0; i < P; ++i) {
          const cpx<T> e = unpack(jj, i);
          if (valid) st_seg<SEG>(a.smain + so + t + TR * i, e);
        }
      }
    }
  }
  const double sum = block_sum<256>(part, red);
  if (tid == 0) a.partials[(long long)l * a.pstride + blockIdx.x] = sum;
}

// ----------------------------------------------------------------------------
// y pass: strided pencils of the main spectrum, contiguous rows of the Nyquist plane
// ----------------------------------------------------------------------------
// Spectrum layouts of the y pass (LAY): 0 in place in the plain layout
// (component-major rows of mx wave-vectors); 1 reads the plain layout and
// writes the component-paired one; 2 reads the paired layout and writes the
// plain one.  In the paired layout (six-component FP32 fields, the z pass of
// 8-pencil tiles) components 2m and 2m+1 of a wave-vector are adjacent:
//   ((m nz + kz) ny + ky) 2 mx + 2 kx + (j & 1),   j = 2m or 2m + 1,
// so an 8-pencil z tile reads whole 128-byte lines for every component pair.
// A converting tile holds TX/2 wave-vectors of two components (columns
// xl < TX/2 the even one).  3 runs in place on the paired layout: each
// component pair is a row of 2 mx entries, cut into tiles of TX.  The Nyquist
// rows stay in place in every layout.
enum : int { YL_INPLACE = 0, YL_TO_PAIRED = 1, YL_FROM_PAIRED = 2, YL_PAIRED = 3 };

template <typename T, int NY, int P, int TX, int DIR, int LAY>
__global__ __launch_bounds__(TX*(NY / P)) void k_y(const Geo g, cpx<T>* __restrict__ smain,
                                                  cpx<T>* __restrict__ snyq, const cpx<T>* __restrict__ twy,
                                                  const LoadState* __restrict__ st, const int main_tiles,
                                                  cpx<T>* __restrict__ sout) {
  constexpr int TY = NY / P;
  constexpr bool INPL = LAY == YL_INPLACE || LAY == YL_PAIRED;
  constexpr int H = INPL ? TX : TX / 2;   // row entries (wave-vectors, or pair entries) per component in a main tile
  constexpr int SEG = H * (int)sizeof(cpx<T>);       // contiguous bytes per plain-layout access
  constexpr int SEGP = TX * (int)sizeof(cpx<T>);     // contiguous bytes per paired-layout access
  __shared__ cpx<T> lds[TX * NY];
  __shared__ cpx<T> twl[NY];
  const int l = blockIdx.y;
  if (st != nullptr && !st[l].active) return;
  const int tid = threadIdx.x;
  cpx<T>* base;
  cpx<T>* obase;
  long long es_g, es_o;
  cpx<T>* lp;
  int es_l, t;
  bool valid, main = false;
  if ((int)blockIdx.x < main_tiles) {
    main = true;
    const int mrow = LAY == YL_PAIRED ? 2 * g.mx : g.mx;   // entries per row
    const int xtiles = (mrow + H - 1) / H;
    const int tile = INPL ? xcd_tile<line_share<T, TX>()>(blockIdx.x, main_tiles) : (int)blockIdx.x;
    const int xc = tile % xtiles;
    const long long jz = tile / xtiles;
    const int xl = tid % TX;
    t = tid / TX;
    const int kx = xc * H + xl % H;
    valid = kx < mrow;
    const int kxc = valid ? kx : 0;
    const long long lo = (long long)l * main_cpx(g);
    if constexpr (INPL) {
      base = smain + lo + jz * g.ny * mrow + kxc;
      obase = base;
      es_g = es_o = mrow;
    } else {
      // jz = m nz + kz over component pairs; this column's component j = 2m + xl / H
      const long long m = jz / g.nz, kz = jz % g.nz;
      const int s = xl / H;
      cpx<T>* plain = (LAY == YL_TO_PAIRED ? smain : sout) + lo + ((2 * m + s) * g.nz + kz) * g.ny * g.mx + kxc;
      cpx<T>* paired = (LAY == YL_TO_PAIRED ? sout : smain) + lo + (m * g.nz + kz) * g.ny * 2 * g.mx + 2 * kxc + s;
      base = LAY == YL_TO_PAIRED ? plain : paired;
      obase = LAY == YL_TO_PAIRED ? paired : plain;
      es_g = LAY == YL_TO_PAIRED ? g.mx : 2 * g.mx;
      es_o = LAY == YL_TO_PAIRED ? 2 * g.mx : g.mx;
    }
    lp = lds + xl;
    es_l = TX;
  } else {
    const int slot = tid / TY;
    t = tid % TY;
    const long long row = (long long)(blockIdx.x - main_tiles) * TX + slot;
    valid = row < (long long)g.c * g.nz;
    base = snyq + (long long)l * nyq_cpx(g) + (valid ? row : 0) * g.ny;
    obase = base;
    es_g = es_o = 1;
    lp = lds + slot * NY;
    es_l = 1;
  }
  cpx<T> v[P];
  if (!main || LAY != YL_FROM_PAIRED) {
#pragma unroll
    for (int i = 0; i < P; ++i) v[i] = valid ? ld_seg<SEG>(base + (long long)(t + TY * i) * es_g) : cpx<T>{0, 0};
  } else {
#pragma unroll
    for (int i = 0; i < P; ++i) v[i] = valid ? ld_seg<SEGP>(base + (long long)(t + TY * i) * es_g) : cpx<T>{0, 0};
  }
  // twiddles staged after the pencil reads are issued (their wait would hold the reads back)
  for (int i = tid; i < NY; i += TX * TY) twl[i] = twy[i];
  __syncthreads();
  fft_pencil<NY, P, DIR, T>(v, t, lp, es_l, twl, 1);
  if (valid) {
    if (!main || LAY != YL_TO_PAIRED) {
#pragma unroll
      for (int i = 0; i < P; ++i) st_seg<SEG>(obase + (long long)(t + TY * i) * es_o, v[i]);
    } else {
#pragma unroll
      for (int i = 0; i < P; ++i) st_seg<SEGP>(obase + (long long)(t + TY * i) * es_o, v[i]);
    }
  }
}

// Global access of the z passes: streaming in FP64 on whole-line segments;
// plain in FP32, where the issue-bound pass measured slower with streaming
// hints (2.00 against 1.85 ms at 256^3 x 6 elastic loads) while the FP64
// pass measured faster.
template <typename T, int W>
__device__ __forceinline__ cpx<T> z_load(const cpx<T>* p) {
  if constexpr (sizeof(T) == 8) return ld_seg<W>(p);
  else return *p;
}
template <typename T, int W>
__device__ __forceinline__ void z_store(cpx<T>* p, const cpx<T>& v) {
  if constexpr (sizeof(T) == 8) st_seg<W>(p, v);
  else *p = v;
}

// ----------------------------------------------------------------------------
// z pass fused with the Green operator: forward z FFT, Gamma_hat, inverse z FFT
// ----------------------------------------------------------------------------
// With qpart, the pass also sums the spectral quadratic form
// (1/V) sum_k w_k Re(conj(tau_hat_k) . Gamma_hat_k tau_hat_k) = tau . Gamma tau
// (Parseval), w_k = 1 on the kx = 0 and kx = nx/2 planes and 2 elsewhere
// (the half spectrum of a real field), one FP64 partial per workgroup at
// qpart[load * pstride + blockIdx.x].
// Workgroup id -> (tile, load) of the z pass with the stored operator: the
// nload workgroups of one tile are dispatched one after another on one XCD
// (ids are dealt round-robin to the 8 XCDs), so the operator entries of the
// tile are read from HBM once and then from that XCD's L2.  Tiles past the
// last whole group of 8 keep a plain order.
__device__ __forceinline__ void xcd_load_tile(const int id, const int ntile, const int nload, int& tile, int& l) {
  const int full = (ntile / 8) * 8 * nload;
  if (id < full) {
    const int x = id % 8, slot = id / 8;
    tile = (slot / nload) * 8 + x;
    l = slot % nload;
  } else {
    const int r = id - full;
    tile = (ntile / 8) * 8 + r / nload;
    l = r % nload;
  }
}

// PR: the main spectrum is in the component-paired layout of the y pass
// (YL_TO_PAIRED), each pair of components read and written as one 16-byte
// access; the Nyquist rows keep the plain layout.  Its 8-pencil workgroups
// (48 KB of LDS) run three per CU: at most 168 VGPRs, without the operator
// prefetch below, whose registers the three workgroups hide better (256^3 x 6
// elastic FP32: 1.23 ms against 1.30 ms at two per CU with the prefetch).
template <typename T, int NZ, int P, int TX, int C, bool GS, bool PR = false>
__global__ __launch_bounds__(TX*(NZ / P)) __attribute__((amdgpu_waves_per_eu(PR ? 3 : 1))) void k_zg(const Geo g, const GreenParams gp, const GreenTabs<T> tb,
                                                   const int zmode, cpx<T>* __restrict__ smain,
                                                   cpx<T>* __restrict__ snyq, const cpx<T>* __restrict__ twz,
                                                   const LoadState* __restrict__ st, const int main_tiles,
                                                   double* __restrict__ qpart, const int pstride, const int nload) {
  constexpr int TZ = NZ / P;
  constexpr int SEG = TX * (int)sizeof(cpx<T>);   // contiguous bytes per access instruction
  constexpr int NT = TX * TZ;
  // six components: three (FP32) or two (FP64) components share each FFT
  // exchange where their buffers fit in 96 KiB of LDS (FP64 at 256^3 x 6,
  // 8 pencils: 3.61 -> 3.50 ms with two, 3.94 with three)
  constexpr int CG = (sizeof(T) == 4 && C == 6 && 3 * TX * NZ * (int)sizeof(cpx<T>) <= 96 * 1024)   ? 3
                     : (sizeof(T) == 8 && C == 6 && 2 * TX * NZ * (int)sizeof(cpx<T>) <= 96 * 1024) ? 2
                                                                                                      : 1;
  __shared__ cpx<T> lds[CG * TX * NZ];
  __shared__ cpx<T> twl[NZ];
  __shared__ double red[(NT + 63) / 64];
  int l, tid_tile;
  if constexpr (GS) {
    xcd_load_tile(blockIdx.x, main_tiles + (g.ny + TX - 1) / TX, nload, tid_tile, l);
  } else {
    l = blockIdx.y;
    tid_tile = blockIdx.x;
  }
  if (st != nullptr && !st[l].active) return;
  const int tid = threadIdx.x;
  const int xl = tid % TX, t = tid / TX;
  cpx<T>* base;
  long long es_g, cstride;
  int kx, ky;
  bool valid;
  if (tid_tile < main_tiles) {
    const int xtiles = (g.mx + TX - 1) / TX;
    const int tile = xcd_tile<line_share<T, TX>()>(tid_tile, main_tiles);
    const int xc = tile % xtiles;
    ky = tile / xtiles;
    kx = xc * TX + xl;
    valid = kx < g.mx;
    base = smain + (long long)l * main_cpx(g) + (long long)ky * g.mx + (valid ? kx : 0);
    es_g = (long long)g.ny * g.mx;
    cstride = (long long)g.nz * g.ny * g.mx;
  } else {
    ky = (tid_tile - main_tiles) * TX + xl;
    kx = g.mx;
    valid = ky < g.ny;
    base = snyq + (long long)l * nyq_cpx(g) + (valid ? ky : 0);
    es_g = g.ny;
    cstride = (long long)g.nz * g.ny;
  }
  cpx<T>* lp = lds + xl;
  // paired layout (main tiles): pair m of wave-vector (kx, ky, kz) at
  // pbase + 2 m cstride + kz pes, 16-byte aligned
  static_assert(!PR || (GS && C % 2 == 0 && sizeof(T) == 4), "paired z pass: stored operator, FP32 component pairs");
  using Q4 = float4;
  const bool pm = PR && tid_tile < main_tiles;
  cpx<T>* pbase = nullptr;
  long long pes = 0;
  if (pm) {
    pbase = smain + (long long)l * main_cpx(g) + (long long)ky * 2 * g.mx + 2 * (valid ? kx : 0);
    pes = (long long)g.ny * 2 * g.mx;
  }

  // all components' loads are issued before the first transform (guarded
  // reads: unguarded ones let the scheduler raise this kernel past 256 VGPRs),
  // and before the twiddles are staged, whose wait would otherwise hold them back
  cpx<T> v[C][P];
  if (pm) {
    if constexpr (PR) {
#pragma unroll
      for (int j = 0; j < C; j += 2)
#pragma unroll
        for (int i = 0; i < P; ++i) {
          const Q4 q = valid ? *reinterpret_cast<const Q4*>(pbase + (long long)j * cstride + (long long)(t + TZ * i) * pes)
                             : Q4{0, 0, 0, 0};
          v[j][i] = cpx<T>{q.x, q.y};
          v[j + 1][i] = cpx<T>{q.z, q.w};
        }
    }
  } else {
#pragma unroll
    for (int j = 0; j < C; ++j)
#pragma unroll
      for (int i = 0; i < P; ++i)
        v[j][i] = valid ? z_load<T, SEG>(base + j * cstride + (long long)(t + TZ * i) * es_g) : cpx<T>{0, 0};
  }
  for (int i = tid; i < NZ; i += TX * TZ) twl[i] = twz[i];
  __syncthreads();
  fft_pencil_multi<NZ, P, -1, T, C, CG>(v, t, lp, TX, twl, 1, TX * NZ);
  if (zmode == Z_GAMMA) {
    double quad = 0.0;
    if (valid) {
      // stored operator: group 0 of (kx, ky, kz = t) and the steps between
      // groups and between the thread's wave-vectors (kz += TZ)
      constexpr int NG = store_groups<C>();
      const Quad<T>* sq = nullptr;
      long long sgs = 0, skz = 0;
      if constexpr (GS) {
        const Quad<T>* s4 = reinterpret_cast<const Quad<T>*>(tb.st);
        const long long nmain = (long long)g.nz * g.ny * g.mx;
        if (kx < g.mx) {
          sq = s4 + (((long long)t * g.ny + ky) * NG) * g.mx + kx;
          sgs = g.mx;
          skz = (long long)TZ * g.ny * NG * g.mx;
        } else {
          sq = s4 + nmain * NG + ((long long)t * NG) * g.ny + ky;
          sgs = g.ny;
          skz = (long long)TZ * NG * g.ny;
        }
      }
      // stored operator: the entries of the next wave-vector are read while
      // the current one is applied (one round trip per wave-vector otherwise;
      // the paired shape leaves that to its third workgroup per CU)
      constexpr int NE = C * (C + 1) / 2;
      constexpr bool PF = GS && !PR;
      T Gn[NE];
      if constexpr (PF) stored_matrix<T, C>(sq, sgs, Gn);
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const int kz = t + TZ * i;
        cpx<T> w[C];
#pragma unroll
        for (int j = 0; j < C; ++j) w[j] = v[j][i];
        if constexpr (PF) {
          T Gm[NE];
#pragma unroll
          for (int e = 0; e < NE; ++e) Gm[e] = Gn[e];
          if (i + 1 < P) stored_matrix<T, C>(sq + (i + 1) * skz, sgs, Gn);
          __builtin_amdgcn_sched_barrier(0);
          sym_apply<T, C>(Gm, w);
        } else if constexpr (GS) {
          T Gm[NE];
          stored_matrix<T, C>(sq + i * skz, sgs, Gm);
          sym_apply<T, C>(Gm, w);
        } else {
          const int k[3] = {kx, ky, kz};
          const long long tidx = (kx < g.mx) ? ((long long)kz * g.ny + ky) * g.mx + kx
                                             : (long long)g.nz * g.ny * g.mx + (long long)kz * g.ny + ky;
          green_apply<T, C>(gp, tb, k, tidx, w);
        }
        if (qpart != nullptr) {
          // one wave-vector's terms in the field type (tau_hat . Gamma_hat tau_hat >= 0:
          // no cancellation), the sum over wave-vectors in FP64
          T d = T(0);
#pragma unroll
          for (int j = 0; j < C; ++j) d += v[j][i].x * w[j].x + v[j][i].y * w[j].y;
          quad += (double)d;
        }
#pragma unroll
        for (int j = 0; j < C; ++j) v[j][i] = w[j];
        // one wave-vector's operator at a time: bounds the registers of the alias sums
        if constexpr (!GS) __builtin_amdgcn_sched_barrier(0);
      }
    }
    if (qpart != nullptr) {
      const double wk = (kx == 0 || kx == g.mx) ? 1.0 : 2.0;
      const double s = block_sum<NT>(quad * wk / (double)g.nvox, red);
      if (tid == 0) qpart[(long long)l * pstride + tid_tile] = s;
    }
    fft_pencil_multi<NZ, P, 1, T, C, CG>(v, t, lp, TX, twl, 1, TX * NZ);
  }
  if (valid && pm) {
    if constexpr (PR) {
#pragma unroll
      for (int j = 0; j < C; j += 2)
#pragma unroll
        for (int i = 0; i < P; ++i)
          *reinterpret_cast<Q4*>(pbase + (long long)j * cstride + (long long)(t + TZ * i) * pes) =
              Q4{v[j][i].x, v[j][i].y, v[j + 1][i].x, v[j + 1][i].y};
    }
  } else if (valid) {
#pragma unroll
    for (int j = 0; j < C; ++j)
#pragma unroll
      for (int i = 0; i < P; ++i) z_store<T, SEG>(base + j * cstride + (long long)(t + TZ * i) * es_g, v[j][i]);
  }
}

// ----------------------------------------------------------------------------
// The same z pass for every load of a tile in one workgroup (truncated,
// filtered and consistent operators): the operator matrices of the thread's
// wave-vectors are formed once and applied to each load in turn, so the alias
// sums (or the stored-table reads) are shared by all loads.  The pencils of
// the next active load are read into a second register set before the
// current one is transformed: workgroup barriers wait on LDS traffic only, so
// those HBM reads overlap the transforms.  With qpart, the per-load Parseval
// partials of k_zg (one per workgroup and load).
// ----------------------------------------------------------------------------
template <typename T, int NZ, int P, int TX, int C>
__global__ __launch_bounds__(TX*(NZ / P)) void k_zgm(const Geo g, const GreenParams gp, const GreenTabs<T> tb,
                                                    cpx<T>* __restrict__ smain, cpx<T>* __restrict__ snyq,
                                                    const cpx<T>* __restrict__ twz, const LoadState* __restrict__ st,
                                                    const int main_tiles, const int nload,
                                                    double* __restrict__ qpart, const int pstride) {
  constexpr int TZ = NZ / P;
  constexpr int SEG = TX * (int)sizeof(cpx<T>);   // contiguous bytes per access instruction
  constexpr int NT = TX * TZ;
  constexpr int NE = C * (C + 1) / 2;
  __shared__ cpx<T> lds[TX * NZ];
  __shared__ cpx<T> twl[NZ];
  __shared__ double red[(NT + 63) / 64];
  const int tid = threadIdx.x;
  for (int i = tid; i < NZ; i += NT) twl[i] = twz[i];
  const int xl = tid % TX, t = tid / TX;
  cpx<T>* base;
  long long es_g, cstride, lstride;
  int kx, ky;
  bool valid;
  if ((int)blockIdx.x < main_tiles) {
    const int xtiles = (g.mx + TX - 1) / TX;
    const int tile = xcd_tile<line_share<T, TX>()>(blockIdx.x, main_tiles);
    const int xc = tile % xtiles;
    ky = tile / xtiles;
    kx = xc * TX + xl;
    valid = kx < g.mx;
    base = smain + (long long)ky * g.mx + (valid ? kx : 0);
    es_g = (long long)g.ny * g.mx;
    cstride = (long long)g.nz * g.ny * g.mx;
    lstride = main_cpx(g);
  } else {
    ky = (blockIdx.x - main_tiles) * TX + xl;
    kx = g.mx;
    valid = ky < g.ny;
    base = snyq + (valid ? ky : 0);
    es_g = g.ny;
    cstride = (long long)g.nz * g.ny;
    lstride = nyq_cpx(g);
  }
  T G[P][NE];
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const int kz = t + TZ * i;
    const int k[3] = {kx, ky, kz};
    const long long tidx = (kx < g.mx) ? ((long long)kz * g.ny + ky) * g.mx + kx
                                       : (long long)g.nz * g.ny * g.mx + (long long)kz * g.ny + ky;
    if (valid) {
      green_matrix<T, C>(gp, tb, k, tidx, G[i]);
    } else {
#pragma unroll
      for (int q = 0; q < NE; ++q) G[i][q] = T(0);
    }
  }
  // the same for every thread of the workgroup
  auto next_active = [&](int l) {
    while (l < nload && st != nullptr && !st[l].active) ++l;
    return l;
  };
  // base is clamped to an existing pencil, so every lane reads in bounds and
  // the reads need no branch; lanes past the edge never store
  auto read = [&](cpx<T> (&dst)[C][P], int l) {
    const cpx<T>* b = base + (long long)l * lstride;
#pragma unroll
    for (int j = 0; j < C; ++j)
#pragma unroll
      for (int i = 0; i < P; ++i) dst[j][i] = z_load<T, SEG>(b + j * cstride + (long long)(t + TZ * i) * es_g);
  };
  const double wk = (kx == 0 || kx == g.mx) ? 1.0 : 2.0;
  cpx<T>* lp = lds + xl;
  int l = next_active(0);
  cpx<T> nx[C][P];
  if (l < nload) read(nx, l);
  __syncthreads();
  while (l < nload) {
    cpx<T> v[C][P];
#pragma unroll
    for (int j = 0; j < C; ++j)
#pragma unroll
      for (int i = 0; i < P; ++i) v[j][i] = nx[j][i];
    const int ln = next_active(l + 1);
    if (ln < nload) read(nx, ln);
    fft_pencil_multi<NZ, P, -1, T, C>(v, t, lp, TX, twl, 1);
    double quad = 0.0;
#pragma unroll
    for (int i = 0; i < P; ++i) {
      cpx<T> w[C];
#pragma unroll
      for (int j = 0; j < C; ++j) w[j] = v[j][i];
      sym_apply<T, C>(G[i], w);
      if (qpart != nullptr) {
        T d = T(0);
#pragma unroll
        for (int j = 0; j < C; ++j) d += v[j][i].x * w[j].x + v[j][i].y * w[j].y;
        quad += (double)d;
      }
#pragma unroll
      for (int j = 0; j < C; ++j) v[j][i] = w[j];
    }
    if (qpart != nullptr) {
      const double s = block_sum<NT>(valid ? quad * wk / (double)g.nvox : 0.0, red);
      if (tid == 0) qpart[(long long)l * pstride + blockIdx.x] = s;
    }
    fft_pencil_multi<NZ, P, 1, T, C>(v, t, lp, TX, twl, 1);
    if (valid) {
      cpx<T>* b = base + (long long)l * lstride;
#pragma unroll
      for (int j = 0; j < C; ++j)
#pragma unroll
        for (int i = 0; i < P; ++i) z_store<T, SEG>(b + j * cstride + (long long)(t + TZ * i) * es_g, v[j][i]);
    }
    l = ln;
  }
}

// ----------------------------------------------------------------------------
// x inverse: C2R, scaling, local term and solver epilogue
// ----------------------------------------------------------------------------
template <typename T>
struct XinvArgs {
  Geo g;
  int mode;
  int nphase;
  int iso;                // every phase has the short (a Id + b m m^T) form
  const cpx<T>* smain;    // input spectrum (may alias out)
  const cpx<T>* snyq;
  const cpx<T>* twx;
  const T* tau;           // field the spectrum was taken of (p, tau, x)
  T* out;                 // real output (q, new tau, strain, updated r); may alias smain or rin
  const T* rin;           // residual updated in place by XI_CGR
  float* rout;            // FP32 residual (refinement)
  const T* ptab;          // [nphase][2 c c + 5], see phase_row
  const uint8_t* phase;
  const T* vcoef;         // per-voxel mode: [2][nvox] (a_inv, b_inv), else null
  const double* loads;    // [load][c]
  const LoadState* st;
  double* partials;
  int pstride;
  T scale;                // 1/N^d times the factor of the half-length route
  T em2[9];               // 2 A0: c x c (scalar), or (4 mu0, 2 lambda0) of the isotropic elastic A0
  int paired;             // main spectrum in the component-paired layout (FP32, even c)
};

template <typename T, int MX, int P, int C>
__global__ __launch_bounds__(256) void k_xinv(const XinvArgs<T> a) {
  constexpr int TR = MX / P;
  constexpr int RPW = 256 / TR;
  constexpr int SEG = TR * (int)sizeof(cpx<T>);   // contiguous bytes per access instruction
  constexpr int TABW = 2 * C * C + 5;
  // six components: three components share each FFT exchange
  constexpr int CG = C == 6 ? 3 : 1;
  __shared__ cpx<T> lds[CG * RPW * MX];
  __shared__ cpx<T> twl[2 * MX];
  __shared__ T tab[kMaxPhases * TABW];
  __shared__ double red[4];
  const Geo& g = a.g;
  const int l = blockIdx.y;
  if (a.st != nullptr && !a.st[l].active) return;
  const int tid = threadIdx.x;
  for (int i = tid; i < a.nphase * TABW; i += 256) tab[i] = a.ptab[i];
  for (int i = tid; i < 2 * MX; i += 256) twl[i] = a.twx[i];
  const int slot = tid / TR, t = tid % TR;
  const long long vrows = (long long)g.nz * g.ny;
  const long long vr = (long long)blockIdx.x * RPW + slot;
  const bool valid = vr < vrows;
  const long long vrc = valid ? vr : 0;
  cpx<T>* lrow = lds + slot * MX;
  const bool iso = a.iso != 0;
  const bool vm = a.vcoef != nullptr;

  // all components' spectrum rows are loaded before the first transform
  cpx<T> gam[C][P];
  cpx<T> nqs[C];
  bool loaded = false;
  if constexpr (C % 2 == 0 && sizeof(T) == 4) {
    if (a.paired) {
      // component pairs side by side: one 16-byte read per pair and point
#pragma unroll
      for (int j = 0; j < C; j += 2) {
        const float4* pr = reinterpret_cast<const float4*>(a.smain + (long long)l * main_cpx(g) +
                                                           ((long long)(j / 2) * vrows + vrc) * 2 * MX);
#pragma unroll
        for (int i = 0; i < P; ++i) {
          const float4 q = ld_stream4(pr + t + TR * i);
          gam[j][i] = cpx<T>{q.x, q.y};
          gam[j + 1][i] = cpx<T>{q.z, q.w};
        }
      }
      loaded = true;
    }
  }
  if (!loaded) {
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const cpx<T>* sm = a.smain + (long long)l * main_cpx(g) + ((long long)j * vrows + vrc) * MX;
#pragma unroll
      for (int i = 0; i < P; ++i) gam[j][i] = ld_seg<SEG>(sm + t + TR * i);
    }
  }
#pragma unroll
  for (int j = 0; j < C; ++j) nqs[j] = a.snyq[(long long)l * nyq_cpx(g) + (long long)j * vrows + vrc];
  // repack each component's half spectrum as the half-length complex
  // transform 2Z = 2E + i 2O (CG components per exchange, in the exchange
  // buffers of the transforms), then the inverse transforms of all components
#pragma unroll
  for (int j0 = 0; j0 < C; j0 += CG) {
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < CG; ++jj)
#pragma unroll
      for (int i = 0; i < P; ++i) lrow[jj * RPW * MX + t + TR * i] = gam[j0 + jj][i];
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < CG; ++jj) {
      const int j = j0 + jj;
      const cpx<T> nq = nqs[j];
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const int k = t + TR * i;
        const cpx<T> xk = gam[j][i];
        const cpx<T> xm = (k == 0) ? nq : lrow[jj * RPW * MX + MX - k];
        const cpx<T> e = cpx<T>{xk.x + xm.x, xk.y - xm.y};          // 2E = X + conj(Xm)
        const cpx<T> d = cpx<T>{xk.x - xm.x, xk.y + xm.y};          // X - conj(Xm)
        const cpx<T> o = cmulc(d, twl[k]);                          // 2O = (X - conj Xm) W^{-k}
        gam[j][i] = cadd(e, mul_i(o));
      }
    }
  }
  __syncthreads();
  fft_pencil_multi<MX, P, 1, T, C, CG>(gam, t, lrow, 1, twl, 2, RPW * MX);

  // the route above returns N^d times the inverse DFT: a.scale = 1/N^d
  const T sc = a.scale;
  const long long fo = (long long)l * field_elems(g);
  double part = 0.0;
  T pl[C];
#pragma unroll
  for (int j = 0; j < C; ++j) pl[j] = static_cast<T>(a.loads[l * C + j]);
  // unrolled by template recursion: the body is too large for the unroll
  // pragma at P >= 8, and a run-time i would index gam and force it to scratch
  static_for<0, P>([&](auto i_) {
    constexpr int i = decltype(i_)::value;
    const int n = t + TR * i;
    const long long vox = vrc * (2 * MX) + 2 * n;   // first voxel of the pair
    T t0[C], t1[C], g0[C], g1[C];
#pragma unroll
    for (int j = 0; j < C; ++j) {
      g0[j] = gam[j][i].x * sc;
      g1[j] = gam[j][i].y * sc;
      t0[j] = t1[j] = T(0);
    }
    if (a.mode != XI_STRAIN) {
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const cpx<T> tv = ld_seg<SEG>(reinterpret_cast<const cpx<T>*>(a.tau + fo + (long long)j * g.nvox + vox));
        t0[j] = tv.x;
        t1[j] = tv.y;
      }
    }
    Loc<T> L0, L1;
    if (vm) {
      const cpx<T> ai = *reinterpret_cast<const cpx<T>*>(a.vcoef + vox);
      const cpx<T> bi = *reinterpret_cast<const cpx<T>*>(a.vcoef + g.nvox + vox);
      L0 = Loc<T>{nullptr, ai.x != T(0) ? T(1) : T(0), ai.x, bi.x};
      L1 = Loc<T>{nullptr, ai.y != T(0) ? T(1) : T(0), ai.y, bi.y};
    } else {
      const uint16_t ph2 = *reinterpret_cast<const uint16_t*>(a.phase + vox);
      const T* tb0 = tab + (ph2 & 0xff) * TABW;
      const T* tb1 = tab + (ph2 >> 8) * TABW;
      L0 = Loc<T>{tb0, tb0[2 * C * C], T(0), T(0)};
      L1 = Loc<T>{tb1, tb1[2 * C * C], T(0), T(0)};
    }
    const T in0 = L0.in, in1 = L1.in;
    cpx<T> res[C];
    if (a.mode == XI_APPLY || a.mode == XI_CG) {
#pragma unroll
      for (int j = 0; j < C; ++j)
        res[j] = cpx<T>{in0 * (loc_row<T, C>(L0, vm, 0, iso, j, t0) + g0[j]),
                        in1 * (loc_row<T, C>(L1, vm, 0, iso, j, t1) + g1[j])};
#pragma unroll
      for (int j = 0; j < C; ++j) part += (double)t0[j] * res[j].x + (double)t1[j] * res[j].y;
    } else if (a.mode == XI_CGR) {
      // r -= alpha L p in place (alpha known from the quadratic forms), and ||r||^2
      const T al = static_cast<T>(a.st[l].alpha);
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const cpx<T> rv = ld_seg<SEG>(reinterpret_cast<const cpx<T>*>(a.rin + fo + (long long)j * g.nvox + vox));
        const T q0 = in0 * (loc_row<T, C>(L0, vm, 0, iso, j, t0) + g0[j]);
        const T q1 = in1 * (loc_row<T, C>(L1, vm, 0, iso, j, t1) + g1[j]);
        res[j] = cpx<T>{rv.x - al * q0, rv.y - al * q1};
        part += (double)res[j].x * res[j].x + (double)res[j].y * res[j].y;
      }
    } else if (a.mode == XI_BASIC) {
      // new tau = (A - A0)(p - Gamma tau); residual (p - Gamma tau) - (A - A0)^{-1} tau
      T u0[C], u1[C];
#pragma unroll
      for (int m = 0; m < C; ++m) {
        u0[m] = pl[m] - g0[m];
        u1[m] = pl[m] - g1[m];
      }
#pragma unroll
      for (int j = 0; j < C; ++j) {
        res[j] = cpx<T>{in0 * loc_row<T, C>(L0, vm, 1, iso, j, u0), in1 * loc_row<T, C>(L1, vm, 1, iso, j, u1)};
        const double rx = in0 * (u0[j] - loc_row<T, C>(L0, vm, 0, iso, j, t0));
        const double ry = in1 * (u1[j] - loc_row<T, C>(L1, vm, 0, iso, j, t1));
        part += rx * rx + ry * ry;
      }
    } else if (a.mode == XI_EM) {
      // new tau = (A - A0)(A + A0)^{-1} (tau + 2 A0 u), u = p - Gamma tau;
      // residual u - (A - A0)^{-1} tau
      T u0[C], u1[C], w0[C], w1[C];
#pragma unroll
      for (int m = 0; m < C; ++m) {
        u0[m] = pl[m] - g0[m];
        u1[m] = pl[m] - g1[m];
      }
#pragma unroll
      for (int j = 0; j < C; ++j) {
        T e0 = 0, e1 = 0;
        if (C == 6) {
          e0 = a.em2[0] * u0[j];
          e1 = a.em2[0] * u1[j];
          if (j < 3) {
            e0 += a.em2[1] * (u0[0] + u0[1] + u0[2]);
            e1 += a.em2[1] * (u1[0] + u1[1] + u1[2]);
          }
        } else {
#pragma unroll
          for (int m = 0; m < C; ++m) {
            e0 += a.em2[j * C + m] * u0[m];
            e1 += a.em2[j * C + m] * u1[m];
          }
        }
        w0[j] = t0[j] + e0;
        w1[j] = t1[j] + e1;
      }
      const int wm = vm ? 2 : 1;
#pragma unroll
      for (int j = 0; j < C; ++j) {
        res[j] = cpx<T>{in0 * loc_row<T, C>(L0, vm, wm, iso, j, w0, a.em2[0], a.em2[1]),
                        in1 * loc_row<T, C>(L1, vm, wm, iso, j, w1, a.em2[0], a.em2[1])};
        const double rx = in0 * (u0[j] - loc_row<T, C>(L0, vm, 0, iso, j, t0));
        const double ry = in1 * (u1[j] - loc_row<T, C>(L1, vm, 0, iso, j, t1));
        part += rx * rx + ry * ry;
      }
    } else if (a.mode == XI_IRRES || a.mode == XI_RESNORM) {
#pragma unroll
      for (int j = 0; j < C; ++j) {
        res[j] = cpx<T>{in0 * (pl[j] - loc_row<T, C>(L0, vm, 0, iso, j, t0) - g0[j]),
                        in1 * (pl[j] - loc_row<T, C>(L1, vm, 0, iso, j, t1) - g1[j])};
        part += (double)res[j].x * res[j].x + (double)res[j].y * res[j].y;
      }
    } else {  // XI_STRAIN: p - Gamma tau everywhere
#pragma unroll
      for (int j = 0; j < C; ++j) res[j] = cpx<T>{pl[j] - g0[j], pl[j] - g1[j]};
    }
    if (valid) {
      if (a.mode == XI_IRRES) {
#pragma unroll
        for (int j = 0; j < C; ++j)
          st_seg<TR * (int)sizeof(float2)>(reinterpret_cast<float2*>(a.rout + fo + (long long)j * g.nvox + vox),
                    float2{static_cast<float>(res[j].x), static_cast<float>(res[j].y)});
      } else if (a.mode != XI_RESNORM) {
#pragma unroll
        for (int j = 0; j < C; ++j) st_seg<SEG>(reinterpret_cast<cpx<T>*>(a.out + fo + (long long)j * g.nvox + vox), res[j]);
      }
    }
  });
  if (!valid) part = 0.0;
  if (a.partials != nullptr) {
    const double s = block_sum<256>(part, red);
    if (tid == 0) a.partials[(long long)l * a.pstride + blockIdx.x] = s;
  }
}

// ----------------------------------------------------------------------------
// Consistent operator of eq. (11), stored: one thread per wave-vector of the
// packed half spectrum (main part, then the Nyquist plane) sums
// F(2 pi (k/N + n))^2 Gamma0_hat(k + n N) over the aliases whose reduced
// frequency k_a/N_a + n_a lies in [-(nmax+1/2), nmax+1/2] on every axis
// (a cut that keeps the truncated series even in k), in FP64, and writes the
// upper triangle in FP64 and FP32.
// ----------------------------------------------------------------------------
__device__ __forceinline__ double sinc_pi(double x) {   // sin(pi x)/(pi x)
  if (x == 0.0) return 1.0;
  return sinpi(x) / (3.14159265358979323846 * x);
}

// Stored operator of the z pass (layout in green_dev.hpp): green_matrix in
// FP64 at every wave-vector of the half spectrum, rounded to TO.
template <typename TO, int C>
__global__ __launch_bounds__(256) void k_green_store(const Geo g, const GreenParams gp, const GreenTabs<double> tb,
                                                     Quad<TO>* __restrict__ out) {
  constexpr int NE = C * (C + 1) / 2, NG = store_groups<C>();
  const long long nmain = (long long)g.nz * g.ny * g.mx;
  const long long total = nmain + (long long)g.nz * g.ny;
  const long long id = (long long)blockIdx.x * 256 + threadIdx.x;
  if (id >= total) return;
  int k[3];
  Quad<TO>* q;
  long long gs;
  if (id < nmain) {
    k[0] = (int)(id % g.mx);
    k[1] = (int)((id / g.mx) % g.ny);
    k[2] = (int)(id / ((long long)g.mx * g.ny));
    q = out + (((long long)k[2] * g.ny + k[1]) * NG) * g.mx + k[0];
    gs = g.mx;
  } else {
    const long long r = id - nmain;
    k[0] = g.mx;
    k[1] = (int)(r % g.ny);
    k[2] = (int)(r / g.ny);
    q = out + nmain * NG + ((long long)k[2] * NG) * g.ny + k[1];
    gs = g.ny;
  }
  double G[NE];
  green_matrix<double, C>(gp, tb, k, 0, G);
  double e[4 * NG];
  for (int i = 0; i < 4 * NG; ++i) e[i] = i < NE ? G[i] : 0.0;
  for (int j = 0; j < NG; ++j)
    q[j * gs] = Quad<TO>{(TO)e[4 * j], (TO)e[4 * j + 1], (TO)e[4 * j + 2], (TO)e[4 * j + 3]};
}

template <int C>
__global__ __launch_bounds__(256) void k_consistent_table(const Geo g, const GreenParams gp, const int nmax,
                                                          double* __restrict__ tab64, float* __restrict__ tab32) {
  constexpr int NE = C * (C + 1) / 2;
  const long long nmain = (long long)g.nz * g.ny * g.mx;
  const long long total = nmain + (long long)g.nz * g.ny;
  const long long id = (long long)blockIdx.x * 256 + threadIdx.x;
  if (id >= total) return;
  int k[3];
  if (id < nmain) {
    k[0] = (int)(id % g.mx);
    k[1] = (int)((id / g.mx) % g.ny);
    k[2] = (int)(id / ((long long)g.mx * g.ny));
  } else {
    const long long r = id - nmain;
    k[0] = g.mx;
    k[1] = (int)(r % g.ny);
    k[2] = (int)(r / g.ny);
  }
  const int dim = (C == 2) ? 2 : 3;
  double acc[C][C];
  for (int i = 0; i < C; ++i)
    for (int j = 0; j < C; ++j) acc[i][j] = 0.0;
  const double lim = nmax + 0.5;
  int lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = 0;
    hi[a] = 0;
  }
  for (int a = 0; a < dim; ++a) {
    lo[a] = -nmax - 1;
    hi[a] = nmax + 1;
  }
  for (int n2 = lo[2]; n2 <= hi[2]; ++n2)
    for (int n1 = lo[1]; n1 <= hi[1]; ++n1)
      for (int n0 = lo[0]; n0 <= hi[0]; ++n0) {
        const int nn[3] = {n0, n1, n2};
        double w = 1.0, xi[3] = {0.0, 0.0, 0.0};
        bool inside = true;
        for (int a = 0; a < dim; ++a) {
          const double frac = (double)k[a] / gp.n[a] + nn[a];
          inside &= fabs(frac) <= lim;
          const double sc = sinc_pi(frac);
          w *= sc * sc;
          xi[a] = frac * gp.n[a];
        }
        if (!inside || w == 0.0) continue;
        // Gamma0_hat at xi, as a c x c matrix (columns: images of the unit vectors)
        if constexpr (C == 6) {
          BD<double> s;
          bd_zero(s);
          bd_add(s, 1.0, xi[0], xi[1], xi[2]);
          for (int j = 0; j < 6; ++j) {
            double e[6], o[6];
            for (int i = 0; i < 6; ++i) e[i] = i == j ? 1.0 : 0.0;
            bd_apply_real(s, 0.5 / gp.mu0, gp.kappa, e, o);
            for (int i = 0; i < 6; ++i) acc[i][j] += w * o[i];
          }
        } else {
          double den = 0.0;
          for (int a = 0; a < C; ++a)
            for (int b = 0; b < C; ++b) den += xi[a] * gp.a0[3 * a + b] * xi[b];
          if (den > 0.0)
            for (int i = 0; i < C; ++i)
              for (int j = 0; j < C; ++j) acc[i][j] += w * xi[i] * xi[j] / den;
        }
      }
  int q = 0;
  for (int i = 0; i < C; ++i)
    for (int j = i; j < C; ++j) {
      const double val = 0.5 * (acc[i][j] + acc[j][i]);
      tab64[id * NE + q] = val;
      tab32[id * NE + q] = (float)val;
      ++q;
    }
}

// ----------------------------------------------------------------------------
// elementwise kernels
// ----------------------------------------------------------------------------

template <typename V> __device__ __forceinline__ double vdot(const V& a, const V& b);
template <> __device__ __forceinline__ double vdot<float4>(const float4& a, const float4& b) {
  return (double)a.x * b.x + (double)a.y * b.y + (double)a.z * b.z + (double)a.w * b.w;
}
template <> __device__ __forceinline__ double vdot<double2>(const double2& a, const double2& b) {
  return a.x * b.x + a.y * b.y;
}
__device__ __forceinline__ float4 vaxpy(float4 x, float s, float4 y) {
  return float4{x.x + s * y.x, x.y + s * y.y, x.z + s * y.z, x.w + s * y.w};
}
__device__ __forceinline__ double2 vaxpy(double2 x, double s, double2 y) {
  return double2{x.x + s * y.x, x.y + s * y.y};
}

constexpr int kEwUnroll = 4;

// Workgroups per load (or per component group) of the grid-stride
// initialisation and mean passes over n elements: at least 1024 elements per
// workgroup, at most 1024 workgroups, so that each workgroup's fixed cost
// (its reduction) is amortised; every count stays within the partials stride.
inline int ew_blocks(long long n) { return (int)std::min<long long>((n + 1023) / 1024, 1024); }

// r -= alpha q;  partial r.r      (per load, 16-byte vectors; x is updated
// one step later inside the x forward pass, or by k_xflush)
template <typename T>
__global__ __launch_bounds__(256) void k_cgupd(const long long nvec, T* __restrict__ r, const T* __restrict__ q,
                                               const LoadState* __restrict__ st, double* __restrict__ partials,
                                               const int pstride) {
  using V = typename Vec16<T>::type;
  __shared__ double red[4];
  const int l = blockIdx.y;
  if (!st[l].active) return;
  const T al = static_cast<T>(st[l].alpha);
  const long long off = (long long)l * nvec;
  V* rv = reinterpret_cast<V*>(r) + off;
  const V* qv = reinterpret_cast<const V*>(q) + off;
  double part = 0.0;
  const long long b0 = (long long)blockIdx.x * 256 * kEwUnroll + threadIdx.x;
#pragma unroll
  for (int u = 0; u < kEwUnroll; ++u) {
    const long long i = b0 + (long long)u * 256;
    if (i < nvec) {
      const V rn = vaxpy(rv[i], -al, qv[i]);
      rv[i] = rn;
      part += vdot(rn, rn);
    }
  }
  const double s = block_sum<256>(part, red);
  if (threadIdx.x == 0) partials[(long long)l * pstride + blockIdx.x] = s;
}

// x += alpha p for the loads whose last CG step is still pending
template <typename T>
__global__ __launch_bounds__(256) void k_xflush(const long long nvec, T* __restrict__ x, const T* __restrict__ p,
                                                const LoadState* __restrict__ st) {
  using V = typename Vec16<T>::type;
  const int l = blockIdx.y;
  if (!st[l].pending) return;
  const T al = static_cast<T>(st[l].alpha);
  const long long off = (long long)l * nvec;
  V* xv = reinterpret_cast<V*>(x) + off;
  const V* pv = reinterpret_cast<const V*>(p) + off;
  const long long b0 = (long long)blockIdx.x * 256 * kEwUnroll + threadIdx.x;
#pragma unroll
  for (int u = 0; u < kEwUnroll; ++u) {
    const long long i = b0 + (long long)u * 256;
    if (i < nvec) xv[i] = vaxpy(xv[i], al, pv[i]);
  }
}

// End of a fused CG solve: the pending steps of every load, x += alpha
// p[pbuf] (+ alpha2 p[1 - pbuf] when two are pending), p[0] and p[1] the two
// direction buffers.
template <typename T>
__global__ __launch_bounds__(256) void k_xflush2(const long long nvec, T* __restrict__ x, const T* __restrict__ p0,
                                                 const T* __restrict__ p1, const LoadState* __restrict__ st) {
  using V = typename Vec16<T>::type;
  const int l = blockIdx.y;
  const int np = st[l].pending;
  if (np == 0) return;
  const T al = static_cast<T>(st[l].alpha);
  const T al2 = static_cast<T>(np == 2 ? st[l].alpha2 : 0.0);
  const long long off = (long long)l * nvec;
  V* xv = reinterpret_cast<V*>(x) + off;
  const V* pn = reinterpret_cast<const V*>(st[l].pbuf ? p1 : p0) + off;
  const V* po = reinterpret_cast<const V*>(st[l].pbuf ? p0 : p1) + off;
  const long long b0 = (long long)blockIdx.x * 256 * kEwUnroll + threadIdx.x;
#pragma unroll
  for (int u = 0; u < kEwUnroll; ++u) {
    const long long i = b0 + (long long)u * 256;
    if (i < nvec) {
      V y = vaxpy(xv[i], al, pn[i]);
      if (np == 2) y = vaxpy(y, al2, po[i]);
      xv[i] = y;
    }
  }
}

// x = 0;  r = 1_{I0} p_l;  partial ||r||^2 (I0 from the phase flags, or from
// a_inv != 0 in per-voxel mode)
template <typename T>
__global__ __launch_bounds__(256) void k_cginit(const Geo g, T* __restrict__ x, T* __restrict__ r,
                                                const uint8_t* __restrict__ phase, const uint8_t* __restrict__ i0,
                                                const double* __restrict__ vcoef, const double* __restrict__ loads,
                                                double* __restrict__ partials, const int pstride) {
  __shared__ double red[4];
  const int l = blockIdx.y;
  const long long F = field_elems(g);
  double part = 0.0;
  // grid-stride over the voxels (ew_blocks workgroups per load), all
  // components of a voxel by one thread: one I0 test per voxel
  for (long long v = (long long)blockIdx.x * 256 + threadIdx.x; v < g.nvox; v += (long long)gridDim.x * 256) {
    const bool inside = vcoef != nullptr ? vcoef[v] != 0.0 : i0[phase[v]] != 0;
    for (int j = 0; j < g.c; ++j) {
      const T val = inside ? static_cast<T>(loads[l * g.c + j]) : T(0);
      const long long e = (long long)l * F + (long long)j * g.nvox + v;
      if (x != nullptr) x[e] = T(0);
      if (r != nullptr) r[e] = val;
      part += (double)val * val;
    }
  }
  const double s = block_sum<256>(part, red);
  if (threadIdx.x == 0) partials[(long long)l * pstride + blockIdx.x] = s;
}

// Initial guesses (flag per load in gflag): the guess is kept on I0 and
// zeroed elsewhere; the other loads, and zero loads (whose solution is 0 and
// which never iterate), start from x = 0.
template <typename T>
__global__ __launch_bounds__(256) void k_guessmask(const Geo g, T* __restrict__ x, const uint8_t* __restrict__ phase,
                                                   const uint8_t* __restrict__ i0, const double* __restrict__ vcoef,
                                                   const uint8_t* __restrict__ gflag, const double* __restrict__ loads) {
  const int l = blockIdx.y;
  const long long F = field_elems(g);
  bool nonzero = false;
  for (int j = 0; j < g.c; ++j) nonzero |= loads[l * g.c + j] != 0.0;
  const bool guessed = gflag[l] != 0 && nonzero;
  for (long long v = (long long)blockIdx.x * 256 + threadIdx.x; v < g.nvox; v += (long long)gridDim.x * 256) {
    const bool inside = vcoef != nullptr ? vcoef[v] != 0.0 : i0[phase[v]] != 0;
    for (int j = 0; j < g.c; ++j) {
      T* xe = x + (long long)l * F + (long long)j * g.nvox + v;
      *xe = (guessed && inside) ? *xe : T(0);
    }
  }
}

// r = b - q with q = L x0 on the guessed loads, r = b on the others (b = p on
// I0); partial ||b||^2 into group l and ||r||^2 into group ngroups + l.
template <typename T>
__global__ __launch_bounds__(256) void k_guessinit(const Geo g, const T* __restrict__ q, T* __restrict__ r,
                                                   const uint8_t* __restrict__ phase, const uint8_t* __restrict__ i0,
                                                   const double* __restrict__ vcoef, const double* __restrict__ loads,
                                                   const uint8_t* __restrict__ gflag, double* __restrict__ partials,
                                                   const int pstride, const int ngroups) {
  __shared__ double red[4];
  const int l = blockIdx.y;
  const long long F = field_elems(g);
  const bool guessed = gflag[l] != 0;
  double pb = 0.0, pr = 0.0;
  for (long long v = (long long)blockIdx.x * 256 + threadIdx.x; v < g.nvox; v += (long long)gridDim.x * 256) {
    const bool inside = vcoef != nullptr ? vcoef[v] != 0.0 : i0[phase[v]] != 0;
    for (int j = 0; j < g.c; ++j) {
      const long long e = (long long)l * F + (long long)j * g.nvox + v;
      const T bv = inside ? static_cast<T>(loads[l * g.c + j]) : T(0);
      const T rv = guessed ? bv - q[e] : bv;
      r[e] = rv;
      pb += (double)bv * bv;
      pr += (double)rv * rv;
    }
  }
  const double sb = block_sum<256>(pb, red);
  if (threadIdx.x == 0) partials[(long long)l * pstride + blockIdx.x] = sb;
  const double sr = block_sum<256>(pr, red);
  if (threadIdx.x == 0) partials[(long long)(ngroups + l) * pstride + blockIdx.x] = sr;
}

// d = 0 and partial ||r||^2 for the loads still refined (inner solve start)
template <typename T>
__global__ __launch_bounds__(256) void k_innerinit(const long long F, T* __restrict__ d, const T* __restrict__ r,
                                                   const LoadState* __restrict__ outer,
                                                   double* __restrict__ partials, const int pstride) {
  __shared__ double red[4];
  const int l = blockIdx.y;
  if (!outer[l].active) return;
  double part = 0.0;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < F; e += (long long)gridDim.x * 256) {
    d[(long long)l * F + e] = T(0);
    const double rv = r[(long long)l * F + e];
    part += rv * rv;
  }
  const double s = block_sum<256>(part, red);
  if (threadIdx.x == 0) partials[(long long)l * pstride + blockIdx.x] = s;
}

// partial sums of one component of one load: group (l, j)
template <typename T>
__global__ __launch_bounds__(256) void k_mean(const Geo g, const T* __restrict__ x, double* __restrict__ partials,
                                              const int pstride) {
  __shared__ double red[4];
  const int grp = blockIdx.y;   // l * c + j
  const T* xp = x + (long long)grp * g.nvox;
  double part = 0.0;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < g.nvox; e += (long long)gridDim.x * 256)
    part += (double)xp[e];
  const double s = block_sum<256>(part, red);
  if (threadIdx.x == 0) partials[(long long)grp * pstride + blockIdx.x] = s;
}

// ----------------------------------------------------------------------------
// Per-voxel isotropic moduli.  Input m[ncoef][nvox]: a (scalar, A = a Id) or
// bulk and shear moduli (K, mu) (elasticity, Mandel form).  Against the
// isotropic reference (a0, or K0 and mu0), (A - A0)^{-1} = a_inv Id + b_inv m m^T
// with a_inv = 1/(a - a0), b_inv = 0 (scalar) or a_inv = 1/(2 dmu),
// b_inv = 1/(9 dK) - 1/(6 dmu) (elasticity).  Hypothesis (2): A - A0 is zero
// (voxel outside I0, a_inv = b_inv = 0) or definite: a - a0 != 0, or dK and
// dmu nonzero of one sign.  Differences below 1e-12 of the moduli count as
// singular.  With out64 == null the kernel only counts violations (one partial
// per workgroup) over voxels [v0, vend); otherwise it writes the coefficients
// (FP64, and FP32 when out32 is given).
// ----------------------------------------------------------------------------
template <typename TI>
__global__ __launch_bounds__(256) void k_voxset(const long long v0, const long long vend, const long long nvox,
                                                const int elastic, const TI* __restrict__ m, const double a0,
                                                const double K0, const double mu0, double* __restrict__ out64,
                                                float* __restrict__ out32, double* __restrict__ partials) {
  __shared__ double red[4];
  const long long v = v0 + (long long)blockIdx.x * 256 + threadIdx.x;
  double bad = 0.0;
  if (v < vend) {
    double ai = 0.0, bi = 0.0;
    if (!elastic) {
      const double a = (double)m[v];
      const double d = a - a0;
      if (!isfinite(a)) bad = 1.0;
      else if (d != 0.0) {
        if (fabs(d) <= 1e-12 * (fabs(a) + fabs(a0))) bad = 1.0;
        else ai = 1.0 / d;
      }
    } else {
      const double K = (double)m[v], mu = (double)m[nvox + v];
      const double dK = K - K0, dm = mu - mu0;
      if (!isfinite(K) || !isfinite(mu)) {
        bad = 1.0;
      } else if (dK != 0.0 || dm != 0.0) {
        const bool tiny = fabs(dK) <= 1e-12 * (fabs(K) + fabs(K0)) || fabs(dm) <= 1e-12 * (fabs(mu) + fabs(mu0));
        if (tiny || (dK > 0.0) != (dm > 0.0)) {
          bad = 1.0;
        } else {
          ai = 1.0 / (2.0 * dm);
          bi = 1.0 / (9.0 * dK) - 1.0 / (6.0 * dm);
        }
      }
    }
    if (out64 != nullptr) {
      out64[v] = ai;
      out64[nvox + v] = bi;
      if (out32 != nullptr) {
        out32[v] = (float)ai;
        out32[nvox + v] = (float)bi;
      }
    }
  }
  if (out64 == nullptr) {
    const double s = block_sum<256>(bad, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
  }
}

// Sets *flag when a phase id of a device map is nphase or more (every writer
// stores the same value, so the race is benign); grid-stride over the voxels.
static __global__ __launch_bounds__(256) void k_phase_check(const uint8_t* __restrict__ phase, const long long nvox,
                                                     const int nphase, int* __restrict__ flag) {
  for (long long v = (long long)blockIdx.x * 256 + threadIdx.x; v < nvox; v += (long long)gridDim.x * 256)
    if ((int)phase[v] >= nphase) *flag = 1;
}

// ----------------------------------------------------------------------------
// Gradient of J = sum_lm W_lm p_l . A*_h p_m with respect to the isotropic
// coefficients of every voxel, from the strain estimates eps_l = p_l - Gamma tau_l
// of the solved loads (eps[load][c][nvox]):
//   scalar:      dJ/da  = (1/V) sum_lm W_lm eps_l . eps_m
//   elasticity:  dJ/dK  = (1/V) sum_lm W_lm tr eps_l tr eps_m,
//                dJ/dmu = (2/V) sum_lm W_lm (eps_l . eps_m - tr eps_l tr eps_m / 3)
// (Mandel dot products).  W is symmetric; its zero entries are skipped.
// ----------------------------------------------------------------------------
template <int C, typename TO>
__global__ __launch_bounds__(256) void k_grad(const Geo g, const int nload, const double* __restrict__ eps,
                                              const double* __restrict__ W, TO* __restrict__ grad) {
  const long long v = (long long)blockIdx.x * 256 + threadIdx.x;
  if (v >= g.nvox) return;
  const long long F = field_elems(g);
  double ee = 0.0, tt = 0.0;
  for (int l = 0; l < nload; ++l) {
    double el[C];
#pragma unroll
    for (int j = 0; j < C; ++j) el[j] = eps[(long long)l * F + (long long)j * g.nvox + v];
    for (int m = l; m < nload; ++m) {
      const double w = (m == l ? 1.0 : 2.0) * W[l * nload + m];
      if (w == 0.0) continue;
      double dot = 0.0, trm = 0.0;
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const double em = (m == l) ? el[j] : eps[(long long)m * F + (long long)j * g.nvox + v];
        dot += el[j] * em;
        if (C == 6 && j < 3) trm += em;
      }
      ee += w * dot;
      if (C == 6) tt += w * (el[0] + el[1] + el[2]) * trm;
    }
  }
  const double iv = 1.0 / (double)g.nvox;
  if (C == 6) {
    grad[v] = static_cast<TO>(tt * iv);
    grad[g.nvox + v] = static_cast<TO>(2.0 * (ee - tt / 3.0) * iv);
  } else {
    grad[v] = static_cast<TO>(ee * iv);
  }
}

template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_convert(const long long n, const TI* __restrict__ in, TO* __restrict__ out) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = static_cast<TO>(in[i]);
}

}  // namespace lsh
