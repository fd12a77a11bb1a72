// Persistent conjugate gradients for small grids: one workgroup per load runs
// every iteration of its load in a single launch.  Each iteration is the fused
// CG step of the multi-kernel path -- x rows (p = r + beta p, x += alpha p of
// the previous step, p.(A - A0)^{-1} p, R2C), y pencils, the last axis with the
// Green operator and p.Gamma p (Parseval), the inverse y pencils and the
// x-inverse rows with r -= alpha Lp and ||r||^2 -- with the passes separated by
// workgroup barriers instead of kernel boundaries.  Fields and spectra stay in
// the workspace (cache resident at these sizes); scalars live in registers of
// every thread, from LDS-broadcast reductions in a fixed order.  The loop ends
// at convergence, breakdown, non-finite values or maxit, the same in every
// thread of the workgroup, so no workgroup waits on another.
#pragma once

#include "kernels.hpp"

namespace lsh {

template <typename T>
struct TinyArgs {
  Geo g;
  GreenParams gp;
  GreenTabs<T> tb;
  T* x;
  T* r;
  T* p;
  cpx<T>* sm;
  cpx<T>* sn;
  const cpx<T>* tw[3];
  int nphase, iso;
  const T* ptab;
  const uint8_t* phase;
  const T* vcoef;
  LoadState* st;
  int maxit;
  double guard;   // CG breakdown when |p.Lp| <= guard r.r (see k_scal)
  HistRef hist;   // residual history (see hist_push)
};

// workgroup sum of one double, returned to every thread (fixed order)
template <int NT>
__device__ __forceinline__ double block_allsum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) s += red[i];
  return s;
}

template <typename T, int NX, int NY, int NZ, int C, int NT>
__global__ __launch_bounds__(NT) void k_tiny_cg(const TinyArgs<T> a) {
  constexpr int MX = NX / 2;
  constexpr int PR = MX < 4 ? MX : 4;                 // row passes
  constexpr int TR = MX / PR;
  constexpr int SLOTS = NT / TR;
  constexpr int ROWS = NY * NZ;
  constexpr int ROW_IT = (ROWS + SLOTS - 1) / SLOTS;
  constexpr int PY = NY < 4 ? NY : 4;                 // y pencils
  constexpr int TY = NY / PY;
  constexpr int PENY = NT / TY;
  constexpr int PZ = NZ < 4 ? NZ : 4;                 // z pencils (3D)
  constexpr int TZ = NZ / PZ;
  constexpr int PENZ = NT / TZ;
  constexpr int TABW = 2 * C * C + 5;
  constexpr int B1 = SLOTS * MX, B2 = PENY * NY, B3 = PENZ * NZ;
  constexpr int BUF = B1 > B2 ? (B1 > B3 ? B1 : B3) : (B2 > B3 ? B2 : B3);
  __shared__ cpx<T> buf[BUF];
  __shared__ cpx<T> tw0[NX];
  __shared__ cpx<T> tw1[NY];
  __shared__ cpx<T> tw2[NZ];
  __shared__ T tab[kMaxPhases * TABW];
  __shared__ double red[NT / 64];

  const Geo& g = a.g;
  const int l = blockIdx.x;
  const int tid = threadIdx.x;
  LoadState* st = a.st + l;
  if (!st->active) return;
  for (int i = tid; i < a.nphase * TABW; i += NT) tab[i] = a.ptab[i];
  for (int i = tid; i < NX; i += NT) tw0[i] = a.tw[0][i];
  for (int i = tid; i < NY; i += NT) tw1[i] = a.tw[1][i];
  for (int i = tid; i < NZ; i += NT) tw2[i] = a.tw[2][i];
  const long long F = field_elems(g);
  T* x = a.x + (long long)l * F;
  T* r = a.r + (long long)l * F;
  T* p = a.p + (long long)l * F;
  cpx<T>* sm = a.sm + (long long)l * main_cpx(g);
  cpx<T>* sn = a.sn + (long long)l * nyq_cpx(g);
  const bool iso = a.iso != 0;
  const bool vm = a.vcoef != nullptr;
  const double tol2 = st->tol2;
  double rr = st->rr;
  double alpha = 0.0, beta = 0.0;
  bool first = true, pend = false;
  int iters = st->iters, status = kStatusOk;
  bool done = false;
  __syncthreads();

  for (int it = 0; it < a.maxit; ++it) {
    double part = 0.0;
    // ---------------- x rows: p, x, local form, R2C ----------------
    {
      const int slot = tid / TR, t = tid % TR;
      cpx<T>* lrow = buf + slot * MX;
      for (int ri = 0; ri < ROW_IT; ++ri) {
        const int vr = ri * SLOTS + slot;
        const bool valid = vr < ROWS;
        const long long vrc = valid ? vr : 0;
        cpx<T> v[C][PR];
#pragma unroll
        for (int j = 0; j < C; ++j) {
          const long long roff = (long long)j * g.nvox + vrc * NX;
          const cpx<T>* r2 = reinterpret_cast<const cpx<T>*>(r + roff);
          cpx<T>* p2 = reinterpret_cast<cpx<T>*>(p + roff);
          cpx<T>* x2 = reinterpret_cast<cpx<T>*>(x + roff);
#pragma unroll
          for (int i = 0; i < PR; ++i) {
            const int n = t + TR * i;
            cpx<T> pv{0, 0};
            if (valid) {
              const cpx<T> rv = r2[n];
              if (first) {
                pv = rv;
              } else {
                const cpx<T> po = p2[n];
                if (pend) {
                  const cpx<T> xo = x2[n];
                  x2[n] = cpx<T>{xo.x + static_cast<T>(alpha) * po.x, xo.y + static_cast<T>(alpha) * po.y};
                }
                pv = cpx<T>{rv.x + static_cast<T>(beta) * po.x, rv.y + static_cast<T>(beta) * po.y};
              }
              p2[n] = pv;
            }
            v[j][i] = pv;
          }
        }
        if (valid) {
#pragma unroll
          for (int i = 0; i < PR; ++i) {
            const long long vox = vrc * NX + 2 * (t + TR * i);
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
            part += (double)(L0.in * loc_quad<T, C>(L0, vm, iso, p0)) +
                    (double)(L1.in * loc_quad<T, C>(L1, vm, iso, p1));
          }
        }
        fft_pencil_multi<MX, PR, -1, T, C>(v, t, lrow, 1, tw0, 2);
#pragma unroll
        for (int j = 0; j < C; ++j) {
          __syncthreads();
#pragma unroll
          for (int i = 0; i < PR; ++i) lrow[t + TR * i] = v[j][i];
          __syncthreads();
          const long long row = (long long)j * ROWS + vrc;
#pragma unroll
          for (int i = 0; i < PR; ++i) {
            const int k = t + TR * i;
            const cpx<T> z = v[j][i];
            if (k == 0) {
              if (valid) {
                sm[row * MX] = cpx<T>{z.x + z.y, T(0)};
                sn[row] = cpx<T>{z.x - z.y, T(0)};
              }
            } else {
              const cpx<T> zm = lrow[MX - k];
              const cpx<T> s1 = cpx<T>{z.x + zm.x, z.y - zm.y};
              const cpx<T> d1 = cpx<T>{z.x - zm.x, z.y + zm.y};
              const cpx<T> wo = cmul(tw0[k], mul_neg_i(d1));
              if (valid) sm[row * MX + k] = cpx<T>{T(0.5) * (s1.x + wo.x), T(0.5) * (s1.y + wo.y)};
            }
          }
        }
        __syncthreads();
      }
    }
    // ---------------- y pencils (3D: plain forward transforms) ----------------
    auto y_pass = [&](auto dir_) {
      constexpr int DIR = decltype(dir_)::value;
      const int q0 = tid / TY, t = tid % TY;
      cpx<T>* lp = buf + q0 * NY;
      constexpr int NPEN = C * NZ * (MX + 1);
      for (int pb = 0; pb < NPEN; pb += PENY) {
        const int q = pb + q0;
        const bool valid = q < NPEN;
        const int qq = valid ? q : 0;
        const int j = qq / (NZ * (MX + 1));
        const int rem = qq % (NZ * (MX + 1));
        const int kz = rem / (MX + 1), kx = rem % (MX + 1);
        cpx<T>* base;
        long long es;
        if (kx < MX) {
          base = sm + ((long long)(j * NZ + kz) * NY) * MX + kx;
          es = MX;
        } else {
          base = sn + (long long)(j * NZ + kz) * NY;
          es = 1;
        }
        cpx<T> v[PY];
#pragma unroll
        for (int i = 0; i < PY; ++i) v[i] = valid ? base[(long long)(t + TY * i) * es] : cpx<T>{0, 0};
        fft_pencil<NY, PY, DIR, T>(v, t, lp, 1, tw1, 1);
        if (valid) {
#pragma unroll
          for (int i = 0; i < PY; ++i) base[(long long)(t + TY * i) * es] = v[i];
        }
        __syncthreads();
      }
    };
    if constexpr (NZ > 1) y_pass(std::integral_constant<int, -1>{});
    // ---------------- last axis with the Green operator ----------------
    {
      // pencils along z (3D) or y (2D), all C components per thread
      constexpr int NL = NZ > 1 ? NZ : NY;
      constexpr int PL = NZ > 1 ? PZ : PY;
      constexpr int TL = NL / PL;
      constexpr int PENL = NT / TL;
      constexpr int NPEN = NZ > 1 ? NY * (MX + 1) : (MX + 1);
      const cpx<T>* twl = NZ > 1 ? tw2 : tw1;
      const int q0 = tid / TL, t = tid % TL;
      cpx<T>* lp = buf + q0 * NL;
      for (int pb = 0; pb < NPEN; pb += PENL) {
        const int q = pb + q0;
        const bool valid = q < NPEN;
        const int qq = valid ? q : 0;
        int kx, ky = 0;
        cpx<T>* base;
        long long es, cs;
        if constexpr (NZ > 1) {
          ky = qq / (MX + 1);
          kx = qq % (MX + 1);
          if (kx < MX) {
            base = sm + (long long)ky * MX + kx;
            es = (long long)NY * MX;
            cs = (long long)NZ * NY * MX;
          } else {
            base = sn + ky;
            es = NY;
            cs = (long long)NZ * NY;
          }
        } else {
          kx = qq;
          if (kx < MX) {
            base = sm + kx;
            es = MX;
            cs = (long long)NY * MX;
          } else {
            base = sn;
            es = 1;
            cs = NY;
          }
        }
        cpx<T> v[C][PL];
#pragma unroll
        for (int j = 0; j < C; ++j)
#pragma unroll
          for (int i = 0; i < PL; ++i) v[j][i] = valid ? base[j * cs + (long long)(t + TL * i) * es] : cpx<T>{0, 0};
        fft_pencil_multi<NL, PL, -1, T, C>(v, t, lp, 1, twl, 1);
        double quad = 0.0;
        if (valid) {
#pragma unroll
          for (int i = 0; i < PL; ++i) {
            const int kl = t + TL * i;
            int k[3];
            long long tidx;
            if constexpr (NZ > 1) {
              k[0] = kx; k[1] = ky; k[2] = kl;
              tidx = (kx < MX) ? ((long long)kl * NY + ky) * MX + kx
                               : (long long)NZ * NY * MX + (long long)kl * NY + ky;
            } else {
              k[0] = kx; k[1] = kl; k[2] = 0;
              tidx = (kx < MX) ? (long long)kl * MX + kx : (long long)NY * MX + kl;
            }
            cpx<T> w[C];
#pragma unroll
            for (int j = 0; j < C; ++j) w[j] = v[j][i];
            green_apply<T, C>(a.gp, a.tb, k, tidx, w);
#pragma unroll
            for (int j = 0; j < C; ++j) {
              quad += (double)v[j][i].x * w[j].x + (double)v[j][i].y * w[j].y;
              v[j][i] = w[j];
            }
          }
        }
        part += quad * ((kx == 0 || kx == MX) ? 1.0 : 2.0) / (double)g.nvox;
        fft_pencil_multi<NL, PL, 1, T, C>(v, t, lp, 1, twl, 1);
        if (valid) {
#pragma unroll
          for (int j = 0; j < C; ++j)
#pragma unroll
            for (int i = 0; i < PL; ++i) base[j * cs + (long long)(t + TL * i) * es] = v[j][i];
        }
        __syncthreads();
      }
    }
    // ---------------- alpha ----------------
    const double pq = block_allsum<NT>(part, red);
    if (!isfinite(pq)) {
      status = kStatusNumeric;
      break;
    }
    if (fabs(pq) <= a.guard * rr) {
      status = kStatusBreakdown;
      break;
    }
    alpha = rr / pq;
    first = false;
    pend = true;
    if constexpr (NZ > 1) y_pass(std::integral_constant<int, 1>{});
    // ---------------- x-inverse rows: r -= alpha L p, ||r||^2 ----------------
    part = 0.0;
    {
      const int slot = tid / TR, t = tid % TR;
      cpx<T>* lrow = buf + slot * MX;
      const T al = static_cast<T>(alpha);
      const T sc = static_cast<T>(1.0 / (double)g.nvox);
      for (int ri = 0; ri < ROW_IT; ++ri) {
        const int vr = ri * SLOTS + slot;
        const bool valid = vr < ROWS;
        const long long vrc = valid ? vr : 0;
        cpx<T> gam[C][PR];
        cpx<T> nqs[C];
#pragma unroll
        for (int j = 0; j < C; ++j) {
          const long long srow = (long long)j * ROWS + vrc;
#pragma unroll
          for (int i = 0; i < PR; ++i) gam[j][i] = sm[srow * MX + t + TR * i];
          nqs[j] = sn[srow];
        }
#pragma unroll
        for (int j = 0; j < C; ++j) {
          __syncthreads();
#pragma unroll
          for (int i = 0; i < PR; ++i) lrow[t + TR * i] = gam[j][i];
          __syncthreads();
#pragma unroll
          for (int i = 0; i < PR; ++i) {
            const int k = t + TR * i;
            const cpx<T> xk = gam[j][i];
            const cpx<T> xm = (k == 0) ? nqs[j] : lrow[MX - k];
            const cpx<T> e = cpx<T>{xk.x + xm.x, xk.y - xm.y};
            const cpx<T> d = cpx<T>{xk.x - xm.x, xk.y + xm.y};
            const cpx<T> o = cmulc(d, tw0[k]);
            gam[j][i] = cadd(e, mul_i(o));
          }
        }
        __syncthreads();
        fft_pencil_multi<MX, PR, 1, T, C>(gam, t, lrow, 1, tw0, 2);
        if (valid) {
#pragma unroll
          for (int i = 0; i < PR; ++i) {
            const long long vox = vrc * NX + 2 * (t + TR * i);
            T t0[C], t1[C];
#pragma unroll
            for (int j = 0; j < C; ++j) {
              const cpx<T> tv = *reinterpret_cast<const cpx<T>*>(p + (long long)j * g.nvox + vox);
              t0[j] = tv.x;
              t1[j] = tv.y;
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
#pragma unroll
            for (int j = 0; j < C; ++j) {
              cpx<T>* rp = reinterpret_cast<cpx<T>*>(r + (long long)j * g.nvox + vox);
              const cpx<T> rv = *rp;
              const T q0 = L0.in * (loc_row<T, C>(L0, vm, 0, iso, j, t0) + gam[j][i].x * sc);
              const T q1 = L1.in * (loc_row<T, C>(L1, vm, 0, iso, j, t1) + gam[j][i].y * sc);
              const cpx<T> rn{rv.x - al * q0, rv.y - al * q1};
              *rp = rn;
              part += (double)rn.x * rn.x + (double)rn.y * rn.y;
            }
          }
        }
        __syncthreads();
      }
    }
    const double rr_new = block_allsum<NT>(part, red);
    ++iters;
    if (!isfinite(rr_new)) {
      status = kStatusNumeric;
      break;
    }
    beta = rr_new / rr;
    rr = rr_new;
    if (tid == 0) hist_push(a.hist, l, rr / st->bb);
    if (rr <= tol2) {
      done = true;
      break;
    }
  }
  // apply the last step's x += alpha p
  if (pend && status == kStatusOk) {
    for (long long e = tid; e < F; e += NT) x[e] += static_cast<T>(alpha) * p[e];
  }
  __syncthreads();
  if (tid == 0) {
    st->rr = rr;
    st->res2 = rr;
    st->alpha = alpha;
    st->beta = beta;
    st->iters = iters;
    st->status = status;
    st->pending = 0;
    st->first = first ? 1 : 0;
    st->active = (done || status != kStatusOk) ? 0 : 1;
  }
}

}  // namespace lsh
