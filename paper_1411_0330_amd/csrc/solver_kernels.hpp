// Solver-scalar kernels (non-template, one instance in the library): the
// deterministic reductions and scalar updates of CG, the fixed-point schemes
// and the refinement, and the MINRES recurrences with their vector kernels.
#pragma once

#include "kernels.hpp"

namespace lsh {

// ----------------------------------------------------------------------------
// MINRES (Paige--Saunders) on the FP64 fields: per-load rotation state and the
// two vector kernels of one step, around the operator application q = L v_k.
// ----------------------------------------------------------------------------
struct MinresState {
  double alpha, beta, c, s, delta1, eps, phi;  // recurrences (beta = beta_k, eps = eps_k)
  double delta2, epsk, gamma2, t, inv_beta;    // coefficients of this step's vector update
  double z1, z2, first, zbar, wc, ws;          // SYMMLQ: z_{k-1}, z_{k-2}, row k's right-hand side,
                                               // CG-point coefficient, rotation of this step
  int apply, pad;
};

enum : int { MR_INIT = 0, MR_ALPHA = 1, MR_ROT = 2 };
enum : int { SY_INIT = 0, SY_ROT = 1 };
enum : int { SY_NONE = 0, SY_STEP = 1, SY_TRANSFER = 2 };

// v = b / ||b||, v_prev = w_{k-1} = w_{k-2} = 0 on the loads that iterate
static __global__ __launch_bounds__(256) void k_mr_start(const long long F, double* __restrict__ v,
                                                  double* __restrict__ vp, double* __restrict__ w1,
                                                  double* __restrict__ w2, const LoadState* __restrict__ st) {
  const int l = blockIdx.y;
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= F) return;
  const long long o = (long long)l * F + i;
  const double sc = st[l].rr > 0.0 ? 1.0 / sqrt(st[l].rr) : 0.0;
  v[o] *= sc;
  vp[o] = 0.0;
  w1[o] = 0.0;
  w2[o] = 0.0;
}

// vp = q - alpha v - beta vp (the unnormalised v_{k+1}); partial ||vp||^2
static __global__ __launch_bounds__(256) void k_mr_lanczos(const long long F, const double* __restrict__ q,
                                                    const double* __restrict__ v, double* __restrict__ vp,
                                                    const LoadState* __restrict__ st,
                                                    const MinresState* __restrict__ ms, double* __restrict__ partials,
                                                    const int pstride) {
  __shared__ double red[4];
  const int l = blockIdx.y;
  if (!st[l].active) return;
  const double al = ms[l].alpha, be = ms[l].beta;
  double part = 0.0;
  const long long b0 = (long long)blockIdx.x * 256 * kEwUnroll + threadIdx.x;
#pragma unroll
  for (int u = 0; u < kEwUnroll; ++u) {
    const long long i = b0 + (long long)u * 256;
    if (i < F) {
      const long long o = (long long)l * F + i;
      const double z = q[o] - al * v[o] - be * vp[o];
      vp[o] = z;
      part += z * z;
    }
  }
  const double sum = block_sum<256>(part, red);
  if (threadIdx.x == 0) partials[(long long)l * pstride + blockIdx.x] = sum;
}

// w_k = (v_k - delta2 w_{k-1} - eps_k w_{k-2}) / gamma2 into the w_{k-2} slot,
// x += t w_k, and v_{k+1} = vp / beta_{k+1} in place
static __global__ __launch_bounds__(256) void k_mr_update(const long long F, const double* __restrict__ v,
                                                   double* __restrict__ vp, const double* __restrict__ w1,
                                                   double* __restrict__ w2, double* __restrict__ x,
                                                   const MinresState* __restrict__ ms) {
  const int l = blockIdx.y;
  const MinresState& m = ms[l];
  if (!m.apply) return;
  const double ig = 1.0 / m.gamma2;
  const long long b0 = (long long)blockIdx.x * 256 * kEwUnroll + threadIdx.x;
#pragma unroll
  for (int u = 0; u < kEwUnroll; ++u) {
    const long long i = b0 + (long long)u * 256;
    if (i < F) {
      const long long o = (long long)l * F + i;
      const double w = (v[o] - m.delta2 * w1[o] - m.epsk * w2[o]) * ig;
      w2[o] = w;
      x[o] += m.t * w;
      vp[o] *= m.inv_beta;
    }
  }
}

__device__ __forceinline__ double group_sum(const double* __restrict__ partials, int pstride, int nparts, int grp,
                                            double* red) {
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 256) s += partials[(long long)grp * pstride + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  return red[0];
}

// Scalar steps of MINRES (one workgroup per load).  MR_ROT applies the
// previous rotation to the new tridiagonal column (beta_k, alpha_k,
// beta_{k+1}), forms the next rotation, the step t_k = c_k phi_{k-1} and the
// residual norm phi_k = s_k phi_{k-1}; the load stops at |phi_k| <= tol ||b||,
// at beta_{k+1} = 0 (exact solution) or, with gamma2 = 0, on breakdown.
static __global__ __launch_bounds__(256) void k_mr_scal(const int mode, const double* __restrict__ partials,
                                                        const int pstride, const int nparts,
                                                        LoadState* __restrict__ st, MinresState* __restrict__ ms,
                                                        const HistRef hist) {
  __shared__ double red[256];
  const int l = blockIdx.x;
  const double S = mode == MR_INIT ? 0.0 : group_sum(partials, pstride, nparts, l, red);
  if (threadIdx.x != 0) return;
  LoadState& L = st[l];
  MinresState& M = ms[l];
  if (mode == MR_INIT) {
    M.alpha = M.beta = M.delta1 = M.eps = 0.0;
    M.c = -1.0;
    M.s = 0.0;
    M.phi = sqrt(L.rr);   // ||r_0|| (= ||b|| from x_0 = 0)
    M.delta2 = M.epsk = M.t = M.inv_beta = 0.0;
    M.gamma2 = 1.0;
    M.apply = 0;
    return;
  }
  if (mode == MR_ALPHA) {
    if (L.active) M.alpha = S;
    return;
  }
  M.apply = 0;
  if (!L.active) return;
  if (!isfinite(S) || !isfinite(M.alpha)) {
    L.status = kStatusNumeric;
    L.active = 0;
    return;
  }
  const double bn = sqrt(S);
  const double delta2 = M.c * M.delta1 + M.s * M.alpha;
  const double gamma1 = M.s * M.delta1 - M.c * M.alpha;
  const double eps_next = M.s * bn;
  const double delta1_next = -M.c * bn;
  const double gamma2 = hypot(gamma1, bn);
  L.iters += 1;
  if (gamma2 == 0.0) {
    L.status = kStatusBreakdown;
    L.active = 0;
    return;
  }
  const double c = gamma1 / gamma2, s = bn / gamma2;
  M.delta2 = delta2;
  M.epsk = M.eps;
  M.gamma2 = gamma2;
  M.t = c * M.phi;
  M.phi = s * M.phi;
  M.inv_beta = bn > 0.0 ? 1.0 / bn : 0.0;
  M.apply = 1;
  M.beta = bn;
  M.delta1 = delta1_next;
  M.eps = eps_next;
  M.c = c;
  M.s = s;
  L.res2 = M.phi * M.phi;
  hist_push(hist, l, L.res2 / L.bb);
  if (L.res2 <= L.tol2 || bn == 0.0) L.active = 0;
}

// ----------------------------------------------------------------------------
// SYMMLQ (Paige--Saunders) on the same fields: the Lanczos step is MINRES's
// (k_mr_scal MR_ALPHA, k_mr_lanczos); the LQ factorisation of the tridiagonal
// matrix by reflectors [c s; s -c] on columns (k, k+1) has MINRES's rotation
// recurrences (dbar in delta1), then forward substitution gives
// z_k = num_k / gamma_k and the CG-point coefficient zbar_k = num_k / gbar_k,
// num_k = [k = 1] ||b|| - delta_k z_{k-1} - eps_k z_{k-2}.  The fields are
// v_{k-1} (overwritten by v_{k+1}), v_k, wbar_k and the iterate x^L.
// ----------------------------------------------------------------------------

// v = b / ||b||, v_prev = 0, wbar_1 = v on the loads that iterate
static __global__ __launch_bounds__(256) void k_sy_start(const long long F, double* __restrict__ v,
                                                  double* __restrict__ vp, double* __restrict__ wbar,
                                                  const LoadState* __restrict__ st) {
  const int l = blockIdx.y;
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= F) return;
  const long long o = (long long)l * F + i;
  const double sc = st[l].rr > 0.0 ? 1.0 / sqrt(st[l].rr) : 0.0;
  const double vv = v[o] * sc;
  v[o] = vv;
  vp[o] = 0.0;
  wbar[o] = vv;
}

// Scalar step of SYMMLQ after the Lanczos step (one workgroup per load).  The
// CG point's residual |beta_{k+1}| |s_{k-1} z_{k-1} - c_{k-1} zbar_k| is the
// stopping quantity: at tol ||b|| the load transfers to the CG point
// (x = x^L_{k-1} + zbar_k wbar_k) and stops; on the last allowed step it
// transfers without stopping (the host reports the iteration limit); with
// gbar_k = 0 there is no CG point and the LQ step is taken; gamma_k = 0 (the
// system singular on the Krylov space) is a breakdown.
static __global__ __launch_bounds__(256) void k_sy_scal(const int mode, const double* __restrict__ partials,
                                                        const int pstride, const int nparts, const int last,
                                                        LoadState* __restrict__ st, MinresState* __restrict__ ms,
                                                        const HistRef hist) {
  __shared__ double red[256];
  const int l = blockIdx.x;
  const double S = mode == SY_INIT ? 0.0 : group_sum(partials, pstride, nparts, l, red);
  if (threadIdx.x != 0) return;
  LoadState& L = st[l];
  MinresState& M = ms[l];
  if (mode == SY_INIT) {
    M.alpha = M.beta = M.delta1 = M.eps = 0.0;
    M.c = -1.0;
    M.s = 0.0;
    M.z1 = M.z2 = M.zbar = M.wc = M.ws = M.t = M.inv_beta = 0.0;
    M.first = sqrt(L.rr);   // ||r_0|| (= ||b|| from x_0 = 0)
    M.apply = SY_NONE;
    return;
  }
  M.apply = SY_NONE;
  if (!L.active) return;
  if (!isfinite(S) || !isfinite(M.alpha)) {
    L.status = kStatusNumeric;
    L.active = 0;
    return;
  }
  const double bn = sqrt(S);
  const double delta = M.c * M.delta1 + M.s * M.alpha;
  const double gbar = M.s * M.delta1 - M.c * M.alpha;
  const double eps_next = M.s * bn;
  const double dbar_next = -M.c * bn;
  const double num = M.first - delta * M.z1 - M.eps * M.z2;
  L.iters += 1;
  // the CG point and its residual (none, an infinite residual, when gbar = 0)
  double zbar = 0.0, rc = (double)INFINITY;
  if (gbar != 0.0) {
    zbar = num / gbar;
    rc = bn * fabs(M.s * M.z1 - M.c * zbar);
  }
  hist_push(hist, l, rc * rc / L.bb);
  if (gbar != 0.0) {
    L.res2 = rc * rc;
    if (L.res2 <= L.tol2) {
      M.zbar = zbar;
      M.apply = SY_TRANSFER;
      L.active = 0;
      return;
    }
  }
  const double gamma = hypot(gbar, bn);
  if (gamma == 0.0) {
    L.status = kStatusBreakdown;
    L.active = 0;
    return;
  }
  if (last && gbar != 0.0) {
    M.zbar = zbar;
    M.apply = SY_TRANSFER;
    return;
  }
  const double c = gbar / gamma, s = bn / gamma;
  const double z = num / gamma;
  M.wc = c;
  M.ws = s;
  M.t = z;
  M.inv_beta = 1.0 / bn;   // bn > 0: bn = 0 gives a zero CG residual or gamma = 0 above
  M.apply = SY_STEP;
  M.beta = bn;
  M.delta1 = dbar_next;
  M.eps = eps_next;
  M.c = c;
  M.s = s;
  M.z2 = M.z1;
  M.z1 = z;
  M.first = 0.0;
}

// SY_STEP: v_{k+1} = vp / beta_{k+1} in place, w_k = c wbar_k + s v_{k+1},
// wbar_{k+1} = s wbar_k - c v_{k+1}, x += z_k w_k.  SY_TRANSFER: x += zbar_k wbar_k.
static __global__ __launch_bounds__(256) void k_sy_update(const long long F, double* __restrict__ vp,
                                                   double* __restrict__ wbar, double* __restrict__ x,
                                                   const MinresState* __restrict__ ms) {
  const int l = blockIdx.y;
  const MinresState& m = ms[l];
  if (m.apply == SY_NONE) return;
  const long long b0 = (long long)blockIdx.x * 256 * kEwUnroll + threadIdx.x;
  if (m.apply == SY_TRANSFER) {
#pragma unroll
    for (int u = 0; u < kEwUnroll; ++u) {
      const long long i = b0 + (long long)u * 256;
      if (i < F) {
        const long long o = (long long)l * F + i;
        x[o] += m.zbar * wbar[o];
      }
    }
    return;
  }
#pragma unroll
  for (int u = 0; u < kEwUnroll; ++u) {
    const long long i = b0 + (long long)u * 256;
    if (i < F) {
      const long long o = (long long)l * F + i;
      const double vn = vp[o] * m.inv_beta;
      const double wb = wbar[o];
      vp[o] = vn;
      wbar[o] = m.ws * wb - m.wc * vn;
      x[o] += m.t * (m.wc * wb + m.ws * vn);
    }
  }
}

// Deterministic final reduction of the partials of group blockIdx.x, then the
// scalar update of the solver (one workgroup per group).
// aux (SC_ALPHA): -1 for the unfused CG step (its x pass applies the pending
// step every iteration); 0 or 1 for the fused step, the buffer this iteration's
// direction went to (its x pass applies pending steps in pairs).
static __global__ __launch_bounds__(256) void k_scal(const int mode, const double* __restrict__ partials, const int pstride,
                                              const int nparts, LoadState* __restrict__ st,
                                              double* __restrict__ sums, const double tol, const int aux,
                                              const HistRef hist) {
  __shared__ double red[256];
  const int grp = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 256) s += partials[(long long)grp * pstride + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double S = red[0];
  double S2 = S;
  if (mode == SC_INITG) {
    // ||r_0||^2 of a start from initial guesses, group ngroups + grp
    __syncthreads();
    double s2 = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 256) s2 += partials[(long long)(gridDim.x + grp) * pstride + i];
    red[threadIdx.x] = s2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    S2 = red[0];
  }
  if (threadIdx.x != 0) return;
  if (mode == SC_SUM) {
    sums[grp] = S;
    return;
  }
  LoadState& L = st[grp];
  if (mode == SC_INIT || mode == SC_INITG) {
    // SC_INITG: S = ||b||^2 (tolerance), S2 = ||b - L x_0||^2 (start)
    L.bb = S;
    L.rr = S2;
    L.res2 = S2;
    L.tol2 = tol * tol * S;
    L.alpha = 0.0;
    L.beta = 0.0;
    L.pq = 0.0;
    L.iters = 0;
    L.first = 1;
    L.pending = 0;
    const bool fin = isfinite(S) && isfinite(S2);
    L.status = fin ? kStatusOk : kStatusNumeric;
    // a guess that already meets the tolerance needs no iteration
    L.active = (S > 0.0 && fin && (mode == SC_INIT || S2 > L.tol2)) ? 1 : 0;
    return;
  }
  if (!L.active) return;
  if (mode == SC_ALPHA) {
    L.pq = S;
    // p.Lp may be negative when A0 lies between the phases (indefinite
    // system): CG proceeds; it breaks down when p.Lp is at rounding level,
    // |p.Lp| <= g r.r with g = eps ||L|| from the host (tol argument): the
    // Rayleigh quotient of p (p.p >= r.r) is then below eps times the bound
    // of the operator, beyond what the field precision resolves.
    // pending steps this iteration's x pass applied: the previous one
    // (unfused), or the pair when two were pending (fused)
    if (aux < 0 || L.pending == 2) L.pending = 0;
    if (!isfinite(S)) {
      L.status = kStatusNumeric;
      L.active = 0;
    } else if (fabs(S) <= tol * L.rr) {
      L.status = kStatusBreakdown;
      L.active = 0;
    } else {
      if (L.pending == 1) L.alpha2 = L.alpha;
      L.alpha = L.rr / S;
      L.first = 0;
      L.pending += 1;
      if (aux >= 0) L.pbuf = aux;
    }
  } else if (mode == SC_BETA) {
    L.iters += 1;
    if (!isfinite(S)) {
      L.status = kStatusNumeric;
      L.active = 0;
      return;
    }
    L.beta = S / L.rr;
    L.rr = S;
    L.res2 = S;
    hist_push(hist, grp, S / L.bb);
    if (S <= L.tol2) L.active = 0;
  } else if (mode == SC_BASIC || mode == SC_OUTER) {
    L.iters += 1;
    L.res2 = S;
    hist_push(hist, grp, S / L.bb);
    if (!isfinite(S)) {
      L.status = kStatusNumeric;
      L.active = 0;
    } else if (S <= L.tol2) {
      L.active = 0;
    }
  }
}

// Deterministic smooth test pattern (kernel-shape timing inputs).
template <typename T>
__global__ __launch_bounds__(256) void k_fill(const long long n, T* __restrict__ x) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) x[i] = static_cast<T>(1.0 + 1e-3 * (double)(i % 977));
}

}  // namespace lsh
