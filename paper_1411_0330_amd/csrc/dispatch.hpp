// Launchers of the transform passes, dispatched on the axis lengths (powers
// of two, and 3 or 5 times a power of two) to the compile-time kernel instances.  Each launcher returns the
// number of workgroups along x of the grid it queued (the number of partial
// sums a reducing kernel wrote per load), or -1 for an unsupported size.
#pragma once

#include "kernels.hpp"

namespace lsh {

// ---------------------------------------------------------------------------
// tile configuration (compile time)
// ---------------------------------------------------------------------------
template <typename T> constexpr int min_tx() { return sizeof(T) == 4 ? 16 : 8; }  // 128-byte rows

constexpr int cmin(int a, int b) { return a < b ? a : b; }
constexpr int cmax(int a, int b) { return a > b ? a : b; }

// points per thread.  For an axis length F 2^m with F = 3 or 5 the points per
// thread are F 2^a (the first FFT stage then has radix F 2^a): 2^a = 4 where
// the exchange buffer of the row passes stays within 48 KiB, else 2.
template <typename T> constexpr int p_odd(int n, int q) {
  const int f = odd_part(n);
  // at most 12 points per thread (radix 5: 10); 20 needs more registers than
  // the pencil buffers leave and drops occupancy to one or two waves
  while (q > 2 && (256 * f * q * 2 * (int)sizeof(T) > 48 * 1024 || f * q > 12)) q /= 2;
  return f * cmin(q, pow2_part(n));
}
// row passes over a power-of-two half row: the most points per thread (at most
// 8, at least 2) that still leave 128 contiguous bytes per access instruction
// (16 FP32 or 8 FP64 threads per row); measured at mx = 64 (128^3 scalar, FP32
// C2R): 8 points per thread, 5.1 TB/s; 4 points, 6.2 TB/s
template <typename T> constexpr int p_row(int mx) {
  return cmin(mx, cmax(2, cmin(8, mx / (128 / (2 * (int)sizeof(T))))));
}
template <typename T> constexpr int p_xfwd(int mx) { return odd_part(mx) > 1 ? p_odd<T>(mx, 4) : p_row<T>(mx); }
template <typename T, int C> constexpr int p_xinv(int mx) {
  // six components: fewer points per thread keep the register file for occupancy
  if (odd_part(mx) > 1) return p_odd<T>(mx, C == 6 ? 2 : 4);
  return C == 6 ? cmin(sizeof(T) == 8 ? 2 : 4, mx) : p_row<T>(mx);
}
template <typename T> constexpr int p_y(int n) {
  return odd_part(n) > 1 ? p_odd<T>(n, 4) : cmin(sizeof(T) == 4 ? 16 : 8, n);
}
template <typename T, int C> constexpr int p_z(int n) {
  if (odd_part(n) > 1) return p_odd<T>(n, C == 6 ? 2 : 4);
  return cmin(C == 6 ? (sizeof(T) == 4 ? 8 : 4) : (sizeof(T) == 4 ? 16 : 8), n);
}

// pencils per workgroup for strided passes: >= 128-byte rows, about 256 threads,
// at most 64 KiB of exchange space and 1024 threads
template <typename T> constexpr int tx_strided(int n, int p) {
  const int threads_per_pencil = n / p;
  int tx = cmax(min_tx<T>(), 256 / threads_per_pencil);
  tx = cmin(tx, 64);
  while (tx > 1 && (long)tx * n * 2 * (int)sizeof(T) > 65536) tx /= 2;
  while (tx > 1 && tx * threads_per_pencil > 1024) tx /= 2;
  return tx;
}

template <typename T>
struct XfwdArgs {
  Geo g;
  int mode;
  const T* src;
  T* pdir;
  T* xacc;
  const float* dsrc;
  cpx<T>* smain;
  cpx<T>* snyq;
  const cpx<T>* twx;
  const LoadState* st;
  IrxFold fold;   // XF_IRX: the inner solve's pending steps, x starting at zero
};

// Kernel-shape variants of each pass (0 = the default shape).  For the axis
// lengths 128 and 256 every pass is compiled in kVariants shapes:
//   strided passes (y, zg): 1 = half the pencils per workgroup,
//                           2 = half the points per thread (at most 256 threads),
//                           3 = twice the pencils per workgroup;
//   row passes (xfwd, xinv): 1 = half the points per thread, 2 = twice,
//                            3 = a quarter.
// Shapes that break a limit (threads, LDS, points) fall back to the default.
constexpr int kVariants = 4;
// The z pass has one more shape: 4 = all loads of a tile in one workgroup with
// the operator matrices formed once (FP32 fields, operators other than the
// finite-difference one, 128- and 256-point z axes; elsewhere it falls back
// to shape 0).  And 5 = 8-pencil tiles on the component-paired spectrum
// layout, whose y passes convert the layout out of place (FP32 six-component
// fields with the stored operator, 128- and 256-point y and z axes; elsewhere
// shape 0).
constexpr int kVariantsZ = 6;
constexpr int kZPaired = 5;
enum : int { PASS_XFWD = 0, PASS_Y = 1, PASS_ZG = 2, PASS_XINV = 3, NPASS = 4 };
constexpr int pass_variants(int pass) { return pass == PASS_ZG ? kVariantsZ : kVariants; }

// multi-load z pass shape: points per thread (registers hold the operator
// matrices of every point) and at most 512 threads
template <typename T, int C> constexpr int p_zm(int n) {
  if (odd_part(n) > 1) return p_odd<T>(n, 2);
  return cmin(C == 6 ? 4 : 8, n);
}
template <typename T> constexpr int tx_zm(int n, int p) {
  int tx = tx_strided<T>(n, p);
  while (tx > 1 && tx * (n / p) > 512) tx /= 2;
  return tx;
}

template <typename T> int launch_xfwd(hipStream_t s, const XfwdArgs<T>& a, int nload, int variant = 0);
template <typename T> int launch_y(hipStream_t s, const Geo& g, int dir, cpx<T>* sm, cpx<T>* sn, const cpx<T>* tw,
                                   const LoadState* st, int nload, int variant = 0);
// y passes into (dir < 0) and out of (dir > 0) the component-paired layout
// held in sp; -1 where the shape has no such instance
template <typename T> int launch_y_paired(hipStream_t s, const Geo& g, int dir, cpx<T>* sm, cpx<T>* sp, cpx<T>* sn,
                                          const cpx<T>* tw, const LoadState* st, int nload, int variant = 0);
// both y passes in place on the paired layout (the fused CG step's); -1 where none exists
template <typename T> int launch_y_paired_inplace(hipStream_t s, const Geo& g, int dir, cpx<T>* sm, cpx<T>* sn,
                                                  const cpx<T>* tw, const LoadState* st, int nload, int variant = 0);
// the Green pass on the paired layout (stored operator); -1 where none exists
template <typename T> int launch_zg_paired(hipStream_t s, const Geo& g, const GreenParams& gp, const GreenTabs<T>& tb,
                                           cpx<T>* sp, cpx<T>* sn, const cpx<T>* tw, const LoadState* st, int nload,
                                           double* qpart, int pstride);
template <typename T> int launch_zg(hipStream_t s, const Geo& g, const GreenParams& gp, const GreenTabs<T>& tb,
                                    int zmode, cpx<T>* sm, cpx<T>* sn, const cpx<T>* tw, const LoadState* st,
                                    int nload, int variant = 0, double* qpart = nullptr, int pstride = 0);
// the Green pass with the stored operator tb.st (3D, three or six components;
// -1 elsewhere); launch_zg forwards to it when tb.st is bound
template <typename T> int launch_zg_stored(hipStream_t s, const Geo& g, const GreenParams& gp, const GreenTabs<T>& tb,
                                           cpx<T>* sm, cpx<T>* sn, const cpx<T>* tw, const LoadState* st, int nload,
                                           int variant, double* qpart, int pstride);
// x forward of conjugate gradients over all components of a voxel row (returns
// the workgroups per load, i.e. the partials written per load)
template <typename T> int launch_xfwdc(hipStream_t s, const XfwdcArgs<T>& a, int nload);
// persistent CG for small grids (returns -1 for grids without an instance)
template <typename T> struct TinyArgs;
template <typename T> int launch_tiny_cg(hipStream_t s, const TinyArgs<T>& a, int nload);
// Grids where one workgroup per load beats the multi-kernel loop on MI355X
// (measured): at most 12288 unknowns per load -- squares 8..64 (2D), cubes of
// 8 (scalar and elastic) and 16 (scalar).  Larger grids keep every CU busy
// with the multi-kernel loop instead.
inline bool tiny_grid(const Geo& g) {
  if (g.nz == 1) return g.c == 2 && g.nx == g.ny && (g.nx == 8 || g.nx == 16 || g.nx == 32 || g.nx == 64);
  if (g.nx != g.ny || g.ny != g.nz) return false;
  return (g.nx == 8 && (g.c == 3 || g.c == 6)) || (g.nx == 16 && g.c == 3);
}
template <typename T> int launch_xinv(hipStream_t s, const XinvArgs<T>& a, int nload, int variant = 0);
// the C2R pass of C components (launch_xinv dispatches on the component count)
template <typename T, int C> int launch_xinv_c(hipStream_t s, const XinvArgs<T>& a, int nload, int variant);

// strided-pass shape of a variant: (pencils per workgroup, points per thread)
template <typename T> constexpr int sv_tx(int n, int p0, int v) {
  const int tx0 = tx_strided<T>(n, p0);
  if (v == 2) {
    // half the points per thread, at most 256 threads per workgroup
    const int tpp = n / (p0 / 2 >= 2 ? p0 / 2 : p0);
    const int tx = 256 / tpp;
    return tx < 1 ? 1 : (tx < tx0 ? tx : tx0);
  }
  return v == 1 ? (tx0 / 2 >= 2 ? tx0 / 2 : tx0) : (v == 3 ? 2 * tx0 : tx0);
}
constexpr int sv_p(int p0, int v) { return v == 2 ? (p0 / 2 >= 2 ? p0 / 2 : p0) : p0; }
// a shape is compiled when it fits 1024 threads and the 160 KiB of LDS a gfx950
// workgroup may hold (exchange buffer, twiddles and the reduction slots)
constexpr long kLdsPerWorkgroup = 160 * 1024;
template <typename T> constexpr bool sv_ok(int n, int tx, int p) {
  return p >= 1 && p <= n && tx >= 1 && tx * (n / p) <= 1024 &&
         (long)(tx + 1) * n * 2 * (int)sizeof(T) + 128 <= kLdsPerWorkgroup;
}
// row-pass points per thread of a variant
constexpr int rv_p(int mx, int p0, int v) {
  const int p = v == 1 ? p0 / 2 : (v == 2 ? p0 * 2 : (v == 3 ? p0 / 4 : p0));
  return (p >= 2 && p <= mx && p <= 16 && mx / p <= 256) ? p : p0;
}

// number of workgroups per load of the reducing passes (partials sizing)
// workgroups per load of the z pass (partials of its spectral form), any shape
template <typename T> inline long long zg_blocks_max(const Geo& g) {
  // the narrowest tile of any shape: 1 pencil along x
  return (long long)g.ny * g.mx + g.ny;
}
inline long long xinv_blocks(const Geo& g, int p) {
  const int tr = g.mx / p;
  const int rpw = 256 / tr;
  return ((long long)g.nz * g.ny + rpw - 1) / rpw;
}

}  // namespace lsh
