// x passes (R2C / C2R with the local term), FP32 and FP64 instances.  Built
// per element type (LSH_X_TYPE) in parts that compile in parallel:
// LSH_X_PART = 0 the R2C pass and the C2R dispatch, 2, 3 or 6 the C2R pass of
// that many components.
#include "dispatch.hpp"

#ifndef LSH_X_PART
#error "define LSH_X_PART"
#endif

namespace lsh {

#if LSH_X_PART == 0

template <typename T, int MX, int P>
static int xfwd_inst(hipStream_t s, const XfwdArgs<T>& a, int nload) {
  constexpr int TR = MX / P;
  constexpr int RPW = 256 / TR;
  const long long rows = (long long)a.g.c * a.g.nz * a.g.ny;
  const int nb = (int)((rows + RPW - 1) / RPW);
  hipLaunchKernelGGL((k_xfwd<T, MX, P>), dim3(nb, nload), dim3(256), 0, s, a.g, a.mode, a.src, a.pdir, a.xacc,
                     a.dsrc, a.smain, a.snyq, a.twx, a.st, a.fold);
  return nb;
}

template <typename T, int MX>
static int xfwd_one(hipStream_t s, const XfwdArgs<T>& a, int nload, int v = 0) {
  constexpr int P0 = p_xfwd<T>(MX);
  if constexpr (MX == 64 || MX == 128) {
    switch (v) {
      case 1: return xfwd_inst<T, MX, rv_p(MX, P0, 1)>(s, a, nload);
      case 2: return xfwd_inst<T, MX, rv_p(MX, P0, 2)>(s, a, nload);
      case 3: return xfwd_inst<T, MX, rv_p(MX, P0, 3)>(s, a, nload);
      default: break;
    }
  }
  return xfwd_inst<T, MX, P0>(s, a, nload);
}

template <typename T>
int launch_xfwd(hipStream_t s, const XfwdArgs<T>& a, int nload, int v) {
  switch (a.g.mx) {
    case 2: return xfwd_one<T, 2>(s, a, nload);
    case 4: return xfwd_one<T, 4>(s, a, nload);
    case 8: return xfwd_one<T, 8>(s, a, nload);
    case 16: return xfwd_one<T, 16>(s, a, nload);
    case 32: return xfwd_one<T, 32>(s, a, nload);
    case 64: return xfwd_one<T, 64>(s, a, nload, v);
    case 128: return xfwd_one<T, 128>(s, a, nload, v);
    case 256: return xfwd_one<T, 256>(s, a, nload);
    case 512: return xfwd_one<T, 512>(s, a, nload);
    case 24: return xfwd_one<T, 24>(s, a, nload);
    case 48: return xfwd_one<T, 48>(s, a, nload);
    case 96: return xfwd_one<T, 96>(s, a, nload);
    case 40: return xfwd_one<T, 40>(s, a, nload);
    case 80: return xfwd_one<T, 80>(s, a, nload);
    default: return -1;
  }
}

#endif  // LSH_X_PART == 0

#if LSH_X_PART != 0
template <typename T, int MX, int C, int P>
static int xinv_inst(hipStream_t s, const XinvArgs<T>& a, int nload) {
  const int nb = (int)xinv_blocks(a.g, P);
  hipLaunchKernelGGL((k_xinv<T, MX, P, C>), dim3(nb, nload), dim3(256), 0, s, a);
  return nb;
}

template <typename T, int MX, int C>
static int xinv_one(hipStream_t s, const XinvArgs<T>& a, int nload, int v) {
  constexpr int P0 = p_xinv<T, C>(MX);
  if constexpr (MX == 64 || MX == 128) {
    switch (v) {
      case 1: return xinv_inst<T, MX, C, rv_p(MX, P0, 1)>(s, a, nload);
      case 2: return xinv_inst<T, MX, C, rv_p(MX, P0, 2)>(s, a, nload);
      case 3: return xinv_inst<T, MX, C, rv_p(MX, P0, 3)>(s, a, nload);
      default: break;
    }
  }
  return xinv_inst<T, MX, C, P0>(s, a, nload);
}

template <typename T, int C>
int launch_xinv_c(hipStream_t s, const XinvArgs<T>& a, int nload, int v) {
  switch (a.g.mx) {
    case 2: return xinv_one<T, 2, C>(s, a, nload, v);
    case 4: return xinv_one<T, 4, C>(s, a, nload, v);
    case 8: return xinv_one<T, 8, C>(s, a, nload, v);
    case 16: return xinv_one<T, 16, C>(s, a, nload, v);
    case 32: return xinv_one<T, 32, C>(s, a, nload, v);
    case 64: return xinv_one<T, 64, C>(s, a, nload, v);
    case 128: return xinv_one<T, 128, C>(s, a, nload, v);
    case 256: return xinv_one<T, 256, C>(s, a, nload, v);
    case 512: return xinv_one<T, 512, C>(s, a, nload, v);
    case 24: return xinv_one<T, 24, C>(s, a, nload, v);
    case 48: return xinv_one<T, 48, C>(s, a, nload, v);
    case 96: return xinv_one<T, 96, C>(s, a, nload, v);
    case 40: return xinv_one<T, 40, C>(s, a, nload, v);
    case 80: return xinv_one<T, 80, C>(s, a, nload, v);
    default: return -1;
  }
}
#endif  // LSH_X_PART != 0

#ifndef LSH_X_TYPE
#error "define LSH_X_TYPE"
#endif
#if LSH_X_PART == 0
template <typename T>
int launch_xinv(hipStream_t s, const XinvArgs<T>& a, int nload, int v) {
  switch (a.g.c) {
    case 2: return launch_xinv_c<T, 2>(s, a, nload, v);
    case 3: return launch_xinv_c<T, 3>(s, a, nload, v);
    case 6: return launch_xinv_c<T, 6>(s, a, nload, v);
    default: return -1;
  }
}
template int launch_xfwd<LSH_X_TYPE>(hipStream_t, const XfwdArgs<LSH_X_TYPE>&, int, int);
template int launch_xinv<LSH_X_TYPE>(hipStream_t, const XinvArgs<LSH_X_TYPE>&, int, int);
#else
template int launch_xinv_c<LSH_X_TYPE, LSH_X_PART>(hipStream_t, const XinvArgs<LSH_X_TYPE>&, int, int);
#endif

}  // namespace lsh
