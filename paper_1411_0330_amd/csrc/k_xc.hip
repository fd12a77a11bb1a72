// x forward pass of conjugate gradients over all components of a voxel row
// (with the local quadratic form); instances for one element type (LSH_XC_TYPE).
#include "dispatch.hpp"

namespace lsh {

template <typename T, int MX, int C>
static int xfwdc_inst(hipStream_t s, const XfwdcArgs<T>& a, int nload) {
  constexpr int P = p_xinv<T, C>(MX);
  const int nb = (int)xinv_blocks(a.g, P);
  hipLaunchKernelGGL((k_xfwdc<T, MX, P, C>), dim3(nb, nload), dim3(256), 0, s, a);
  return nb;
}

template <typename T, int MX>
static int xfwdc_c(hipStream_t s, const XfwdcArgs<T>& a, int nload) {
  switch (a.g.c) {
    case 2: return xfwdc_inst<T, MX, 2>(s, a, nload);
    case 3: return xfwdc_inst<T, MX, 3>(s, a, nload);
    case 6: return xfwdc_inst<T, MX, 6>(s, a, nload);
    default: return -1;
  }
}

template <typename T>
int launch_xfwdc(hipStream_t s, const XfwdcArgs<T>& a, int nload) {
  switch (a.g.mx) {
    case 2: return xfwdc_c<T, 2>(s, a, nload);
    case 4: return xfwdc_c<T, 4>(s, a, nload);
    case 8: return xfwdc_c<T, 8>(s, a, nload);
    case 16: return xfwdc_c<T, 16>(s, a, nload);
    case 32: return xfwdc_c<T, 32>(s, a, nload);
    case 64: return xfwdc_c<T, 64>(s, a, nload);
    case 128: return xfwdc_c<T, 128>(s, a, nload);
    case 256: return xfwdc_c<T, 256>(s, a, nload);
    case 512: return xfwdc_c<T, 512>(s, a, nload);
    case 24: return xfwdc_c<T, 24>(s, a, nload);
    case 48: return xfwdc_c<T, 48>(s, a, nload);
    case 96: return xfwdc_c<T, 96>(s, a, nload);
    case 40: return xfwdc_c<T, 40>(s, a, nload);
    case 80: return xfwdc_c<T, 80>(s, a, nload);
    default: return -1;
  }
}

#ifndef LSH_XC_TYPE
#error "define LSH_XC_TYPE"
#endif
template int launch_xfwdc<LSH_XC_TYPE>(hipStream_t, const XfwdcArgs<LSH_XC_TYPE>&, int);

}  // namespace lsh
