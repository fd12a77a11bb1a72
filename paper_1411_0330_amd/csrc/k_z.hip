// z pass fused with the Green operator; instances for one element type
// (LSH_Z_TYPE) so that FP32 and FP64 compile in parallel.  Built twice per
// type: without LSH_Z_STORED the operator is formed on the fly (launch_zg);
// with it, from the stored table (launch_zg_stored, three- and
// six-component 3D fields), in a unit of its own so both compile in parallel.
#include "dispatch.hpp"

namespace lsh {

#ifdef LSH_Z_STORED
constexpr bool kGS = true;
#else
constexpr bool kGS = false;
#endif

template <typename T, int NZ, int C, int TX, int P, bool PR = false>
static int z_inst(hipStream_t s, const Geo& g, const GreenParams& gp, const GreenTabs<T>& tb, int zmode, cpx<T>* sm,
                  cpx<T>* sn, const cpx<T>* tw, const LoadState* st, int nload, double* qp, int ps) {
  constexpr int NT = TX * (NZ / P);
  const int xtiles = (g.mx + TX - 1) / TX;
  const int main_tiles = g.ny * xtiles;
  const int nyq_tiles = (g.ny + TX - 1) / TX;
  // stored operator: one workgroup per (tile, load), the loads of a tile adjacent on one XCD
  const dim3 grid = kGS ? dim3((main_tiles + nyq_tiles) * nload, 1) : dim3(main_tiles + nyq_tiles, nload);
  hipLaunchKernelGGL((k_zg<T, NZ, P, TX, C, kGS, PR>), grid, dim3(NT), 0, s, g, gp, tb, zmode, sm, sn, tw, st,
                     main_tiles, qp, ps, nload);
  return main_tiles + nyq_tiles;
}

template <typename T, int NZ, int C>
static int zm_inst(hipStream_t s, const Geo& g, const GreenParams& gp, const GreenTabs<T>& tb, cpx<T>* sm,
                   cpx<T>* sn, const cpx<T>* tw, const LoadState* st, int nload, double* qp, int ps) {
  constexpr int P = p_zm<T, C>(NZ);
  constexpr int TX = tx_zm<T>(NZ, P);
  constexpr int NT = TX * (NZ / P);
  const int xtiles = (g.mx + TX - 1) / TX;
  const int main_tiles = g.ny * xtiles;
  const int nyq_tiles = (g.ny + TX - 1) / TX;
  hipLaunchKernelGGL((k_zgm<T, NZ, P, TX, C>), dim3(main_tiles + nyq_tiles, 1), dim3(NT), 0, s, g, gp, tb, sm, sn,
                     tw, st, main_tiles, nload, qp, ps);
  return main_tiles + nyq_tiles;
}

template <typename T, int NZ, int C, int V>
static int z_var(hipStream_t s, const Geo& g, const GreenParams& gp, const GreenTabs<T>& tb, int zmode, cpx<T>* sm,
                 cpx<T>* sn, const cpx<T>* tw, const LoadState* st, int nload, double* qp, int ps) {
  constexpr int P0 = (NZ == 1) ? 1 : p_z<T, C>(NZ);
  constexpr int TX0 = (NZ == 1) ? 64 : tx_strided<T>(NZ, P0);
  constexpr int TXV = sv_tx<T>(NZ, P0, V), PV = sv_p(P0, V);
  if constexpr (V != 0 && NZ > 1 && sv_ok<T>(NZ, TXV, PV))
    return z_inst<T, NZ, C, TXV, PV>(s, g, gp, tb, zmode, sm, sn, tw, st, nload, qp, ps);
  else
    return z_inst<T, NZ, C, TX0, P0>(s, g, gp, tb, zmode, sm, sn, tw, st, nload, qp, ps);
}

template <typename T, int NZ, int C>
static int z_one(hipStream_t s, const Geo& g, const GreenParams& gp, const GreenTabs<T>& tb, int zmode, cpx<T>* sm,
                 cpx<T>* sn, const cpx<T>* tw, const LoadState* st, int nload, double* qp, int ps, int variant = 0) {
  if constexpr (!kGS && sizeof(T) == 4 && (NZ == 128 || NZ == 256) && C != 2) {
    if (variant == 4 && zmode == Z_GAMMA && gp.variant != kGreenFD)
      return zm_inst<T, NZ, C>(s, g, gp, tb, sm, sn, tw, st, nload, qp, ps);
  }
  if constexpr (NZ == 128 || NZ == 256) {
    switch (variant) {
      case 1: return z_var<T, NZ, C, 1>(s, g, gp, tb, zmode, sm, sn, tw, st, nload, qp, ps);
      case 2: return z_var<T, NZ, C, 2>(s, g, gp, tb, zmode, sm, sn, tw, st, nload, qp, ps);
      case 3: return z_var<T, NZ, C, 3>(s, g, gp, tb, zmode, sm, sn, tw, st, nload, qp, ps);
      default: break;
    }
  }
  return z_var<T, NZ, C, 0>(s, g, gp, tb, zmode, sm, sn, tw, st, nload, qp, ps);
}

template <typename T, int C>
static int z_c(hipStream_t s, const Geo& g, const GreenParams& gp, const GreenTabs<T>& tb, int zmode, cpx<T>* sm,
               cpx<T>* sn, const cpx<T>* tw, const LoadState* st, int nload, int v, double* qp, int ps) {
  switch (g.nz) {
    case 2: return z_one<T, 2, C>(s, g, gp, tb, zmode, sm, sn, tw, st, nload, qp, ps);
    case 4: return z_one<T, 4, C>(s, g, gp, tb, zmode, sm, sn, tw, st, nload, qp, ps);
    case 8: return z_one<T, 8, C>(s, g, gp, tb, zmode, sm, sn, tw, st, nload, qp, ps);
    case 16: return z_one<T, 16, C>(s, g, gp, tb, zmode, sm, sn, tw, st, nload, qp, ps);
    case 32: return z_one<T, 32, C>(s, g, gp, tb, zmode, sm, sn, tw, st, nload, qp, ps);
    case 64: return z_one<T, 64, C>(s, g, gp, tb, zmode, sm, sn, tw, st, nload, qp, ps);
    case 128: return z_one<T, 128, C>(s, g, gp, tb, zmode, sm, sn, tw, st, nload, qp, ps, v);
    case 256: return z_one<T, 256, C>(s, g, gp, tb, zmode, sm, sn, tw, st, nload, qp, ps, v);
    case 512: return z_one<T, 512, C>(s, g, gp, tb, zmode, sm, sn, tw, st, nload, qp, ps);
    case 1024: return z_one<T, 1024, C>(s, g, gp, tb, zmode, sm, sn, tw, st, nload, qp, ps);
    case 48: return z_one<T, 48, C>(s, g, gp, tb, zmode, sm, sn, tw, st, nload, qp, ps);
    case 96: return z_one<T, 96, C>(s, g, gp, tb, zmode, sm, sn, tw, st, nload, qp, ps);
    case 192: return z_one<T, 192, C>(s, g, gp, tb, zmode, sm, sn, tw, st, nload, qp, ps);
    case 80: return z_one<T, 80, C>(s, g, gp, tb, zmode, sm, sn, tw, st, nload, qp, ps);
    case 160: return z_one<T, 160, C>(s, g, gp, tb, zmode, sm, sn, tw, st, nload, qp, ps);
    default: return -1;
  }
}

#ifdef LSH_Z_STORED
template <typename T>
int launch_zg_stored(hipStream_t s, const Geo& g, const GreenParams& gp, const GreenTabs<T>& tb, cpx<T>* sm,
                     cpx<T>* sn, const cpx<T>* tw, const LoadState* st, int nload, int v, double* qp, int ps) {
  if (g.nz == 1 || tb.st == nullptr) return -1;
  if (g.c == 3) return z_c<T, 3>(s, g, gp, tb, Z_GAMMA, sm, sn, tw, st, nload, v, qp, ps);
  if (g.c == 6) return z_c<T, 6>(s, g, gp, tb, Z_GAMMA, sm, sn, tw, st, nload, v, qp, ps);
  return -1;
}

// 8-pencil tiles of the component-paired layout: two workgroups per compute
// unit, every access a whole 128-byte line
template <typename T>
int launch_zg_paired(hipStream_t s, const Geo& g, const GreenParams& gp, const GreenTabs<T>& tb, cpx<T>* sp,
                     cpx<T>* sn, const cpx<T>* tw, const LoadState* st, int nload, double* qp, int ps) {
  if constexpr (sizeof(T) == 4) {
    if (g.c != 6 || tb.st == nullptr) return -1;
    if (g.nz == 128)
      return z_inst<T, 128, 6, 8, p_z<T, 6>(128), true>(s, g, gp, tb, Z_GAMMA, sp, sn, tw, st, nload, qp, ps);
    if (g.nz == 256)
      return z_inst<T, 256, 6, 8, p_z<T, 6>(256), true>(s, g, gp, tb, Z_GAMMA, sp, sn, tw, st, nload, qp, ps);
  }
  return -1;
}
#else
template <typename T>
int launch_zg(hipStream_t s, const Geo& g, const GreenParams& gp, const GreenTabs<T>& tb, int zmode, cpx<T>* sm,
              cpx<T>* sn, const cpx<T>* tw, const LoadState* st, int nload, int v, double* qp, int ps) {
  if (g.c == 2) {
    if (g.nz != 1) return -1;
    return z_one<T, 1, 2>(s, g, gp, tb, zmode, sm, sn, tw, st, nload, qp, ps);
  }
  // the stored operator (where bound) serves the Green pass of every shape
  // except the multi-load one (4), which forms its matrices itself
  if (zmode == Z_GAMMA && tb.st != nullptr && g.nz > 1 && v != 4)
    return launch_zg_stored<T>(s, g, gp, tb, sm, sn, tw, st, nload, v, qp, ps);
  if (g.c == 3) return z_c<T, 3>(s, g, gp, tb, zmode, sm, sn, tw, st, nload, v, qp, ps);
  if (g.c == 6) return z_c<T, 6>(s, g, gp, tb, zmode, sm, sn, tw, st, nload, v, qp, ps);
  return -1;
}
#endif

#ifndef LSH_Z_TYPE
#error "define LSH_Z_TYPE"
#endif
#ifdef LSH_Z_STORED
template int launch_zg_stored<LSH_Z_TYPE>(hipStream_t, const Geo&, const GreenParams&, const GreenTabs<LSH_Z_TYPE>&,
                                          cpx<LSH_Z_TYPE>*, cpx<LSH_Z_TYPE>*, const cpx<LSH_Z_TYPE>*,
                                          const LoadState*, int, int, double*, int);
template int launch_zg_paired<LSH_Z_TYPE>(hipStream_t, const Geo&, const GreenParams&, const GreenTabs<LSH_Z_TYPE>&,
                                          cpx<LSH_Z_TYPE>*, cpx<LSH_Z_TYPE>*, const cpx<LSH_Z_TYPE>*,
                                          const LoadState*, int, double*, int);
#else
template int launch_zg<LSH_Z_TYPE>(hipStream_t, const Geo&, const GreenParams&, const GreenTabs<LSH_Z_TYPE>&, int,
                                   cpx<LSH_Z_TYPE>*, cpx<LSH_Z_TYPE>*, const cpx<LSH_Z_TYPE>*, const LoadState*,
                                   int, int, double*, int);
#endif

}  // namespace lsh
