// y passes (forward and inverse); instances for one element type (LSH_Y_TYPE).
#include "dispatch.hpp"

namespace lsh {

template <typename T, int NY, int DIR, int TX, int P>
static int y_inst(hipStream_t s, const Geo& g, cpx<T>* sm, cpx<T>* sn, const cpx<T>* tw, const LoadState* st,
                  int nload) {
  constexpr int NT = TX * (NY / P);
  const int xtiles = (g.mx + TX - 1) / TX;
  const int main_tiles = g.c * g.nz * xtiles;
  const int nyq_tiles = (g.c * g.nz + TX - 1) / TX;
  hipLaunchKernelGGL((k_y<T, NY, P, TX, DIR>), dim3(main_tiles + nyq_tiles, nload), dim3(NT), 0, s, g, sm, sn, tw,
                     st, main_tiles);
  return main_tiles + nyq_tiles;
}

template <typename T, int NY, int DIR, int V>
static int y_var(hipStream_t s, const Geo& g, cpx<T>* sm, cpx<T>* sn, const cpx<T>* tw, const LoadState* st,
                 int nload) {
  constexpr int P0 = p_y<T>(NY);
  constexpr int TX0 = tx_strided<T>(NY, P0);
  constexpr int TXV = sv_tx<T>(NY, P0, V), PV = sv_p(P0, V);
  if constexpr (V != 0 && sv_ok<T>(NY, TXV, PV))
    return y_inst<T, NY, DIR, TXV, PV>(s, g, sm, sn, tw, st, nload);
  else
    return y_inst<T, NY, DIR, TX0, P0>(s, g, sm, sn, tw, st, nload);
}

template <typename T, int NY, int DIR>
static int y_one(hipStream_t s, const Geo& g, cpx<T>* sm, cpx<T>* sn, const cpx<T>* tw, const LoadState* st,
                 int nload, int v = 0) {
  if constexpr (NY == 128 || NY == 256) {
    switch (v) {
      case 1: return y_var<T, NY, DIR, 1>(s, g, sm, sn, tw, st, nload);
      case 2: return y_var<T, NY, DIR, 2>(s, g, sm, sn, tw, st, nload);
      case 3: return y_var<T, NY, DIR, 3>(s, g, sm, sn, tw, st, nload);
      default: break;
    }
  }
  return y_var<T, NY, DIR, 0>(s, g, sm, sn, tw, st, nload);
}

template <typename T, int DIR>
static int y_dir(hipStream_t s, const Geo& g, cpx<T>* sm, cpx<T>* sn, const cpx<T>* tw, const LoadState* st,
                 int nload, int v) {
  switch (g.ny) {
    case 2: return y_one<T, 2, DIR>(s, g, sm, sn, tw, st, nload);
    case 4: return y_one<T, 4, DIR>(s, g, sm, sn, tw, st, nload);
    case 8: return y_one<T, 8, DIR>(s, g, sm, sn, tw, st, nload);
    case 16: return y_one<T, 16, DIR>(s, g, sm, sn, tw, st, nload);
    case 32: return y_one<T, 32, DIR>(s, g, sm, sn, tw, st, nload);
    case 64: return y_one<T, 64, DIR>(s, g, sm, sn, tw, st, nload);
    case 128: return y_one<T, 128, DIR>(s, g, sm, sn, tw, st, nload, v);
    case 256: return y_one<T, 256, DIR>(s, g, sm, sn, tw, st, nload, v);
    case 512: return y_one<T, 512, DIR>(s, g, sm, sn, tw, st, nload);
    case 1024: return y_one<T, 1024, DIR>(s, g, sm, sn, tw, st, nload);
    case 48: return y_one<T, 48, DIR>(s, g, sm, sn, tw, st, nload);
    case 96: return y_one<T, 96, DIR>(s, g, sm, sn, tw, st, nload);
    case 192: return y_one<T, 192, DIR>(s, g, sm, sn, tw, st, nload);
    case 80: return y_one<T, 80, DIR>(s, g, sm, sn, tw, st, nload);
    case 160: return y_one<T, 160, DIR>(s, g, sm, sn, tw, st, nload);
    default: return -1;
  }
}

template <typename T>
int launch_y(hipStream_t s, const Geo& g, int dir, cpx<T>* sm, cpx<T>* sn, const cpx<T>* tw, const LoadState* st,
             int nload, int v) {
  return dir < 0 ? y_dir<T, -1>(s, g, sm, sn, tw, st, nload, v) : y_dir<T, 1>(s, g, sm, sn, tw, st, nload, v);
}

#ifndef LSH_Y_TYPE
#error "define LSH_Y_TYPE"
#endif
template int launch_y<LSH_Y_TYPE>(hipStream_t, const Geo&, int, cpx<LSH_Y_TYPE>*, cpx<LSH_Y_TYPE>*,
                                  const cpx<LSH_Y_TYPE>*, const LoadState*, int, int);

}  // namespace lsh
