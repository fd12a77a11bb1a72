// y passes (forward and inverse), FP32 and FP64 instances.
#include "dispatch.hpp"

namespace lsh {

template <typename T, int NY, int DIR>
static int y_one(hipStream_t s, const Geo& g, cpx<T>* sm, cpx<T>* sn, const cpx<T>* tw, const LoadState* st,
                 int nload) {
  constexpr int P = p_y<T>(NY);
  constexpr int TX = tx_strided<T>(NY, P);
  constexpr int NT = TX * (NY / P);
  const int xtiles = (g.mx + TX - 1) / TX;
  const int main_tiles = g.c * g.nz * xtiles;
  const int nyq_tiles = (g.c * g.nz + TX - 1) / TX;
  hipLaunchKernelGGL((k_y<T, NY, P, TX, DIR>), dim3(main_tiles + nyq_tiles, nload), dim3(NT), 0, s, g, sm, sn, tw,
                     st, main_tiles);
  return main_tiles + nyq_tiles;
}

template <typename T, int DIR>
static int y_dir(hipStream_t s, const Geo& g, cpx<T>* sm, cpx<T>* sn, const cpx<T>* tw, const LoadState* st,
                 int nload) {
  switch (g.ny) {
    case 2: return y_one<T, 2, DIR>(s, g, sm, sn, tw, st, nload);
    case 4: return y_one<T, 4, DIR>(s, g, sm, sn, tw, st, nload);
    case 8: return y_one<T, 8, DIR>(s, g, sm, sn, tw, st, nload);
    case 16: return y_one<T, 16, DIR>(s, g, sm, sn, tw, st, nload);
    case 32: return y_one<T, 32, DIR>(s, g, sm, sn, tw, st, nload);
    case 64: return y_one<T, 64, DIR>(s, g, sm, sn, tw, st, nload);
    case 128: return y_one<T, 128, DIR>(s, g, sm, sn, tw, st, nload);
    case 256: return y_one<T, 256, DIR>(s, g, sm, sn, tw, st, nload);
    case 512: return y_one<T, 512, DIR>(s, g, sm, sn, tw, st, nload);
    case 1024: return y_one<T, 1024, DIR>(s, g, sm, sn, tw, st, nload);
    default: return -1;
  }
}

template <typename T>
int launch_y(hipStream_t s, const Geo& g, int dir, cpx<T>* sm, cpx<T>* sn, const cpx<T>* tw, const LoadState* st,
             int nload) {
  return dir < 0 ? y_dir<T, -1>(s, g, sm, sn, tw, st, nload) : y_dir<T, 1>(s, g, sm, sn, tw, st, nload);
}

template int launch_y<float>(hipStream_t, const Geo&, int, cpx<float>*, cpx<float>*, const cpx<float>*,
                             const LoadState*, int);
template int launch_y<double>(hipStream_t, const Geo&, int, cpx<double>*, cpx<double>*, const cpx<double>*,
                              const LoadState*, int);

}  // namespace lsh
