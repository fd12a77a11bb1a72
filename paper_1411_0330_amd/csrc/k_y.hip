// y passes (forward and inverse); instances for one element type (LSH_Y_TYPE).
#include "dispatch.hpp"

namespace lsh {

template <typename T, int NY, int DIR, int TX, int P, int LAY = YL_INPLACE>
static int y_inst(hipStream_t s, const Geo& g, cpx<T>* sm, cpx<T>* sn, const cpx<T>* tw, const LoadState* st,
                  int nload, cpx<T>* sout = nullptr) {
  constexpr int NT = TX * (NY / P);
  constexpr bool INPL = LAY == YL_INPLACE || LAY == YL_PAIRED;
  constexpr int H = INPL ? TX : TX / 2;
  const int mrow = LAY == YL_PAIRED ? 2 * g.mx : g.mx;
  const int xtiles = (mrow + H - 1) / H;
  // paired layouts: tiles over component pairs
  const int main_tiles = (LAY == YL_INPLACE ? g.c : g.c / 2) * g.nz * xtiles;
  const int nyq_tiles = (g.c * g.nz + TX - 1) / TX;
  hipLaunchKernelGGL((k_y<T, NY, P, TX, DIR, LAY>), dim3(main_tiles + nyq_tiles, nload), dim3(NT), 0, s, g, sm, sn,
                     tw, st, main_tiles, sout);
  return main_tiles + nyq_tiles;
}

template <typename T, int NY, int DIR, int V, int LAY = YL_INPLACE>
static int y_var(hipStream_t s, const Geo& g, cpx<T>* sm, cpx<T>* sn, const cpx<T>* tw, const LoadState* st,
                 int nload) {
  constexpr int P0 = p_y<T>(NY);
  constexpr int TX0 = tx_strided<T>(NY, P0);
  constexpr int TXV = sv_tx<T>(NY, P0, V), PV = sv_p(P0, V);
  if constexpr (V != 0 && sv_ok<T>(NY, TXV, PV))
    return y_inst<T, NY, DIR, TXV, PV, LAY>(s, g, sm, sn, tw, st, nload);
  else
    return y_inst<T, NY, DIR, TX0, P0, LAY>(s, g, sm, sn, tw, st, nload);
}

template <typename T, int NY, int DIR, int LAY = YL_INPLACE>
static int y_one(hipStream_t s, const Geo& g, cpx<T>* sm, cpx<T>* sn, const cpx<T>* tw, const LoadState* st,
                 int nload, int v = 0) {
  if constexpr (NY == 128 || NY == 256) {
    switch (v) {
      case 1: return y_var<T, NY, DIR, 1, LAY>(s, g, sm, sn, tw, st, nload);
      case 2: return y_var<T, NY, DIR, 2, LAY>(s, g, sm, sn, tw, st, nload);
      case 3: return y_var<T, NY, DIR, 3, LAY>(s, g, sm, sn, tw, st, nload);
      default: break;
    }
  }
  return y_var<T, NY, DIR, 0, LAY>(s, g, sm, sn, tw, st, nload);
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

// Forward y into the component-paired layout (sm plain in, sp paired out) or
// inverse y back from it (sp paired in, sm plain out): six-component FP32
// fields with 128 or 256 points along y.  Tiles hold at least 16
// wave-vectors of each component (whole 128-byte lines in both layouts):
// variant 3 takes twice the pencils of the others.  Returns -1 where no
// instance exists.
template <typename T>
int launch_y_paired(hipStream_t s, const Geo& g, int dir, cpx<T>* sm, cpx<T>* sp, cpx<T>* sn, const cpx<T>* tw,
                    const LoadState* st, int nload, int v) {
  if constexpr (sizeof(T) == 4) {
    if (g.c != 6 || g.nz < 2) return -1;
    auto go = [&](auto ny_tag, auto var_tag) -> int {
      constexpr int NY = decltype(ny_tag)::value, V = decltype(var_tag)::value;
      constexpr int P = p_y<T>(NY);
      constexpr int TX0 = tx_strided<T>(NY, P);
      // at least 32 pencils (16 wave-vectors of each component); shape 3 twice shape 0's
      constexpr int TXA = TX0 >= 32 ? TX0 : 32;
      constexpr int TXB = sv_ok<T>(NY, 2 * TXA, P) ? 2 * TXA : TXA;
      constexpr int TX = V == 3 ? TXB : TXA;
      static_assert(sv_ok<T>(NY, TX, P), "paired y shape within the workgroup limits");
      if (dir < 0) return y_inst<T, NY, -1, TX, P, YL_TO_PAIRED>(s, g, sm, sn, tw, st, nload, sp);
      return y_inst<T, NY, 1, TX, P, YL_FROM_PAIRED>(s, g, sp, sn, tw, st, nload, sm);
    };
    using V0 = std::integral_constant<int, 0>;
    using V3 = std::integral_constant<int, 3>;
    if (g.ny == 128) return v == 3 ? go(std::integral_constant<int, 128>{}, V3{}) : go(std::integral_constant<int, 128>{}, V0{});
    if (g.ny == 256) return v == 3 ? go(std::integral_constant<int, 256>{}, V3{}) : go(std::integral_constant<int, 256>{}, V0{});
  }
  return -1;
}

// Both y passes in place on the component-paired layout (written by the
// fused CG x pass, read by its x inverse pass): six-component FP32 fields,
// 128 or 256 points along y, every shape variant; -1 elsewhere.
template <typename T>
int launch_y_paired_inplace(hipStream_t s, const Geo& g, int dir, cpx<T>* sm, cpx<T>* sn, const cpx<T>* tw,
                            const LoadState* st, int nload, int v) {
  if constexpr (sizeof(T) == 4) {
    if (g.c != 6 || g.nz < 2) return -1;
    if (g.ny == 128)
      return dir < 0 ? y_one<T, 128, -1, YL_PAIRED>(s, g, sm, sn, tw, st, nload, v)
                     : y_one<T, 128, 1, YL_PAIRED>(s, g, sm, sn, tw, st, nload, v);
    if (g.ny == 256)
      return dir < 0 ? y_one<T, 256, -1, YL_PAIRED>(s, g, sm, sn, tw, st, nload, v)
                     : y_one<T, 256, 1, YL_PAIRED>(s, g, sm, sn, tw, st, nload, v);
  }
  return -1;
}

#ifndef LSH_Y_TYPE
#error "define LSH_Y_TYPE"
#endif
template int launch_y<LSH_Y_TYPE>(hipStream_t, const Geo&, int, cpx<LSH_Y_TYPE>*, cpx<LSH_Y_TYPE>*,
                                  const cpx<LSH_Y_TYPE>*, const LoadState*, int, int);
template int launch_y_paired<LSH_Y_TYPE>(hipStream_t, const Geo&, int, cpx<LSH_Y_TYPE>*, cpx<LSH_Y_TYPE>*,
                                         cpx<LSH_Y_TYPE>*, const cpx<LSH_Y_TYPE>*, const LoadState*, int, int);
template int launch_y_paired_inplace<LSH_Y_TYPE>(hipStream_t, const Geo&, int, cpx<LSH_Y_TYPE>*, cpx<LSH_Y_TYPE>*,
                                                 const cpx<LSH_Y_TYPE>*, const LoadState*, int, int);

}  // namespace lsh
