// Persistent CG for small grids; instances for one element type (LSH_TINY_TYPE).
#include "dispatch.hpp"
#include "tiny.hpp"

namespace lsh {

// 2D scalar grids have few registers per point: a 512-thread workgroup takes
// the rows of a 64^2 grid in one sweep; 3D grids use 256 threads
template <typename T, int NX, int NY, int NZ, int C>
static int tiny_inst(hipStream_t s, const TinyArgs<T>& a, int nload) {
  constexpr int NT = (NZ == 1) ? 512 : 256;
  hipLaunchKernelGGL((k_tiny_cg<T, NX, NY, NZ, C, NT>), dim3(nload), dim3(NT), 0, s, a);
  return nload;
}

// grids of tiny_grid(): squares 8..64 (2D), cubes of 8 and (scalar) 16
template <typename T>
int launch_tiny_cg(hipStream_t s, const TinyArgs<T>& a, int nload) {
  const Geo& g = a.g;
  if (g.nz == 1 && g.c == 2 && g.nx == g.ny) {
    switch (g.nx) {
      case 8: return tiny_inst<T, 8, 8, 1, 2>(s, a, nload);
      case 16: return tiny_inst<T, 16, 16, 1, 2>(s, a, nload);
      case 32: return tiny_inst<T, 32, 32, 1, 2>(s, a, nload);
      case 64: return tiny_inst<T, 64, 64, 1, 2>(s, a, nload);
      default: return -1;
    }
  }
  if (g.nz > 1 && g.nx == g.ny && g.ny == g.nz) {
    if (g.nx == 8 && g.c == 3) return tiny_inst<T, 8, 8, 8, 3>(s, a, nload);
    if (g.nx == 8 && g.c == 6) return tiny_inst<T, 8, 8, 8, 6>(s, a, nload);
    if (g.nx == 16 && g.c == 3) return tiny_inst<T, 16, 16, 16, 3>(s, a, nload);
  }
  return -1;
}

#ifndef LSH_TINY_TYPE
#error "define LSH_TINY_TYPE"
#endif
template int launch_tiny_cg<LSH_TINY_TYPE>(hipStream_t, const TinyArgs<LSH_TINY_TYPE>&, int);

}  // namespace lsh
