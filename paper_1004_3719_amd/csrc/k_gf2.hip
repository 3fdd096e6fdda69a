// Tile kernels over GF(2) with bit-packed blocks of 32-bit words.
#include "launch.h"
#include "tiles.h"

namespace ffx {
hipError_t launch_tiles_gf2(const DevMat& A, int64_t mte, const void* X, int64_t ldx, void* Y, int64_t ldy, int w,
                            hipStream_t st) {
  // words are moved as int32 bit patterns: conversions to and from uint32 keep every bit
  return launch_tiles_t<ArGF2, int32_t>(A, mte, X, ldx, Y, ldy, w, 1, 0, st, nullptr, 0);
}
}  // namespace ffx
