// Tile kernels, m <= 65536 (16-bit values, 32-bit terms, 64-bit sums).
#include "launch.h"
#include "tiles.h"

namespace ffx {
hipError_t launch_tiles_small(const DevMat& A, int64_t mte, ffx_dtype dt, const void* X, int64_t ldx, void* Y,
                              int64_t ldy, int s, uint32_t alpha, uint32_t beta, hipStream_t st, const uint16_t* x16,
                              uint32_t nb) {
  if (dt == FFX_I32) return launch_tiles_t<ArSmall, int32_t>(A, mte, X, ldx, Y, ldy, s, alpha, beta, st, x16, nb);
  return launch_tiles_t<ArSmall, int64_t>(A, mte, X, ldx, Y, ldy, s, alpha, beta, st, x16, nb);
}

hipError_t launch_compact_x(ffx_dtype dt, const void* X, int64_t ldx, uint16_t* out, int64_t n, hipStream_t st) {
  if (dt == FFX_I32) return launch_to_u16<int32_t>(X, ldx, out, n, st);
  return launch_to_u16<int64_t>(X, ldx, out, n, st);
}
}  // namespace ffx
