// Tile kernels, m > 65536 on 64-bit integer sums.
#include "launch.h"
#include "tiles.h"

namespace ffx {
hipError_t launch_tiles_big(bool chunk, const DevMat& A, int64_t mte, ffx_dtype dt, const void* X, int64_t ldx,
                            void* Y, int64_t ldy, int s, uint32_t alpha, uint32_t beta, hipStream_t st, uint32_t nb) {
  if (chunk) {
    if (dt == FFX_I32) return launch_tiles_t<ArBig<true>, int32_t>(A, mte, X, ldx, Y, ldy, s, alpha, beta, st, nullptr, nb);
    return launch_tiles_t<ArBig<true>, int64_t>(A, mte, X, ldx, Y, ldy, s, alpha, beta, st, nullptr, nb);
  }
  if (dt == FFX_I32) return launch_tiles_t<ArBig<false>, int32_t>(A, mte, X, ldx, Y, ldy, s, alpha, beta, st, nullptr, nb);
  return launch_tiles_t<ArBig<false>, int64_t>(A, mte, X, ldx, Y, ldy, s, alpha, beta, st, nullptr, nb);
}
}  // namespace ffx
