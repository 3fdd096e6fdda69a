// Tile kernels, m > 65536 on 64-bit integer sums.
#include "launch.h"
#include "tiles.h"

namespace ffx {
template <class AR>
static hipError_t go(const DevMat& A, int64_t mte, ffx_dtype dt, const void* X, int64_t ldx, void* Y, int64_t ldy,
                     int s, uint32_t alpha, uint32_t beta, hipStream_t st, uint32_t nb) {
  if (dt == FFX_I32) return launch_tiles_t<AR, int32_t>(A, mte, X, ldx, Y, ldy, s, alpha, beta, st, nullptr, nb);
  return launch_tiles_t<AR, int64_t>(A, mte, X, ldx, Y, ldy, s, alpha, beta, st, nullptr, nb);
}
hipError_t launch_tiles_big(int ak, const DevMat& A, int64_t mte, ffx_dtype dt, const void* X, int64_t ldx,
                            void* Y, int64_t ldy, int s, uint32_t alpha, uint32_t beta, hipStream_t st, uint32_t nb) {
  if (ak == AK_M31) return go<ArM31>(A, mte, dt, X, ldx, Y, ldy, s, alpha, beta, st, nb);
  if (ak == AK_BIG_CH) return go<ArBig<true>>(A, mte, dt, X, ldx, Y, ldy, s, alpha, beta, st, nb);
  return go<ArBig<false>>(A, mte, dt, X, ldx, Y, ldy, s, alpha, beta, st, nb);
}
}  // namespace ffx
