// Tile kernels on centered doubles, 32-bit values.
#include "launch.h"
#include "tiles.h"

namespace ffx {
template <class AR>
static hipError_t go(const DevMat& A, int64_t mte, ffx_dtype dt, const void* X, int64_t ldx, void* Y, int64_t ldy,
                     int s, uint32_t alpha, uint32_t beta, hipStream_t st, const uint16_t* x16, uint32_t nb) {
  if (dt == FFX_I32) return launch_tiles_t<AR, int32_t>(A, mte, X, ldx, Y, ldy, s, alpha, beta, st, x16, nb);
  return launch_tiles_t<AR, int64_t>(A, mte, X, ldx, Y, ldy, s, alpha, beta, st, x16, nb);
}
hipError_t launch_tiles_f64c32(bool chunk, const DevMat& A, int64_t mte, ffx_dtype dt, const void* X, int64_t ldx, void* Y,
                              int64_t ldy, int s, uint32_t alpha, uint32_t beta, hipStream_t st, const uint16_t* x16,
                              uint32_t nb) {
  if (chunk) return go<ArCentered<double, uint32_t, true>>(A, mte, dt, X, ldx, Y, ldy, s, alpha, beta, st, nullptr, nb);
  return go<ArCentered<double, uint32_t, false>>(A, mte, dt, X, ldx, Y, ldy, s, alpha, beta, st, nullptr, nb);
}
}  // namespace ffx
