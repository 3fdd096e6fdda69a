// Tile kernels on exact doubles.
#include "launch.h"
#include "tiles.h"

namespace ffx {
template <typename V, bool CH>
static hipError_t go(const DevMat& A, int64_t mte, ffx_dtype dt, const void* X, int64_t ldx, void* Y, int64_t ldy,
                     int s, uint32_t alpha, uint32_t beta, hipStream_t st, const uint16_t* x16, uint32_t nb) {
  if (dt == FFX_I32) return launch_tiles_t<ArF64<V, CH>, int32_t>(A, mte, X, ldx, Y, ldy, s, alpha, beta, st, x16, nb);
  return launch_tiles_t<ArF64<V, CH>, int64_t>(A, mte, X, ldx, Y, ldy, s, alpha, beta, st, x16, nb);
}
hipError_t launch_tiles_f64(bool v16, bool chunk, const DevMat& A, int64_t mte, ffx_dtype dt, const void* X,
                            int64_t ldx, void* Y, int64_t ldy, int s, uint32_t alpha, uint32_t beta, hipStream_t st,
                            const uint16_t* x16, uint32_t nb) {
  if (v16) return chunk ? go<uint16_t, true>(A, mte, dt, X, ldx, Y, ldy, s, alpha, beta, st, x16, nb)
                        : go<uint16_t, false>(A, mte, dt, X, ldx, Y, ldy, s, alpha, beta, st, x16, nb);
  return chunk ? go<uint32_t, true>(A, mte, dt, X, ldx, Y, ldy, s, alpha, beta, st, nullptr, nb)
               : go<uint32_t, false>(A, mte, dt, X, ldx, Y, ldy, s, alpha, beta, st, nullptr, nb);
}
}  // namespace ffx
