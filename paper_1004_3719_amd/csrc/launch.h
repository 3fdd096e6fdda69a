// Arithmetic-class dispatch of the tile kernels.
#pragma once

#include "ffx_impl.h"

namespace ffx {

// Accumulator classes (see tiles.h): integer for m <= 65536; 64-bit integer
// for larger m, with or without reductions inside a row; exact doubles with
// 16- or 32-bit stored values, with or without reductions inside a row.
enum ArithKind { AK_SMALL = 0, AK_BIG, AK_BIG_CH, AK_F64_16, AK_F64_16_CH, AK_F64_32, AK_F64_32_CH, AK_COUNT };

hipError_t launch_tiles_small(const DevMat& A, int64_t mte, ffx_dtype dt, const void* X, int64_t ldx, void* Y,
                              int64_t ldy, int s, uint32_t alpha, uint32_t beta, hipStream_t st, const uint16_t* x16);
hipError_t launch_tiles_big(bool chunk, const DevMat& A, int64_t mte, ffx_dtype dt, const void* X, int64_t ldx,
                            void* Y, int64_t ldy, int s, uint32_t alpha, uint32_t beta, hipStream_t st);
hipError_t launch_tiles_f64(bool v16, bool chunk, const DevMat& A, int64_t mte, ffx_dtype dt, const void* X,
                            int64_t ldx, void* Y, int64_t ldy, int s, uint32_t alpha, uint32_t beta, hipStream_t st,
                            const uint16_t* x16);

// x16: a 16-bit copy of X (only for s = 1 and m <= 65536), or null.
inline hipError_t launch_tiles(int ak, const DevMat& A, int64_t mte, ffx_dtype dt, const void* X, int64_t ldx, void* Y,
                               int64_t ldy, int s, uint32_t alpha, uint32_t beta, hipStream_t st,
                               const uint16_t* x16 = nullptr) {
  switch (ak) {
    case AK_SMALL: return launch_tiles_small(A, mte, dt, X, ldx, Y, ldy, s, alpha, beta, st, x16);
    case AK_BIG: return launch_tiles_big(false, A, mte, dt, X, ldx, Y, ldy, s, alpha, beta, st);
    case AK_BIG_CH: return launch_tiles_big(true, A, mte, dt, X, ldx, Y, ldy, s, alpha, beta, st);
    case AK_F64_16: return launch_tiles_f64(true, false, A, mte, dt, X, ldx, Y, ldy, s, alpha, beta, st, x16);
    case AK_F64_16_CH: return launch_tiles_f64(true, true, A, mte, dt, X, ldx, Y, ldy, s, alpha, beta, st, x16);
    case AK_F64_32: return launch_tiles_f64(false, false, A, mte, dt, X, ldx, Y, ldy, s, alpha, beta, st, nullptr);
    default: return launch_tiles_f64(false, true, A, mte, dt, X, ldx, Y, ldy, s, alpha, beta, st, nullptr);
  }
}

// 16-bit copy of one vector of n residues (stride ldx) for the compact-x path.
hipError_t launch_compact_x(ffx_dtype dt, const void* X, int64_t ldx, uint16_t* out, int64_t n, hipStream_t st);

// Projection S[a][b] = sum_k U[k][a] * W[k][b] mod m (n x s operands), as
// per-workgroup partial sums followed by one combining launch. `partial`
// holds at least proj_partials() * s * s uint64 values.
int proj_partials();
hipError_t launch_projection(bool small, const DevMat& A, ffx_dtype dt, const void* U, int64_t ldu, const void* W,
                             int64_t ldw, int64_t n, int s, uint64_t* partial, void* S, hipStream_t st);

// Strided copy of an n x s block (ld_in -> ld_out) of dtype elements.
hipError_t launch_copy_block(ffx_dtype dt, const void* in, int64_t ldi, void* out, int64_t ldo, int64_t n, int s,
                             hipStream_t st);

}  // namespace ffx
