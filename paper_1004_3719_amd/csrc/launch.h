// Arithmetic-class dispatch of the tile kernels.
#pragma once

#include <algorithm>

#include "ffx_impl.h"

namespace ffx {

// Accumulator classes (see tiles.h): integer for m <= 65536; 64-bit integer
// for larger m, with or without reductions inside a row; exact doubles with
// 16- or 32-bit stored values, with or without reductions inside a row; the
// folding integer class of m = 2^31 - 1; exact floats (m <= 4096); centered
// floats and doubles.
enum ArithKind {
  AK_SMALL = 0, AK_BIG, AK_BIG_CH, AK_F64_16, AK_F64_16_CH, AK_F64_32, AK_F64_32_CH, AK_M31,
  AK_F32, AK_F32_CH, AK_F32C, AK_F32C_CH, AK_F64C_16, AK_F64C_16_CH, AK_F64C_32, AK_F64C_32_CH, AK_COUNT
};

hipError_t launch_tiles_small(const DevMat& A, int64_t mte, ffx_dtype dt, const void* X, int64_t ldx, void* Y,
                              int64_t ldy, int s, uint32_t alpha, uint32_t beta, hipStream_t st, const uint16_t* x16,
                              uint32_t nblocks);
// ak: AK_BIG, AK_BIG_CH or AK_M31
hipError_t launch_tiles_big(int ak, const DevMat& A, int64_t mte, ffx_dtype dt, const void* X, int64_t ldx,
                            void* Y, int64_t ldy, int s, uint32_t alpha, uint32_t beta, hipStream_t st,
                            uint32_t nblocks);
hipError_t launch_tiles_f64(bool v16, bool chunk, const DevMat& A, int64_t mte, ffx_dtype dt, const void* X,
                            int64_t ldx, void* Y, int64_t ldy, int s, uint32_t alpha, uint32_t beta, hipStream_t st,
                            const uint16_t* x16, uint32_t nblocks);
hipError_t launch_tiles_f32(bool chunk, const DevMat& A, int64_t mte, ffx_dtype dt, const void* X, int64_t ldx, void* Y,
                           int64_t ldy, int s, uint32_t alpha, uint32_t beta, hipStream_t st, const uint16_t* x16,
                           uint32_t nblocks);
hipError_t launch_tiles_f32c(bool chunk, const DevMat& A, int64_t mte, ffx_dtype dt, const void* X, int64_t ldx, void* Y,
                            int64_t ldy, int s, uint32_t alpha, uint32_t beta, hipStream_t st, const uint16_t* x16,
                            uint32_t nblocks);
hipError_t launch_tiles_f64c16(bool chunk, const DevMat& A, int64_t mte, ffx_dtype dt, const void* X, int64_t ldx, void* Y,
                              int64_t ldy, int s, uint32_t alpha, uint32_t beta, hipStream_t st, const uint16_t* x16,
                              uint32_t nblocks);
hipError_t launch_tiles_f64c32(bool chunk, const DevMat& A, int64_t mte, ffx_dtype dt, const void* X, int64_t ldx, void* Y,
                              int64_t ldy, int s, uint32_t alpha, uint32_t beta, hipStream_t st, const uint16_t* x16,
                              uint32_t nblocks);

// x16: a 16-bit copy of X (only for s = 1 and m <= 65536), or null. nblocks:
// the grid size (0: one workgroup per tile; larger grids repeat the tiles).
inline hipError_t launch_tiles(int ak, const DevMat& A, int64_t mte, ffx_dtype dt, const void* X, int64_t ldx, void* Y,
                               int64_t ldy, int s, uint32_t alpha, uint32_t beta, hipStream_t st,
                               const uint16_t* x16 = nullptr, uint32_t nb = 0) {
  switch (ak) {
    case AK_SMALL: return launch_tiles_small(A, mte, dt, X, ldx, Y, ldy, s, alpha, beta, st, x16, nb);
    case AK_BIG:
    case AK_BIG_CH:
    case AK_M31: return launch_tiles_big(ak, A, mte, dt, X, ldx, Y, ldy, s, alpha, beta, st, nb);
    case AK_F64_16: return launch_tiles_f64(true, false, A, mte, dt, X, ldx, Y, ldy, s, alpha, beta, st, x16, nb);
    case AK_F64_16_CH: return launch_tiles_f64(true, true, A, mte, dt, X, ldx, Y, ldy, s, alpha, beta, st, x16, nb);
    case AK_F64_32: return launch_tiles_f64(false, false, A, mte, dt, X, ldx, Y, ldy, s, alpha, beta, st, nullptr, nb);
    case AK_F64_32_CH: return launch_tiles_f64(false, true, A, mte, dt, X, ldx, Y, ldy, s, alpha, beta, st, nullptr, nb);
    case AK_F32:
    case AK_F32_CH: return launch_tiles_f32(ak == AK_F32_CH, A, mte, dt, X, ldx, Y, ldy, s, alpha, beta, st, x16, nb);
    case AK_F32C:
    case AK_F32C_CH: return launch_tiles_f32c(ak == AK_F32C_CH, A, mte, dt, X, ldx, Y, ldy, s, alpha, beta, st, x16, nb);
    case AK_F64C_16:
    case AK_F64C_16_CH:
      return launch_tiles_f64c16(ak == AK_F64C_16_CH, A, mte, dt, X, ldx, Y, ldy, s, alpha, beta, st, x16, nb);
    default:
      return launch_tiles_f64c32(ak == AK_F64C_32_CH, A, mte, dt, X, ldx, Y, ldy, s, alpha, beta, st, nullptr, nb);
  }
}

// Y = A X over GF(2), X and Y bit-packed blocks of w 32-bit words per row (A built with m = 2).
hipError_t launch_tiles_gf2(const DevMat& A, int64_t mte, const void* X, int64_t ldx, void* Y, int64_t ldy, int w,
                            hipStream_t st);

// S_i = U^T A^i W0 over GF(2) for i < L (L >= 1), packed blocks of w words per row (ld w); S holds
// L * 32w * w words. Workspace: w1 (n x w words), part (G * 32w * w words, G = ceil(n / 256)); W0 is
// overwritten.
// Wlast (n x w, or null) receives A^L W0.
// Words of the partial buffers of launch_sequence_gf2.
size_t gf2_sequence_part_words(const DevMat& A, int w);
hipError_t launch_sequence_gf2(const DevMat& A, int64_t mte, int w, const uint32_t* U, const uint32_t* W0, int64_t L,
                               uint32_t* S, uint32_t* w1, uint32_t* part, uint32_t* Wlast, hipStream_t st);

// 16-bit copy of one vector of n residues (stride ldx) for the compact-x path.
hipError_t launch_compact_x(ffx_dtype dt, const void* X, int64_t ldx, uint16_t* out, int64_t n, hipStream_t st);

// The sequence S_i = U^T A^i V, i < L (L >= 1), and A^L V into Wlast when not
// null. Workspace: w0, w1, u32 (n x s int32 each), p0, p1 ((4 * ntiles + 64) *
// s * s uint64 each), counter (one int64). Steps are replayed from a hipGraph
// in batches of `batch` iterations (0: no graph).
// ak: an integer class (AK_SMALL, AK_BIG, AK_BIG_CH or AK_M31); only_sell: the
// matrix has SELL tiles only.
hipError_t launch_sequence(int ak, bool only_sell, const DevMat& A, int64_t mte, ffx_dtype dt, const void* U,
                           int64_t ldu, const void* V, int64_t ldv, int64_t L, int s, void* S, void* Wlast, void* w0,
                           void* w1, void* u32, uint64_t* p0, uint64_t* p1, int64_t* counter, int batch,
                           hipStream_t st);

// Y = alpha*A^T*X + beta*Y by scattering the entries of A (no stored A^T);
// acc is workspace of ncols * s uint64.
hipError_t launch_transpose_scatter(bool small, const DevMat& A, ffx_dtype dt, const void* X, int64_t ldx, void* Y,
                                    int64_t ldy, int s, uint32_t alpha, uint32_t beta, unsigned long long* acc,
                                    hipStream_t st);

// *first = the smallest flat index k*ldx + c of an entry of the n x s block X
// outside [0, m-1], or ~0 when there is none (device memory, set by the launch).
hipError_t launch_check_block(ffx_dtype dt, const void* X, int64_t n, int s, int64_t ldx, uint32_t m,
                              unsigned long long* first, hipStream_t st);

// Row permutation of an n x s block of esize-byte elements (4 or 8) by perm
// (n entries, each < n): gather out[i] = in[perm[i]], or scatter
// out[perm[i]] = in[i]. in and out must not overlap.
hipError_t launch_permute_rows(size_t esize, const void* in, int64_t ldi, void* out, int64_t ldo, const uint32_t* perm,
                               int64_t n, int s, bool scatter, hipStream_t st);
// out[i] = x[perm[i] * ldx] as 16 bits, i < n (m <= 65536); out 16-byte aligned.
hipError_t launch_permute_to_u16(ffx_dtype dt, const void* x, int64_t ldx, uint16_t* out, const uint32_t* perm,
                                 int64_t n, hipStream_t st);

// Strided copy of an n x s block (ld_in -> ld_out) of dtype elements.
hipError_t launch_copy_block(ffx_dtype dt, const void* in, int64_t ldi, void* out, int64_t ldo, int64_t n, int s,
                             hipStream_t st);

}  // namespace ffx
