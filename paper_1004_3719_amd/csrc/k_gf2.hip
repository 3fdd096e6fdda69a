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

// ------------------------------------------------------------------------
// Block-Wiedemann sequence over GF(2) with packed blocks (Section 3, step 1,
// with the GF(2) compression of Section 4): S_i = U^T A^i V for 32w vectors.
// S_i is a 32w x 32w bit matrix; its row a is w words, bit b of word c being
// entry (a, 32c + b), the parity of the rows j where bit a of U[j] and bit b of
// word c of (A^i V)[j] are both set.
namespace ffx {

// Partial projection: workgroup g stages rows [256g, 256g + 256) of U and W in
// LDS, then thread t takes pair p = t % (32w*w), p = a*w + c, over every
// (256 / pairs)-th staged row (or, with more pairs than threads, the pairs t,
// t + 256, ... over all staged rows); the row groups meet in LDS.
constexpr int GF2_ROWS = 256;

__global__ __launch_bounds__(256) void k_proj_gf2(const uint32_t* __restrict__ U, const uint32_t* __restrict__ W,
                                                  int64_t n, int w, uint32_t* __restrict__ part) {
  extern __shared__ __align__(16) uint32_t sh[];  // U rows [256*w], W rows [256*w], groups [256]
  uint32_t* su = sh;
  uint32_t* sw = sh + GF2_ROWS * w;
  uint32_t* red = sw + GF2_ROWS * w;
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * GF2_ROWS;
  const int rows = (int)(n - r0 < GF2_ROWS ? n - r0 : GF2_ROWS);
  for (int k = tid; k < rows * w; k += 256) {
    su[k] = U[r0 * w + k];
    sw[k] = W[r0 * w + k];
  }
  __syncthreads();
  const int npairs = 32 * w * w;
  uint32_t* out = part + (int64_t)blockIdx.x * npairs;
  if (npairs <= 256) {
    const int ngrp = 256 / npairs, grp = tid / npairs, p = tid % npairs;
    const int a = p / w, c = p - a * w, ua = a >> 5, ub = a & 31;
    uint32_t acc = 0;
    if (grp < ngrp)
      for (int j = grp; j < rows; j += ngrp) acc ^= (0u - ((su[j * w + ua] >> ub) & 1u)) & sw[j * w + c];
    red[tid] = acc;
    __syncthreads();
    if (tid < npairs) {
      uint32_t x = 0;
      for (int g = 0; g < ngrp; ++g) x ^= red[g * npairs + tid];
      out[tid] = x;
    }
  } else {
    for (int p = tid; p < npairs; p += 256) {
      const int a = p / w, c = p - a * w, ua = a >> 5, ub = a & 31;
      uint32_t acc = 0;
      for (int j = 0; j < rows; ++j) acc ^= (0u - ((su[j * w + ua] >> ub) & 1u)) & sw[j * w + c];
      out[p] = acc;
    }
  }
}

// S_i[p] = XOR of the G partials of pair p: one workgroup per pair.
__global__ __launch_bounds__(256) void k_fold_gf2(const uint32_t* __restrict__ part, int G, int npairs,
                                                  uint32_t* __restrict__ S) {
  __shared__ uint32_t red[256];
  const int p = blockIdx.x, tid = threadIdx.x;
  uint32_t acc = 0;
  for (int g = tid; g < G; g += 256) acc ^= part[(int64_t)g * npairs + p];
  red[tid] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) red[tid] ^= red[tid + o];
    __syncthreads();
  }
  if (tid == 0) S[p] = red[0];
}

hipError_t launch_sequence_gf2(const DevMat& A, int64_t mte, int w, const uint32_t* U, const uint32_t* W0, int64_t L,
                               uint32_t* S, uint32_t* w1, uint32_t* part, int G, uint32_t* Wlast, hipStream_t st) {
  const int64_t n = A.nrows;
  const int npairs = 32 * w * w;
  const size_t lds = (size_t)(2 * GF2_ROWS * w + 256) * 4;
  const uint32_t* cur = W0;
  uint32_t* bufs[2] = {const_cast<uint32_t*>(W0), w1};
  for (int64_t i = 0; i < L; ++i) {
    hipLaunchKernelGGL(k_proj_gf2, dim3(G), dim3(256), lds, st, U, cur, n, w, part);
    hipLaunchKernelGGL(k_fold_gf2, dim3(npairs), dim3(256), 0, st, part, G, npairs, S + i * (int64_t)npairs);
    const bool last = i + 1 == L;
    if (last && !Wlast) break;
    uint32_t* next = last ? Wlast : bufs[(i + 1) & 1];
    hipError_t e = launch_tiles_gf2(A, mte, cur, w, next, w, w, st);
    if (e != hipSuccess) return e;
    cur = next;
  }
  return hipGetLastError();
}

}  // namespace ffx
