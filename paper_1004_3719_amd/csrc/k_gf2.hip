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

// Partial projection: workgroup g takes rows [g*chunk, (g+1)*chunk), thread t
// the pairs p = t, t + 256, ... of the 32w*w pairs (a, c), p = a*w + c.
__global__ __launch_bounds__(256) void k_proj_gf2(const uint32_t* __restrict__ U, const uint32_t* __restrict__ W,
                                                  int64_t n, int w, int64_t chunk, uint32_t* __restrict__ part) {
  const int npairs = 32 * w * w;
  const int64_t r0 = (int64_t)blockIdx.x * chunk, r1 = r0 + chunk < n ? r0 + chunk : n;
  for (int p = threadIdx.x; p < npairs; p += blockDim.x) {
    const int a = p / w, c = p - a * w;
    const int ua = a >> 5, ub = a & 31;
    uint32_t acc = 0;
    for (int64_t j = r0; j < r1; ++j) {
      const uint32_t bit = (U[j * w + ua] >> ub) & 1u;
      acc ^= (0u - bit) & W[j * w + c];
    }
    part[(int64_t)blockIdx.x * npairs + p] = acc;
  }
}

// S_i[p] = XOR of the G partials of pair p.
__global__ void k_fold_gf2(const uint32_t* __restrict__ part, int G, int npairs, uint32_t* __restrict__ S) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  uint32_t acc = 0;
  for (int g = 0; g < G; ++g) acc ^= part[(int64_t)g * npairs + p];
  S[p] = acc;
}

hipError_t launch_sequence_gf2(const DevMat& A, int64_t mte, int w, const uint32_t* U, const uint32_t* W0, int64_t L,
                               uint32_t* S, uint32_t* w1, uint32_t* part, int G, uint32_t* Wlast, hipStream_t st) {
  const int64_t n = A.nrows;
  const int npairs = 32 * w * w;
  const int64_t chunk = (n + G - 1) / G;
  const uint32_t* cur = W0;
  uint32_t* bufs[2] = {const_cast<uint32_t*>(W0), w1};
  for (int64_t i = 0; i < L; ++i) {
    hipLaunchKernelGGL(k_proj_gf2, dim3(G), dim3(256), 0, st, U, cur, n, w, chunk, part);
    hipLaunchKernelGGL(k_fold_gf2, dim3((npairs + 255) / 256), dim3(256), 0, st, part, G, npairs,
                       S + i * (int64_t)npairs);
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
