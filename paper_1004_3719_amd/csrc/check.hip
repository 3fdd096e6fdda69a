// Checked mode: find the first entry of an n x s block that is not a residue
// in [0, m-1] (vector entries must be canonical residues, Section 2.2).
#include "launch.h"

namespace ffx {

__global__ void k_check_init(unsigned long long* first) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *first = ~0ull;
}

template <typename Tv>
__global__ void k_check_block(const Tv* __restrict__ X, int64_t n, int s, int64_t ldx, uint32_t m,
                              unsigned long long* first) {
  const int64_t total = n * s;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = t / s;
    const int c = (int)(t - k * s);
    const int64_t v = (int64_t)X[k * ldx + c];
    if (v < 0 || v >= (int64_t)m) atomicMin(first, (unsigned long long)(k * ldx + c));
  }
}

hipError_t launch_check_block(ffx_dtype dt, const void* X, int64_t n, int s, int64_t ldx, uint32_t m,
                              unsigned long long* first, hipStream_t st) {
  hipLaunchKernelGGL(k_check_init, dim3(1), dim3(64), 0, st, first);
  const int64_t total = n * s;
  if (total > 0) {
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 8192);
    if (dt == FFX_I32)
      hipLaunchKernelGGL(k_check_block<int32_t>, dim3(blocks), dim3(256), 0, st, (const int32_t*)X, n, s, ldx, m,
                         first);
    else
      hipLaunchKernelGGL(k_check_block<int64_t>, dim3(blocks), dim3(256), 0, st, (const int64_t*)X, n, s, ldx, m,
                         first);
  }
  return hipGetLastError();
}

}  // namespace ffx
