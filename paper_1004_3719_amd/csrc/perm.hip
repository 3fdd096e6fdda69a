// Row permutations of n x s blocks for reordered matrices: the caller's
// vectors are gathered into the stored order before the products and the
// results scattered back after them.
#include "launch.h"

namespace ffx {

// gather: out[i][c] = in[perm[i]][c]; scatter: out[perm[i]][c] = in[i][c].
// One thread per element; the compact side (i) is read or written coalesced.
template <typename T, bool SCATTER>
__global__ void k_permute_rows(const T* __restrict__ in, int64_t ldi, T* __restrict__ out, int64_t ldo,
                               const uint32_t* __restrict__ perm, int64_t n, int s) {
  const int64_t total = n * s;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t / s;
    const int c = (int)(t - i * s);
    const int64_t p = perm[i];
    if (SCATTER) out[p * ldo + c] = in[i * ldi + c];
    else out[i * ldo + c] = in[p * ldi + c];
  }
}

// out[i] = x[perm[i]] as 16 bits (residues below 65536): the gather of a
// reordered one-vector product fused with its compact copy of x.
// Each thread takes 8 consecutive outputs and issues its 8 independent gathers
// before any of them is used, so a wave keeps 512 gathers in flight.
template <typename Tv>
__global__ void k_permute_to_u16(const Tv* __restrict__ x, int64_t ldx, uint16_t* __restrict__ out,
                                 const uint32_t* __restrict__ perm, int64_t n) {
  const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 8;
  if (i0 >= n) return;
  if (i0 + 8 <= n) {
    uint32_t p[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) p[k] = perm[i0 + k];
    uint32_t v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = (uint32_t)x[(int64_t)p[k] * ldx];
    typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
    u32x4_t o;  // one 16-byte store (out is 16-byte aligned, i0 a multiple of 8)
    o.x = (v[0] & 0xffffu) | (v[1] << 16);
    o.y = (v[2] & 0xffffu) | (v[3] << 16);
    o.z = (v[4] & 0xffffu) | (v[5] << 16);
    o.w = (v[6] & 0xffffu) | (v[7] << 16);
    *(u32x4_t*)(out + i0) = o;
  } else {
    for (int64_t i = i0; i < n; ++i) out[i] = (uint16_t)x[(int64_t)perm[i] * ldx];
  }
}

hipError_t launch_permute_to_u16(ffx_dtype dt, const void* x, int64_t ldx, uint16_t* out, const uint32_t* perm,
                                 int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  if ((uintptr_t)out & 15) return hipErrorInvalidValue;
  const unsigned blocks = (unsigned)((n + 8 * 256 - 1) / (8 * 256));  // n <= 2^30: at most 2^19 blocks
  if (dt == FFX_I32)
    hipLaunchKernelGGL((k_permute_to_u16<int32_t>), dim3(blocks), dim3(256), 0, st, (const int32_t*)x, ldx, out, perm, n);
  else
    hipLaunchKernelGGL((k_permute_to_u16<int64_t>), dim3(blocks), dim3(256), 0, st, (const int64_t*)x, ldx, out, perm, n);
  return hipGetLastError();
}

hipError_t launch_permute_rows(size_t esize, const void* in, int64_t ldi, void* out, int64_t ldo, const uint32_t* perm,
                               int64_t n, int s, bool scatter, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int64_t total = n * s;
  const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 16384);
  if (esize == 4) {
    if (scatter)
      hipLaunchKernelGGL((k_permute_rows<uint32_t, true>), dim3(blocks), dim3(256), 0, st, (const uint32_t*)in, ldi,
                         (uint32_t*)out, ldo, perm, n, s);
    else
      hipLaunchKernelGGL((k_permute_rows<uint32_t, false>), dim3(blocks), dim3(256), 0, st, (const uint32_t*)in, ldi,
                         (uint32_t*)out, ldo, perm, n, s);
  } else {
    if (scatter)
      hipLaunchKernelGGL((k_permute_rows<uint64_t, true>), dim3(blocks), dim3(256), 0, st, (const uint64_t*)in, ldi,
                         (uint64_t*)out, ldo, perm, n, s);
    else
      hipLaunchKernelGGL((k_permute_rows<uint64_t, false>), dim3(blocks), dim3(256), 0, st, (const uint64_t*)in, ldi,
                         (uint64_t*)out, ldo, perm, n, s);
  }
  return hipGetLastError();
}

}  // namespace ffx
