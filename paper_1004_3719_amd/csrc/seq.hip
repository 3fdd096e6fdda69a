// Projection U^T W of the block-Wiedemann sequence (paper Section 3, step 1:
// S_i = U^T A^i V) and a strided block copy.
#include "launch.h"
#include "tiles.h"

namespace ffx {

constexpr int PROJ_WG = 512;
int proj_partials() { return PROJ_WG; }

// Each lane owns one column b of W and all s columns a of U for a strided set
// of rows, and accumulates U[k][a]*W[k][b] with the same delayed reduction as
// the products. Residues of the lanes meet in LDS; one partial per workgroup.
template <class AR, typename Tv, int S>
__global__ __launch_bounds__(256) void k_proj_partial(DevMat A, const Tv* __restrict__ U, int64_t ldu,
                                                      const Tv* __restrict__ W, int64_t ldw, int64_t n, int s,
                                                      uint64_t* __restrict__ partial) {
  __shared__ uint64_t red[256 * S];
  const int tid = threadIdx.x;
  const int b = tid % S, rsub = tid / S, rpw = 256 / S;
  LaneAcc<AR, S> acc;
  acc.init(A);
  if (b < s) {
    for (int64_t k = (int64_t)blockIdx.x * rpw + rsub; k < n; k += (int64_t)gridDim.x * rpw) {
      uint32_t w = (uint32_t)W[k * ldw + b];
      const Tv* ur = U + k * ldu;
#pragma unroll
      for (int a = 0; a < S; ++a)
        if (a < s) acc.a[a] += AR::mul((uint32_t)ur[a], w);
      acc.tick(A);
    }
  }
#pragma unroll
  for (int a = 0; a < S; ++a) red[(rsub * S + a) * S + b] = (b < s && a < s) ? AR::reduce(acc.a[a], A) : 0u;
  __syncthreads();
  if (tid < S * S) {
    const int a = tid / S, bb = tid % S;
    uint64_t t = 0;
    for (int q = 0; q < rpw; ++q) t += red[(q * S + a) * S + bb];
    if (a < s && bb < s) partial[(int64_t)blockIdx.x * s * s + a * s + bb] = t;
  }
}

template <typename Tv>
__global__ __launch_bounds__(256) void k_proj_final(DevMat A, const uint64_t* __restrict__ partial, int nparts, int s,
                                                    Tv* __restrict__ S) {
  const int t = threadIdx.x;
  if (t >= s * s) return;
  uint64_t acc = 0;  // nparts * 256 * m < 2^49
  for (int q = 0; q < nparts; ++q) acc += partial[(int64_t)q * s * s + t];
  S[t] = (Tv)mod_u64(acc, A.m, A.mu);
}

template <class AR, typename Tv>
static hipError_t proj_go(const DevMat& A, const void* U, int64_t ldu, const void* W, int64_t ldw, int64_t n, int s,
                          uint64_t* partial, void* S, hipStream_t st) {
  const Tv* u = (const Tv*)U;
  const Tv* w = (const Tv*)W;
  dim3 g(PROJ_WG), b(256);
  if (s <= 1) hipLaunchKernelGGL((k_proj_partial<AR, Tv, 1>), g, b, 0, st, A, u, ldu, w, ldw, n, s, partial);
  else if (s <= 2) hipLaunchKernelGGL((k_proj_partial<AR, Tv, 2>), g, b, 0, st, A, u, ldu, w, ldw, n, s, partial);
  else if (s <= 4) hipLaunchKernelGGL((k_proj_partial<AR, Tv, 4>), g, b, 0, st, A, u, ldu, w, ldw, n, s, partial);
  else if (s <= 8) hipLaunchKernelGGL((k_proj_partial<AR, Tv, 8>), g, b, 0, st, A, u, ldu, w, ldw, n, s, partial);
  else hipLaunchKernelGGL((k_proj_partial<AR, Tv, 16>), g, b, 0, st, A, u, ldu, w, ldw, n, s, partial);
  hipLaunchKernelGGL((k_proj_final<Tv>), dim3(1), dim3(256), 0, st, A, partial, PROJ_WG, s, (Tv*)S);
  return hipGetLastError();
}

hipError_t launch_projection(bool small, const DevMat& A, ffx_dtype dt, const void* U, int64_t ldu, const void* W,
                             int64_t ldw, int64_t n, int s, uint64_t* partial, void* S, hipStream_t st) {
  if (small) {
    if (dt == FFX_I32) return proj_go<ArSmall, int32_t>(A, U, ldu, W, ldw, n, s, partial, S, st);
    return proj_go<ArSmall, int64_t>(A, U, ldu, W, ldw, n, s, partial, S, st);
  }
  if (dt == FFX_I32) return proj_go<ArBig<true>, int32_t>(A, U, ldu, W, ldw, n, s, partial, S, st);
  return proj_go<ArBig<true>, int64_t>(A, U, ldu, W, ldw, n, s, partial, S, st);
}

template <typename Tv>
__global__ void k_copy_block(const Tv* __restrict__ in, int64_t ldi, Tv* __restrict__ out, int64_t ldo, int64_t n,
                             int s) {
  int64_t total = n * s;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    int64_t k = t / s;
    int c = (int)(t - k * s);
    out[k * ldo + c] = in[k * ldi + c];
  }
}

hipError_t launch_copy_block(ffx_dtype dt, const void* in, int64_t ldi, void* out, int64_t ldo, int64_t n, int s,
                             hipStream_t st) {
  if (n == 0) return hipSuccess;
  int64_t total = n * s;
  int blocks = (int)((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
  if (dt == FFX_I32)
    hipLaunchKernelGGL(k_copy_block<int32_t>, dim3(blocks), dim3(256), 0, st, (const int32_t*)in, ldi, (int32_t*)out,
                       ldo, n, s);
  else
    hipLaunchKernelGGL(k_copy_block<int64_t>, dim3(blocks), dim3(256), 0, st, (const int64_t*)in, ldi, (int64_t*)out,
                       ldo, n, s);
  return hipGetLastError();
}

}  // namespace ffx
