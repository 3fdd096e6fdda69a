// Gather-rate calibration: the ceiling that bounds the products on this GPU.
//
// A product reads its matrix as a coalesced stream and gathers one element (or
// one row of s elements) of x per entry at the entry's column. Section 2.5
// ("Performance issues") names memory access as what limits sparse products;
// on MI355X the limit of the large products is the rate at which random
// gathers are served from the vector L1/L2 caches, not HBM bandwidth. This
// kernel measures that rate in the products' own pattern: each lane reads a
// streamed index word and gathers the row it names from a table of a given
// size, and the gathered values are folded into one word per lane so the loads
// cannot be dropped.
#include <algorithm>
#include <vector>

#include "host.h"

namespace ffx {
namespace {

__device__ inline uint64_t mixg(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// idx[i]: uniform over [0, rows) (window 0), or uniform within the aligned window of `window` rows
// that the position i/per_window falls in (the locality of a reordered or banded matrix)
__global__ void k_gather_indices(uint32_t* __restrict__ idx, int64_t count, uint64_t rows, uint64_t window,
                                 uint64_t seed) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t r = mixg(seed + (uint64_t)i * 0x9E3779B97F4A7C15ULL);
    uint64_t v;
    if (window == 0) {
      v = r % rows;
    } else {
      uint64_t nwin = (rows + window - 1) / window;
      uint64_t w = ((uint64_t)i * nwin / (uint64_t)count) % nwin;
      v = std::min<uint64_t>(rows - 1, w * window + r % window);
    }
    idx[i] = (uint32_t)v;
  }
}

// ROWW 32-bit words per row (a 2-byte row reads half a word); PER gathers per lane in flight
template <int ROWW, bool HALF, int PER>
__global__ __launch_bounds__(256) void k_gather(const uint32_t* __restrict__ idx, const uint32_t* __restrict__ table,
                                                int64_t count, uint32_t* __restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * PER;
  uint32_t acc = 0;
  for (int64_t base = ((int64_t)blockIdx.x * blockDim.x) * PER + threadIdx.x; base < count; base += stride) {
    uint32_t ix[PER];
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      int64_t i = base + (int64_t)p * blockDim.x;
      ix[p] = i < count ? __builtin_nontemporal_load(idx + i) : 0xFFFFFFFFu;
    }
    uint32_t v[PER][ROWW];
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      if (ix[p] == 0xFFFFFFFFu) {
#pragma unroll
        for (int w = 0; w < ROWW; ++w) v[p][w] = 0;
        continue;
      }
      if constexpr (HALF) {
        v[p][0] = ((const uint16_t*)table)[ix[p]];
      } else {
#pragma unroll
        for (int w = 0; w < ROWW; ++w) v[p][w] = table[(int64_t)ix[p] * ROWW + w];
      }
    }
#pragma unroll
    for (int p = 0; p < PER; ++p)
#pragma unroll
      for (int w = 0; w < ROWW; ++w) acc ^= v[p][w] + (uint32_t)w;
  }
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

template <int ROWW, bool HALF>
hipError_t launch_gather(const uint32_t* idx, const uint32_t* table, int64_t count, uint32_t* out, int grid,
                         hipStream_t st) {
  hipLaunchKernelGGL((k_gather<ROWW, HALF, 8>), dim3(grid), dim3(256), 0, st, idx, table, count, out);
  return hipGetLastError();
}

struct Buf {
  void* p = nullptr;
  ~Buf() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace
}  // namespace ffx

using namespace ffx;

extern "C" ffx_status ffx_gather_rate(int64_t table_bytes, int32_t row_bytes, int64_t count, int64_t window,
                                      int32_t reps, void* stream, double* rate) {
  return guard([&] {
    if (!rate) fail(FFX_EINVAL, "rate is NULL");
    if (row_bytes != 2 && row_bytes != 4 && row_bytes != 8 && row_bytes != 16 && row_bytes != 32 && row_bytes != 64)
      fail(FFX_EINVAL, "row_bytes %d (2, 4, 8, 16, 32 or 64)", row_bytes);
    const int64_t rows = table_bytes / row_bytes;
    if (rows < 1 || rows > ((int64_t)1 << 31)) fail(FFX_EINVAL, "table of %lld bytes", (long long)table_bytes);
    if (count < 1 || count > ((int64_t)1 << 31)) fail(FFX_EINVAL, "count %lld", (long long)count);
    if (window < 0 || window > rows) fail(FFX_EINVAL, "window %lld", (long long)window);
    if (reps < 1 || reps > 1000) fail(FFX_EINVAL, "reps %d", reps);
    hipStream_t st = (hipStream_t)stream;
    int dev = 0, ncu = 0;
    FFX_HIP(hipGetDevice(&dev));
    FFX_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const int grid = std::max(1, ncu) * 8;
    Buf tab, ix, out;
    const size_t tbytes = (size_t)rows * row_bytes;
    FFX_HIP(hipMalloc(&tab.p, (tbytes + 3) / 4 * 4));
    FFX_HIP(hipMalloc(&ix.p, (size_t)count * 4));
    FFX_HIP(hipMalloc(&out.p, (size_t)grid * 256 * 4));
    FFX_HIP(hipMemsetAsync(tab.p, 0x5A, (tbytes + 3) / 4 * 4, st));
    hipLaunchKernelGGL(k_gather_indices, dim3(2048), dim3(256), 0, st, (uint32_t*)ix.p, count, (uint64_t)rows,
                       (uint64_t)window, (uint64_t)0x9A7E5EEDULL);
    FFX_HIP(hipGetLastError());
    auto go = [&]() -> hipError_t {
      const uint32_t* I = (const uint32_t*)ix.p;
      const uint32_t* T = (const uint32_t*)tab.p;
      uint32_t* O = (uint32_t*)out.p;
      switch (row_bytes) {
        case 2: return launch_gather<1, true>(I, T, count, O, grid, st);
        case 4: return launch_gather<1, false>(I, T, count, O, grid, st);
        case 8: return launch_gather<2, false>(I, T, count, O, grid, st);
        case 16: return launch_gather<4, false>(I, T, count, O, grid, st);
        case 32: return launch_gather<8, false>(I, T, count, O, grid, st);
        default: return launch_gather<16, false>(I, T, count, O, grid, st);
      }
    };
    FFX_HIP(go());  // warm: the table's lines reach the caches as they would in a product
    hipEvent_t e0, e1;
    FFX_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
      (void)hipEventDestroy(e0);
      fail(FFX_EDEVICE, "hipEventCreate failed");
    }
    std::vector<float> ms;
    hipError_t e = hipSuccess;
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
      e = hipEventRecord(e0, st);
      if (e == hipSuccess) e = go();
      if (e == hipSuccess) e = hipEventRecord(e1, st);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float t = 0;
      if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
      ms.push_back(t);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    FFX_HIP(e);
    std::sort(ms.begin(), ms.end());
    *rate = (double)count / (ms[ms.size() / 2] * 1e-3);
  });
}
