// The one-vector product on column-sorted row groups (layout in sg.h).
#include <algorithm>
#include <mutex>

#include "sg.h"

namespace ffx {

constexpr int SG_THREADS = 1024;  // one workgroup per compute unit: 16 waves
constexpr int SG_U = 2;           // chunks per wave in flight
// Dynamic LDS of one group is at least this much, so that a compute unit never
// holds two groups (the groups are sized to be about one per compute unit, and
// two on one CU would leave another CU idle).
constexpr size_t SG_LDS_FLOOR = 96 * 1024;

__device__ inline uint32_t sg_lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// GF2: a matrix mod 2 times one bit-packed word per row (32 vectors over GF(2)): x and y are words
// (stride ldx, ldy), a row's sum is the exclusive or of its columns' words (32-bit LDS sums).
template <typename Tx, typename Tv, int NT, int U, bool GF2>
__global__ __launch_bounds__(NT) void k_sg(SgMat G, const Tx* __restrict__ x, Tv* __restrict__ y, uint32_t alpha,
                                           uint32_t beta, uint16_t* __restrict__ y16, int64_t ldx, int64_t ldy) {
  extern __shared__ __align__(16) unsigned long long acc[];
  uint32_t* accx = (uint32_t*)acc;  // GF2
  constexpr uint32_t NW = NT / WAVE;
  const SgGroup g = G.groups[blockIdx.x];
  const uint32_t tid = threadIdx.x, lane = tid & (WAVE - 1), wave = tid / WAVE;
  for (uint32_t r = tid; r < g.nrows; r += NT) {
    if constexpr (GF2) accx[r] = 0u;
    else acc[r] = 0ull;
  }
  __syncthreads();
  // the entry words of the next U chunks are requested before the values and gathers of the
  // current ones, so each pass waits on one round trip to memory instead of two
  uint32_t w[U][4], vo[U], cb[U];
  auto load_words = [&](uint32_t ch0, uint32_t (&ww)[U][4], uint32_t (&vv)[U], uint32_t (&cc)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t ch = ch0 + u * NW;
      const bool ok = ch < g.nchunks;
      typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
      const u32x4_t q = ok ? __builtin_nontemporal_load((const u32x4_t*)(G.ent + (size_t)(g.c0 + ch) * SG_CHUNK) + lane)
                           : (u32x4_t)(PAD_WORD);
      ww[u][0] = q.x;
      ww[u][1] = q.y;
      ww[u][2] = q.z;
      ww[u][3] = q.w;
      vv[u] = ok ? G.choff[g.c0 + ch] : 0u;
      cc[u] = ok ? G.cbase[g.c0 + ch] : 0u;
    }
  };
  load_words(wave, w, vo, cb);
  for (uint32_t ch0 = wave; ch0 < g.nchunks; ch0 += NW * U) {
    uint32_t wn[U][4], von[U], cbn[U];
    load_words(ch0 + NW * U, wn, von, cbn);
    // values: a lane's general values are consecutive, after those of the lanes below it (four
    // ballots give their count), and one 12-byte load brings all of them; then x
    uint32_t v[U][4], xv[U][4];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      uint32_t idx = vo[u], ng = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const bool gen = (w[u][k] >> TAG_SHIFT) == TAG_GEN;
        idx += sg_lanes_below(__ballot(gen));
        ng += gen ? 1u : 0u;
      }
      uint32_t q0 = 0, q1 = 0, q2 = 0;
      if (ng) {
        typedef uint32_t u32x3_t __attribute__((ext_vector_type(3)));
        const u32x3_t q = __builtin_nontemporal_load((const u32x3_t*)((const uint32_t*)G.val + (idx >> 1)));
        q0 = q.x;
        q1 = q.y;
        q2 = q.z;
      }
      uint32_t j = idx & 1u;  // position of the lane's first value in the 12 bytes (16-bit units)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t tag = w[u][k] >> TAG_SHIFT;
        const uint32_t d = j < 2 ? q0 : j < 4 ? q1 : q2;
        v[u][k] = tag == TAG_GEN ? (d >> ((j & 1u) * 16)) & 0xFFFFu : 0u;
        j += tag == TAG_GEN ? 1u : 0u;
        const uint32_t col = cb[u] + (w[u][k] & SG_COL_MASK);
        xv[u][k] = tag != TAG_PAD ? (uint32_t)(GF2 ? x[(int64_t)col * ldx] : x[col]) : 0u;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t tag = w[u][k] >> TAG_SHIFT;
        if (tag != TAG_PAD) {
          const uint32_t row = (w[u][k] >> SG_ROW_SHIFT) & (SG_MAX_ROWS - 1);
          if constexpr (GF2) {  // entries are 1 (with values off, a stored value is odd)
            atomicXor(&accx[row], (tag != TAG_GEN || (v[u][k] & 1u)) ? xv[u][k] : 0u);
          } else {
            // a term is below 2^32: (m-1)^2, x or m - x
            const uint32_t t = tag == TAG_GEN ? v[u][k] * xv[u][k] : tag == TAG_PLUS ? xv[u][k] : G.m - xv[u][k];
            atomicAdd(&acc[row], (unsigned long long)t);
          }
        }
      }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      vo[u] = von[u];
      cb[u] = cbn[u];
#pragma unroll
      for (int k = 0; k < 4; ++k) w[u][k] = wn[u][k];
    }
  }
  __syncthreads();
  if constexpr (GF2) {
    for (uint32_t r = tid; r < g.nrows; r += NT) {
      const uint32_t row = g.row0 + r;
      y[(int64_t)(G.rowmap ? G.rowmap[row] : row) * ldy] = (Tv)accx[r];
    }
    return;
  }
  for (uint32_t r = tid; r < g.nrows; r += NT) {
    const uint32_t row = g.row0 + r;
    Tv* yr = y + (G.rowmap ? G.rowmap[row] : row);
    const uint32_t res = mod_u64(acc[r], G.m, G.mu);
    const uint32_t out = (alpha == 1 && beta == 0) ? res : axpby(alpha, res, beta, beta ? (uint32_t)*yr : 0u, G.m, G.mu);
    *yr = (Tv)out;
    if (y16) y16[G.rowmap ? G.rowmap[row] : row] = (uint16_t)out;  // the next product's 16-bit x
  }
}

// The largest dynamic LDS a group can ask for: SG_MAX_ROWS 64-bit sums.
constexpr size_t SG_LDS_MAX = (size_t)SG_MAX_ROWS * 8;

template <typename Tx, typename Tv, bool GF2 = false>
static hipError_t sg_go(const SgMat& G, const Tx* x, Tv* y, uint32_t alpha, uint32_t beta, uint16_t* y16,
                        hipStream_t st, int64_t ldx = 1, int64_t ldy = 1) {
  const size_t lds = std::max<size_t>((size_t)G.max_rows * 8, SG_LDS_FLOOR);
  auto k = k_sg<Tx, Tv, SG_THREADS, SG_U, GF2>;
  // the kernel's LDS limit is raised once per device to the most any group can need (the
  // attribute is a host call that would otherwise cost a few microseconds per product)
  static std::mutex mu;
  static bool done[64] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  {
    std::lock_guard<std::mutex> lock(mu);
    if (!done[dev]) {
      e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)SG_LDS_MAX);
      if (e != hipSuccess) return e;
      done[dev] = true;
    }
  }
  hipLaunchKernelGGL(k, dim3(G.ngroups), dim3(SG_THREADS), lds, st, G, x, y, alpha, beta, y16, ldx, ldy);
  return hipGetLastError();
}

hipError_t launch_sg(const SgMat& G, ffx_dtype dt, const void* x, const uint16_t* x16, void* y, uint32_t alpha,
                     uint32_t beta, hipStream_t st, uint16_t* y16) {
  if (G.ngroups == 0) return hipSuccess;
  if (dt == FFX_I32) {
    if (x16) return sg_go<uint16_t, int32_t>(G, x16, (int32_t*)y, alpha, beta, y16, st);
    return sg_go<int32_t, int32_t>(G, (const int32_t*)x, (int32_t*)y, alpha, beta, y16, st);
  }
  if (x16) return sg_go<uint16_t, int64_t>(G, x16, (int64_t*)y, alpha, beta, y16, st);
  return sg_go<int64_t, int64_t>(G, (const int64_t*)x, (int64_t*)y, alpha, beta, y16, st);
}

hipError_t launch_sg_gf2(const SgMat& G, const uint32_t* X, int64_t ldx, uint32_t* Y, int64_t ldy, hipStream_t st) {
  if (G.ngroups == 0) return hipSuccess;
  return sg_go<uint32_t, uint32_t, true>(G, X, Y, 1, 0, nullptr, st, ldx, ldy);
}

}  // namespace ffx
