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
//
// One launch per iteration i, as for residues: workgroup t < ntiles computes
// its tile's rows of W_{i+1} = A W_i (the product's tile code) and then the
// XOR over those rows of its share of U^T W_{i+1}, a partial of 32w*w words;
// GF2_NMID workgroups fold the partials of W_i (written by the previous launch)
// into GF2_NMID words per pair, and one workgroup folds those of iteration
// i-1 into S_{i-1}. Partials and folds are double-buffered by parity.
namespace ffx {

constexpr uint32_t GF2_NMID = 64;

struct Gf2SeqArgs {
  const uint32_t* U;   // n x w words
  uint32_t* W[2];      // W_i in W[i & 1]; n x w words
  uint32_t* part[2];   // [ntiles][npairs], by parity
  uint32_t* mid[2];    // [GF2_NMID][npairs], by parity
  uint32_t* S;         // L x npairs
  uint32_t* Wlast;     // W_L (or null)
  int64_t L;
  int32_t w;
};

// Row of slot q of a tile (>= nrows for a padding slot).
__device__ inline uint32_t gf2_tile_row(const DevMat& A, const Tile& T, uint32_t q) {
  return (tile_kind(T.kind) == TK_SELL && (T.kind & TF_SORTED)) ? A.perm[T.row0 + q] : T.row0 + q;
}

// out[p] for the pairs p = a*w + c: XOR over the tile's rows of (bit a of U[row]) * W[row][c]. The
// tile's rows of U and W are staged in LDS first (sh: 2 * 256 * w words, then 256 for the groups).
__device__ inline void tile_projection_gf2(const DevMat& A, const Tile& T, const uint32_t* __restrict__ U,
                                           const uint32_t* W, int w, uint32_t* sh, uint32_t* __restrict__ out) {
  const int tid = threadIdx.x, npairs = 32 * w * w;
  const int nq = tile_kind(T.kind) == TK_LONG ? 1 : (int)tile_rows(T.kind);
  uint32_t* su = sh;
  uint32_t* sw = sh + TILE_THREADS * w;
  uint32_t* red = sw + TILE_THREADS * w;
  for (int k = tid; k < nq * w; k += TILE_THREADS) {
    const uint32_t row = gf2_tile_row(A, T, (uint32_t)(k / w));
    const int c = k % w;
    const bool ok = row < A.nrows;
    su[k] = ok ? U[(int64_t)row * w + c] : 0u;
    sw[k] = ok ? W[(int64_t)row * w + c] : 0u;
  }
  __syncthreads();
  if (npairs <= TILE_THREADS) {
    const int ngrp = TILE_THREADS / npairs, grp = tid / npairs, p = tid % npairs;
    const int a = p / w, c = p - a * w, ua = a >> 5, ub = a & 31;
    uint32_t acc = 0;
    if (grp < ngrp)
      for (int q = grp; q < nq; q += ngrp) acc ^= (0u - ((su[q * w + ua] >> ub) & 1u)) & sw[q * w + c];
    red[tid] = grp < ngrp ? acc : 0u;
    __syncthreads();
    if (tid < npairs) {
      uint32_t x = 0;
      for (int g = 0; g < ngrp; ++g) x ^= red[g * npairs + tid];
      out[tid] = x;
    }
  } else {
    for (int p = tid; p < npairs; p += TILE_THREADS) {
      const int a = p / w, c = p - a * w, ua = a >> 5, ub = a & 31;
      uint32_t acc = 0;
      for (int q = 0; q < nq; ++q) acc ^= (0u - ((su[q * w + ua] >> ub) & 1u)) & sw[q * w + c];
      out[p] = acc;
    }
  }
}

// LDS of tile_projection_gf2.
inline size_t gf2_projection_lds(int w) { return (size_t)(2 * TILE_THREADS * w + TILE_THREADS) * sizeof(uint32_t); }

// XOR of part[g][p] over g = first, first + stride, ... < nparts, for every pair p.
__device__ inline void fold_xor(const uint32_t* __restrict__ part, uint32_t first, uint32_t stride, uint32_t nparts,
                                int npairs, uint32_t* __restrict__ out) {
  for (int p = threadIdx.x; p < npairs; p += TILE_THREADS) {
    uint32_t x = 0;
    for (uint32_t g = first; g < nparts; g += stride) x ^= part[(int64_t)g * npairs + p];
    out[p] = x;
  }
}

// Partials of W_0 = V.
__global__ __launch_bounds__(TILE_THREADS) void k_seq_first_gf2(DevMat A, Gf2SeqArgs q) {
  extern __shared__ __align__(16) unsigned char lds[];
  const Tile T = A.tiles[blockIdx.x];
  tile_projection_gf2(A, T, q.U, q.W[0], q.w, (uint32_t*)lds, q.part[0] + (int64_t)blockIdx.x * 32 * q.w * q.w);
}

template <int S>
__global__ __launch_bounds__(TILE_THREADS) void k_seq_step_gf2(DevMat A, Gf2SeqArgs q, int64_t i) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int w = q.w, npairs = 32 * w * w;
  const uint32_t nt = A.ntiles;
  if (blockIdx.x >= nt) {
    const uint32_t r = blockIdx.x - nt;
    if (r < GF2_NMID) fold_xor(q.part[i & 1], r, GF2_NMID, nt, npairs, q.mid[i & 1] + (int64_t)r * npairs);
    else if (i > 0) fold_xor(q.mid[(i - 1) & 1], 0, 1, GF2_NMID, npairs, q.S + (i - 1) * (int64_t)npairs);
    return;
  }
  const bool last = i + 1 == q.L;
  if (last && !q.Wlast) return;
  const int32_t* X = (const int32_t*)q.W[i & 1];
  int32_t* Y = (int32_t*)(last ? q.Wlast : q.W[(i + 1) & 1]);
  const Tile T = A.tiles[blockIdx.x];
  switch (tile_kind(T.kind)) {
    case TK_SELL: sell_tile_rc<ArGF2, int32_t, int32_t, S>(A, T, X, w, Y, w, w, 1, 0); break;
    case TK_LONG: long_tile<ArGF2, int32_t, int32_t, S, 1>(A, T, X, w, Y, w, w, 1, 0, lds); break;
    default: stream_tile_s<ArGF2, int32_t, int32_t, S>(A, T, X, w, Y, w, w, 1, 0, lds);
  }
  if (last) return;  // W_L only
  // the projection reads back only rows this workgroup wrote: a workgroup barrier orders them
  __syncthreads();
  tile_projection_gf2(A, T, q.U, (const uint32_t*)Y, w, (uint32_t*)lds,
                      q.part[(i + 1) & 1] + (int64_t)blockIdx.x * npairs);
}

// S_{L-1} from the folds of the last iteration.
__global__ __launch_bounds__(TILE_THREADS) void k_seq_finish_gf2(Gf2SeqArgs q) {
  const int npairs = 32 * q.w * q.w;
  fold_xor(q.mid[(q.L - 1) & 1], 0, 1, GF2_NMID, npairs, q.S + (q.L - 1) * (int64_t)npairs);
}

size_t gf2_sequence_part_words(const DevMat& A, int w) {
  return 2 * ((size_t)(A.ntiles > 0 ? A.ntiles : 1) + GF2_NMID) * 32 * w * w;
}

hipError_t launch_sequence_gf2(const DevMat& A, int64_t mte, int w, const uint32_t* U, const uint32_t* W0, int64_t L,
                               uint32_t* S, uint32_t* w1, uint32_t* part, uint32_t* Wlast, hipStream_t st) {
  if (L <= 0) return hipSuccess;
  if (A.ntiles == 0) return hipErrorInvalidValue;  // every row lies in a tile, so n > 0 means tiles
  const int npairs = 32 * w * w;
  const size_t pw = (size_t)(A.ntiles > 0 ? A.ntiles : 1) * npairs, mw = (size_t)GF2_NMID * npairs;
  Gf2SeqArgs q;
  q.U = U;
  q.W[0] = const_cast<uint32_t*>(W0);
  q.W[1] = w1;
  q.part[0] = part;
  q.part[1] = part + pw;
  q.mid[0] = part + 2 * pw;
  q.mid[1] = part + 2 * pw + mw;
  q.S = S;
  q.Wlast = Wlast;
  q.L = L;
  q.w = w;
  const int S_ = w <= 2 ? 2 : w <= 4 ? 4 : w <= 8 ? 8 : 16;  // the multi-vector tiles, as for residues
  size_t lds = tiles_lds_bytes<ArGF2>(mte, S_);
  const size_t plds = gf2_projection_lds(w);
  if (lds < plds) lds = plds;
  hipLaunchKernelGGL(k_seq_first_gf2, dim3(A.ntiles), dim3(TILE_THREADS), plds, st, A, q);
  const dim3 g(A.ntiles + GF2_NMID + 1), b(TILE_THREADS);
  for (int64_t i = 0; i < L; ++i) {
    switch (S_) {
      case 2: hipLaunchKernelGGL((k_seq_step_gf2<2>), g, b, lds, st, A, q, i); break;
      case 4: hipLaunchKernelGGL((k_seq_step_gf2<4>), g, b, lds, st, A, q, i); break;
      case 8: hipLaunchKernelGGL((k_seq_step_gf2<8>), g, b, lds, st, A, q, i); break;
      default: hipLaunchKernelGGL((k_seq_step_gf2<16>), g, b, lds, st, A, q, i); break;
    }
  }
  hipLaunchKernelGGL(k_seq_finish_gf2, dim3(1), dim3(TILE_THREADS), 0, st, q);
  return hipGetLastError();
}

}  // namespace ffx
