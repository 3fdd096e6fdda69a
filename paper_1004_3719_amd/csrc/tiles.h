// gfx950 kernels for y = alpha*A*X + beta*Y over Z/mZ on the tile table.
//
// One launch covers the whole matrix: workgroup g takes tile g, whatever the
// format of its row block. Three tile shapes:
//   STREAM  up to 256 consecutive rows whose entries are read with fully
//           coalesced 64-entry chunks; for one vector the terms (value times
//           gathered x) go to LDS and each row is summed from LDS by a group
//           of lanes sized to the tile (the CSR-Stream scheme of Greathouse
//           and Daga, SC'14, designed for AMD GPUs); for s > 1 vectors the
//           chunk stages words and values in LDS and each lane sums one row.
//   LONG    one row too long for a STREAM tile: all 256 lanes sweep it and
//           the partial sums meet through shuffles and LDS.
//   SELL    up to 4 slices of 64 rows stored column-major (ELL on a GPU is
//           column-major for coalescing, paper Section 2.4 "Basic formats"),
//           one lane per row, no LDS.
// Every tile may carry a band part: dense diagonals with one value per row,
// applied by one lane per row (the DIA idea of Section 2.1).
//
// Arithmetic (Section 2.2): each lane sums its terms in a wide accumulator
// and reduces modulo m only when the next term could overflow what the type
// represents exactly (CHUNK variants; the host sets reduce_every from the
// bound), otherwise once per row. Entries of residue 1 and m-1 carry no value
// and add x or m - x (Section 2.4, "Taking into account the +-1").
#pragma once

#include "ffx_impl.h"

namespace ffx {

// ------------------------------- arithmetic --------------------------------
// m <= 65536: values in 16 bits, one term (m-1)^2 < 2^32, and no row can have
// enough terms to reach 2^63, so a row is reduced once.
struct ArSmall {
  using ValT = uint16_t;
  using Acc = uint64_t;
  using Prod = uint32_t;
  static constexpr bool CHUNK = false;
  __device__ static inline Prod mul(uint32_t v, uint32_t x) { return v * x; }
  __device__ static inline uint32_t reduce(Acc a, const DevMat& A) { return mod_u64(a, A.m, A.mu); }
  __device__ static inline Acc from_residue(uint32_t r) { return r; }
};
// m > 65536 on 64-bit integers: a term is below 2^62.
template <bool CH>
struct ArBig {
  using ValT = uint32_t;
  using Acc = uint64_t;
  using Prod = uint64_t;
  static constexpr bool CHUNK = CH;
  __device__ static inline Prod mul(uint32_t v, uint32_t x) { return (uint64_t)v * x; }
  __device__ static inline uint32_t reduce(Acc a, const DevMat& A) { return mod_u64(a, A.m, A.mu); }
  __device__ static inline Acc from_residue(uint32_t r) { return r; }
};
// exact doubles: integers up to 2^53 add exactly.
template <typename V, bool CH>
struct ArF64 {
  using ValT = V;
  using Acc = double;
  using Prod = double;
  static constexpr bool CHUNK = CH;
  __device__ static inline Prod mul(uint32_t v, uint32_t x) { return (double)v * (double)x; }
  __device__ static inline uint32_t reduce(Acc a, const DevMat& A) { return mod_f64(a, A.m, A.inv_m); }
  __device__ static inline Acc from_residue(uint32_t r) { return (double)r; }
};

template <class AR>
__device__ inline typename AR::Prod term(uint32_t tag, uint32_t v, uint32_t x, uint32_t m) {
  if (tag == TAG_GEN) return AR::mul(v, x);
  if (tag == TAG_PLUS) return (typename AR::Prod)x;
  if (tag == TAG_MINUS) return (typename AR::Prod)(m - x);
  return (typename AR::Prod)0;
}

// S accumulators of one lane with a shared countdown to the next reduction.
template <class AR, int S>
struct LaneAcc {
  typename AR::Acc a[S];
  int64_t left;
  __device__ inline void init(const DevMat& A) {
#pragma unroll
    for (int c = 0; c < S; ++c) a[c] = 0;
    left = A.reduce_every;
  }
  // called once per term position, after the S terms of that position were added
  __device__ inline void tick(const DevMat& A) {
    if (AR::CHUNK) {
      if (--left == 0) {
#pragma unroll
        for (int c = 0; c < S; ++c) a[c] = AR::from_residue(AR::reduce(a[c], A));
        left = A.reduce_every;
      }
    }
  }
  // before partial sums of several lanes are added together
  __device__ inline void to_residues(const DevMat& A) {
    if (AR::CHUNK) {
#pragma unroll
      for (int c = 0; c < S; ++c) a[c] = AR::from_residue(AR::reduce(a[c], A));
    }
  }
};

// ------------------------------- wave helpers ------------------------------
__device__ inline uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}
__device__ inline uint64_t shfl_xor_u64(uint64_t v, int mask, int width) {
  uint32_t lo = __shfl_xor((int)(uint32_t)v, mask, width);
  uint32_t hi = __shfl_xor((int)(uint32_t)(v >> 32), mask, width);
  return ((uint64_t)hi << 32) | lo;
}
__device__ inline double shfl_xor_acc(double v, int mask, int width) { return __shfl_xor(v, mask, width); }
__device__ inline uint64_t shfl_xor_acc(uint64_t v, int mask, int width) { return shfl_xor_u64(v, mask, width); }

template <typename V>
__device__ inline uint32_t ldval(const void* p, uint32_t i) {
  return (uint32_t)((const V*)p)[i];
}

// Writes row `row` of Y from the residues r[0..s).
template <typename Tv, int S>
__device__ inline void write_row(const DevMat& A, Tv* Y, int64_t ldy, uint32_t row, const uint32_t* r, int s,
                                 uint32_t alpha, uint32_t beta) {
  Tv* yr = Y + (int64_t)row * ldy;
#pragma unroll
  for (int c = 0; c < S; ++c) {
    if (c < s) {
      uint32_t yo = beta ? (uint32_t)yr[c] : 0u;
      uint32_t out = (alpha == 1 && beta == 0) ? r[c] : axpby(alpha, r[c], beta, yo, A.m, A.mu);
      yr[c] = (Tv)out;
    }
  }
}

// Adds the band terms of one row (diagonals d = first, first+step, ...).
template <class AR, typename Tv, int S>
__device__ inline void band_terms(const DevMat& A, const Tile& T, LaneAcc<AR, S>& acc, uint32_t row, uint32_t slot,
                                  uint32_t rows_in_tile, uint32_t first, uint32_t step, const Tv* X, int64_t ldx,
                                  int s) {
  const uint32_t nd = tile_nd(T.kind);
  for (uint32_t d = first; d < nd; d += step) {
    uint32_t v = ldval<typename AR::ValT>(A.bval, T.b0 + d * rows_in_tile + slot);
    if (v) {
      int64_t col = (int64_t)row + A.boffs[T.boff + d];
      const Tv* xr = X + col * ldx;
#pragma unroll
      for (int c = 0; c < S; ++c)
        if (c < s) acc.a[c] += AR::mul(v, (uint32_t)xr[c]);
      acc.tick(A);
    }
  }
}

// ------------------------------- SELL tile ---------------------------------
template <class AR, typename Tv, int S>
__device__ inline void sell_tile(const DevMat& A, const Tile& T, const Tv* __restrict__ X, int64_t ldx,
                                 Tv* __restrict__ Y, int64_t ldy, int s, uint32_t alpha, uint32_t beta) {
  const uint32_t lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
  const uint32_t nsl = T.ne;
  if (wave >= nsl) return;
  uint32_t off = 0;
  for (uint32_t k = 0; k < wave; ++k) off += A.swidth[T.aux + k];
  const uint32_t width = A.swidth[T.aux + wave];
  const uint32_t slot = wave * WAVE + lane;
  uint32_t row = (T.kind & TF_SORTED) ? A.perm[T.row0 + slot] : T.row0 + slot;
  const bool valid = row < A.nrows;
  const uint32_t* ent = A.ent + T.e0 + (size_t)off * WAVE + lane;
  const uint32_t* choff = A.choff + T.c0 + off;
  LaneAcc<AR, S> acc;
  acc.init(A);
  for (uint32_t j = 0; j < width; ++j) {
    uint32_t w = ent[(size_t)j * WAVE];
    uint32_t tag = w >> TAG_SHIFT;
    uint64_t gm = __ballot(tag == TAG_GEN);
    if (tag != TAG_PAD) {
      uint32_t v = tag == TAG_GEN ? ldval<typename AR::ValT>(A.val, choff[j] + lanes_below(gm)) : 0u;
      const Tv* xr = X + (int64_t)(w & COL_MASK) * ldx;
#pragma unroll
      for (int c = 0; c < S; ++c)
        if (c < s) acc.a[c] += term<AR>(tag, v, (uint32_t)xr[c], A.m);
      acc.tick(A);
    }
  }
  if (!valid) return;
  band_terms<AR, Tv, S>(A, T, acc, row, slot, tile_rows(T.kind), 0, 1, X, ldx, s);
  uint32_t r[S];
#pragma unroll
  for (int c = 0; c < S; ++c) r[c] = AR::reduce(acc.a[c], A);
  write_row<Tv, S>(A, Y, ldy, row, r, s, alpha, beta);
}

// ------------------------------- LONG tile ---------------------------------
template <class AR, typename Tv, int S>
__device__ inline void long_tile(const DevMat& A, const Tile& T, const Tv* __restrict__ X, int64_t ldx,
                                 Tv* __restrict__ Y, int64_t ldy, int s, uint32_t alpha, uint32_t beta,
                                 unsigned char* lds) {
  using Acc = typename AR::Acc;
  const uint32_t lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
  const uint32_t nchunks = (T.ne + WAVE - 1) / WAVE;
  LaneAcc<AR, S> acc;
  acc.init(A);
  for (uint32_t ch = wave; ch < nchunks; ch += TILE_THREADS / WAVE) {
    uint32_t k = ch * WAVE + lane;
    uint32_t w = k < T.ne ? A.ent[T.e0 + k] : PAD_WORD;
    uint32_t tag = w >> TAG_SHIFT;
    uint64_t gm = __ballot(tag == TAG_GEN);
    if (tag != TAG_PAD) {
      uint32_t v = tag == TAG_GEN ? ldval<typename AR::ValT>(A.val, A.choff[T.c0 + ch] + lanes_below(gm)) : 0u;
      const Tv* xr = X + (int64_t)(w & COL_MASK) * ldx;
#pragma unroll
      for (int c = 0; c < S; ++c)
        if (c < s) acc.a[c] += term<AR>(tag, v, (uint32_t)xr[c], A.m);
      acc.tick(A);
    }
  }
  band_terms<AR, Tv, S>(A, T, acc, T.row0, 0, 1, threadIdx.x, TILE_THREADS, X, ldx, s);
  acc.to_residues(A);
  Acc* red = (Acc*)lds;  // [4 waves][S]
#pragma unroll
  for (int c = 0; c < S; ++c) {
    Acc v = acc.a[c];
    for (int o = WAVE / 2; o > 0; o >>= 1) v += shfl_xor_acc(v, o, WAVE);
    if (lane == 0) red[wave * S + c] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t r[S];
#pragma unroll
    for (int c = 0; c < S; ++c) {
      Acc t = 0;
      for (int q = 0; q < TILE_THREADS / WAVE; ++q) t += red[q * S + c];
      r[c] = AR::reduce(t, A);
    }
    write_row<Tv, S>(A, Y, ldy, T.row0, r, s, alpha, beta);
  }
}

// ------------------------------- STREAM tile -------------------------------
// one vector: terms to LDS, then groups of lanes per row
template <class AR, typename Tv>
__device__ inline void stream_tile_1(const DevMat& A, const Tile& T, const Tv* __restrict__ X, int64_t ldx,
                                     Tv* __restrict__ Y, int64_t ldy, uint32_t alpha, uint32_t beta,
                                     unsigned char* lds) {
  using Prod = typename AR::Prod;
  using Acc = typename AR::Acc;
  Prod* prod = (Prod*)lds;
  const uint32_t tid = threadIdx.x, lane = tid & (WAVE - 1), wave = tid / WAVE;
  const uint32_t nchunks = (T.ne + WAVE - 1) / WAVE;
  for (uint32_t ch = wave; ch < nchunks; ch += TILE_THREADS / WAVE) {
    uint32_t k = ch * WAVE + lane;
    bool in = k < T.ne;
    uint32_t w = in ? A.ent[T.e0 + k] : PAD_WORD;
    uint32_t tag = w >> TAG_SHIFT;
    uint64_t gm = __ballot(tag == TAG_GEN);
    Prod p = 0;
    if (tag != TAG_PAD) {
      uint32_t v = tag == TAG_GEN ? ldval<typename AR::ValT>(A.val, A.choff[T.c0 + ch] + lanes_below(gm)) : 0u;
      p = term<AR>(tag, v, (uint32_t)X[(int64_t)(w & COL_MASK) * ldx], A.m);
    }
    if (in) prod[k] = p;
  }
  __syncthreads();
  const uint32_t nr = tile_rows(T.kind);
  uint32_t lpr = 1;
  while (lpr < WAVE && lpr * 2 * nr <= TILE_THREADS) lpr <<= 1;
  const uint32_t r = tid / lpr, sub = tid & (lpr - 1);
  const bool active = r < nr;
  LaneAcc<AR, 1> acc;
  acc.init(A);
  if (active) {
    uint32_t kb = A.rowp[T.aux + r] - T.e0, ke = A.rowp[T.aux + r + 1] - T.e0;
    for (uint32_t k = kb + sub; k < ke; k += lpr) {
      acc.a[0] += prod[k];
      acc.tick(A);
    }
    band_terms<AR, Tv, 1>(A, T, acc, T.row0 + r, r, nr, sub, lpr, X, ldx, 1);
  }
  Acc v = acc.a[0];
  if (lpr > 1) {
    acc.to_residues(A);
    v = acc.a[0];
    for (uint32_t o = lpr / 2; o > 0; o >>= 1) v += shfl_xor_acc(v, (int)o, (int)lpr);
  }
  if (active && sub == 0) {
    uint32_t res = AR::reduce(v, A);
    write_row<Tv, 1>(A, Y, ldy, T.row0 + r, &res, 1, alpha, beta);
  }
}

// s > 1 vectors: stage words and values in LDS, one lane per row
template <class AR, typename Tv, int S>
__device__ inline void stream_tile_s(const DevMat& A, const Tile& T, const Tv* __restrict__ X, int64_t ldx,
                                     Tv* __restrict__ Y, int64_t ldy, int s, uint32_t alpha, uint32_t beta,
                                     unsigned char* lds) {
  uint32_t* sw = (uint32_t*)lds;
  uint32_t* sv = sw + T.ne;
  const uint32_t tid = threadIdx.x, lane = tid & (WAVE - 1), wave = tid / WAVE;
  const uint32_t nchunks = (T.ne + WAVE - 1) / WAVE;
  for (uint32_t ch = wave; ch < nchunks; ch += TILE_THREADS / WAVE) {
    uint32_t k = ch * WAVE + lane;
    bool in = k < T.ne;
    uint32_t w = in ? A.ent[T.e0 + k] : PAD_WORD;
    uint32_t tag = w >> TAG_SHIFT;
    uint64_t gm = __ballot(tag == TAG_GEN);
    uint32_t v = tag == TAG_GEN ? ldval<typename AR::ValT>(A.val, A.choff[T.c0 + ch] + lanes_below(gm)) : 0u;
    if (in) {
      sw[k] = w;
      sv[k] = v;
    }
  }
  __syncthreads();
  const uint32_t nr = tile_rows(T.kind);
  if (tid >= nr) return;
  const uint32_t row = T.row0 + tid;
  LaneAcc<AR, S> acc;
  acc.init(A);
  uint32_t kb = A.rowp[T.aux + tid] - T.e0, ke = A.rowp[T.aux + tid + 1] - T.e0;
  for (uint32_t k = kb; k < ke; ++k) {
    uint32_t w = sw[k], tag = w >> TAG_SHIFT, v = sv[k];
    const Tv* xr = X + (int64_t)(w & COL_MASK) * ldx;
#pragma unroll
    for (int c = 0; c < S; ++c)
      if (c < s) acc.a[c] += term<AR>(tag, v, (uint32_t)xr[c], A.m);
    acc.tick(A);
  }
  band_terms<AR, Tv, S>(A, T, acc, row, tid, nr, 0, 1, X, ldx, s);
  uint32_t r[S];
#pragma unroll
  for (int c = 0; c < S; ++c) r[c] = AR::reduce(acc.a[c], A);
  write_row<Tv, S>(A, Y, ldy, row, r, s, alpha, beta);
}

// ------------------------------- the launch --------------------------------
template <class AR, typename Tv, int S>
__global__ __launch_bounds__(TILE_THREADS) void k_tiles(DevMat A, const Tv* __restrict__ X, int64_t ldx,
                                                        Tv* __restrict__ Y, int64_t ldy, int s, uint32_t alpha,
                                                        uint32_t beta) {
  extern __shared__ __align__(16) unsigned char lds[];
  const Tile T = A.tiles[blockIdx.x];
  switch (tile_kind(T.kind)) {
    case TK_SELL: sell_tile<AR, Tv, S>(A, T, X, ldx, Y, ldy, s, alpha, beta); break;
    case TK_LONG: long_tile<AR, Tv, S>(A, T, X, ldx, Y, ldy, s, alpha, beta, lds); break;
    default:
      if (S == 1) stream_tile_1<AR, Tv>(A, T, X, ldx, Y, ldy, alpha, beta, lds);
      else stream_tile_s<AR, Tv, S>(A, T, X, ldx, Y, ldy, s, alpha, beta, lds);
  }
}

// Dynamic LDS of one launch.
template <class AR>
inline size_t tiles_lds_bytes(int64_t max_tile_entries, int S) {
  size_t stream = (size_t)max_tile_entries * (S == 1 ? sizeof(typename AR::Prod) : 8);
  size_t red = (size_t)(TILE_THREADS / WAVE) * S * sizeof(typename AR::Acc);
  size_t b = stream > red ? stream : red;
  return b < 16 ? 16 : b;
}

template <class AR, typename Tv>
hipError_t launch_tiles_t(const DevMat& A, int64_t max_tile_entries, const void* X, int64_t ldx, void* Y, int64_t ldy,
                          int s, uint32_t alpha, uint32_t beta, hipStream_t st) {
  if (A.ntiles == 0) return hipSuccess;
  const int S = s <= 1 ? 1 : s <= 2 ? 2 : s <= 4 ? 4 : s <= 8 ? 8 : 16;
  size_t lds = tiles_lds_bytes<AR>(max_tile_entries, S);
  dim3 grid(A.ntiles), block(TILE_THREADS);
  const Tv* x = (const Tv*)X;
  Tv* y = (Tv*)Y;
  switch (S) {
    case 1: hipLaunchKernelGGL((k_tiles<AR, Tv, 1>), grid, block, lds, st, A, x, ldx, y, ldy, s, alpha, beta); break;
    case 2: hipLaunchKernelGGL((k_tiles<AR, Tv, 2>), grid, block, lds, st, A, x, ldx, y, ldy, s, alpha, beta); break;
    case 4: hipLaunchKernelGGL((k_tiles<AR, Tv, 4>), grid, block, lds, st, A, x, ldx, y, ldy, s, alpha, beta); break;
    case 8: hipLaunchKernelGGL((k_tiles<AR, Tv, 8>), grid, block, lds, st, A, x, ldx, y, ldy, s, alpha, beta); break;
    default: hipLaunchKernelGGL((k_tiles<AR, Tv, 16>), grid, block, lds, st, A, x, ldx, y, ldy, s, alpha, beta); break;
  }
  return hipGetLastError();
}

}  // namespace ffx
