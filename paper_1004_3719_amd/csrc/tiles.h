// gfx950 kernels for Y = alpha*A*X + beta*Y over Z/mZ on the tile table.
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
// Latency: a lane issues the loads of U chunks (entry words, then values and
// gathers) before it uses any of them, and the band part and row pointers,
// which do not depend on the entry stream, are loaded before it.
//
// Arithmetic (Section 2.2): each lane sums its terms in a wide accumulator
// and reduces modulo m only when the next term could overflow what the type
// represents exactly (CHUNK variants; the host sets reduce_every from the
// bound), otherwise once per row. Entries of residue 1 and m-1 carry no value
// and add x or m - x (Section 2.4, "Taking into account the +-1").
//
// Tx is the element type read from X (int32, int64, or a 16-bit copy of x
// when m <= 65536), Tv the element type of Y.
#pragma once

#include <algorithm>

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
  static constexpr bool CENTERED = false;
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
  static constexpr bool CENTERED = false;
  __device__ static inline Prod mul(uint32_t v, uint32_t x) { return (uint64_t)v * x; }
  __device__ static inline uint32_t reduce(Acc a, const DevMat& A) { return mod_u64(a, A.m, A.mu); }
  __device__ static inline Acc from_residue(uint32_t r) { return r; }
};
// m = 2^31 - 1: since 2^31 = 1 (mod m), a product below 2^62 folds below
// 2^32 with one shift and one add, so a row needs no reduction inside it (a
// row of at most 2^30 + 64 folded terms stays below 2^63).
struct ArM31 {
  using ValT = uint32_t;
  using Acc = uint64_t;
  using Prod = uint64_t;
  static constexpr bool CHUNK = false;
  static constexpr bool CENTERED = false;
  static constexpr uint64_t M = 0x7FFFFFFFull;
  __device__ static inline Prod mul(uint32_t v, uint32_t x) {
    uint64_t p = (uint64_t)v * x;
    return (p & M) + (p >> 31);
  }
  __device__ static inline uint32_t reduce(Acc a, const DevMat&) {
    a = (a & M) + (a >> 31);  // below 2^32 + 2^31 for a < 2^63
    a = (a & M) + (a >> 31);  // at most M + 2
    return (uint32_t)(a >= M ? a - M : a);
  }
  __device__ static inline Acc from_residue(uint32_t r) { return r; }
};
// GF(2) with bit-packed blocks: every 32-bit word of X holds bit j of 32
// vectors, an entry of A is 1 (m = 2 keeps only residue 1), and a sum over GF(2)
// is an exclusive or, so one word operation adds 32 products. The accumulator
// type makes + an exclusive or, so the tile code runs unchanged.
struct Gf2 {
  uint32_t v;
  Gf2() = default;
  __host__ __device__ Gf2(uint32_t x) : v(x) {}
  __device__ Gf2& operator+=(Gf2 o) {
    v ^= o.v;
    return *this;
  }
  __device__ Gf2 operator+(Gf2 o) const { return Gf2(v ^ o.v); }
};
using ::atomicAdd;  // the overload below must not hide the runtime's
__device__ inline void atomicAdd(Gf2* p, Gf2 x) { atomicXor(&p->v, x.v); }
struct ArGF2 {
  using ValT = uint16_t;
  using Acc = Gf2;
  using Prod = Gf2;
  static constexpr bool CHUNK = false;
  static constexpr bool CENTERED = false;
  __device__ static inline Prod mul(uint32_t v, uint32_t x) { return Gf2((v & 1u) ? x : 0u); }
  __device__ static inline uint32_t reduce(Acc a, const DevMat&) { return a.v; }
  __device__ static inline Acc from_residue(uint32_t r) { return Gf2(r); }
};
// exact doubles: integers up to 2^53 add exactly.
template <typename V, bool CH>
struct ArF64 {
  using ValT = V;
  using Acc = double;
  using Prod = double;
  static constexpr bool CHUNK = CH;
  static constexpr bool CENTERED = false;
  __device__ static inline Prod mul(uint32_t v, uint32_t x) { return (double)v * (double)x; }
  __device__ static inline uint32_t reduce(Acc a, const DevMat& A) { return mod_f64(a, A.m, A.inv_m); }
  __device__ static inline Acc from_residue(uint32_t r) { return (double)r; }
};

// exact floats: integers up to 2^24 add exactly (m <= 4096, values in 16 bits).
template <bool CH>
struct ArF32 {
  using ValT = uint16_t;
  using Acc = float;
  using Prod = float;
  static constexpr bool CHUNK = CH;
  static constexpr bool CENTERED = false;
  __device__ static inline Prod mul(uint32_t v, uint32_t x) { return (float)v * (float)x; }
  __device__ static inline uint32_t reduce(Acc a, const DevMat& A) { return mod_f32(a, A.m, A.inv_mf); }
  __device__ static inline Acc from_residue(uint32_t r) { return (float)r; }
};
// Centered residues (Section 2.2): a residue r is used as r - m when r > m/2,
// so every operand lies in [-h, h], h = floor(m/2), a product is at most h^2
// (about a quarter of (m-1)^2) in magnitude, and sums of both signs use the
// whole symmetric range of the floating type: about four times as many
// terms between reductions, and fp32 holds one product up to m = 8191. The
// stored entries and x stay canonical; operands are centered as they are
// used, partial reductions keep accumulators centered, and the final one
// returns the canonical residue.
template <typename F, typename V, bool CH>
struct ArCentered {
  using ValT = V;
  using Acc = F;
  using Prod = F;
  static constexpr bool CHUNK = CH;
  static constexpr bool CENTERED = true;
  __device__ static inline F lift(uint32_t r, uint32_t m) { return (F)(int32_t)(r > (m >> 1) ? r - m : r); }
  __device__ static inline F crem(F a, const DevMat& A) {
    if constexpr (sizeof(F) == 4) return crem_f32(a, A.m, A.inv_mf);
    else return crem_f64(a, A.m, A.inv_m);
  }
  __device__ static inline uint32_t reduce(Acc a, const DevMat& A) {
    F r = crem(a, A);
    return (uint32_t)(int32_t)(r < 0 ? r + (F)A.m : r);
  }
};

// one term v*x (the +-1 entries pass x or m - x), and a partial reduction
// that keeps an accumulator in the class's representation
template <class AR>
__device__ inline typename AR::Prod lift(uint32_t r, uint32_t m) {
  if constexpr (AR::CENTERED) return AR::lift(r, m);
  else return (typename AR::Prod)r;
}
template <class AR>
__device__ inline typename AR::Prod mul_term(uint32_t v, uint32_t x, uint32_t m) {
  if constexpr (AR::CENTERED) return AR::lift(v, m) * AR::lift(x, m);
  else return AR::mul(v, x);
}
template <class AR>
__device__ inline typename AR::Acc renorm(typename AR::Acc a, const DevMat& A) {
  if constexpr (AR::CENTERED) return AR::crem(a, A);
  else return AR::from_residue(AR::reduce(a, A));
}
template <class AR>
__device__ inline typename AR::Prod term(uint32_t tag, uint32_t v, uint32_t x, uint32_t m) {
  if (tag == TAG_GEN) return mul_term<AR>(v, x, m);
  if (tag == TAG_PLUS) return lift<AR>(x, m);
  if (tag == TAG_MINUS) return lift<AR>(m - x, m);
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
        for (int c = 0; c < S; ++c) a[c] = renorm<AR>(a[c], A);
        left = A.reduce_every;
      }
    }
  }
  // before partial sums of several lanes are added together
  __device__ inline void to_residues(const DevMat& A) {
    if (AR::CHUNK) {
#pragma unroll
      for (int c = 0; c < S; ++c) a[c] = renorm<AR>(a[c], A);
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
__device__ inline float shfl_xor_acc(float v, int mask, int width) { return __shfl_xor(v, mask, width); }
__device__ inline uint64_t shfl_xor_acc(uint64_t v, int mask, int width) { return shfl_xor_u64(v, mask, width); }
__device__ inline Gf2 shfl_xor_acc(Gf2 v, int mask, int width) { return Gf2((uint32_t)__shfl_xor((int)v.v, mask, width)); }

// stored values are streamed once: non-temporal loads keep them out of the way of x in L2
template <typename V>
__device__ inline uint32_t ldval(const void* p, uint32_t i) {
  return (uint32_t)__builtin_nontemporal_load((const V*)p + i);
}

// Writes row `row` of Y from the residues r[0..s).
template <typename Tv, int S>
__device__ inline void write_row(const DevMat& A, Tv* Y, int64_t ldy, uint32_t row, const uint32_t* r, int s,
                                 uint32_t alpha, uint32_t beta) {
  Tv* yr = Y + (int64_t)(A.rowmap ? A.rowmap[row] : row) * ldy;
#pragma unroll
  for (int c = 0; c < S; ++c) {
    if (c < s) {
      uint32_t yo = beta ? (uint32_t)yr[c] : 0u;
      uint32_t out = (alpha == 1 && beta == 0) ? r[c] : axpby(alpha, r[c], beta, yo, A.m, A.mu);
      yr[c] = (Tv)out;
    }
  }
}

// Adds the band terms of one row (diagonals d = first, first+step, ...). The
// x address depends only on the row and the offset, never on the stored value
// (absent entries hold 0), so all loads of a batch are issued together.
// Diagonals per batch: 16 gathers in flight per lane whatever S (more would
// only cost registers).
template <int S>
constexpr int band_batch() { return S >= 16 ? 1 : 16 / S > 8 ? 8 : 16 / S; }
template <class AR, typename Tx, int S>
__device__ inline void band_terms(const DevMat& A, const Tile& T, LaneAcc<AR, S>& acc, uint32_t row, uint32_t slot,
                                  uint32_t rows_in_tile, uint32_t first, uint32_t step, const Tx* X, int64_t ldx,
                                  int s) {
  constexpr int BAND_BATCH = band_batch<S>();
  const uint32_t nd = tile_nd(T.kind);
  for (uint32_t d0 = first; d0 < nd; d0 += BAND_BATCH * step) {
    uint32_t v[BAND_BATCH];
    uint32_t xv[BAND_BATCH][S];
#pragma unroll
    for (int q = 0; q < BAND_BATCH; ++q) {
      uint32_t d = d0 + q * step;
      bool in = d < nd;
      v[q] = in ? ldval<typename AR::ValT>(A.bval, T.b0 + d * rows_in_tile + slot) : 0u;
      int64_t col = in ? (int64_t)row + A.boffs[T.boff + d] : -1;
      bool ok = col >= 0 && col < (int64_t)A.ncols;
      const Tx* xr = X + (ok ? col : 0) * ldx;
#pragma unroll
      for (int c = 0; c < S; ++c) xv[q][c] = (ok && c < s) ? (uint32_t)xr[c] : 0u;
    }
#pragma unroll
    for (int q = 0; q < BAND_BATCH; ++q) {
      if (d0 + q * step < nd) {
#pragma unroll
        for (int c = 0; c < S; ++c) acc.a[c] += mul_term<AR>(v[q], xv[q][c], A.m);
        acc.tick(A);
      }
    }
  }
}

// Index of the first general value of this lane's four entry words w
// (entries 4*lane .. 4*lane+3 of a chunk whose value offset is vo). Values
// follow the entry order, so the lane's general values are consecutive, after
// those of lower lanes (four ballots over the wave).
__device__ inline uint32_t value_index4(const uint32_t* w, uint32_t vo) {
  uint32_t idx = vo;
#pragma unroll
  for (int k = 0; k < WIDE; ++k) idx += lanes_below(__ballot((w[k] >> TAG_SHIFT) == TAG_GEN));
  return idx;
}

// The general values of four entry words w whose first value is at index idx:
// one 12-byte (16-bit values) or 16-byte load fetches them all. Per lane: any
// lane may load the values of any row once it holds that row's words and index.
template <class AR>
__device__ inline void load_values_at(const DevMat& A, const uint32_t* w, uint32_t idx, uint32_t* v) {
  uint32_t g = 0;
#pragma unroll
  for (int k = 0; k < WIDE; ++k) g += (w[k] >> TAG_SHIFT) == TAG_GEN ? 1u : 0u;
  uint32_t q0 = 0, q1 = 0, q2 = 0, q3 = 0, j = 0;
  if constexpr (sizeof(typename AR::ValT) == 2) {
    if (g) {
      const uint32_t* p = (const uint32_t*)A.val + (idx >> 1);
      q0 = __builtin_nontemporal_load(p);
      q1 = __builtin_nontemporal_load(p + 1);
      q2 = __builtin_nontemporal_load(p + 2);
    }
    j = idx & 1u;
  } else {
    if (g) {
      const uint32_t* p = (const uint32_t*)A.val + idx;
      q0 = __builtin_nontemporal_load(p);
      q1 = __builtin_nontemporal_load(p + 1);
      q2 = __builtin_nontemporal_load(p + 2);
      q3 = __builtin_nontemporal_load(p + 3);
    }
  }
#pragma unroll
  for (int k = 0; k < WIDE; ++k) {
    bool gen = (w[k] >> TAG_SHIFT) == TAG_GEN;
    uint32_t val;
    if constexpr (sizeof(typename AR::ValT) == 2) {
      uint32_t d = j < 2 ? q0 : j < 4 ? q1 : q2;
      val = (d >> ((j & 1u) * 16)) & 0xffffu;
    } else {
      val = j == 0 ? q0 : j == 1 ? q1 : j == 2 ? q2 : q3;
    }
    v[k] = gen ? val : 0u;
    j += gen ? 1u : 0u;
  }
}

// Values of the four entry words w of this lane (entries 4*lane .. 4*lane+3
// of a chunk whose value offset is vo).
template <class AR>
__device__ inline void load_values4(const DevMat& A, const uint32_t* w, uint32_t vo, uint32_t* v) {
  load_values_at<AR>(A, w, value_index4(w, vo), v);
}

// U chunks of 256 entries, 4 words (16 bytes) per lane: the chunks of STREAM
// and LONG tiles, and the 4-column groups of SELL slices (where the 4 words of
// a lane are 4 consecutive entries of its row).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
template <class AR, typename Tx, int S, int U>
struct Chunk4 {
  uint32_t w[U][WIDE];
  uint32_t vo[U];
  uint32_t v[U][WIDE];
  uint32_t xv[U][WIDE][S];
  // step 1: at(u): this lane's 16-byte word group in chunk u, or null
  template <class At, class ChOff>
  __device__ inline void load_words(At at, ChOff choff_at) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const u32x4* p = at(u);
      u32x4 q = p ? __builtin_nontemporal_load(p) : (u32x4)(PAD_WORD);
      w[u][0] = q.x;
      w[u][1] = q.y;
      w[u][2] = q.z;
      w[u][3] = q.w;
      vo[u] = choff_at(u);
    }
  }
  // step 2: values and gathered x
  __device__ inline void load_gathers(const DevMat& A, const Tx* X, int64_t ldx, int s) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      load_values4<AR>(A, w[u], vo[u], v[u]);
#pragma unroll
      for (int k = 0; k < WIDE; ++k) {
        const uint32_t tag = w[u][k] >> TAG_SHIFT;
        const Tx* xr = X + (int64_t)(w[u][k] & COL_MASK) * ldx;
#pragma unroll
        for (int c = 0; c < S; ++c) xv[u][k][c] = (tag != TAG_PAD && c < s) ? (uint32_t)xr[c] : 0u;
      }
    }
  }
  __device__ inline void accumulate(const DevMat& A, LaneAcc<AR, S>& acc, int s) const {
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < WIDE; ++k) {
        uint32_t tag = w[u][k] >> TAG_SHIFT;
        if (tag != TAG_PAD) {
#pragma unroll
          for (int c = 0; c < S; ++c)
            if (c < s) acc.a[c] += term<AR>(tag, v[u][k], xv[u][k][c], A.m);
          acc.tick(A);
        }
      }
  }
};

// ------------------------------- SELL tile ---------------------------------
// A slice stores its rows in groups of 4 columns: group g is 256 words, word
// 4*lane + k being entry 4g + k of the slice's row `lane`; swidth holds the
// number of groups of each slice.
template <class AR, typename Tx, typename Tv, int S, int U>
__device__ inline void sell_tile(const DevMat& A, const Tile& T, const Tx* __restrict__ X, int64_t ldx,
                                 Tv* __restrict__ Y, int64_t ldy, int s, uint32_t alpha, uint32_t beta) {
  const uint32_t lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
  const uint32_t nsl = T.ne;
  if (wave >= nsl) return;
  uint32_t off = 0;
  for (uint32_t k = 0; k < wave; ++k) off += A.swidth[T.aux + k];
  const uint32_t groups = A.swidth[T.aux + wave];
  const uint32_t slot = wave * WAVE + lane;
  uint32_t row = (T.kind & TF_SORTED) ? A.perm[T.row0 + slot] : T.row0 + slot;
  const bool valid = row < A.nrows;
  const uint32_t* ent = A.ent + T.e0 + (size_t)off * SELL_GROUP + lane * WIDE;
  const uint32_t* choff = A.choff + T.c0 + off;
  auto words = [&](Chunk4<AR, Tx, S, U>& b, uint32_t g0) {
    b.load_words(
        [&](int u) -> const u32x4* {
          return g0 + u < groups ? (const u32x4*)(ent + (size_t)(g0 + u) * SELL_GROUP) : nullptr;
        },
        [&](int u) -> uint32_t { return g0 + u < groups ? choff[g0 + u] : 0u; });
  };
  // the first batch of entry words is requested before the band part, whose
  // loads then overlap its latency
  Chunk4<AR, Tx, S, U> first;
  words(first, 0);
  LaneAcc<AR, S> acc;
  acc.init(A);
  if (valid) band_terms<AR, Tx, S>(A, T, acc, row, slot, tile_rows(T.kind), 0, 1, X, ldx, s);
  first.load_gathers(A, X, ldx, s);  // groups past the last hold padding words and add nothing
  first.accumulate(A, acc, s);
  for (uint32_t g0 = U; g0 < groups; g0 += U) {
    Chunk4<AR, Tx, S, U> b;
    words(b, g0);
    b.load_gathers(A, X, ldx, s);
    b.accumulate(A, acc, s);
  }
  if (!valid) return;
  uint32_t r[S];
#pragma unroll
  for (int c = 0; c < S; ++c) r[c] = AR::reduce(acc.a[c], A);
  write_row<Tv, S>(A, Y, ldy, row, r, s, alpha, beta);
}

// SELL with s > 1 vectors: lane (r, c) of a pass handles component c of row
// r, so the S lanes of one row gather one contiguous piece of X (one cache
// line for s = 8 int64) instead of S separate lookups per lane. The entry
// words and values of each row are loaded once per 4-column group with lane =
// row and broadcast to the pass lanes with shuffles.
template <class AR, typename Tx, typename Tv, int S>
__device__ inline void sell_tile_rc(const DevMat& A, const Tile& T, const Tx* __restrict__ X, int64_t ldx,
                                    Tv* __restrict__ Y, int64_t ldy, int s, uint32_t alpha, uint32_t beta) {
  constexpr int RPW = WAVE / S;                       // rows per pass; S passes cover the slice
  constexpr int KB = S >= 16 ? 1 : S >= 8 ? 2 : WIDE;  // group columns per batch: 16 gathers in flight
  const uint32_t lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
  const uint32_t nsl = T.ne;
  if (wave >= nsl) return;
  uint32_t off = 0;
  for (uint32_t k = 0; k < wave; ++k) off += A.swidth[T.aux + k];
  const uint32_t groups = A.swidth[T.aux + wave];
  const uint32_t comp = lane % S, sub = lane / S;
  const bool cok = (int)comp < s;
  const uint32_t* ent = A.ent + T.e0 + (size_t)off * SELL_GROUP + lane * WIDE;
  const uint32_t* choff = A.choff + T.c0 + off;
  uint32_t prow[S];  // row of each pass
#pragma unroll
  for (int p = 0; p < S; ++p) {
    uint32_t slot = wave * WAVE + p * RPW + sub;
    prow[p] = (T.kind & TF_SORTED) ? A.perm[T.row0 + slot] : T.row0 + slot;
  }
  LaneAcc<AR, S> acc;  // acc.a[p]: pass p
  acc.init(A);
  // band part
  const uint32_t nd = tile_nd(T.kind), rows_in_tile = tile_rows(T.kind);
  for (uint32_t d = 0; d < nd; ++d) {
    const int32_t o = A.boffs[T.boff + d];
#pragma unroll
    for (int p = 0; p < S; ++p) {
      uint32_t slot = wave * WAVE + p * RPW + sub;
      int64_t col = (int64_t)prow[p] + o;
      bool ok = prow[p] < A.nrows && col >= 0 && col < (int64_t)A.ncols && cok;
      uint32_t v = ok ? ldval<typename AR::ValT>(A.bval, T.b0 + d * rows_in_tile + slot) : 0u;
      uint32_t x = ok ? (uint32_t)X[col * ldx + comp] : 0u;
      acc.a[p] += mul_term<AR>(v, x, A.m);
    }
    acc.tick(A);
  }
  for (uint32_t g = 0; g < groups; ++g) {
    uint32_t w[WIDE], v[WIDE];
    {
      u32x4 q = __builtin_nontemporal_load((const u32x4*)(ent + (size_t)g * SELL_GROUP));
      w[0] = q.x;
      w[1] = q.y;
      w[2] = q.z;
      w[3] = q.w;
    }
    load_values4<AR>(A, w, choff[g], v);
#pragma unroll
    for (int k0 = 0; k0 < WIDE; k0 += KB) {
      // every gather of the batch is issued before the first term is added
      uint32_t xv[KB][S];
#pragma unroll
      for (int k = 0; k < KB; ++k)
#pragma unroll
        for (int p = 0; p < S; ++p) {
          uint32_t wp = (uint32_t)__shfl((int)w[k0 + k], p * RPW + (int)sub);
          xv[k][p] = ((wp >> TAG_SHIFT) != TAG_PAD && cok) ? (uint32_t)X[(int64_t)(wp & COL_MASK) * ldx + comp] : 0u;
        }
#pragma unroll
      for (int k = 0; k < KB; ++k) {
#pragma unroll
        for (int p = 0; p < S; ++p) {
          int src = p * RPW + (int)sub;
          uint32_t wp = (uint32_t)__shfl((int)w[k0 + k], src), vp = (uint32_t)__shfl((int)v[k0 + k], src);
          acc.a[p] += term<AR>(wp >> TAG_SHIFT, vp, xv[k][p], A.m);
        }
        acc.tick(A);
      }
    }
  }
#pragma unroll
  for (int p = 0; p < S; ++p) {
    if (prow[p] < A.nrows && cok) {
      uint32_t r = AR::reduce(acc.a[p], A);
      Tv* yr = Y + (int64_t)(A.rowmap ? A.rowmap[prow[p]] : prow[p]) * ldy + comp;
      uint32_t yo = beta ? (uint32_t)*yr : 0u;
      *yr = (Tv)((alpha == 1 && beta == 0) ? r : axpby(alpha, r, beta, yo, A.m, A.mu));
    }
  }
}

// ------------------------------- LONG tile ---------------------------------
template <class AR, typename Tx, typename Tv, int S, int U>
__device__ inline void long_tile(const DevMat& A, const Tile& T, const Tx* __restrict__ X, int64_t ldx,
                                 Tv* __restrict__ Y, int64_t ldy, int s, uint32_t alpha, uint32_t beta,
                                 unsigned char* lds) {
  using Acc = typename AR::Acc;
  constexpr uint32_t NW = TILE_THREADS / WAVE;
  const uint32_t lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
  const uint32_t nchunks = (T.ne + WCHUNK - 1) / WCHUNK;
  LaneAcc<AR, S> acc;
  acc.init(A);
  band_terms<AR, Tx, S>(A, T, acc, T.row0, 0, 1, threadIdx.x, TILE_THREADS, X, ldx, s);
  auto words = [&](Chunk4<AR, Tx, S, U>& b, uint32_t ch0) {
    b.load_words(
        [&](int u) -> const u32x4* {
          uint32_t ch = ch0 + u * NW, k = ch * WCHUNK + lane * WIDE;
          return (ch < nchunks && k < T.ne) ? (const u32x4*)(A.ent + T.e0 + k) : nullptr;
        },
        [&](int u) -> uint32_t {
          uint32_t ch = ch0 + u * NW;
          return ch < nchunks ? A.choff[T.c0 + ch] : 0u;
        });
  };
  for (uint32_t ch0 = wave; ch0 < nchunks; ch0 += NW * U) {
    Chunk4<AR, Tx, S, U> b;
    words(b, ch0);
    b.load_gathers(A, X, ldx, s);
    b.accumulate(A, acc, s);
  }
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
      for (uint32_t q = 0; q < NW; ++q) t += red[q * S + c];
      r[c] = AR::reduce(t, A);
    }
    write_row<Tv, S>(A, Y, ldy, T.row0, r, s, alpha, beta);
  }
}

// ------------------------------- STREAM tile -------------------------------
// One vector. The tile's terms (value times gathered x) go to LDS; then every
// thread sums an equal run of consecutive terms and adds each row's piece to
// that row's LDS sum with an LDS atomic (exact in any order: integers, or
// integer-valued doubles below 2^53), so one long row inside a tile does not
// serialize on one lane. Row pointers and the band part are loaded first.
template <class AR, typename Tx, typename Tv, int U>
__device__ inline void stream_tile_1(const DevMat& A, const Tile& T, const Tx* __restrict__ X, int64_t ldx,
                                     Tv* __restrict__ Y, int64_t ldy, uint32_t alpha, uint32_t beta,
                                     unsigned char* lds) {
  using Prod = typename AR::Prod;
  using Acc = typename AR::Acc;
  constexpr uint32_t NW = TILE_THREADS / WAVE;
  Acc* rowsum = (Acc*)lds;                                 // [256]
  uint32_t* rps = (uint32_t*)(rowsum + TILE_THREADS);     // [257] tile-relative row starts
  Prod* prod = (Prod*)(rps + TILE_THREADS + 4);            // [ne]
  const uint32_t tid = threadIdx.x, lane = tid & (WAVE - 1), wave = tid / WAVE;
  const uint32_t ne = T.ne;
  const uint32_t nchunks = (ne + WCHUNK - 1) / WCHUNK;
  const uint32_t nr = tile_rows(T.kind);
  auto words = [&](Chunk4<AR, Tx, 1, U>& b, uint32_t ch0) {
    b.load_words(
        [&](int u) -> const u32x4* {
          uint32_t ch = ch0 + u * NW, k = ch * WCHUNK + lane * WIDE;
          return (ch < nchunks && k < ne) ? (const u32x4*)(A.ent + T.e0 + k) : nullptr;
        },
        [&](int u) -> uint32_t {
          uint32_t ch = ch0 + u * NW;
          return ch < nchunks ? A.choff[T.c0 + ch] : 0u;
        });
  };
  auto terms = [&](Chunk4<AR, Tx, 1, U>& b, uint32_t ch0) {
    b.load_gathers(A, X, ldx, 1);
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < WIDE; ++k) {
        uint32_t e = (ch0 + u * NW) * WCHUNK + lane * WIDE + k;
        if (e < ne) prod[e] = term<AR>(b.w[u][k] >> TAG_SHIFT, b.v[u][k], b.xv[u][k][0], A.m);
      }
  };
  // the first batch of entry words is requested before the row pointers and
  // the band part, whose loads then overlap its latency
  Chunk4<AR, Tx, 1, U> first;
  words(first, wave);
  if (tid < nr) rps[tid] = A.rowp[T.aux + tid] - T.e0;
  if (tid == 0) rps[nr] = ne;  // nr may be 256: the sentinel needs its own writer
  if (tid < nr) {
    LaneAcc<AR, 1> band;
    band.init(A);
    band_terms<AR, Tx, 1>(A, T, band, T.row0 + tid, tid, nr, 0, 1, X, ldx, 1);
    band.to_residues(A);
    rowsum[tid] = band.a[0];
  }
  terms(first, wave);  // chunks past the end hold padding words and store nothing
  for (uint32_t ch0 = wave + NW * U; ch0 < nchunks; ch0 += NW * U) {
    Chunk4<AR, Tx, 1, U> b;
    words(b, ch0);
    terms(b, ch0);
  }
  __syncthreads();
  // entry-balanced segmented sum
  const uint32_t per = (ne + TILE_THREADS - 1) / TILE_THREADS;
  const uint32_t p0 = tid * per, p1 = min(ne, p0 + per);
  if (p0 < p1) {
    uint32_t lo = 0, hi = nr;  // last row r with rps[r] <= p0
    while (hi - lo > 1) {
      uint32_t mid = (lo + hi) >> 1;
      if (rps[mid] <= p0) lo = mid;
      else hi = mid;
    }
    uint32_t r = lo, next = rps[r + 1];
    LaneAcc<AR, 1> acc;
    acc.init(A);
    for (uint32_t p = p0; p < p1; ++p) {
      while (p >= next) {
        acc.to_residues(A);
        atomicAdd(&rowsum[r], acc.a[0]);
        acc.init(A);
        next = rps[++r + 1];
      }
      acc.a[0] += prod[p];
      acc.tick(A);
    }
    acc.to_residues(A);
    atomicAdd(&rowsum[r], acc.a[0]);
  }
  __syncthreads();
  if (tid < nr) {
    uint32_t res = AR::reduce(rowsum[tid], A);
    write_row<Tv, 1>(A, Y, ldy, T.row0 + tid, &res, 1, alpha, beta);
  }
}

// s > 1 vectors on a tile whose rows are skewed (TF_LONGROWS): a row of up to
// STREAM_LONG_ROW entries is summed by its own lane, a longer one by the whole
// workgroup, lane = (slot, component), so a power-law row inside a tile does
// not serialize on one lane. The workgroup's partial sums of a long row meet
// through shuffles and LDS atomics.

// LDS of stream_tile_s for a tile of ne entries (see the layout there).
template <class AR, int S>
__host__ __device__ inline size_t stream_s_lds_bytes(int64_t ne) {
  const size_t maxl = (size_t)ne / (STREAM_LONG_ROW + 1) + 1;
  return (size_t)ne * 8 + 16 + 4 + maxl * 4 + 16 + maxl * S * sizeof(typename AR::Acc);  // with alignment slack
}

template <class AR, typename Tx, typename Tv, int S>
__device__ inline void stream_tile_s_long(const DevMat& A, const Tile& T, const Tx* __restrict__ X, int64_t ldx,
                                     Tv* __restrict__ Y, int64_t ldy, int s, uint32_t alpha, uint32_t beta,
                                     unsigned char* lds) {
  using Acc = typename AR::Acc;
  constexpr uint32_t NW = TILE_THREADS / WAVE;
  constexpr int U = 2;
  // LDS: words [ne], values [ne], long-row count, long rows [maxl], their sums [maxl][S]
  uint32_t* sw = (uint32_t*)lds;
  uint32_t* sv = sw + T.ne;
  const uint32_t maxl = T.ne / (STREAM_LONG_ROW + 1) + 1;
  uint32_t* lcount = (uint32_t*)(((uintptr_t)(sv + T.ne) + 15) & ~(uintptr_t)15);
  uint32_t* lrows = lcount + 1;
  Acc* lacc = (Acc*)(((uintptr_t)(lrows + maxl) + 15) & ~(uintptr_t)15);
  const uint32_t tid = threadIdx.x, lane = tid & (WAVE - 1), wave = tid / WAVE;
  const uint32_t nchunks = (T.ne + WCHUNK - 1) / WCHUNK;
  const uint32_t nr = tile_rows(T.kind);
  if (tid == 0) *lcount = 0;
  uint32_t kb = 0, ke = 0;
  if (tid < nr) {
    kb = A.rowp[T.aux + tid] - T.e0;
    ke = A.rowp[T.aux + tid + 1] - T.e0;
  }
  for (uint32_t ch0 = wave; ch0 < nchunks; ch0 += NW * U) {
    uint32_t w[U][WIDE], vo[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      uint32_t ch = ch0 + u * NW, k = ch * WCHUNK + lane * WIDE;
      u32x4 q = (ch < nchunks && k < T.ne) ? __builtin_nontemporal_load((const u32x4*)(A.ent + T.e0 + k))
                                           : (u32x4)(PAD_WORD);
      w[u][0] = q.x;
      w[u][1] = q.y;
      w[u][2] = q.z;
      w[u][3] = q.w;
      vo[u] = ch < nchunks ? A.choff[T.c0 + ch] : 0u;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      uint32_t v[WIDE];
      load_values4<AR>(A, w[u], vo[u], v);
#pragma unroll
      for (int k = 0; k < WIDE; ++k) {
        uint32_t e = (ch0 + u * NW) * WCHUNK + lane * WIDE + k;
        if (e < T.ne) {
          sw[e] = w[u][k];
          sv[e] = v[k];
        }
      }
    }
  }
  __syncthreads();
  const bool mine = tid < nr;
  const bool islong = mine && ke - kb > STREAM_LONG_ROW;
  uint32_t lidx = 0;
  if (islong) {
    lidx = atomicAdd(lcount, 1u);
    lrows[lidx] = tid;
  }
  const uint32_t row = T.row0 + tid;
  if (mine) {
    LaneAcc<AR, S> acc;
    acc.init(A);
    band_terms<AR, Tx, S>(A, T, acc, row, tid, nr, 0, 1, X, ldx, s);
    if (islong) {  // a long row's sums start from its band part, as residues; the workgroup adds the rest
      acc.to_residues(A);
#pragma unroll
      for (int c = 0; c < S; ++c) lacc[lidx * S + c] = acc.a[c];
    } else {
      // EU entries of the row at a time: their gathers are all issued before the
      // first term is added (16 in flight per lane)
      constexpr int EU = S >= 16 ? 1 : 16 / S;
      for (uint32_t k0 = kb; k0 < ke; k0 += EU) {
        uint32_t w[EU], xv[EU][S];
#pragma unroll
        for (int e = 0; e < EU; ++e) {
          w[e] = k0 + e < ke ? sw[k0 + e] : PAD_WORD;
          const Tx* xr = X + (int64_t)(w[e] & COL_MASK) * ldx;
          const bool live = (w[e] >> TAG_SHIFT) != TAG_PAD;
#pragma unroll
          for (int c = 0; c < S; ++c) xv[e][c] = (live && c < s) ? (uint32_t)xr[c] : 0u;
        }
#pragma unroll
        for (int e = 0; e < EU; ++e) {
          const uint32_t tag = w[e] >> TAG_SHIFT, v = k0 + e < ke ? sv[k0 + e] : 0u;
#pragma unroll
          for (int c = 0; c < S; ++c)
            if (c < s) acc.a[c] += term<AR>(tag, v, xv[e][c], A.m);
          acc.tick(A);
        }
      }
      uint32_t r[S];
#pragma unroll
      for (int c = 0; c < S; ++c) r[c] = AR::reduce(acc.a[c], A);
      write_row<Tv, S>(A, Y, ldy, row, r, s, alpha, beta);
    }
  }
  __syncthreads();  // the long-row list and the band sums of long rows are complete
  const uint32_t nl = *lcount;
  if (nl) {
    constexpr uint32_t SLOTS = TILE_THREADS / S;
    constexpr int EU2 = 4;
    const uint32_t comp = tid % S, slot = tid / S;
    const bool cok = (int)comp < s;
    for (uint32_t q = 0; q < nl; ++q) {
      const uint32_t r = lrows[q];
      const uint32_t b = A.rowp[T.aux + r] - T.e0, e = A.rowp[T.aux + r + 1] - T.e0;
      LaneAcc<AR, 1> pa;
      pa.init(A);
      for (uint32_t k0 = b + slot; k0 < e; k0 += SLOTS * EU2) {
        uint32_t w[EU2], xv[EU2];
#pragma unroll
        for (int u = 0; u < EU2; ++u) {
          const uint32_t k = k0 + u * SLOTS;
          w[u] = k < e ? sw[k] : PAD_WORD;
          xv[u] = ((w[u] >> TAG_SHIFT) != TAG_PAD && cok) ? (uint32_t)X[(int64_t)(w[u] & COL_MASK) * ldx + comp] : 0u;
        }
#pragma unroll
        for (int u = 0; u < EU2; ++u) {
          const uint32_t k = k0 + u * SLOTS;
          pa.a[0] += term<AR>(w[u] >> TAG_SHIFT, k < e ? sv[k] : 0u, xv[u], A.m);
          pa.tick(A);
        }
      }
      pa.to_residues(A);
      Acc t = pa.a[0];
      for (int o = S; o < WAVE; o <<= 1) t += shfl_xor_acc(t, o, WAVE);  // the wave's slots of one component
      if (lane < (uint32_t)S && cok) atomicAdd(&lacc[q * S + comp], t);
    }
    __syncthreads();
    if (islong) {
      uint32_t r[S];
#pragma unroll
      for (int c = 0; c < S; ++c) r[c] = AR::reduce(lacc[lidx * S + c], A);
      write_row<Tv, S>(A, Y, ldy, row, r, s, alpha, beta);
    }
  }
}

// s > 1 vectors: stage words and values in LDS, one lane per row (correct
// for every tile; tiles flagged TF_LONGROWS are faster with stream_tile_s_long)
template <class AR, typename Tx, typename Tv, int S>
__device__ inline void stream_tile_s(const DevMat& A, const Tile& T, const Tx* __restrict__ X, int64_t ldx,
                                     Tv* __restrict__ Y, int64_t ldy, int s, uint32_t alpha, uint32_t beta,
                                     unsigned char* lds) {
  constexpr uint32_t NW = TILE_THREADS / WAVE;
  constexpr int U = 2;
  uint32_t* sw = (uint32_t*)lds;
  uint32_t* sv = sw + T.ne;
  const uint32_t tid = threadIdx.x, lane = tid & (WAVE - 1), wave = tid / WAVE;
  const uint32_t nchunks = (T.ne + WCHUNK - 1) / WCHUNK;
  const uint32_t nr = tile_rows(T.kind);
  uint32_t kb = 0, ke = 0;
  if (tid < nr) {
    kb = A.rowp[T.aux + tid] - T.e0;
    ke = A.rowp[T.aux + tid + 1] - T.e0;
  }
  for (uint32_t ch0 = wave; ch0 < nchunks; ch0 += NW * U) {
    uint32_t w[U][WIDE], vo[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      uint32_t ch = ch0 + u * NW, k = ch * WCHUNK + lane * WIDE;
      u32x4 q = (ch < nchunks && k < T.ne) ? __builtin_nontemporal_load((const u32x4*)(A.ent + T.e0 + k))
                                           : (u32x4)(PAD_WORD);
      w[u][0] = q.x;
      w[u][1] = q.y;
      w[u][2] = q.z;
      w[u][3] = q.w;
      vo[u] = ch < nchunks ? A.choff[T.c0 + ch] : 0u;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      uint32_t idx = vo[u];
#pragma unroll
      for (int k = 0; k < WIDE; ++k) idx += lanes_below(__ballot((w[u][k] >> TAG_SHIFT) == TAG_GEN));
#pragma unroll
      for (int k = 0; k < WIDE; ++k) {
        bool gen = (w[u][k] >> TAG_SHIFT) == TAG_GEN;
        uint32_t v = gen ? ldval<typename AR::ValT>(A.val, idx) : 0u;
        idx += gen ? 1u : 0u;
        uint32_t e = (ch0 + u * NW) * WCHUNK + lane * WIDE + k;
        if (e < T.ne) {
          sw[e] = w[u][k];
          sv[e] = v;
        }
      }
    }
  }
  __syncthreads();
  if (tid >= nr) return;
  const uint32_t row = T.row0 + tid;
  LaneAcc<AR, S> acc;
  acc.init(A);
  band_terms<AR, Tx, S>(A, T, acc, row, tid, nr, 0, 1, X, ldx, s);
  // EU entries of the row at a time: their gathers are all issued before the
  // first term is added (16 in flight per lane)
  constexpr int EU = S >= 16 ? 1 : 16 / S;
  // s = S with 16-byte aligned rows of X: a row is gathered in 16-byte loads
  // (two for s = 8 int32 instead of eight 4-byte ones), so the vector cache
  // looks up each line once per load, not once per component
  constexpr bool VT = sizeof(Tx) == 4 || sizeof(Tx) == 8;  // int32 or int64 rows (not a 16-bit copy)
  constexpr int NV = VT && (S * sizeof(Tx)) % 16 == 0 ? (int)((S * sizeof(Tx)) / 16) : 0;
  const bool vx = NV > 0 && s == S && ((uintptr_t)X & 15) == 0 && ((ldx * (int64_t)sizeof(Tx)) & 15) == 0;
  for (uint32_t k0 = kb; k0 < ke; k0 += EU) {
    uint32_t w[EU], xv[EU][S];
#pragma unroll
    for (int e = 0; e < EU; ++e) {
      w[e] = k0 + e < ke ? sw[k0 + e] : PAD_WORD;
      const Tx* xr = X + (int64_t)(w[e] & COL_MASK) * ldx;
      const bool live = (w[e] >> TAG_SHIFT) != TAG_PAD;
      if (NV > 0 && vx) {
#pragma unroll
        for (int j = 0; j < (NV > 0 ? NV : 1); ++j) {
          const u32x4 q = live ? ((const u32x4*)xr)[j] : (u32x4){0u, 0u, 0u, 0u};
          if constexpr (sizeof(Tx) == 4) {
            xv[e][4 * j] = q.x;
            xv[e][4 * j + 1] = q.y;
            xv[e][4 * j + 2] = q.z;
            xv[e][4 * j + 3] = q.w;
          } else if constexpr (sizeof(Tx) == 8) {  // residues: the low words of two int64
            xv[e][2 * j] = q.x;
            xv[e][2 * j + 1] = q.z;
          }
        }
      } else {
#pragma unroll
        for (int c = 0; c < S; ++c) xv[e][c] = (live && c < s) ? (uint32_t)xr[c] : 0u;
      }
    }
#pragma unroll
    for (int e = 0; e < EU; ++e) {
      const uint32_t tag = w[e] >> TAG_SHIFT, v = k0 + e < ke ? sv[k0 + e] : 0u;
#pragma unroll
      for (int c = 0; c < S; ++c)
        if (c < s) acc.a[c] += term<AR>(tag, v, xv[e][c], A.m);
      acc.tick(A);
    }
  }
  uint32_t r[S];
#pragma unroll
  for (int c = 0; c < S; ++c) r[c] = AR::reduce(acc.a[c], A);
  write_row<Tv, S>(A, Y, ldy, row, r, s, alpha, beta);
}

// ------------------------------- the launch --------------------------------
template <class AR, typename Tx, typename Tv, int S, int U>
__global__ __launch_bounds__(TILE_THREADS) void k_tiles(DevMat A, const Tx* __restrict__ X, int64_t ldx,
                                                        Tv* __restrict__ Y, int64_t ldy, int s, uint32_t alpha,
                                                        uint32_t beta) {
  extern __shared__ __align__(16) unsigned char lds[];
  // a grid larger than the tile table repeats it (per-block timing)
  const Tile T = A.tiles[blockIdx.x % A.ntiles];
  switch (tile_kind(T.kind)) {
    case TK_SELL:
      if constexpr (S == 1) sell_tile<AR, Tx, Tv, 1, 4>(A, T, X, ldx, Y, ldy, s, alpha, beta);
      else sell_tile_rc<AR, Tx, Tv, S>(A, T, X, ldx, Y, ldy, s, alpha, beta);
      break;
    case TK_LONG: long_tile<AR, Tx, Tv, S, (S == 1 ? U : 1)>(A, T, X, ldx, Y, ldy, s, alpha, beta, lds); break;
    default:
      if constexpr (S == 1) stream_tile_1<AR, Tx, Tv, U>(A, T, X, ldx, Y, ldy, alpha, beta, lds);
      else if (!(T.kind & TF_LONGROWS)) stream_tile_s<AR, Tx, Tv, S>(A, T, X, ldx, Y, ldy, s, alpha, beta, lds);
      // (flagged tiles, s > 1: k_tiles_long)
  }
}

// The STREAM tiles flagged TF_LONGROWS, for s > 1 (one workgroup each).
template <class AR, typename Tx, typename Tv, int S>
__global__ __launch_bounds__(TILE_THREADS) void k_tiles_long(DevMat A, const Tx* __restrict__ X, int64_t ldx,
                                                             Tv* __restrict__ Y, int64_t ldy, int s, uint32_t alpha,
                                                             uint32_t beta) {
  extern __shared__ __align__(16) unsigned char lds[];
  const Tile T = A.tiles[A.ltiles[blockIdx.x]];
  stream_tile_s_long<AR, Tx, Tv, S>(A, T, X, ldx, Y, ldy, s, alpha, beta, lds);
}

template <typename Tv>
__global__ void k_to_u16(const Tv* __restrict__ x, int64_t ldx, uint16_t* __restrict__ out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (uint16_t)x[i * ldx];
}

// Contiguous x with 16-byte alignment: eight residues per thread, read with
// 16-byte loads and written with one 16-byte store.
template <typename Tv>
__global__ void k_to_u16_x8(const Tv* __restrict__ x, uint16_t* __restrict__ out, int64_t n) {
  typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, base = t * 8;
  if (base + 8 <= n) {
    constexpr int NV = (int)(8 * sizeof(Tv) / 16);  // 16-byte loads per thread
    constexpr int PER = 16 / (int)sizeof(Tv);       // residues per load
    uint32_t r[8];
    const u32x4_t* src = (const u32x4_t*)(x + base);
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      u32x4_t q = __builtin_nontemporal_load(src + k);
      if constexpr (PER == 4) {
        r[4 * k] = q.x; r[4 * k + 1] = q.y; r[4 * k + 2] = q.z; r[4 * k + 3] = q.w;
      } else {  // two int64 residues: their low words
        r[2 * k] = q.x; r[2 * k + 1] = q.z;
      }
    }
    u32x4_t o;
    o.x = (r[0] & 0xffffu) | (r[1] << 16);
    o.y = (r[2] & 0xffffu) | (r[3] << 16);
    o.z = (r[4] & 0xffffu) | (r[5] << 16);
    o.w = (r[6] & 0xffffu) | (r[7] << 16);
    *(u32x4_t*)(out + base) = o;
  } else {
    for (int64_t i = base; i < n; ++i) out[i] = (uint16_t)x[i];
  }
}

// Dynamic LDS of one launch.
template <class AR>
inline size_t tiles_lds_bytes(int64_t max_tile_entries, int S) {
  size_t stream = S == 1 ? TILE_THREADS * sizeof(typename AR::Acc) + (TILE_THREADS + 4) * 4 +
                               (size_t)max_tile_entries * sizeof(typename AR::Prod)
                  : S == 2  ? stream_s_lds_bytes<AR, 2>(max_tile_entries)
                  : S == 4  ? stream_s_lds_bytes<AR, 4>(max_tile_entries)
                  : S == 8  ? stream_s_lds_bytes<AR, 8>(max_tile_entries)
                            : stream_s_lds_bytes<AR, 16>(max_tile_entries);
  size_t red = (size_t)(TILE_THREADS / WAVE) * S * sizeof(typename AR::Acc);
  size_t b = stream > red ? stream : red;
  return b < 16 ? 16 : b;
}

// Unroll of the one-vector STREAM/LONG paths: every chunk of a tile in one batch.
inline int unroll_for(int64_t max_tile_entries) {
  int64_t per_wave = (max_tile_entries + (int64_t)WCHUNK * (TILE_THREADS / WAVE) - 1) / ((int64_t)WCHUNK * (TILE_THREADS / WAVE));
  return per_wave <= 1 ? 1 : per_wave <= 2 ? 2 : 4;
}

template <class AR, typename Tx, typename Tv, int U>
static void launch_s1(const DevMat& A, dim3 grid, size_t lds, const Tx* x, int64_t ldx, Tv* y, int64_t ldy,
                      uint32_t alpha, uint32_t beta, hipStream_t st) {
  hipLaunchKernelGGL((k_tiles<AR, Tx, Tv, 1, U>), grid, dim3(TILE_THREADS), lds, st, A, x, ldx, y, ldy, 1, alpha,
                     beta);
}

// x16: when not null, a 16-bit copy of the one vector (s must be 1)
template <class AR, typename Tv>
hipError_t launch_tiles_t(const DevMat& A, int64_t max_tile_entries, const void* X, int64_t ldx, void* Y, int64_t ldy,
                          int s, uint32_t alpha, uint32_t beta, hipStream_t st, const uint16_t* x16,
                          uint32_t nblocks = 0) {
  if (A.ntiles == 0) return hipSuccess;
  const int S = s <= 1 ? 1 : s <= 2 ? 2 : s <= 4 ? 4 : s <= 8 ? 8 : 16;
  size_t lds = tiles_lds_bytes<AR>(max_tile_entries, S);
  dim3 grid(nblocks ? nblocks : A.ntiles), block(TILE_THREADS);
  const Tv* x = (const Tv*)X;
  Tv* y = (Tv*)Y;
  if (S == 1) {
    const int U = unroll_for(max_tile_entries);
    if (x16) {
      if (U == 1) launch_s1<AR, uint16_t, Tv, 1>(A, grid, lds, x16, 1, y, ldy, alpha, beta, st);
      else if (U == 2) launch_s1<AR, uint16_t, Tv, 2>(A, grid, lds, x16, 1, y, ldy, alpha, beta, st);
      else launch_s1<AR, uint16_t, Tv, 4>(A, grid, lds, x16, 1, y, ldy, alpha, beta, st);
    } else {
      if (U == 1) launch_s1<AR, Tv, Tv, 1>(A, grid, lds, x, ldx, y, ldy, alpha, beta, st);
      else if (U == 2) launch_s1<AR, Tv, Tv, 2>(A, grid, lds, x, ldx, y, ldy, alpha, beta, st);
      else launch_s1<AR, Tv, Tv, 4>(A, grid, lds, x, ldx, y, ldy, alpha, beta, st);
    }
    return hipGetLastError();
  }
  switch (S) {
    case 2: hipLaunchKernelGGL((k_tiles<AR, Tv, Tv, 2, 4>), grid, block, lds, st, A, x, ldx, y, ldy, s, alpha, beta); break;
    case 4: hipLaunchKernelGGL((k_tiles<AR, Tv, Tv, 4, 4>), grid, block, lds, st, A, x, ldx, y, ldy, s, alpha, beta); break;
    case 8: hipLaunchKernelGGL((k_tiles<AR, Tv, Tv, 8, 4>), grid, block, lds, st, A, x, ldx, y, ldy, s, alpha, beta); break;
    default: hipLaunchKernelGGL((k_tiles<AR, Tv, Tv, 16, 4>), grid, block, lds, st, A, x, ldx, y, ldy, s, alpha, beta); break;
  }
  if (A.nltiles && !nblocks) {  // the flagged tiles the launch above left out
    dim3 lg(A.nltiles);
    switch (S) {
      case 2: hipLaunchKernelGGL((k_tiles_long<AR, Tv, Tv, 2>), lg, block, lds, st, A, x, ldx, y, ldy, s, alpha, beta); break;
      case 4: hipLaunchKernelGGL((k_tiles_long<AR, Tv, Tv, 4>), lg, block, lds, st, A, x, ldx, y, ldy, s, alpha, beta); break;
      case 8: hipLaunchKernelGGL((k_tiles_long<AR, Tv, Tv, 8>), lg, block, lds, st, A, x, ldx, y, ldy, s, alpha, beta); break;
      default: hipLaunchKernelGGL((k_tiles_long<AR, Tv, Tv, 16>), lg, block, lds, st, A, x, ldx, y, ldy, s, alpha, beta); break;
    }
  }
  return hipGetLastError();
}

// 16-bit copy of one vector (residues < 65536), for the compact-x path.
template <typename Tv>
hipError_t launch_to_u16(const void* X, int64_t ldx, uint16_t* out, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (ldx == 1 && ((uintptr_t)X & 15) == 0 && ((uintptr_t)out & 15) == 0) {
    int64_t threads = (n + 7) / 8;
    hipLaunchKernelGGL((k_to_u16_x8<Tv>), dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, (const Tv*)X,
                       out, n);
    return hipGetLastError();
  }
  int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL((k_to_u16<Tv>), dim3(blocks), dim3(256), 0, st, (const Tv*)X, ldx, out, n);
  return hipGetLastError();
}

}  // namespace ffx
