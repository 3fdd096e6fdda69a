// Internal definitions shared by the host planner and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ffx.h"

namespace ffx {

// ---------------------------------------------------------------------------
// Entry words. Each stored entry is one 32-bit word: the column in the low 30
// bits and a 2-bit tag on top. Entries with residue 1 or m-1 carry no value
// (paper Section 2.4, "Taking into account the +-1"): the tag says which.
// General entries take their value from a compacted value stream (uint16 when
// m <= 65536, else uint32); the value index of a general entry is the offset
// stored for its 64-entry chunk plus the number of general entries before it
// in that chunk, which a wavefront gets from one ballot and a bit count.
// ---------------------------------------------------------------------------
constexpr uint32_t TAG_SHIFT = 30;
constexpr uint32_t COL_MASK = (1u << TAG_SHIFT) - 1;
constexpr uint32_t TAG_GEN = 0u, TAG_PLUS = 1u, TAG_MINUS = 2u, TAG_PAD = 3u;
constexpr uint32_t PAD_WORD = TAG_PAD << TAG_SHIFT;
constexpr int64_t MAX_DIM = int64_t(1) << TAG_SHIFT;

// ---------------------------------------------------------------------------
// Tiles: the unit of work of one 256-lane workgroup. A matrix is a list of
// row blocks, each block has one format, and each block is cut into tiles.
// One kernel launch walks the whole tile table, whatever the formats.
// ---------------------------------------------------------------------------
enum TileKind : uint32_t {
  TK_STREAM = 0,  // up to 256 consecutive rows, entries staged through LDS
  TK_LONG = 1,    // one row longer than a STREAM tile; all lanes sweep it
  TK_SELL = 2,    // up to 4 slices of 64 rows in padded 4-column groups
};
constexpr uint32_t TF_SORTED = 1u << 4;  // SELL slots map to rows through perm[]
// A STREAM tile with a row of more than STREAM_LONG_ROW entries is flagged
// TF_LONGROWS: with s > 1 vectors a kernel of its own sums its long rows with
// the whole workgroup instead of one lane.
constexpr uint32_t TF_LONGROWS = 1u << 5;
constexpr uint32_t STREAM_LONG_ROW = 64;

constexpr int TILE_THREADS = 256;
constexpr int WAVE = 64;
// STREAM and LONG tiles are read 4 consecutive entry words (16 bytes) per
// lane: their entries start 16-byte aligned, are padded to a multiple of 4,
// and their value chunks cover 256 entries. SELL chunks cover 64 entries.
constexpr int WIDE = 4;
constexpr int WCHUNK = WAVE * WIDE;
constexpr int SELL_SLICES = TILE_THREADS / WAVE;  // 4
constexpr int SELL_GROUP = WAVE * WIDE;           // words of one 4-column group of a SELL slice
constexpr int MAX_BAND = 64;                      // diagonals per band part
constexpr int MAX_S = 16;

struct Tile {
  uint32_t kind;   // TileKind | flags; bits 8..15 band diagonals; bits 16..31 rows (slots for SELL)
  uint32_t row0;   // first row (STREAM, LONG) or first slot (SELL)
  uint32_t e0;     // first entry word
  uint32_t ne;     // STREAM/LONG: entries; SELL: slices
  uint32_t c0;     // first value chunk
  uint32_t aux;    // STREAM: first index in rowp[]; SELL: first index in swidth[]
  uint32_t b0;     // first band value
  uint32_t boff;   // first band offset in boffs[]
};
static_assert(sizeof(Tile) == 32, "tile layout");

__host__ __device__ inline uint32_t tile_kind(uint32_t k) { return k & 0xF; }
__host__ __device__ inline uint32_t tile_nd(uint32_t k) { return (k >> 8) & 0xFF; }
__host__ __device__ inline uint32_t tile_rows(uint32_t k) { return k >> 16; }

// Everything a kernel needs about one encoded matrix (passed by value).
struct DevMat {
  const Tile* tiles;
  const uint32_t* ent;
  const void* val;       // uint16_t or uint32_t, by the modulus
  const uint32_t* choff; // value offset of each 256-entry chunk
  const uint32_t* rowp;  // STREAM tiles: rows+1 absolute entry offsets per tile
  const uint32_t* perm;  // sorted SELL: slot -> row (0xFFFFFFFF for padding slots)
  const uint32_t* swidth;// SELL: 4-column groups of each slice
  const void* bval;      // band values, diagonal-major inside each tile
  const int32_t* boffs;  // band diagonal offsets (column - row)
  const uint32_t* ltiles;// STREAM tiles flagged TF_LONGROWS
  const uint32_t* rowmap;// when not null, row r of the product is written to row rowmap[r] of Y
  uint32_t nltiles;
  uint32_t ntiles;
  uint32_t nrows, ncols;
  uint32_t m;
  uint64_t mu;           // floor((2^64-1)/m), for Barrett reduction
  double inv_m;          // 1/m rounded, for the fp64 path
  float inv_mf;          // 1/m rounded to float, for the fp32 paths
  int64_t reduce_every;  // terms summed between two reductions
};

// ---------------------------------------------------------------------------
// Modular arithmetic (paper Section 2.2): delayed reduction of wide sums.
// ---------------------------------------------------------------------------
__host__ __device__ inline uint64_t umulhi64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul64hi(a, b);
#else
  return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

// a mod m for any 64-bit a and 2 <= m < 2^31. Barrett (1986) with the
// precomputed mu = floor((2^64-1)/m): q = floor(a*mu/2^64) is at most two
// below floor(a/m), so r = a - q*m < 3m and two conditional subtractions
// finish.
__host__ __device__ inline uint32_t mod_u64(uint64_t a, uint32_t m, uint64_t mu) {
  uint64_t q = umulhi64(a, mu);
  uint64_t r = a - q * (uint64_t)m;
  if (r >= m) r -= m;
  if (r >= m) r -= m;
  return (uint32_t)r;
}

// a mod m for an integer-valued double 0 <= a <= 2^53, by one multiplication
// with the rounded reciprocal: the quotient estimate is within 2 of the true
// floor (relative error of a*inv_m below 2^-52 and a/m <= 2^52), the
// remainder a - q*m is an exact integer computed exactly by one fma, and at
// most two corrections each way bring it into [0, m).
__host__ __device__ inline uint32_t mod_f64(double a, uint32_t m, double inv_m) {
  double q = floor(a * inv_m);
  double r = fma(-q, (double)m, a);
  double md = (double)m;
  if (r < 0) r += md;
  if (r < 0) r += md;
  if (r >= md) r -= md;
  if (r >= md) r -= md;
  return (uint32_t)r;
}

// a mod m for an integer-valued float 0 <= a <= 2^24 (m <= 8191): as in
// mod_f64, with a quotient estimate within 1 of the floor (a/m * 2^-23 < 1)
// and one correction each way.
__host__ __device__ inline uint32_t mod_f32(float a, uint32_t m, float inv_m) {
  float q = floorf(a * inv_m);
  float md = (float)m;
  float r = fmaf(-q, md, a);
  if (r < 0) r += md;
  if (r >= md) r -= md;
  return (uint32_t)r;
}

// Centered remainder (Section 2.2, the representation on
// [-floor((m-1)/2), ceil((m-1)/2)]): for an integer-valued a with |a| at most
// 2^53 (double) or 2^24 (float), returns the r = a (mod m) with
// -h <= r <= h, h = floor(m/2) = ceil((m-1)/2). The nearest-integer quotient
// estimate is within 1 of the true nearest quotient, so |a - q*m| <= h + m is
// an exact integer that one fma computes exactly and one correction each way
// brings into [-h, h].
__host__ __device__ inline double crem_f64(double a, uint32_t m, double inv_m) {
  double md = (double)m, h = (double)(m >> 1);
  double q = rint(a * inv_m);
  double r = fma(-q, md, a);
  if (r > h) r -= md;
  if (r < -h) r += md;
  return r;
}
__host__ __device__ inline float crem_f32(float a, uint32_t m, float inv_m) {
  float md = (float)m, h = (float)(m >> 1);
  float q = rintf(a * inv_m);
  float r = fmaf(-q, md, a);
  if (r > h) r -= md;
  if (r < -h) r += md;
  return r;
}

// (alpha*r + beta*y) mod m with every operand in [0, m): both products are
// below 2^62, so their sum fits 64 bits.
__host__ __device__ inline uint32_t axpby(uint32_t alpha, uint32_t r, uint32_t beta, uint32_t y, uint32_t m,
                                          uint64_t mu) {
  return mod_u64((uint64_t)alpha * r + (uint64_t)beta * y, m, mu);
}

// The largest number of terms, each at most tmax in magnitude, that can be
// added to a reduced accumulator (magnitude at most rmax) while the sum stays
// at most limit in magnitude.
__host__ __device__ inline int64_t terms_before_reduce(uint64_t limit, uint64_t rmax, uint64_t tmax) {
  if (limit < rmax) return 0;
  return (int64_t)((limit - rmax) / tmax);
}

}  // namespace ffx
