// Column-sorted row groups: a second encoding of A for the one-vector
// product y = alpha*A*x + beta*y when m <= 65536.
//
// The tile kernels gather one x entry per matrix entry at a random column, and
// on MI355X such random 2-byte gathers cost a whole cache line each: the
// large products run at the rate the vector caches serve random lines, not at
// HBM bandwidth. Here the rows are cut into about one group per compute unit,
// and inside a group the entries are sorted by column, so the 64 lanes of one
// gather instruction read 64 consecutive columns of the group's sorted list
// and share a few cache lines of x. Each workgroup keeps the sums of its
// group's rows in LDS (64-bit integers, updated with LDS atomics) and writes
// its rows of y once at the end. This is the paper's delayed reduction
// (Section 2.2) with the reduction taken once per row at the end: for
// m <= 65536 a term is below 2^32, so no row can overflow 64 bits.
//
// Layout. Entry word: tag (2 bits, as in the tiles) | row in the group (14
// bits) | column - panel base (16 bits). The entries of a group are sorted by
// column and cut into chunks of 256 words; a chunk never spans two panels of
// 65,536 columns (the last chunk of a panel is padded), and stores its panel
// base in `cbase` and the offset of its general values in `choff`. Entry e of
// a chunk is gathered by lane e mod 64 of the e/64-th gather instruction, so
// one instruction covers 64 consecutive sorted columns; the chunk stores entry
// 64k + l at word 4l + k, so lane l reads its four entries with one 16-byte
// load. General values follow the same lane-major order, so a lane's (at most
// four) values are consecutive and one 12-byte load fetches them: each chunk
// costs a lane one entry load, one value load and four gathers.
#pragma once

#include "ffx_impl.h"

namespace ffx {

constexpr int SG_CHUNK = 256;
constexpr uint32_t SG_MAX_ROWS = 1u << 14;  // rows of one group (14-bit row field)
constexpr uint32_t SG_ROW_SHIFT = 16;
constexpr uint32_t SG_COL_MASK = 0xFFFFu;

struct SgGroup {
  uint32_t row0;     // first row
  uint32_t nrows;    // rows (at most SG_MAX_ROWS)
  uint32_t c0;       // first chunk
  uint32_t nchunks;  // chunks
};
static_assert(sizeof(SgGroup) == 16, "group layout");

struct SgMat {
  const SgGroup* groups;
  const uint32_t* ent;     // SG_CHUNK words per chunk
  const uint16_t* val;     // general values, in entry order
  const uint32_t* choff;   // per chunk: index of its first general value
  const uint32_t* cbase;   // per chunk: column of its panel's first column
  const uint32_t* rowmap;  // when not null, row r of the product is written to row rowmap[r] of y
  uint32_t ngroups;
  uint32_t max_rows;       // largest group (sizes the LDS)
  uint32_t nrows;
  uint32_t m;
  uint64_t mu;
};

// y = alpha*A*x + beta*y from the groups; x16: 16-bit copy of x, or null to gather from x (Tv);
// y16: when not null, also receives y as 16-bit residues (row rowmap[r] when there is a row map), the
// next product's x16 in a chain of products.
hipError_t launch_sg(const SgMat& G, ffx_dtype dt, const void* x, const uint16_t* x16, void* y, uint32_t alpha,
                     uint32_t beta, hipStream_t st, uint16_t* y16 = nullptr);
// Y = A X over GF(2) for a matrix mod 2 and one bit-packed word per row (32 vectors): X ncols x 1
// words with stride ldx, Y nrows x 1 with stride ldy (through the row map when there is one).
hipError_t launch_sg_gf2(const SgMat& G, const uint32_t* X, int64_t ldx, uint32_t* Y, int64_t ldy, hipStream_t st);

}  // namespace ffx
