// Block-Wiedemann sequence S_i = U^T A^i V (paper Section 3, step 1; Section
// 3.1) and the projection U^T W it is made of.
//
// One launch per iteration i covers the whole tile table. Workgroup g < ntiles
// computes its tile's rows of W_{i+1} = A W_i (the same tile code as the
// products) and then the s x s partial sum of U^T W_{i+1} over those rows.
// Workgroup ntiles reduces the partials of iteration i, written by the
// previous launch, into S_i. Partials are double-buffered by iteration parity,
// so launch i reads one parity while writing the other. The launches of a
// batch of iterations are captured into a hipGraph and replayed; the
// iteration number comes from a device counter that the last node of the
// graph advances, so the same graph serves every batch.
#include "launch.h"
#include "tiles.h"

namespace ffx {

// --------------------------------------------------------------- helpers ---
// Row of index q (0 <= q < tile_rows) of a tile, or >= nrows for a padding slot.
__device__ inline uint32_t tile_row(const DevMat& A, const Tile& T, uint32_t q) {
  switch (tile_kind(T.kind)) {
    case TK_SELL: return (T.kind & TF_SORTED) ? A.perm[T.row0 + q] : T.row0 + q;
    default: return T.row0 + q;
  }
}

// Sum over the tile's rows of U[row][a] * W[row][b] for the s*s pairs (a, b),
// into out[a*s + b] as residues (mod m) in uint64. Thread t takes pair
// t % (s*s) and every (256/(s*s))-th row.
template <class AR, typename Tv>
__device__ inline void tile_projection(const DevMat& A, const Tile& T, const Tv* __restrict__ U, int64_t ldu,
                                       const Tv* W, int64_t ldw, int s, uint64_t* red /* LDS [256] */,
                                       uint64_t* __restrict__ out) {
  const uint32_t tid = threadIdx.x;
  const uint32_t ss = (uint32_t)(s * s);
  const uint32_t pair = tid % ss, grp = tid / ss, ngrp = TILE_THREADS / ss;
  const uint32_t a = pair / s, b = pair % s;
  const uint32_t nq = tile_kind(T.kind) == TK_LONG ? 1u : tile_rows(T.kind);
  LaneAcc<AR, 1> acc;
  acc.init(A);
  if (grp < ngrp) {
    for (uint32_t q = grp; q < nq; q += ngrp) {
      uint32_t row = tile_row(A, T, q);
      if (row >= A.nrows) continue;
      acc.a[0] += AR::mul((uint32_t)U[(int64_t)row * ldu + a], (uint32_t)W[(int64_t)row * ldw + b]);
      acc.tick(A);
    }
  }
  red[tid] = (grp < ngrp) ? (uint64_t)AR::reduce(acc.a[0], A) : 0ull;
  __syncthreads();
  if (tid < ss) {
    uint64_t t = 0;  // at most 256 residues: below 2^39
    for (uint32_t q = 0; q < ngrp; ++q) t += red[q * ss + tid];
    out[tid] = t;
  }
}

// out[pair] = sum of part[g][pair] over g = first, first + stride, ... < nparts,
// reduced mod m when `reduce` (else left as a sum of residues). Each input is
// below 2^40, and at most 2^20 inputs are added.
__device__ inline uint64_t fold_partials(const DevMat& A, const uint64_t* __restrict__ part, uint32_t first,
                                         uint32_t stride, uint32_t nparts, int s, uint64_t* red /* LDS [256] */,
                                         uint32_t* pair_out) {
  const uint32_t tid = threadIdx.x, ss = (uint32_t)(s * s);
  const uint32_t pair = tid % ss, grp = tid / ss, ngrp = TILE_THREADS / ss;
  uint64_t acc = 0;
  if (grp < ngrp)
    for (uint32_t g = first + grp * stride; g < nparts; g += ngrp * stride) acc += part[(int64_t)g * ss + pair];
  red[tid] = grp < ngrp ? (uint64_t)mod_u64(acc, A.m, A.mu) : 0ull;
  __syncthreads();
  uint64_t t = 0;
  if (tid < ss)
    for (uint32_t q = 0; q < ngrp; ++q) t += red[q * ss + tid];
  *pair_out = tid;
  return t;
}

// One 64-row SELL slice by a whole workgroup, for s > 1: the slice's S passes
// (RPW = 64/S rows each, lane = (row, component)) are split over the 4 waves,
// so a launch has four times the waves of one-slice-per-wave. Every wave reads
// the slice's 4-column groups (entry words and values, lane = row) and keeps
// the passes it owns. With PROJ the slice also adds U^T W_{i+1} over its rows: a
// lane holds W_{i+1}[row][c] and U[row][c]; the U values of the row's other
// components come by shuffle, so out[a*s + c] gets sum_row U[row][a] W[row][c].
template <class AR, typename Tv, int S, bool PROJ>
__device__ inline void sell_slice_rc(const DevMat& A, const Tile& T, uint32_t slice, const Tv* __restrict__ X,
                                     int64_t ldx, Tv* __restrict__ Y, int64_t ldy, int s, const Tv* __restrict__ U,
                                     int64_t ldu, uint64_t* __restrict__ out, uint64_t* red /* LDS [4][256] */) {
  using Acc = typename AR::Acc;
  constexpr int RPW = WAVE / S;
  constexpr int NW = TILE_THREADS / WAVE;
  constexpr int PPW = (S + NW - 1) / NW;  // passes per wave
  constexpr int GU = PPW >= 4 ? 1 : 2;  // 4-column groups loaded together
  const uint32_t lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
  const uint32_t comp = lane % S, sub = lane / S;
  const bool cok = (int)comp < s;
  const bool live = slice < T.ne;
  uint32_t off = 0;
  for (uint32_t k = 0; k < slice && live; ++k) off += A.swidth[T.aux + k];
  const uint32_t groups = live ? A.swidth[T.aux + slice] : 0u;
  const uint32_t* ent = A.ent + T.e0 + (size_t)off * SELL_GROUP + lane * WIDE;
  const uint32_t* choff = A.choff + T.c0 + off;
  uint32_t prow[PPW];
  bool pok[PPW];
#pragma unroll
  for (int q = 0; q < PPW; ++q) {
    int p = (int)wave * PPW + q;
    uint32_t slot = slice * WAVE + p * RPW + sub;
    prow[q] = (!live || p >= S) ? 0xFFFFFFFFu : (T.kind & TF_SORTED) ? A.perm[T.row0 + slot] : T.row0 + slot;
    pok[q] = prow[q] < A.nrows;
  }
  // U of the projection does not depend on the product: its loads go out first
  uint32_t urow[PPW];
#pragma unroll
  for (int q = 0; q < PPW; ++q) urow[q] = (PROJ && pok[q] && cok) ? (uint32_t)U[(int64_t)prow[q] * ldu + comp] : 0u;
  LaneAcc<AR, PPW> acc;
  acc.init(A);
  const uint32_t nd = tile_nd(T.kind), rows_in_tile = tile_rows(T.kind);
  for (uint32_t d = 0; d < nd && live; ++d) {
    const int32_t o = A.boffs[T.boff + d];
#pragma unroll
    for (int q = 0; q < PPW; ++q) {
      uint32_t slot = slice * WAVE + ((int)wave * PPW + q) * RPW + sub;
      int64_t col = (int64_t)prow[q] + o;
      bool ok = pok[q] && col >= 0 && col < (int64_t)A.ncols && cok;
      uint32_t v = ok ? ldval<typename AR::ValT>(A.bval, T.b0 + d * rows_in_tile + slot) : 0u;
      uint32_t x = ok ? (uint32_t)X[col * ldx + comp] : 0u;
      acc.a[q] += AR::mul(v, x);
    }
    acc.tick(A);
  }
  for (uint32_t g0 = 0; g0 < groups; g0 += GU) {
    uint32_t w[GU][WIDE], v[GU][WIDE];
#pragma unroll
    for (int u = 0; u < GU; ++u) {
      u32x4 q = g0 + u < groups ? __builtin_nontemporal_load((const u32x4*)(ent + (size_t)(g0 + u) * SELL_GROUP))
                                : (u32x4)(PAD_WORD);
      w[u][0] = q.x;
      w[u][1] = q.y;
      w[u][2] = q.z;
      w[u][3] = q.w;
    }
#pragma unroll
    for (int u = 0; u < GU; ++u) load_values4<AR>(A, w[u], g0 + u < groups ? choff[g0 + u] : 0u, v[u]);
    // every gather of the GU groups is issued before the first term is added
    // (groups past the last hold padding words and add nothing)
    uint32_t xv[GU][WIDE][PPW];
#pragma unroll
    for (int u = 0; u < GU; ++u)
#pragma unroll
      for (int k = 0; k < WIDE; ++k)
#pragma unroll
        for (int q = 0; q < PPW; ++q) {
          int src = (((int)wave * PPW + q) % S) * RPW + (int)sub;
          uint32_t wp = (uint32_t)__shfl((int)w[u][k], src);
          xv[u][k][q] = ((wp >> TAG_SHIFT) != TAG_PAD && cok && pok[q])
                            ? (uint32_t)X[(int64_t)(wp & COL_MASK) * ldx + comp]
                            : 0u;
        }
#pragma unroll
    for (int u = 0; u < GU; ++u)
#pragma unroll
      for (int k = 0; k < WIDE; ++k) {
#pragma unroll
        for (int q = 0; q < PPW; ++q) {
          int src = (((int)wave * PPW + q) % S) * RPW + (int)sub;
          uint32_t wp = (uint32_t)__shfl((int)w[u][k], src), vp = (uint32_t)__shfl((int)v[u][k], src);
          acc.a[q] += term<AR>(wp >> TAG_SHIFT, vp, xv[u][k][q], A.m);
        }
        acc.tick(A);
      }
  }
  uint32_t r[PPW];
#pragma unroll
  for (int q = 0; q < PPW; ++q) {
    r[q] = AR::reduce(acc.a[q], A);
    if (pok[q] && cok) Y[(int64_t)prow[q] * ldy + comp] = (Tv)r[q];
  }
  if constexpr (PROJ) {
    LaneAcc<AR, S> pj;  // pj.a[a]: sum over this lane's rows of U[row][a] * W[row][comp]
    pj.init(A);
#pragma unroll
    for (int q = 0; q < PPW; ++q) {
      uint32_t u = urow[q];
      uint32_t w = (pok[q] && cok) ? r[q] : 0u;
#pragma unroll
      for (int a = 0; a < S; ++a) {
        uint32_t ua = (uint32_t)__shfl((int)u, (int)(sub * S) + a);
        pj.a[a] += AR::mul(ua, w);
      }
      pj.tick(A);
    }
    pj.to_residues(A);
    // sum over the RPW lanes of the same component (lane bits above log2 S)
#pragma unroll
    for (int a = 0; a < S; ++a) {
      Acc t = pj.a[a];
      for (int o = S; o < WAVE; o <<= 1) t += shfl_xor_acc(t, o, WAVE);
      pj.a[a] = t;
    }
    if (sub == 0) {
#pragma unroll
      for (int a = 0; a < S; ++a)
        if (a < s && cok) red[wave * 256 + a * s + comp] = (uint64_t)AR::reduce(pj.a[a], A);
    }
    __syncthreads();
    const uint32_t ss = (uint32_t)(s * s);
    if (threadIdx.x < ss) {
      uint64_t t = 0;
      for (int q = 0; q < NW; ++q) t += red[q * 256 + threadIdx.x];
      out[threadIdx.x] = t;
    }
  }
}

// Two SELL slices by one workgroup for s = 8, the common block width: a wave
// takes 32 rows of a slice, two lanes per row, and a lane keeps four of the
// row's eight components. Each gather is then one 16-byte load (half a row of
// W_i) and a wave instruction covers 32 rows, against 8 rows and 4-byte loads
// in the (row, component) layout. Both lanes of a row load the row's entry
// words themselves. Its values are found without the other half's words: a
// group's values lie in row order, so the lower half's start at the group's
// offset and the upper half's end where the next chunk's begin (the offsets
// end with the total), and ballots over one lane per row count those before a
// row within the half. With PROJ the wave writes its rows of U and W_{i+1} to
// LDS and lane p = 8a + c sums U[row][a] W_{i+1}[row][c] over its 32 rows.
// X, Y and U have leading dimension 8.
// GU: 4-column groups loaded together.
template <class AR, bool PROJ, int GU>
__device__ inline void sell_slice_h8(const DevMat& A, const Tile& T, uint32_t slice, uint32_t half,
                                     const int32_t* __restrict__ X, int32_t* __restrict__ Y,
                                     const int32_t* __restrict__ U, uint32_t* wl /* LDS [2][32][8] of this wave */,
                                     uint64_t* red /* LDS [TILE_THREADS] */) {
  const uint32_t lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
  const uint32_t rr = lane >> 1, h = lane & 1u;
  const bool live = slice < T.ne;
  uint32_t off = 0;
  for (uint32_t k = 0; k < slice && live; ++k) off += A.swidth[T.aux + k];
  const uint32_t groups = live ? A.swidth[T.aux + slice] : 0u;
  const uint32_t srow = half * 32u + rr;  // this lane's row in the slice
  const uint32_t* ent = A.ent + T.e0 + (size_t)off * SELL_GROUP + srow * WIDE;
  const uint32_t* choff = A.choff + T.c0 + off;
  const uint32_t slot = slice * WAVE + srow;
  const uint32_t prow = !live ? 0xFFFFFFFFu : (T.kind & TF_SORTED) ? A.perm[T.row0 + slot] : T.row0 + slot;
  const bool pok = prow < A.nrows;
  // U of the projection does not depend on the product: its load goes out first
  u32x4 uq = {0u, 0u, 0u, 0u};
  if (PROJ && pok) uq = *(const u32x4*)(U + (int64_t)prow * 8 + 4 * h);
  LaneAcc<AR, 4> acc;
  acc.init(A);
  const uint32_t nd = tile_nd(T.kind), rows_in_tile = tile_rows(T.kind);
  for (uint32_t d = 0; d < nd && live; ++d) {
    const int64_t col = (int64_t)prow + A.boffs[T.boff + d];
    const bool ok = pok && col >= 0 && col < (int64_t)A.ncols;
    const uint32_t v = ok ? ldval<typename AR::ValT>(A.bval, T.b0 + d * rows_in_tile + slot) : 0u;
    u32x4 x = {0u, 0u, 0u, 0u};
    if (ok) x = *(const u32x4*)(X + col * 8 + 4 * h);
    acc.a[0] += AR::mul(v, x.x);
    acc.a[1] += AR::mul(v, x.y);
    acc.a[2] += AR::mul(v, x.z);
    acc.a[3] += AR::mul(v, x.w);
    acc.tick(A);
  }
  const uint64_t even = 0x5555555555555555ull;  // one lane per row
  for (uint32_t g0 = 0; g0 < groups; g0 += GU) {
    uint32_t w[GU][WIDE], v[GU][WIDE];
    u32x4 xv[GU][WIDE];
#pragma unroll
    for (int u = 0; u < GU; ++u) {
      u32x4 q = g0 + u < groups ? __builtin_nontemporal_load((const u32x4*)(ent + (size_t)(g0 + u) * SELL_GROUP))
                                : (u32x4)(PAD_WORD);
      w[u][0] = q.x;
      w[u][1] = q.y;
      w[u][2] = q.z;
      w[u][3] = q.w;
      // general values of the rows before this one in the half (even lanes only), and in the half
      uint32_t below = 0, total = 0, mine = 0;
#pragma unroll
      for (int k = 0; k < WIDE; ++k) {
        const bool gen = (w[u][k] >> TAG_SHIFT) == TAG_GEN;
        const uint64_t mk = __ballot(gen && h == 0) & even;
        below += lanes_below(mk);
        total += (uint32_t)__builtin_popcountll(mk);
        mine += gen ? 1u : 0u;
      }
      if (h) below -= mine;  // an odd lane's count includes its own row's even lane
      uint32_t base = 0;
      if (g0 + u < groups) base = half ? choff[g0 + u + 1] - total : choff[g0 + u];
      if (pok) {
        load_values_at<AR>(A, w[u], base + below, v[u]);
      } else {
#pragma unroll
        for (int k = 0; k < WIDE; ++k) v[u][k] = 0u;
      }
#pragma unroll
      for (int k = 0; k < WIDE; ++k) {
        xv[u][k] = (u32x4){0u, 0u, 0u, 0u};
        if ((w[u][k] >> TAG_SHIFT) != TAG_PAD && pok)
          xv[u][k] = *(const u32x4*)(X + (int64_t)(w[u][k] & COL_MASK) * 8 + 4 * h);
      }
    }
#pragma unroll
    for (int u = 0; u < GU; ++u)
#pragma unroll
      for (int k = 0; k < WIDE; ++k) {
        const uint32_t tag = w[u][k] >> TAG_SHIFT;
        acc.a[0] += term<AR>(tag, v[u][k], xv[u][k].x, A.m);
        acc.a[1] += term<AR>(tag, v[u][k], xv[u][k].y, A.m);
        acc.a[2] += term<AR>(tag, v[u][k], xv[u][k].z, A.m);
        acc.a[3] += term<AR>(tag, v[u][k], xv[u][k].w, A.m);
        acc.tick(A);
      }
  }
  u32x4 r;
  r.x = AR::reduce(acc.a[0], A);
  r.y = AR::reduce(acc.a[1], A);
  r.z = AR::reduce(acc.a[2], A);
  r.w = AR::reduce(acc.a[3], A);
  if (pok) *(u32x4*)(Y + (int64_t)prow * 8 + 4 * h) = r;
  if constexpr (PROJ) {
    // this wave's rows of W_{i+1} (wl[0]) and U (wl[1]); rows outside the matrix hold zeros
    const u32x4 z = {0u, 0u, 0u, 0u};
    *(u32x4*)(wl + rr * 8 + 4 * h) = pok ? r : z;
    *(u32x4*)(wl + 256 + rr * 8 + 4 * h) = pok ? uq : z;
    __syncthreads();
    const uint32_t a = lane >> 3, c = lane & 7u;
    LaneAcc<AR, 1> pj;
    pj.init(A);
#pragma unroll 8
    for (uint32_t q = 0; q < 32; ++q) {
      pj.a[0] += AR::mul(wl[256 + q * 8 + a], wl[q * 8 + c]);
      pj.tick(A);
    }
    red[wave * WAVE + lane] = (uint64_t)AR::reduce(pj.a[0], A);
  }
}

// ------------------------------------------------------------- kernels -----
// The blocks W_i and U live in workspace as int32 (n x s, ld = s), whatever the
// caller's element type: residues are below 2^31, and the 32-bit copies halve
// the bytes every iteration gathers, writes and projects. Only S (and the
// final W_L) take the caller's type.
using Tw = int32_t;

struct SeqArgs {
  const Tw* U;         // n x s, ld s
  Tw* W[2];            // W_i lives in W[i & 1]; n x s, ld s
  uint64_t* part[2];   // [4*ntiles][s*s] partial sums, by parity
  uint64_t* mid[2];    // [NMID][s*s] folded partial sums, by parity
  void* S;             // L*s*s entries of the caller's type
  const int64_t* base; // device counter: iteration number of node 0 of this batch
  int64_t L;
  int32_t s;
  int32_t last_w;      // compute W_L too (at i = L-1)
};

// Projection of W_0 = V into the partials of iteration 0.
template <class AR>
__global__ __launch_bounds__(TILE_THREADS) void k_seq_first(DevMat A, SeqArgs q) {
  __shared__ uint64_t red[TILE_THREADS];
  const Tile T = A.tiles[blockIdx.x];
  const int64_t ss = (int64_t)q.s * q.s;
  uint64_t* out = q.part[0] + (int64_t)blockIdx.x * SELL_SLICES * ss;
  tile_projection<AR, Tw>(A, T, q.U, q.s, q.W[0], q.s, q.s, red, out);
  for (int64_t k = ss + threadIdx.x; k < SELL_SLICES * ss; k += TILE_THREADS) out[k] = 0;
}

// Iteration i = *base + j. Four workgroups per tile (one per SELL slice; for
// the other tile kinds only the first works), then NMID workgroups that fold
// the partials of W_i into NMID sums (mid, by parity), then one workgroup that
// turns the sums of iteration i-1 into S_{i-1}.
constexpr uint32_t NMID = 64;

// groups per load round of the s = 8 step (sell_slice_h8)
constexpr int SEQ_H8_GROUPS = 1;

// ONLY_SELL: the matrix has SELL tiles only, and the kernel is built without
// the STREAM/LONG path, whose registers would otherwise set the occupancy.
// H8 > 0 (s = 8): two workgroups per tile, each taking two SELL slices (two
// waves per slice, sell_slice_h8 loading H8 groups together); workgroup
// 2t + h writes the partial of slot 4t + 2h and zeros into slot 4t + 2h + 1,
// so the partial buffers keep four slots per tile either way.
template <class AR, typename Ts, int S, bool ONLY_SELL, int H8>
__device__ __forceinline__ void seq_step(const DevMat& A, const SeqArgs& q, int32_t j, unsigned char* lds) {
  const int64_t i = *q.base + j;
  if (i >= q.L) return;
  const int s = q.s;
  const int64_t ss = (int64_t)s * s;
  const uint32_t nparts = A.ntiles * SELL_SLICES;
  const uint32_t nwork = H8 ? A.ntiles * 2 : nparts;
  if (blockIdx.x >= nwork) {
    const uint32_t r = blockIdx.x - nwork;
    uint32_t pair;
    if (r < NMID) {  // stage 1 for iteration i
      uint64_t t = fold_partials(A, q.part[i & 1], r, NMID, nparts, s, (uint64_t*)lds, &pair);
      if (pair < ss) q.mid[i & 1][r * ss + pair] = t;
    } else if (i > 0) {  // stage 2 for iteration i-1
      uint64_t t = fold_partials(A, q.mid[(i - 1) & 1], 0, 1, NMID, s, (uint64_t*)lds, &pair);
      if (pair < ss) ((Ts*)q.S)[(i - 1) * ss + pair] = (Ts)mod_u64(t, A.m, A.mu);
    }
    return;
  }
  const bool last = i + 1 == q.L;
  if (last && !q.last_w) return;
  const Tw* Win = q.W[i & 1];
  Tw* Wout = q.W[(i + 1) & 1];
  const int64_t ldin = s;
  const uint32_t t = H8 ? blockIdx.x / 2 : blockIdx.x / SELL_SLICES;
  const uint32_t slice = H8 ? 2 * (blockIdx.x % 2) : blockIdx.x % SELL_SLICES;  // H8: first of the two slices
  const Tile T = A.tiles[t];
  uint64_t* out = q.part[(i + 1) & 1] + (int64_t)(t * SELL_SLICES + slice) * ss;
  if (tile_kind(T.kind) == TK_SELL) {
    if constexpr (H8 > 0) {
      const uint32_t wave = threadIdx.x / WAVE;
      uint32_t* wl = (uint32_t*)lds + wave * 512;
      uint64_t* red = (uint64_t*)(lds + 4 * 512 * sizeof(uint32_t));
      if (last) {
        sell_slice_h8<AR, false, H8>(A, T, slice + (wave >> 1), wave & 1u, Win, Wout, nullptr, nullptr, nullptr);
        return;
      }
      sell_slice_h8<AR, true, H8>(A, T, slice + (wave >> 1), wave & 1u, Win, Wout, q.U, wl, red);
      __syncthreads();
      if (threadIdx.x < WAVE) {
        uint64_t sum = 0;  // four residues
#pragma unroll
        for (int w = 0; w < 4; ++w) sum += red[w * WAVE + threadIdx.x];
        out[threadIdx.x] = sum;
        out[ss + threadIdx.x] = 0;
      }
    } else {
      if (last) sell_slice_rc<AR, Tw, S, false>(A, T, slice, Win, ldin, Wout, s, s, nullptr, 0, nullptr, nullptr);
      else sell_slice_rc<AR, Tw, S, true>(A, T, slice, Win, ldin, Wout, s, s, q.U, s, out, (uint64_t*)lds);
    }
    return;
  }
  if constexpr (!ONLY_SELL) {
    if (slice != 0) {  // idle slices of a STREAM/LONG tile: empty partials
      if (!last && threadIdx.x < ss) {
        out[threadIdx.x] = 0;
        if (H8) out[ss + threadIdx.x] = 0;
      }
      return;
    }
    if (tile_kind(T.kind) == TK_LONG) long_tile<AR, Tw, Tw, S, 1>(A, T, Win, ldin, Wout, s, s, 1, 0, lds);
    else stream_tile_s<AR, Tw, Tw, S>(A, T, Win, ldin, Wout, s, s, 1, 0, lds);
    if (last) return;  // W_L only: no partials needed
    // the projection reads back only rows this workgroup wrote: a workgroup barrier orders them
    __syncthreads();
    tile_projection<AR, Tw>(A, T, q.U, s, Wout, s, s, (uint64_t*)lds, out);
    if (H8 && threadIdx.x < ss) out[ss + threadIdx.x] = 0;
  }
}

template <class AR, typename Ts, int S, bool ONLY_SELL>
__global__ __launch_bounds__(TILE_THREADS) void k_seq_step(DevMat A, SeqArgs q, int32_t j) {
  extern __shared__ __align__(16) unsigned char lds[];
  seq_step<AR, Ts, S, ONLY_SELL, 0>(A, q, j, lds);
}

// s = 8 (sell_slice_h8): the 6,256 waves of a 200,000-row operand are resident at once with 7 waves
// per SIMD, so the kernel is held to the registers that allow 7
template <class AR, typename Ts, bool ONLY_SELL>
__global__ __launch_bounds__(TILE_THREADS, 7) void k_seq_step_h8(DevMat A, SeqArgs q, int32_t j) {
  extern __shared__ __align__(16) unsigned char lds[];
  seq_step<AR, Ts, 8, ONLY_SELL, SEQ_H8_GROUPS>(A, q, j, lds);
}

// S_{L-1} from the sums of the last iteration.
template <typename Ts>
__global__ __launch_bounds__(TILE_THREADS) void k_seq_finish(DevMat A, SeqArgs q) {
  __shared__ uint64_t red[TILE_THREADS];
  const int64_t i = q.L - 1;
  const int64_t ss = (int64_t)q.s * q.s;
  uint32_t pair;
  uint64_t t = fold_partials(A, q.mid[i & 1], 0, 1, NMID, q.s, red, &pair);
  if (pair < ss) ((Ts*)q.S)[i * ss + pair] = (Ts)mod_u64(t, A.m, A.mu);
}

__global__ void k_seq_counter(int64_t* base, int64_t add, int set) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *base = set ? add : *base + add;
}

template <class AR, typename Ts, bool ONLY_SELL>
static hipError_t seq_go(const DevMat& A, int64_t mte, const SeqArgs& q, int batch, hipStream_t user) {
  const int s = q.s;
  const int S = s <= 2 ? 2 : s <= 4 ? 4 : s <= 8 ? 8 : 16;  // the step always runs the multi-vector tiles
  size_t lds = tiles_lds_bytes<AR>(mte, S);
  if (lds < SELL_SLICES * TILE_THREADS * sizeof(uint64_t)) lds = SELL_SLICES * TILE_THREADS * sizeof(uint64_t);
  // s = 8: half-row lanes (sell_slice_h8), whose LDS holds 4 waves x 2 KB of rows and the 256 sums
  const bool h8 = s == 8;
  const size_t h8_lds = 4 * 512 * sizeof(uint32_t) + TILE_THREADS * sizeof(uint64_t);
  if (h8 && lds < h8_lds) lds = h8_lds;
  int64_t* base = const_cast<int64_t*>(q.base);
  auto step = [&](hipStream_t st, int32_t j) {
    dim3 g((h8 ? A.ntiles * 2 : A.ntiles * SELL_SLICES) + NMID + 1), b(TILE_THREADS);
    switch (S) {
      case 2: hipLaunchKernelGGL((k_seq_step<AR, Ts, 2, ONLY_SELL>), g, b, lds, st, A, q, j); break;
      case 4: hipLaunchKernelGGL((k_seq_step<AR, Ts, 4, ONLY_SELL>), g, b, lds, st, A, q, j); break;
      case 8:
        if (h8) hipLaunchKernelGGL((k_seq_step_h8<AR, Ts, ONLY_SELL>), g, b, lds, st, A, q, j);
        else hipLaunchKernelGGL((k_seq_step<AR, Ts, 8, ONLY_SELL>), g, b, lds, st, A, q, j);
        break;
      default: hipLaunchKernelGGL((k_seq_step<AR, Ts, 16, ONLY_SELL>), g, b, lds, st, A, q, j); break;
    }
  };
  hipLaunchKernelGGL((k_seq_counter), dim3(1), dim3(64), 0, user, base, (int64_t)0, 1);
  hipLaunchKernelGGL((k_seq_first<AR>), dim3(A.ntiles), dim3(TILE_THREADS), 0, user, A, q);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t L = q.L;
  int64_t nbatch = batch > 0 ? L / batch : 0;
  if (nbatch >= 2) {
    // capture one batch on a private stream, replay it on the caller's stream
    hipStream_t cs;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      for (int32_t j = 0; j < batch; ++j) step(cs, j);
      hipLaunchKernelGGL((k_seq_counter), dim3(1), dim3(64), 0, cs, base, (int64_t)batch, 0);
      e = hipStreamEndCapture(cs, &graph);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    for (int64_t r = 0; r < nbatch && e == hipSuccess; ++r) e = hipGraphLaunch(exec, user);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) return e;
  } else {
    nbatch = 0;
  }
  // the remaining iterations, launched directly (the counter holds nbatch*batch)
  for (int64_t i = nbatch * batch; i < L; ++i) step(user, (int32_t)(i - nbatch * batch));
  hipLaunchKernelGGL((k_seq_finish<Ts>), dim3(1), dim3(TILE_THREADS), 0, user, A, q);
  return hipGetLastError();
}

template <typename Ti, typename To>
__global__ void k_convert_block(const Ti* __restrict__ in, int64_t ldi, To* __restrict__ out, int64_t ldo, int64_t n,
                                int s) {
  int64_t total = n * s;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    int64_t k = t / s;
    int c = (int)(t - k * s);
    out[k * ldo + c] = (To)in[k * ldi + c];
  }
}

// n x s block copy from element type `ti` (stride ldi) to `to` (stride ldo); values are residues, so
// narrowing int64 -> int32 keeps them.
static hipError_t convert_block(ffx_dtype ti, const void* in, int64_t ldi, ffx_dtype to, void* out, int64_t ldo,
                                int64_t n, int s, hipStream_t st) {
  if (n == 0) return hipSuccess;
  int64_t total = n * s;
  int blocks = (int)((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
  dim3 g(blocks), b(256);
  if (ti == FFX_I32 && to == FFX_I32)
    hipLaunchKernelGGL((k_convert_block<int32_t, int32_t>), g, b, 0, st, (const int32_t*)in, ldi, (int32_t*)out, ldo, n, s);
  else if (ti == FFX_I32)
    hipLaunchKernelGGL((k_convert_block<int32_t, int64_t>), g, b, 0, st, (const int32_t*)in, ldi, (int64_t*)out, ldo, n, s);
  else if (to == FFX_I32)
    hipLaunchKernelGGL((k_convert_block<int64_t, int32_t>), g, b, 0, st, (const int64_t*)in, ldi, (int32_t*)out, ldo, n, s);
  else
    hipLaunchKernelGGL((k_convert_block<int64_t, int64_t>), g, b, 0, st, (const int64_t*)in, ldi, (int64_t*)out, ldo, n, s);
  return hipGetLastError();
}

hipError_t launch_copy_block(ffx_dtype dt, const void* in, int64_t ldi, void* out, int64_t ldo, int64_t n, int s,
                             hipStream_t st) {
  return convert_block(dt, in, ldi, dt, out, ldo, n, s, st);
}

hipError_t launch_sequence(int ak, bool only_sell, const DevMat& A, int64_t mte, ffx_dtype dt, const void* U,
                           int64_t ldu, const void* V, int64_t ldv, int64_t L, int s, void* S, void* Wlast, void* w0,
                           void* w1, void* u32, uint64_t* p0, uint64_t* p1, int64_t* counter, int batch,
                           hipStream_t st) {
  const int64_t n = A.nrows;
  // int32 copies of U and W_0 = V in workspace
  hipError_t e = convert_block(dt, U, ldu, FFX_I32, u32, s, n, s, st);
  if (e == hipSuccess) e = convert_block(dt, V, ldv, FFX_I32, w0, s, n, s, st);
  if (e != hipSuccess) return e;
  SeqArgs q;
  // the fold buffers live at the end of the partial buffers
  const int64_t ss = (int64_t)s * s;
  q.mid[0] = p0 + (int64_t)A.ntiles * SELL_SLICES * ss;
  q.mid[1] = p1 + (int64_t)A.ntiles * SELL_SLICES * ss;
  q.U = (const Tw*)u32;
  q.W[0] = (Tw*)w0;
  q.W[1] = (Tw*)w1;
  q.part[0] = p0;
  q.part[1] = p1;
  q.S = S;
  q.base = counter;
  q.L = L;
  q.s = s;
  q.last_w = Wlast ? 1 : 0;
  auto go = [&](auto ar) -> hipError_t {
    using AR = decltype(ar);
    if (only_sell) {
      if (dt == FFX_I32) return seq_go<AR, int32_t, true>(A, mte, q, batch, st);
      return seq_go<AR, int64_t, true>(A, mte, q, batch, st);
    }
    if (dt == FFX_I32) return seq_go<AR, int32_t, false>(A, mte, q, batch, st);
    return seq_go<AR, int64_t, false>(A, mte, q, batch, st);
  };
  switch (ak) {
    case AK_SMALL: e = go(ArSmall{}); break;
    case AK_M31: e = go(ArM31{}); break;
    case AK_BIG_CH: e = go(ArBig<true>{}); break;
    default: e = go(ArBig<false>{}); break;
  }
  if (e != hipSuccess || !Wlast) return e;
  return convert_block(FFX_I32, q.W[L & 1], s, dt, Wlast, s, n, s, st);  // W_L, in the caller's type
}

}  // namespace ffx
