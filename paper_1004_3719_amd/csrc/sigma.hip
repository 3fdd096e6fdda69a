// Block Wiedemann steps 2 and 3 (Section 3) over a prime field F_p, p < 2^31:
// the order basis (sigma-basis) of a power series by PM-Basis (Giorgi,
// Jeannerod and Villard, ISSAC 2003; Section 3.2 "Parallelization of the
// sigma-basis computation"), the minimal matrix generator of the sequence, and
// rank = deg det F - codeg det F.
//
// PM-Basis splits the order in two halves: the basis M1 of the first half, the
// middle product R = [x^s1 .. x^(s-1)] (M1 G), the basis M2 of R with M1's
// degrees, and M = M2 M1. Orders up to LEAF are done by the one-order-at-a-time
// M-Basis in a single workgroup whose basis lives in LDS. Because M-Basis only
// looks at the residual coefficient [x^k](M G) and the degrees, the
// divide-and-conquer result is the same basis, step for step, as M-Basis run
// over the whole order.
//
// Large polynomial matrix products go through number-theoretic transforms over
// three word-size primes and a CRT (the paper's DFT multiplication; see the
// NTT section below); the small ones, where the transforms' passes cost more
// than the convolution, are schoolbook convolutions on the vector ALU.
// A workgroup computes 256 consecutive coefficients of one entry; for each
// inner index q and each 256-coefficient chunk of A it stages the chunk of A and
// the 511 coefficients of B that the tile needs in LDS, and every lane adds
// 256 products into a 96-bit accumulator (64-bit sum plus a carry count), so a
// coefficient is reduced once.
#include <algorithm>
#include <atomic>
#include <vector>

#include "host.h"
#include "launch.h"

namespace ffx {

constexpr int SB_LEAF = 32;    // orders done by the in-LDS M-Basis
constexpr int SB_MAXM = 16;    // rows of the basis
constexpr int SB_MAXN = 8;     // columns of the series
constexpr int PM_TILE = 256;   // coefficients per workgroup in the products

struct Field {
  uint32_t p;
  uint64_t mu;    // floor((2^64-1)/p)
  uint32_t r64;   // 2^64 mod p
  int mersenne;   // p = 2^31 - 1: products fold with shifts
};

__device__ inline uint32_t fmul(uint32_t a, uint32_t b, const Field& F) {
  uint64_t x = (uint64_t)a * b;
  if (F.mersenne) {  // x < 2^62: two folds bring it to at most p + 1
    x = (x & 0x7FFFFFFFull) + (x >> 31);
    x = (x & 0x7FFFFFFFull) + (x >> 31);
    return (uint32_t)(x >= 0x7FFFFFFFull ? x - 0x7FFFFFFFull : x);
  }
  return mod_u64(x, F.p, F.mu);
}

// (hi * 2^64 + lo) mod p, hi < 2^32
__device__ inline uint32_t fold96(uint64_t lo, uint32_t hi, const Field& F) {
  uint64_t h = (uint64_t)(hi % F.p) * F.r64;
  return mod_u64(h + mod_u64(lo, F.p, F.mu), F.p, F.mu);
}

__device__ inline uint32_t finv(uint32_t a, const Field& F) {  // a^(p-2), a != 0
  uint32_t r = 1, b = a, e = F.p - 2;
  while (e) {
    if (e & 1) r = fmul(r, b, F);
    b = fmul(b, b, F);
    e >>= 1;
  }
  return r;
}

// Sums of products of two residues: for p = 2^31 - 1 each product is folded
// below 2^32 and added to 64 bits (no reduction for 2^31 terms); otherwise the
// products are added to a 96-bit sum.
template <bool MERS>
struct Acc96 {
  uint64_t lo = 0;
  uint32_t hi = 0;
  __device__ inline void add(uint64_t prod) {
    if (MERS) {
      lo += (prod & 0x7FFFFFFFull) + (prod >> 31);
    } else {
      lo += prod;
      hi += lo < prod;
    }
  }
  __device__ inline uint32_t reduce(const Field& F) const {
    if (MERS) {
      uint64_t x = (lo & 0x7FFFFFFFull) + (lo >> 31);  // below 2^33
      x = (x & 0x7FFFFFFFull) + (x >> 31);             // at most p + 3
      return (uint32_t)(x >= 0x7FFFFFFFull ? x - 0x7FFFFFFFull : x);
    }
    return fold96(lo, hi, F);
  }
};

// C[r][c][t] = sum_q sum_j A[r][q][j] B[q][c][k0 + t - j] for t < len.
// A: R x Q entries of la coefficients (entry (r,q) at A + (r*Q+q)*sa); B: Q x NC
// entries of lb coefficients (stride sb); C: R x NC entries (stride sc).
__global__ void __launch_bounds__(PM_TILE) k_polymul(const uint32_t* __restrict__ A, int64_t sa, int64_t la,
                                                     const uint32_t* __restrict__ B, int64_t sb, int64_t lb,
                                                     uint32_t* __restrict__ C, int64_t sc, int64_t k0, int64_t len,
                                                     int Q, int NC, Field F) {
  __shared__ uint32_t As[PM_TILE];
  __shared__ uint32_t Bs[2 * PM_TILE];
  const int tid = threadIdx.x;
  const int r = blockIdx.y / NC, c = blockIdx.y % NC;
  const int64_t kbase = k0 + (int64_t)blockIdx.x * PM_TILE;
  uint64_t lo = 0;
  uint32_t hi = 0;
  const int64_t jlo = std::max<int64_t>(0, kbase - (lb - 1));
  const int64_t jhi = std::min<int64_t>(la - 1, kbase + PM_TILE - 1);
  for (int q = 0; q < Q; ++q) {
    const uint32_t* a = A + (int64_t)(r * Q + q) * sa;
    const uint32_t* b = B + (int64_t)(q * NC + c) * sb;
    for (int64_t j0 = jlo; j0 <= jhi; j0 += PM_TILE) {
      __syncthreads();
      As[tid] = (j0 + tid <= jhi) ? a[j0 + tid] : 0u;
      // Bs[u] = B[kbase - j0 - (PM_TILE-1) + u], u < 2*PM_TILE - 1
      const int64_t base = kbase - j0 - (PM_TILE - 1);
      for (int u = tid; u < 2 * PM_TILE - 1; u += PM_TILE) {
        const int64_t idx = base + u;
        Bs[u] = (idx >= 0 && idx < lb) ? b[idx] : 0u;
      }
      __syncthreads();
#pragma unroll 8
      for (int jj = 0; jj < PM_TILE; ++jj) {
        const uint64_t prod = (uint64_t)As[jj] * Bs[tid - jj + PM_TILE - 1];
        lo += prod;
        hi += lo < prod;
      }
    }
  }
  const int64_t t = (int64_t)blockIdx.x * PM_TILE + tid;
  if (t < len) C[(int64_t)blockIdx.y * sc + t] = fold96(lo, hi, F);
}

// The same product with PM_OUT = 4 * PM_TILE coefficients per workgroup, four
// consecutive ones per lane, for products large enough to fill the GPU with
// such tiles: a lane keeps the B values of its four outputs in registers and
// shifts them by one per j, reading the next four B values and four A values
// (the same in every lane) with one aligned 16-byte read each, so each LDS read
// serves eight multiply-adds. For p = 2^31 - 1 the four products an output
// gets per group of four j are added raw (below 2^64) and folded once.
constexpr int PM_OUT = 4 * PM_TILE;
template <bool MERS>
__global__ void __launch_bounds__(PM_TILE) k_polymul4(const uint32_t* __restrict__ A, int64_t sa, int64_t la,
                                                      const uint32_t* __restrict__ B, int64_t sb, int64_t lb,
                                                      uint32_t* __restrict__ C, int64_t sc, int64_t k0, int64_t len,
                                                      int Q, int NC, Field F) {
  typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
  __shared__ __align__(16) uint32_t As[PM_TILE];
  __shared__ __align__(16) uint32_t Bs[PM_OUT + PM_TILE];  // Bs[1 + u] = B[kbase - j0 - (PM_TILE - 1) + u]
  const int tid = threadIdx.x;
  const int r = blockIdx.y / NC, c = blockIdx.y % NC;
  const int64_t kbase = k0 + (int64_t)blockIdx.x * PM_OUT;
  Acc96<MERS> acc[4];
  const int64_t jlo = std::max<int64_t>(0, kbase - (lb - 1));
  const int64_t jhi = std::min<int64_t>(la - 1, kbase + PM_OUT - 1);
  for (int q = 0; q < Q; ++q) {
    const uint32_t* a = A + (int64_t)(r * Q + q) * sa;
    const uint32_t* b = B + (int64_t)(q * NC + c) * sb;
    for (int64_t j0 = jlo; j0 <= jhi; j0 += PM_TILE) {
      __syncthreads();
      As[tid] = (j0 + tid <= jhi) ? a[j0 + tid] : 0u;
      const int64_t base = kbase - j0 - (PM_TILE - 1);
      for (int u = tid; u < PM_OUT + PM_TILE - 1; u += PM_TILE) {
        const int64_t idx = base + u;
        Bs[1 + u] = (idx >= 0 && idx < lb) ? b[idx] : 0u;
      }
      if (tid == 0) Bs[0] = 0u;
      __syncthreads();
      // output t = 4 tid + v meets A[j0 + jj] and Bs[t - jj + PM_TILE]
      const int t0 = 4 * tid + PM_TILE;
      uint32_t bv0 = Bs[t0], bv1 = Bs[t0 + 1], bv2 = Bs[t0 + 2], bv3 = Bs[t0 + 3];
      for (int jj = 0; jj < PM_TILE; jj += 4) {
        const u32x4_t a4 = *(const u32x4_t*)&As[jj];
        const u32x4_t nb = *(const u32x4_t*)&Bs[t0 - jj - 4];  // index >= 4 tid >= 0
        uint64_t g0 = 0, g1 = 0, g2 = 0, g3 = 0;
        auto step = [&](uint32_t av, uint32_t next) {
          const uint64_t x = av;
          if (MERS) {
            g0 += x * bv0;
            g1 += x * bv1;
            g2 += x * bv2;
            g3 += x * bv3;
          } else {
            acc[0].add(x * bv0);
            acc[1].add(x * bv1);
            acc[2].add(x * bv2);
            acc[3].add(x * bv3);
          }
          bv3 = bv2;
          bv2 = bv1;
          bv1 = bv0;
          bv0 = next;
        };
        step(a4.x, nb.w);
        step(a4.y, nb.z);
        step(a4.z, nb.y);
        step(a4.w, nb.x);
        if (MERS) {
          acc[0].lo += (g0 & 0x7FFFFFFFull) + (g0 >> 31);
          acc[1].lo += (g1 & 0x7FFFFFFFull) + (g1 >> 31);
          acc[2].lo += (g2 & 0x7FFFFFFFull) + (g2 >> 31);
          acc[3].lo += (g3 & 0x7FFFFFFFull) + (g3 >> 31);
        }
      }
    }
  }
  const int64_t t = (int64_t)blockIdx.x * PM_OUT + 4 * tid;
#pragma unroll
  for (int v = 0; v < 4; ++v)
    if (t + v < len) C[(int64_t)blockIdx.y * sc + t + v] = acc[v].reduce(F);
}

// Products whose A entries have at most PMS_MAXA coefficients and whose output
// entries at most PMS_MAX_TILES * PM_TILE: the lower levels of the recursion,
// where a product is a few thousand multiply-adds per entry and the tile
// kernel's time goes to a barrier and a round trip to memory per inner index.
// Here one workgroup per output entry and PM_TILE outputs stages every A and B
// coefficient it needs in LDS at once, and four groups of PM_TILE lanes each
// take every fourth inner index q; the four partial sums, reduced, meet in LDS.
constexpr int PMS_MAXA = PM_TILE + 1;
constexpr int PMS_NT = 4 * PM_TILE;
constexpr int PMS_MAX_TILES = 4;  // longer outputs go to the tile kernels
inline size_t polymul_small_lds(int Q, int64_t la) {
  return ((size_t)Q * la + (size_t)Q * (PM_TILE + la - 1) + 3 * PM_TILE) * sizeof(uint32_t);
}
template <bool MERS>
__global__ void __launch_bounds__(PMS_NT) k_polymul_small(const uint32_t* __restrict__ A, int64_t sa, int la,
                                                          const uint32_t* __restrict__ B, int64_t sb, int64_t lb,
                                                          uint32_t* __restrict__ C, int64_t sc, int64_t k0, int64_t len,
                                                          int Q, int NC, Field F) {
  extern __shared__ uint32_t pms[];
  const int tid = threadIdx.x;
  const int r = blockIdx.x / NC, c = blockIdx.x % NC;
  // this workgroup's PM_TILE outputs: coefficients t0 .. t0 + tl - 1 of the entry
  const int64_t t0 = (int64_t)blockIdx.y * PM_TILE;
  const int tl = (int)std::min<int64_t>(PM_TILE, len - t0);
  k0 += t0;
  C += t0;
  const int nb = tl + la - 1;  // B[k0 - (la - 1) .. k0 + tl - 1]
  uint32_t* As = pms;
  uint32_t* Bs = pms + Q * la;
  uint32_t* part_s = Bs + Q * nb;
  for (int i = tid; i < Q * la; i += PMS_NT) {
    const int q = i / la, j = i - q * la;
    As[i] = A[(int64_t)(r * Q + q) * sa + j];
  }
  const int64_t b0 = k0 - (la - 1);
  for (int i = tid; i < Q * nb; i += PMS_NT) {
    const int q = i / nb, u = i - q * nb;
    const int64_t idx = b0 + u;
    Bs[i] = (idx >= 0 && idx < lb) ? B[(int64_t)(q * NC + c) * sb + idx] : 0u;
  }
  __syncthreads();
  const int t = tid % PM_TILE, part = tid / PM_TILE;
  Acc96<MERS> acc;
  if (t < tl) {
    // output k0 + t meets A[j] and B[k0 + t - j] = Bs[t - j + la - 1], for j with 0 <= k0 + t - j < lb
    const int64_t kt = k0 + t;
    const int jlo = (int)std::max<int64_t>(0, kt - (lb - 1));
    const int jhi = (int)std::min<int64_t>(la - 1, kt);
    for (int q = part; q < Q; q += 4) {
      const uint32_t* a = As + q * la;
      const uint32_t* b = Bs + q * nb + t + la - 1;
      for (int j = jlo; j <= jhi; ++j) acc.add((uint64_t)a[j] * b[-j]);
    }
  }
  const uint32_t v = acc.reduce(F);
  if (part > 0) part_s[(part - 1) * PM_TILE + t] = v;
  __syncthreads();
  if (part == 0 && t < tl) {
    uint32_t sum = v;
#pragma unroll
    for (int k = 0; k < 3; ++k) {  // residues below p < 2^31: a sum of two stays below 2^32
      sum += part_s[k * PM_TILE + t];
      sum = sum >= F.p ? sum - F.p : sum;
    }
    C[(int64_t)blockIdx.x * sc + t] = sum;
  }
}

// One-order-at-a-time basis (M-Basis) of the m x n series G to order sg <= SB_LEAF
// with shifted degrees d (in/out, device). M: m x m entries of sm >= sg + 1 coefficients.
// LEAF_NT lanes: the residual takes 8 lanes per entry and the basis update 4 lanes per entry, each
// over a share of the inner index or of the coefficients.
constexpr int LEAF_NT = 1024;
template <bool MERS>
__global__ void __launch_bounds__(LEAF_NT) k_mbasis_leaf(const uint32_t* __restrict__ G, int64_t ldg, int m, int n,
                                                         int sg, int32_t* __restrict__ d, uint32_t* __restrict__ M,
                                                         int64_t sm, Field F) {
  constexpr int LC = SB_LEAF + 1;
  __shared__ uint32_t Ms[2][SB_MAXM][SB_MAXM][LC];
  __shared__ uint32_t Gs[SB_MAXM][SB_MAXN][SB_LEAF + 1];  // padded: the 8 columns fall in different banks
  __shared__ uint32_t Dl[SB_MAXM][SB_MAXN];      // residual coefficient, reduced in place
  __shared__ __align__(16) uint32_t T[SB_MAXM][SB_MAXM];  // this order's row transformation
  __shared__ int dl[SB_MAXM];
  __shared__ uint32_t sc[SB_MAXM];              // scale of each row from fraction-free elimination
  __shared__ int order[SB_MAXM];                // rows by (shifted degree, index)
  __shared__ uint32_t rinfo[SB_MAXM][2];        // per row: first nonzero unused column, its value
  const int tid = threadIdx.x;
  for (int i = tid; i < SB_MAXM * SB_MAXN * SB_LEAF; i += LEAF_NT) {
    int r = i / (SB_MAXN * SB_LEAF), c = (i / SB_LEAF) % SB_MAXN, k = i % SB_LEAF;
    Gs[r][c][k] = (r < m && c < n && k < sg) ? G[(int64_t)(r * n + c) * ldg + k] : 0u;
  }
  for (int i = tid; i < SB_MAXM * SB_MAXM * LC; i += LEAF_NT) {  // both buffers: coefficients above the degree stay 0
    int r = i / (SB_MAXM * LC), c = (i / LC) % SB_MAXM, k = i % LC;
    Ms[0][r][c][k] = (r == c && k == 0) ? 1u : 0u;
    Ms[1][r][c][k] = 0u;
  }
  if (tid < m) {
    dl[tid] = d[tid];
    sc[tid] = 1u;
  }
  __syncthreads();
  int cur = 0;
  for (int k = 0; k < sg; ++k) {
    // residual [x^k](M G): eight lanes per entry, each over an eighth of the inner index; the
    // eight reduced parts meet through shuffles, each sum of two residues reduced at once
    {
      const int o = tid >> 3, part8 = tid & 7;
      Acc96<MERS> acc;
      const int r = o / SB_MAXN, c = o % SB_MAXN;
      if (r < m && c < n) {
        for (int q = part8; q < m; q += 8) {
#pragma unroll 8
          for (int j = 0; j <= k; ++j) acc.add((uint64_t)Ms[cur][r][q][j] * Gs[q][c][k - j]);
        }
      }
      uint32_t v = (r < m && c < n) ? acc.reduce(F) : 0u;
#pragma unroll
      for (int sh = 1; sh < 8; sh <<= 1) {
        const uint32_t t = v + (uint32_t)__shfl_xor((int)v, sh);  // below 2p < 2^32
        v = t >= F.p ? t - F.p : t;
      }
      if (part8 == 0 && r < m && c < n) Dl[r][c] = v;
      // the wave holds row r's residual (lane 8c, column c): its first nonzero column and value
      const uint64_t bal = __ballot(part8 == 0 && r < m && c < n && v != 0u);
      const int f = bal ? __builtin_ctzll(bal) / 8 : -1;
      const uint32_t fv = (uint32_t)__shfl((int)v, f < 0 ? 0 : 8 * f);
      if ((tid & (WAVE - 1)) == 0 && r < m) {
        rinfo[r][0] = (uint32_t)f;
        rinfo[r][1] = fv;
      }
    }
    // (no barrier here: the row order reads only the degrees; the barrier after it covers both)
    // Echelon form of the residual, rows by increasing shifted degree (ties by
    // index), right-looking: when a row keeps a nonzero residual it becomes a
    // pivot (column: its first nonzero entry) and every later row is reduced by
    // it at once, so each row meets the pivots before it in the order they were
    // found, as in the one-row-at-a-time elimination. T accumulates the row
    // combinations; pivot rows are multiplied by x below.
    // row order: the position of row i is the number of rows before it by
    // (shifted degree, index)
    if (tid < m) {
      const int di = dl[tid];
      int pos = 0;
      for (int j = 0; j < m; ++j) {
        const int dj = dl[j];
        pos += (dj < di) || (dj == di && j < tid);
      }
      order[pos] = tid;
    }
    for (int idx = tid; idx < m * m; idx += LEAF_NT) T[idx / m][idx % m] = (idx / m == idx % m) ? 1u : 0u;
    __syncthreads();
    // Fraction free: row_j <- pv row_j - x_j row_i is the oracle's
    // row_j - (x_j / pv) row_i times pv. The rows of M (and so of the residual)
    // stay scaled by the product sc[j] of these factors from order to order;
    // the scales are divided out once, when the leaf writes its basis. The
    // pivot column of the later rows becomes zero and is never written: the
    // lanes read it in place, and the scans skip the columns of earlier pivots.
    // Every lane keeps the row order in registers (indexed by the unrolled pivot counter below) and
    // works on one fixed entry of [residual | T] for the whole order: half a wave per row (lane lcol
    // < 8 a residual column, 8 <= lcol < 24 a column of T), so a row's lanes trade values by
    // shuffles. The lane's own entry stays in a register (no other lane writes it) and goes to LDS
    // for the pivot steps of later rows; the scale of a row is kept by its lane 0. Every row's first
    // nonzero unused column and its value (rinfo, by row) come from the residual phase and, after
    // each pivot step, from the lanes of every later row, so a pivot step reads two words and the
    // lane's column of the pivot row, and a row left with zeros costs one read and no barrier.
    int ord[SB_MAXM];
#pragma unroll
    for (int q = 0; q < SB_MAXM; ++q) ord[q] = q < m ? order[q] : 0;
    constexpr int EW = WAVE / 2;
    static_assert(SB_MAXN + SB_MAXM <= EW && SB_MAXM * EW <= LEAF_NT && SB_MAXN <= 32, "lanes of the elimination");
    const int lp = tid / EW, lcol = tid % EW;
    const bool el_wave = tid < SB_MAXM * EW;  // whole waves
    const bool lane_on = el_wave && lp < m && (lcol < SB_MAXN ? lcol < n : lcol - SB_MAXN < m);
    const int lj = lane_on ? order[lp] : 0;
    const int rowbase = tid & ~(EW - 1);
    uint32_t own = 0u, scr = 0u;
    if (lane_on) {
      own = lcol < SB_MAXN ? Dl[lj][lcol] : T[lj][lcol - SB_MAXN];
      if (lcol == 0) scr = sc[lj];
    }
    uint32_t used = 0, pivmask = 0;  // pivot columns and pivot rows so far (the same in every lane)
    // rinfo of the rows at positions after `after`, from their lanes (called by whole waves; the rows
    // at earlier positions are left alone, since slower waves may still read the pivot row's)
    auto publish = [&](int after) {
      const uint64_t bal = __ballot(lane_on && lcol < SB_MAXN && !((used >> lcol) & 1u) && own != 0u);
      const uint32_t rm = (uint32_t)(bal >> (tid & EW)) & ((1u << SB_MAXN) - 1u);
      const int f = rm ? __builtin_ctz(rm) : -1;
      const uint32_t fv = (uint32_t)__shfl((int)own, rowbase + (f < 0 ? 0 : f));
      if (lane_on && lcol == 0 && lp > after) {
        rinfo[lj][0] = (uint32_t)f;
        rinfo[lj][1] = fv;
      }
    };
#pragma unroll
    for (int oi = 0; oi < SB_MAXM; ++oi) {
      if (oi >= m) break;
      const int i = ord[oi];
      const int first = (int)rinfo[i][0];
      const uint32_t pv = rinfo[i][1];
      const uint32_t prv = lane_on ? (lcol < SB_MAXN ? Dl[i][lcol] : T[i][lcol - SB_MAXN]) : 0u;
      if (first < 0) continue;  // the same answer in every lane
      used |= 1u << first;
      pivmask |= 1u << i;
      const uint32_t x = (uint32_t)__shfl((int)own, rowbase + first);  // this row's entry in the pivot column
      if (lane_on && lp > oi && x) {
        if (lcol == 0) scr = fmul(scr, pv, F);
        if (lcol >= SB_MAXN || !((used >> lcol) & 1u)) {  // neither this pivot's column nor an earlier one
          const uint32_t v = fmul(pv, own, F) + fmul(F.p - x, prv, F);
          own = v >= F.p ? v - F.p : v;
          if (lcol < SB_MAXN) Dl[lj][lcol] = own;
          else T[lj][lcol - SB_MAXN] = own;
        }
      }
      if (el_wave) publish(oi);
      __syncthreads();
    }
    if (lane_on && lcol == 0) sc[lj] = scr;
    if (tid < m && ((pivmask >> tid) & 1u)) dl[tid] += 1;
    // (no barrier here: the update reads T, complete at the last pivot's barrier, and takes the
    // pivot rows from pivmask; the scales and degrees are next read after the update's barrier)
    // M <- diag(x^piv) T M: four lanes per entry (i, c), each over every fourth coefficient, T's row
    // in registers. M has degree <= k before order k, so only coefficients 0..k+1 change (the
    // buffers hold zeros above). The 64 lanes of a wave share the row i, so T's zero entries (rows
    // no pivot was combined into) are skipped without divergence.
    const int nxt = cur ^ 1;
    {
      const int e = tid >> 2, j0 = tid & 3;
      const int i = e / SB_MAXM, c = e % SB_MAXM;
      if (i < m && c < m) {
        uint32_t t[SB_MAXM];
#pragma unroll
        for (int q4 = 0; q4 < SB_MAXM; q4 += 4) {  // T's row in 16-byte reads
          typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
          const u32x4_t tv = *(const u32x4_t*)&T[i][q4];
          t[q4] = q4 < m ? tv.x : 0u;
          t[q4 + 1] = q4 + 1 < m ? tv.y : 0u;
          t[q4 + 2] = q4 + 2 < m ? tv.z : 0u;
          t[q4 + 3] = q4 + 3 < m ? tv.w : 0u;
        }
        const int sh = (int)((pivmask >> i) & 1u);
        for (int j = j0; j <= k + 1 && j < LC; j += 4) {
          const int js = j - sh;
          uint32_t out = 0;
          if (js >= 0 && js <= k) {
            Acc96<MERS> acc;
            if (MERS) {  // four products of residues below 2^31 add below 2^64: one fold per four
#pragma unroll
              for (int q0 = 0; q0 < SB_MAXM; q0 += 4) {
                uint64_t g = 0;
#pragma unroll
                for (int q = q0; q < q0 + 4; ++q)
                  if (q < m && t[q]) g += (uint64_t)t[q] * Ms[cur][q][c][js];
                acc.lo += (g & 0x7FFFFFFFull) + (g >> 31);
              }
            } else {
#pragma unroll
              for (int q = 0; q < SB_MAXM; ++q)
                if (q < m && t[q]) acc.add((uint64_t)t[q] * Ms[cur][q][c][js]);
            }
            out = acc.reduce(F);
          }
          Ms[nxt][i][c][j] = out;
        }
      }
    }
    cur = nxt;
    __syncthreads();
  }
  // divide out the row scales: all inverses from one exponentiation (prefix
  // products, one inverse, and back)
  if (tid == 0) {
    uint32_t pre[SB_MAXM + 1];
    pre[0] = 1;
    for (int j = 0; j < m; ++j) pre[j + 1] = fmul(pre[j], sc[j], F);
    uint32_t inv = finv(pre[m], F);
    for (int j = m - 1; j >= 0; --j) {
      const uint32_t ij = fmul(inv, pre[j], F);
      inv = fmul(inv, sc[j], F);
      sc[j] = ij;
    }
  }
  __syncthreads();
  for (int idx = tid; idx < m * m * (sg + 1); idx += LEAF_NT) {
    const int i = idx / (m * (sg + 1)), c = (idx / (sg + 1)) % m, j = idx % (sg + 1);
    M[(int64_t)(i * m + c) * sm + j] = fmul(Ms[cur][i][c][j], sc[i], F);
  }
  if (tid < m) d[tid] = dl[tid];
}

// G = [S(x); -I] as 2s x s entries of L coefficients from S (L x s x s, dtype residues mod p).
template <typename T>
__global__ void k_sequence_series(const T* __restrict__ S, int64_t L, int s, uint32_t p, uint32_t* __restrict__ G) {
  const int64_t total = (int64_t)2 * s * s * L;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = t / L, k = t % L;
    const int r = (int)(e / s), c = (int)(e % s);
    uint32_t v;
    if (r < s) {
      const int64_t x = (int64_t)S[(k * s + r) * s + c] % (int64_t)p;
      v = (uint32_t)(x < 0 ? x + p : x);
    } else {
      v = (k == 0 && r - s == c) ? p - 1 : 0u;
    }
    G[t] = v;
  }
}

// ------------------------------------------------------------------ host ----
static Field make_field(uint32_t p) {
  Field F;
  F.p = p;
  F.mu = UINT64_MAX / p;
  F.r64 = (uint32_t)((((unsigned __int128)1) << 64) % p);
  F.mersenne = p == 0x7FFFFFFFu;
  return F;
}

// ------------------------------------------------------------ NTT products
// The paper multiplies the polynomial matrices of PM-Basis through a DFT
// (Section 3.2, "Parallel polynomial matrix multiplication": transform the
// entries, multiply the transformed matrices point by point, transform back).
// F_p with p = 2^31 - 1 has no roots of unity of large power-of-two order, so
// the product is taken over the integers: exactly modulo three primes below
// 2^31 that have roots of unity of order 2^25 and more, with the coefficients
// recovered by the Chinese remainder theorem (Garner's mixed-radix form) and
// reduced mod p. An integer coefficient of the product is below
// Q * min(la, lb) * (p-1)^2, checked on the host against the product of the
// three primes (about 2^92.6).
//
// Transforms of length N (a power of two) run as log2 N radix-2 passes over
// global memory, each pass one launch over every entry and prime: forward
// passes are decimation in frequency (natural order in, bit-reversed out), the
// pointwise products work in that order, and the inverse passes are
// decimation in time (bit-reversed in, natural out). Products are cyclic of
// length N; N covers the wanted coefficients k0 .. k0+len-1 and is large
// enough that no coefficient of the full product wraps onto them.
constexpr int NTT_NP = 3;
static const uint32_t NTT_PRIME[NTT_NP] = {2013265921u, 1811939329u, 2113929217u};  // 15*2^27+1, 27*2^26+1, 63*2^25+1
static const uint32_t NTT_GEN[NTT_NP] = {31u, 13u, 5u};                            // primitive roots

struct NttPrimes {
  uint32_t p[NTT_NP];
  uint64_t mu[NTT_NP];
};

__device__ inline uint32_t nmul(uint32_t a, uint32_t b, uint32_t p, uint64_t mu) { return mod_u64((uint64_t)a * b, p, mu); }

// dst[i][e][t] = t < len ? src[e][t] mod p_i : 0, for n entries (entry e of src at src + e*stride)
__global__ void k_ntt_load(const uint32_t* __restrict__ src, int64_t stride, int64_t len, int ne, uint32_t* __restrict__ dst,
                           int64_t N, int dst_ne, int e0, NttPrimes P) {
  const int64_t total = (int64_t)NTT_NP * ne * N;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = g % N;
    const int64_t e = (g / N) % ne;
    const int i = (int)(g / (N * ne));
    const uint32_t v = t < len ? src[e * stride + t] % P.p[i] : 0u;
    dst[((int64_t)i * dst_ne + e0 + e) * N + t] = v;
  }
}

// tw[i][k] = w_i^k and itw[i][k] = w_i^-k, k < N/2, w_i a root of unity of order N modulo p_i
__global__ void k_ntt_twiddles(uint32_t* __restrict__ tw, int64_t half, const uint32_t* __restrict__ roots,
                               NttPrimes P) {
  const int64_t total = (int64_t)2 * NTT_NP * half;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = g % half;
    const int q = (int)(g / half);  // 0..2: forward roots, 3..5: inverse roots
    const int i = q % NTT_NP;
    uint32_t r = 1, b = roots[q];
    for (int64_t e = k; e; e >>= 1) {
      if (e & 1) r = nmul(r, b, P.p[i], P.mu[i]);
      b = nmul(b, b, P.p[i], P.mu[i]);
    }
    tw[g] = r;
  }
}

// One radix-2 pass over ne entries of every prime, butterflies of span h: forward (decimation in
// frequency) a, b -> a + b, (a - b) w^(j N / 2h); inverse (decimation in time) a, b -> a + b w', a - b w'.
template <bool INV>
__global__ void k_ntt_pass(uint32_t* __restrict__ X, int64_t N, int64_t h, int ne, const uint32_t* __restrict__ tw,
                           NttPrimes P) {
  const int64_t half = N / 2, total = (int64_t)NTT_NP * ne * half;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = g % half;
    const int64_t row = g / half;  // prime * ne + entry
    const int i = (int)(row / ne);
    const uint32_t p = P.p[i];
    const int64_t j = b % h, blk = b / h;
    uint32_t* x = X + row * N + blk * 2 * h + j;
    const uint32_t w = tw[((INV ? NTT_NP : 0) + i) * half + j * (half / h)];
    const uint32_t u = x[0], v = x[h];
    if (INV) {
      const uint32_t t = nmul(v, w, p, P.mu[i]);
      const uint32_t s = u + t;
      x[0] = s >= p ? s - p : s;
      x[h] = u >= t ? u - t : u + p - t;
    } else {
      const uint32_t s = u + v;
      x[0] = s >= p ? s - p : s;
      x[h] = nmul(u >= v ? u - v : u + p - v, w, p, P.mu[i]);
    }
  }
}

// C^[i][r][c][f] = sum_q A^[i][r][q][f] B^[i][q][c][f] mod p_i; AB holds the R*Q entries of A, then the Q*NC of B
__global__ void k_ntt_pointwise(const uint32_t* __restrict__ AB, uint32_t* __restrict__ Cf, int64_t N, int R, int Q,
                                int NC, NttPrimes P) {
  const int nab = R * Q + Q * NC, nc = R * NC;
  const int64_t total = (int64_t)NTT_NP * nc * N;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t f = g % N;
    const int e = (int)((g / N) % nc);
    const int i = (int)(g / (N * nc));
    const int r = e / NC, c = e % NC;
    const uint32_t* base = AB + (int64_t)i * nab * N;
    uint64_t acc = 0;  // Q <= 16 reduced products: below 2^36
    for (int q = 0; q < Q; ++q)
      acc += nmul(base[(int64_t)(r * Q + q) * N + f], base[(int64_t)(R * Q + q * NC + c) * N + f], P.p[i], P.mu[i]);
    Cf[((int64_t)i * nc + e) * N + f] = (uint32_t)(acc % P.p[i]);
  }
}

struct Garner {
  NttPrimes P;
  uint32_t ninv[NTT_NP];  // N^-1 mod p_i
  uint32_t inv1_2;        // p1^-1 mod p2
  uint32_t inv12_3;       // (p1 p2)^-1 mod p3
  uint32_t p12_3;         // p1 p2 mod p3
  uint32_t p1_f, p12_f;   // p1 and p1 p2 mod the field prime
};

// C[e][t - k0] = the product's coefficient t mod the field prime, for k0 <= t < k0 + len
__global__ void k_ntt_crt(const uint32_t* __restrict__ Cf, int64_t N, int nc, uint32_t* __restrict__ C, int64_t sc,
                          int64_t k0, int64_t len, Garner G, Field F) {
  const int64_t total = (int64_t)nc * len;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = g % len;
    const int e = (int)(g / len);
    uint32_t r[NTT_NP];
#pragma unroll
    for (int i = 0; i < NTT_NP; ++i)
      r[i] = nmul(Cf[((int64_t)i * nc + e) * N + k0 + t], G.ninv[i], G.P.p[i], G.P.mu[i]);
    const uint32_t p1 = G.P.p[0], p2 = G.P.p[1], p3 = G.P.p[2];
    // x = r1 + p1 t1 + p1 p2 t2 with 0 <= t1 < p2, 0 <= t2 < p3
    const uint32_t r1m2 = r[0] % p2;
    const uint32_t t1 = nmul(r[1] >= r1m2 ? r[1] - r1m2 : r[1] + p2 - r1m2, G.inv1_2, p2, G.P.mu[1]);
    const uint64_t x12 = (uint64_t)r[0] + (uint64_t)p1 * t1;  // < p1 p2 < 2^62
    const uint32_t x12m3 = (uint32_t)(x12 % p3);
    const uint32_t t2 = nmul(r[2] >= x12m3 ? r[2] - x12m3 : r[2] + p3 - x12m3, G.inv12_3, p3, G.P.mu[2]);
    const uint64_t lo = (uint64_t)mod_u64(x12, F.p, F.mu) + mod_u64((uint64_t)G.p12_f * t2, F.p, F.mu);
    C[(int64_t)e * sc + t] = (uint32_t)(lo >= F.p ? lo - F.p : lo);
  }
}

static uint32_t host_pow(uint64_t b, uint64_t e, uint32_t p) {
  uint64_t r = 1;
  b %= p;
  while (e) {
    if (e & 1) r = r * b % p;
    b = b * b % p;
    e >>= 1;
  }
  return (uint32_t)r;
}

// process-wide: the smallest la and lb at which a product goes through the NTT (0: never)
static std::atomic<int64_t> g_ntt_min{1024};

static int ntt_grid(int64_t work) { return (int)std::max<int64_t>(1, std::min<int64_t>((work + 255) / 256, 8192)); }

// The NTT form of polymul; returns false (nothing enqueued) when the coefficient bound exceeds the
// three primes' product or the length exceeds the primes' roots of unity.
static bool polymul_ntt(const uint32_t* A, int64_t sa, int64_t la, const uint32_t* B, int64_t sb, int64_t lb,
                        uint32_t* C, int64_t sc, int64_t k0, int64_t len, int R, int Q, int NC, const Field& F,
                        hipStream_t st) {
  const long double bound = (long double)Q * (long double)std::min(la, lb) * (long double)(F.p - 1) * (long double)(F.p - 1);
  const long double prod = (long double)NTT_PRIME[0] * NTT_PRIME[1] * NTT_PRIME[2];
  if (!(bound < prod * 0.999L)) return false;
  // cyclic length: covers k0 + len, and full coefficients at index >= N land below k0
  const int64_t need = std::max<int64_t>(k0 + len, la + lb - 1 - k0);
  int64_t N = 2;
  while (N < need) N *= 2;
  if (N > ((int64_t)1 << 25)) return false;
  NttPrimes P;
  uint32_t roots[2 * NTT_NP];
  Garner G;
  for (int i = 0; i < NTT_NP; ++i) {
    P.p[i] = NTT_PRIME[i];
    P.mu[i] = UINT64_MAX / NTT_PRIME[i];
    const uint32_t w = host_pow(NTT_GEN[i], (NTT_PRIME[i] - 1) / (uint64_t)N, NTT_PRIME[i]);
    if (host_pow(w, N / 2, NTT_PRIME[i]) != NTT_PRIME[i] - 1) fail(FFX_EDEVICE, "NTT root of unity check failed");
    roots[i] = w;
    roots[NTT_NP + i] = host_pow(w, NTT_PRIME[i] - 2, NTT_PRIME[i]);
    G.ninv[i] = host_pow((uint64_t)N % NTT_PRIME[i], NTT_PRIME[i] - 2, NTT_PRIME[i]);
  }
  G.P = P;
  const uint64_t p1 = NTT_PRIME[0], p2 = NTT_PRIME[1], p3 = NTT_PRIME[2];
  G.inv1_2 = host_pow(p1 % p2, p2 - 2, (uint32_t)p2);
  G.p12_3 = (uint32_t)((p1 * p2) % p3);
  G.inv12_3 = host_pow(G.p12_3, p3 - 2, (uint32_t)p3);
  G.p1_f = (uint32_t)(p1 % F.p);
  G.p12_f = (uint32_t)((unsigned __int128)(p1 * p2) % F.p);
  const int nab = R * Q + Q * NC, nc = R * NC;
  const int64_t half = N / 2;
  uint32_t *AB = nullptr, *Cf = nullptr, *tw = nullptr;
  const size_t bab = (size_t)NTT_NP * nab * N * 4, bc = (size_t)NTT_NP * nc * N * 4,
               btw = (size_t)2 * NTT_NP * half * 4 + 2 * NTT_NP * 4;
  if (hipMallocAsync((void**)&AB, bab, st) != hipSuccess || hipMallocAsync((void**)&Cf, bc, st) != hipSuccess ||
      hipMallocAsync((void**)&tw, btw, st) != hipSuccess) {
    for (void* q : {(void*)AB, (void*)Cf, (void*)tw})
      if (q) (void)hipFreeAsync(q, st);
    fail(FFX_ENOMEM, "NTT workspace allocation failed (length %lld)", (long long)N);
  }
  uint32_t* d_roots = tw + 2 * NTT_NP * half;
  hipError_t e = hipMemcpyAsync(d_roots, roots, sizeof roots, hipMemcpyHostToDevice, st);
  // the roots are read by the next kernel before this function returns the host array
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_ntt_twiddles, dim3(ntt_grid(2 * NTT_NP * half)), dim3(256), 0, st, tw, half, d_roots, P);
    hipLaunchKernelGGL(k_ntt_load, dim3(ntt_grid((int64_t)NTT_NP * R * Q * N)), dim3(256), 0, st, A, sa, la, R * Q, AB,
                       N, nab, 0, P);
    hipLaunchKernelGGL(k_ntt_load, dim3(ntt_grid((int64_t)NTT_NP * Q * NC * N)), dim3(256), 0, st, B, sb, lb, Q * NC,
                       AB, N, nab, R * Q, P);
    for (int64_t h = half; h >= 1; h /= 2)
      hipLaunchKernelGGL((k_ntt_pass<false>), dim3(ntt_grid((int64_t)NTT_NP * nab * half)), dim3(256), 0, st, AB, N, h,
                         nab, tw, P);
    hipLaunchKernelGGL(k_ntt_pointwise, dim3(ntt_grid((int64_t)NTT_NP * nc * N)), dim3(256), 0, st, AB, Cf, N, R, Q,
                       NC, P);
    for (int64_t h = 1; h < N; h *= 2)
      hipLaunchKernelGGL((k_ntt_pass<true>), dim3(ntt_grid((int64_t)NTT_NP * nc * half)), dim3(256), 0, st, Cf, N, h,
                         nc, tw, P);
    hipLaunchKernelGGL(k_ntt_crt, dim3(ntt_grid((int64_t)nc * len)), dim3(256), 0, st, Cf, N, nc, C, sc, k0, len, G, F);
    e = hipGetLastError();
    // the host array `roots` must outlive its copy
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  }
  (void)hipFreeAsync(AB, st);
  (void)hipFreeAsync(Cf, st);
  (void)hipFreeAsync(tw, st);
  FFX_HIP(e);
  return true;
}

static void polymul(const uint32_t* A, int64_t sa, int64_t la, const uint32_t* B, int64_t sb, int64_t lb, uint32_t* C,
                    int64_t sc, int64_t k0, int64_t len, int R, int Q, int NC, const Field& F, hipStream_t st) {
  if (len <= 0) return;
  const int64_t nt = g_ntt_min.load();
  if (nt > 0 && la >= nt && lb >= nt && polymul_ntt(A, sa, la, B, sb, lb, C, sc, k0, len, R, Q, NC, F, st)) return;
  const int64_t tiles = (len + PM_TILE - 1) / PM_TILE;
  if (tiles <= PMS_MAX_TILES && la <= PMS_MAXA && polymul_small_lds(Q, std::max<int64_t>(la, 1)) <= 64 * 1024) {
    const int la1 = (int)std::max<int64_t>(la, 1);
    const size_t lds = polymul_small_lds(Q, la1);
    const dim3 grid((unsigned)(R * NC), (unsigned)tiles);
    if (F.mersenne)
      hipLaunchKernelGGL((k_polymul_small<true>), grid, dim3(PMS_NT), lds, st, A, sa, la1, B, sb, lb, C, sc, k0, len,
                         Q, NC, F);
    else
      hipLaunchKernelGGL((k_polymul_small<false>), grid, dim3(PMS_NT), lds, st, A, sa, la1, B, sb, lb, C, sc, k0, len,
                         Q, NC, F);
    FFX_HIP(hipGetLastError());
    return;
  }
  const int64_t tiles4 = (len + PM_OUT - 1) / PM_OUT;
  if (tiles4 * R * NC >= 2048) {  // enough four-per-lane tiles to fill the GPU
    dim3 grid4((unsigned)tiles4, (unsigned)(R * NC));
    if (F.mersenne)
      hipLaunchKernelGGL((k_polymul4<true>), grid4, dim3(PM_TILE), 0, st, A, sa, std::max<int64_t>(la, 1), B, sb, lb,
                         C, sc, k0, len, Q, NC, F);
    else
      hipLaunchKernelGGL((k_polymul4<false>), grid4, dim3(PM_TILE), 0, st, A, sa, std::max<int64_t>(la, 1), B, sb, lb,
                         C, sc, k0, len, Q, NC, F);
    FFX_HIP(hipGetLastError());
    return;
  }
  dim3 grid((unsigned)((len + PM_TILE - 1) / PM_TILE), (unsigned)(R * NC));
  hipLaunchKernelGGL(k_polymul, grid, dim3(PM_TILE), 0, st, A, sa, std::max<int64_t>(la, 1), B, sb, lb, C, sc, k0, len,
                     Q, NC, F);
  FFX_HIP(hipGetLastError());
}

struct SbCtx {
  Field F;
  int m, n;
  hipStream_t st;
  int32_t* d_dev;       // m shifted degrees on the device: the leaves read and update them there
  bool d_host = true;   // the host copy of the degrees is current
};

// Nodes of at most this order take no degrees from the device: their lengths are the bound
// sigma + 1 (the extra coefficients come out zero), so a subtree of such nodes is queued without
// waiting for the GPU; larger nodes read the degrees back to size their products exactly.
constexpr int64_t SB_EXACT_ABOVE = 256;

// The host copy of the degrees, read back when a leaf has run since the last read.
static void host_degrees(SbCtx& X, std::vector<int32_t>& d) {
  if (X.d_host) return;
  FFX_HIP(hipMemcpyAsync(d.data(), X.d_dev, X.m * sizeof(int32_t), hipMemcpyDeviceToHost, X.st));
  FFX_HIP(hipStreamSynchronize(X.st));
  X.d_host = true;
}

// Basis of G (m x n entries, stride sg, order sigma) into M (m x m entries, stride sm >= sigma + 1,
// zero beyond the returned length); the shifted degrees are updated in X.d_dev (and in d when it is
// read back). Returns a bound on the number of coefficients of M that can be nonzero.
static int64_t pmbasis(SbCtx& X, const uint32_t* G, int64_t sg, int64_t sigma, std::vector<int32_t>& d, uint32_t* M,
                       int64_t sm) {
  const int m = X.m, n = X.n;
  if (sigma <= SB_LEAF) {
    if (X.F.mersenne)
      hipLaunchKernelGGL((k_mbasis_leaf<true>), dim3(1), dim3(LEAF_NT), 0, X.st, G, sg, m, n, (int)sigma, X.d_dev, M,
                         sm, X.F);
    else
      hipLaunchKernelGGL((k_mbasis_leaf<false>), dim3(1), dim3(LEAF_NT), 0, X.st, G, sg, m, n, (int)sigma, X.d_dev, M,
                         sm, X.F);
    FFX_HIP(hipGetLastError());
    X.d_host = false;
    return sigma + 1;
  }
  const bool exact = sigma > SB_EXACT_ABOVE;
  int32_t dmin = 0;
  if (exact) {
    host_degrees(X, d);
    dmin = *std::min_element(d.begin(), d.end());
  }
  const int64_t s1 = sigma / 2, s2 = sigma - s1;
  uint32_t *M1 = nullptr, *R = nullptr, *M2 = nullptr;
  const size_t b1 = (size_t)m * m * (s1 + 1) * 4, bR = (size_t)m * n * s2 * 4, b2 = (size_t)m * m * (s2 + 1) * 4;
  if (hipMallocAsync((void**)&M1, b1, X.st) != hipSuccess || hipMallocAsync((void**)&R, bR, X.st) != hipSuccess ||
      hipMallocAsync((void**)&M2, b2, X.st) != hipSuccess) {
    for (void* q : {(void*)M1, (void*)R, (void*)M2})
      if (q) (void)hipFreeAsync(q, X.st);
    fail(FFX_ENOMEM, "order basis workspace allocation failed (order %lld)", (long long)sigma);
  }
  try {
    const int64_t l1 = pmbasis(X, G, sg, s1, d, M1, s1 + 1);
    // R = [x^s1 .. x^(sigma-1)] (M1 G)
    polymul(M1, s1 + 1, l1, G, sg, sigma, R, s2, s1, s2, m, m, n, X.F, X.st);
    const int64_t l2 = pmbasis(X, R, s2, s2, d, M2, s2 + 1);
    int64_t len = std::min<int64_t>(sigma + 1, l1 + l2 - 1);
    if (exact) {
      host_degrees(X, d);
      const int32_t dmax = *std::max_element(d.begin(), d.end());
      len = std::min<int64_t>(len, (int64_t)dmax - dmin + 1);
    }
    polymul(M2, s2 + 1, l2, M1, s1 + 1, l1, M, sm, 0, len, m, m, m, X.F, X.st);
    if (len < sm) FFX_HIP(hipMemset2DAsync(M + len, sm * 4, 0, (sm - len) * 4, (size_t)m * m, X.st));
    (void)hipFreeAsync(M1, X.st);
    (void)hipFreeAsync(R, X.st);
    (void)hipFreeAsync(M2, X.st);
    return len;
  } catch (...) {
    (void)hipFreeAsync(M1, X.st);
    (void)hipFreeAsync(R, X.st);
    (void)hipFreeAsync(M2, X.st);
    throw;
  }
}

static bool is_prime(uint32_t p) {
  if (p < 2) return false;
  for (uint32_t q : {2u, 3u, 5u, 7u}) {
    if (p % q == 0) return p == q;
  }
  uint32_t dd = p - 1;
  int r = 0;
  while (!(dd & 1)) {
    dd >>= 1;
    ++r;
  }
  auto mulm = [&](uint64_t a, uint64_t b) { return a * b % p; };
  for (uint64_t a : {2ull, 3ull, 5ull, 7ull}) {  // deterministic below 3,215,031,751
    uint64_t x = 1, b = a, e = dd;
    while (e) {
      if (e & 1) x = mulm(x, b);
      b = mulm(b, b);
      e >>= 1;
    }
    if (x == 1 || x == p - 1) continue;
    bool comp = true;
    for (int i = 1; i < r && comp; ++i) {
      x = mulm(x, x);
      if (x == p - 1) comp = false;
    }
    if (comp) return false;
  }
  return true;
}

void sigma_basis(uint32_t p, int m, int n, int64_t sigma, const uint32_t* G, int64_t ldg, const int32_t* shift,
                 uint32_t* M, int64_t ldm, int32_t* d_out, hipStream_t st) {
  if (p > 2147483647u) fail(FFX_EINVAL, "the order basis needs a prime p < 2^31 (p = %u)", p);
  if (!is_prime(p)) fail(FFX_EINVAL, "the order basis needs a prime modulus (%u is not prime)", p);
  if (m < 1 || m > SB_MAXM || n < 1 || n > SB_MAXN || n > m)
    fail(FFX_EINVAL, "m = %d, n = %d: need 1 <= n <= m <= %d and n <= %d", m, n, SB_MAXM, SB_MAXN);
  if (sigma < 1) fail(FFX_EINVAL, "sigma = %lld < 1", (long long)sigma);
  if (ldg < sigma || ldm < sigma + 1) fail(FFX_EINVAL, "ldg < sigma or ldm < sigma + 1");
  if (!G || !M || !shift || !d_out) fail(FFX_EINVAL, "NULL argument");
  std::vector<int32_t> d(shift, shift + m);
  for (int32_t v : d)
    if (v < 0 || v > (1 << 28)) fail(FFX_EINVAL, "shift %d outside [0, 2^28]", v);
  SbCtx X{make_field(p), m, n, st, nullptr};
  if (hipMallocAsync((void**)&X.d_dev, SB_MAXM * sizeof(int32_t), st) != hipSuccess)
    fail(FFX_ENOMEM, "order basis workspace allocation failed");
  try {
    FFX_HIP(hipMemcpyAsync(X.d_dev, d.data(), m * sizeof(int32_t), hipMemcpyHostToDevice, st));
    const int64_t len = pmbasis(X, G, ldg, sigma, d, M, ldm);
    if (len < ldm) FFX_HIP(hipMemset2DAsync(M + len, ldm * 4, 0, (ldm - len) * 4, (size_t)m * m, st));
    host_degrees(X, d);
  } catch (...) {
    (void)hipFreeAsync(X.d_dev, st);
    throw;
  }
  (void)hipFreeAsync(X.d_dev, st);
  FFX_HIP(hipStreamSynchronize(st));
  std::copy(d.begin(), d.end(), d_out);
}

// x-adic valuation of det F (s x s entries of K coefficients, row-major [r][c][k]) over F_p by
// elimination over F_p[[x]]/x^K; -1 when det F = 0 mod x^K.
static int64_t det_valuation(std::vector<uint64_t> A, int s, int64_t K, uint32_t p) {
  auto at = [&](int r, int c) { return &A[((size_t)r * s + c) * K]; };
  auto pw = [&](uint64_t a, uint64_t e) {
    uint64_t r = 1;
    a %= p;
    while (e) {
      if (e & 1) r = r * a % p;
      a = a * a % p;
      e >>= 1;
    }
    return r;
  };
  int64_t val = 0;
  std::vector<uint64_t> u(K), ui(K), f(K);
  for (int c = 0; c < s; ++c) {
    int best = -1;
    int64_t bv = K;
    for (int r = c; r < s; ++r) {
      const uint64_t* x = at(r, c);
      for (int64_t k = 0; k < bv; ++k)
        if (x[k]) {
          best = r;
          bv = k;
          break;
        }
    }
    if (best < 0) return -1;
    if (best != c)
      for (int cc = 0; cc < s; ++cc) std::swap_ranges(at(c, cc), at(c, cc) + K, at(best, cc));
    val += bv;
    if (val >= K) return -1;
    // u = A[c][c] / x^bv, ui = 1/u
    std::fill(u.begin(), u.end(), 0);
    for (int64_t k = bv; k < K; ++k) u[k - bv] = at(c, c)[k];
    const uint64_t i0 = pw(u[0], p - 2);
    for (int64_t k = 0; k < K; ++k) {
      uint64_t acc = 0;
      for (int64_t j = 1; j <= k; ++j) acc = (acc + u[j] * ui[k - j]) % p;
      ui[k] = k == 0 ? i0 : (p - acc) % p * i0 % p;
    }
    for (int r = c + 1; r < s; ++r) {
      // f = (A[r][c] / x^bv) * ui; row r -= f * row c
      std::fill(f.begin(), f.end(), 0);
      for (int64_t k = 0; k + bv < K; ++k) {
        const uint64_t q = at(r, c)[k + bv];
        if (!q) continue;
        for (int64_t j = 0; k + j < K; ++j) f[k + j] = (f[k + j] + q * ui[j]) % p;
      }
      for (int cc = c; cc < s; ++cc) {
        uint64_t* y = at(r, cc);
        const uint64_t* x = at(c, cc);
        for (int64_t k = 0; k < K; ++k) {
          if (!f[k]) continue;
          for (int64_t j = 0; k + j < K; ++j) y[k + j] = (y[k + j] + (p - f[k]) * x[j]) % p;
        }
      }
    }
  }
  return val;
}

void sequence_rank(uint32_t p, int s, int64_t L, const void* S, ffx_dtype dt, int32_t* deg_out, int64_t* rank,
                   int64_t* deg_det, int64_t* codeg_det, hipStream_t st) {
  if (s < 1 || s > SB_MAXN) fail(FFX_EINVAL, "s = %d outside [1, %d]", s, SB_MAXN);
  if (L < 1) fail(FFX_EINVAL, "L = %lld < 1", (long long)L);
  if (!S) fail(FFX_EINVAL, "S is NULL");
  if (p > 2147483647u) fail(FFX_EINVAL, "the rank needs a prime p < 2^31 (p = %u)", p);
  if (!is_prime(p)) fail(FFX_EINVAL, "the rank needs a prime modulus (%u is not prime)", p);
  const int m = 2 * s;
  uint32_t *G = nullptr, *M = nullptr;
  if (hipMallocAsync((void**)&G, (size_t)m * s * L * 4, st) != hipSuccess ||
      hipMallocAsync((void**)&M, (size_t)m * m * (L + 1) * 4, st) != hipSuccess) {
    if (G) (void)hipFreeAsync(G, st);
    if (M) (void)hipFreeAsync(M, st);
    fail(FFX_ENOMEM, "rank workspace allocation failed (L = %lld)", (long long)L);
  }
  std::vector<int32_t> d(m);
  std::vector<uint32_t> Mh;
  try {
    const int64_t total = (int64_t)m * s * L;
    const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 16384);
    if (dt == FFX_I32)
      hipLaunchKernelGGL((k_sequence_series<int32_t>), dim3(blocks), dim3(256), 0, st, (const int32_t*)S, L, s, p, G);
    else
      hipLaunchKernelGGL((k_sequence_series<int64_t>), dim3(blocks), dim3(256), 0, st, (const int64_t*)S, L, s, p, G);
    FFX_HIP(hipGetLastError());
    std::vector<int32_t> shift(m, 0);
    for (int i = s; i < m; ++i) shift[i] = 1;
    sigma_basis(p, m, s, L, G, L, shift.data(), M, L + 1, d.data(), st);
    Mh.resize((size_t)m * m * (L + 1));
    FFX_HIP(hipMemcpyAsync(Mh.data(), M, Mh.size() * 4, hipMemcpyDeviceToHost, st));
    FFX_HIP(hipStreamSynchronize(st));
  } catch (...) {
    (void)hipFreeAsync(G, st);
    (void)hipFreeAsync(M, st);
    throw;
  }
  (void)hipFreeAsync(G, st);
  (void)hipFreeAsync(M, st);
  // the generator: the s rows of smallest shifted degree (ties by index), left s x s part
  std::vector<int> rows(m);
  for (int i = 0; i < m; ++i) rows[i] = i;
  std::stable_sort(rows.begin(), rows.end(), [&](int a, int b) { return d[a] < d[b]; });
  rows.resize(s);
  int64_t D = 0;
  for (int i = 0; i < s; ++i) {
    deg_out[i] = d[rows[i]];
    D += d[rows[i]];
    if (d[rows[i]] > L) fail(FFX_EUNSUPPORTED, "generator degree %d exceeds the sequence length", d[rows[i]]);
  }
  auto coef = [&](int r, int c, int64_t k) { return Mh[((size_t)rows[r] * m + c) * (L + 1) + k]; };
  // row reduced: the reversed form's constant coefficients must be nonsingular, else deg det F is
  // not the sum of the row degrees
  {
    std::vector<uint64_t> A0((size_t)s * s);
    for (int r = 0; r < s; ++r)
      for (int c = 0; c < s; ++c) A0[(size_t)r * s + c] = coef(r, c, 0);
    if (det_valuation(A0, s, 1, p) != 0)
      fail(FFX_EUNSUPPORTED, "the generator is not row reduced (sequence too short or degenerate projections)");
  }
  // codeg det F: F row i = lambda^deg_i Frev_i(1/lambda), so [lambda^k] F_i = [x^(deg_i - k)] Frev_i.
  // F is row reduced, so det F has degree D exactly and its valuation is at most D: a truncation
  // order K > D always finds it.
  int64_t e = -1;
  for (int64_t K = 16;; K *= 2) {
    std::vector<uint64_t> A((size_t)s * s * K, 0);
    for (int r = 0; r < s; ++r)
      for (int c = 0; c < s; ++c)
        for (int64_t k = 0; k < K && k <= deg_out[r]; ++k) A[((size_t)r * s + c) * K + k] = coef(r, c, deg_out[r] - k);
    e = det_valuation(A, s, K, p);
    if (e >= 0 || K > D) break;
  }
  if (e < 0) fail(FFX_EUNSUPPORTED, "det F vanishes: no rank from this sequence");
  *deg_det = D;
  *codeg_det = e;
  *rank = D - e;
}

}  // namespace ffx

extern "C" ffx_status ffx_set_ntt_threshold(int64_t min_length) {
  return ffx::guard([&] {
    if (min_length < 0) ffx::fail(FFX_EINVAL, "NTT threshold %lld < 0", (long long)min_length);
    ffx::g_ntt_min.store(min_length);
  });
}
