// Y = alpha*A^T*X + beta*Y without a stored A^T (paper Section 4 notes that A
// and A^T may not fit together): every entry A[i,j] scatters its terms
// A[i,j]*X[i][c] into a 64-bit accumulator of output row j with an integer
// atomic add, which is exact and order-free while the sums stay below 2^64.
// For m <= 65536 a term is below 2^32 and a column has at most 2^30 entries;
// for larger m each term is reduced mod m first. A second launch turns the
// accumulators into residues.
#include "launch.h"
#include "tiles.h"

namespace ffx {

// the value type of the stored entries (all that load_values4 needs to know)
template <typename V>
struct ValsOf {
  using ValT = V;
};

template <typename V, bool SMALL>
__device__ inline uint64_t scatter_term(uint32_t tag, uint32_t v, uint32_t x, const DevMat& A) {
  uint64_t t;
  if (tag == TAG_GEN) t = (uint64_t)v * x;
  else if (tag == TAG_PLUS) t = x;
  else t = (uint64_t)(A.m - x);
  return SMALL ? t : (uint64_t)mod_u64(t, A.m, A.mu);
}

template <typename V, bool SMALL, typename Tv>
__device__ inline void scatter_entry(const DevMat& A, uint32_t row, uint32_t w, uint32_t v, const Tv* X, int64_t ldx,
                                     int s, unsigned long long* acc) {
  const uint32_t tag = w >> TAG_SHIFT;
  if (tag == TAG_PAD || row >= A.nrows) return;
  const uint32_t col = w & COL_MASK;
  const Tv* xr = X + (int64_t)row * ldx;
  for (int c = 0; c < s; ++c)
    atomicAdd(&acc[(int64_t)col * s + c], (unsigned long long)scatter_term<V, SMALL>(tag, v, (uint32_t)xr[c], A));
}

template <typename V, bool SMALL, typename Tv>
__global__ __launch_bounds__(TILE_THREADS) void k_scatter_t(DevMat A, const Tv* __restrict__ X, int64_t ldx, int s,
                                                            unsigned long long* __restrict__ acc) {
  const Tile T = A.tiles[blockIdx.x];
  const uint32_t tid = threadIdx.x, lane = tid & (WAVE - 1), wave = tid / WAVE;
  const uint32_t kind = tile_kind(T.kind);
  if (kind == TK_SELL) {
    if (wave < T.ne) {
      uint32_t off = 0;
      for (uint32_t k = 0; k < wave; ++k) off += A.swidth[T.aux + k];
      const uint32_t groups = A.swidth[T.aux + wave], slot = wave * WAVE + lane;
      const uint32_t row = (T.kind & TF_SORTED) ? A.perm[T.row0 + slot] : T.row0 + slot;
      const uint32_t* ent = A.ent + T.e0 + (size_t)off * SELL_GROUP + lane * WIDE;
      for (uint32_t g = 0; g < groups; ++g) {  // 4-column groups: 4 consecutive entries of the lane's row
        uint32_t w[WIDE], v[WIDE];
        for (int k = 0; k < WIDE; ++k) w[k] = ent[(size_t)g * SELL_GROUP + k];
        load_values4<ValsOf<V>>(A, w, A.choff[T.c0 + off + g], v);
        for (int k = 0; k < WIDE; ++k) scatter_entry<V, SMALL, Tv>(A, row, w[k], v[k], X, ldx, s, acc);
      }
    }
  } else {
    const uint32_t nchunks = (T.ne + WCHUNK - 1) / WCHUNK;
    const uint32_t nr = kind == TK_LONG ? 1u : tile_rows(T.kind);
    for (uint32_t ch = wave; ch < nchunks; ch += TILE_THREADS / WAVE) {
      uint32_t e = ch * WCHUNK + lane * WIDE;
      uint32_t w[WIDE] = {PAD_WORD, PAD_WORD, PAD_WORD, PAD_WORD};
      if (e < T.ne)
        for (int k = 0; k < WIDE; ++k) w[k] = A.ent[T.e0 + e + k];
      uint32_t idx = A.choff[T.c0 + ch];
      for (int k = 0; k < WIDE; ++k) idx += lanes_below(__ballot((w[k] >> TAG_SHIFT) == TAG_GEN));
      // row of entry e: the last row whose start is <= e
      uint32_t r = 0;
      if (kind != TK_LONG && e < T.ne) {
        uint32_t lo = 0, hi = nr;
        while (hi - lo > 1) {
          uint32_t mid = (lo + hi) >> 1;
          if (A.rowp[T.aux + mid] - T.e0 <= e) lo = mid;
          else hi = mid;
        }
        r = lo;
      }
      for (int k = 0; k < WIDE; ++k) {
        if (e + k >= T.ne) break;
        if (kind != TK_LONG)
          while (A.rowp[T.aux + r + 1] - T.e0 <= e + k) ++r;
        bool gen = (w[k] >> TAG_SHIFT) == TAG_GEN;
        uint32_t v = gen ? ldval<V>(A.val, idx) : 0u;
        idx += gen ? 1u : 0u;
        scatter_entry<V, SMALL, Tv>(A, T.row0 + r, w[k], v, X, ldx, s, acc);
      }
    }
  }
  // band part: one (row, diagonal) slot per thread
  const uint32_t nd = tile_nd(T.kind);
  if (nd) {
    const uint32_t rows = kind == TK_LONG ? 1u : tile_rows(T.kind);
    for (uint32_t q = tid; q < rows * nd; q += TILE_THREADS) {
      uint32_t d = q / rows, slot = q % rows;
      uint32_t row = kind == TK_SELL ? ((T.kind & TF_SORTED) ? A.perm[T.row0 + slot] : T.row0 + slot) : T.row0 + slot;
      uint32_t v = ldval<V>(A.bval, T.b0 + d * rows + slot);
      if (!v || row >= A.nrows) continue;
      int64_t col = (int64_t)row + A.boffs[T.boff + d];
      const Tv* xr = X + (int64_t)row * ldx;
      for (int c = 0; c < s; ++c)
        atomicAdd(&acc[col * s + c], (unsigned long long)scatter_term<V, SMALL>(TAG_GEN, v, (uint32_t)xr[c], A));
    }
  }
}

__global__ void k_zero_u64(unsigned long long* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0;
}

template <typename Tv>
__global__ void k_finish_t(DevMat A, const unsigned long long* __restrict__ acc, int64_t n, int s, uint32_t alpha,
                           uint32_t beta, Tv* __restrict__ Y, int64_t ldy) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n * s; i += (int64_t)gridDim.x * blockDim.x) {
    int64_t j = i / s;
    int c = (int)(i - j * s);
    uint32_t r = mod_u64(acc[i], A.m, A.mu);
    Tv* y = Y + j * ldy + c;
    uint32_t yo = beta ? (uint32_t)*y : 0u;
    *y = (Tv)((alpha == 1 && beta == 0) ? r : axpby(alpha, r, beta, yo, A.m, A.mu));
  }
}

template <typename Tv>
static hipError_t scatter_go(bool small, const DevMat& A, const void* X, int64_t ldx, int s,
                             unsigned long long* acc, hipStream_t st) {
  dim3 g(A.ntiles), b(TILE_THREADS);
  if (small) hipLaunchKernelGGL((k_scatter_t<uint16_t, true, Tv>), g, b, 0, st, A, (const Tv*)X, ldx, s, acc);
  else hipLaunchKernelGGL((k_scatter_t<uint32_t, false, Tv>), g, b, 0, st, A, (const Tv*)X, ldx, s, acc);
  return hipGetLastError();
}

hipError_t launch_transpose_scatter(bool small, const DevMat& A, ffx_dtype dt, const void* X, int64_t ldx, void* Y,
                                    int64_t ldy, int s, uint32_t alpha, uint32_t beta, unsigned long long* acc,
                                    hipStream_t st) {
  const int64_t n = A.ncols;  // outputs of A^T
  const int64_t total = n * s;
  int zb = (int)std::min<int64_t>((total + 255) / 256, 8192);
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u64, dim3(zb), dim3(256), 0, st, acc, total);
  hipError_t e = A.ntiles ? (dt == FFX_I32 ? scatter_go<int32_t>(small, A, X, ldx, s, acc, st)
                                           : scatter_go<int64_t>(small, A, X, ldx, s, acc, st))
                          : hipSuccess;
  if (e != hipSuccess) return e;
  if (dt == FFX_I32)
    hipLaunchKernelGGL(k_finish_t<int32_t>, dim3(zb), dim3(256), 0, st, A, acc, n, s, alpha, beta, (int32_t*)Y, ldy);
  else
    hipLaunchKernelGGL(k_finish_t<int64_t>, dim3(zb), dim3(256), 0, st, A, acc, n, s, alpha, beta, (int64_t*)Y, ldy);
  return hipGetLastError();
}

}  // namespace ffx
