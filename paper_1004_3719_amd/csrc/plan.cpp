// Row-block planning and encoding (host side).
//
// A matrix is cut into blocks of block_rows consecutive rows; each block gets
// one storage format (paper Section 2.4, "Hybridization" and "Heuristic
// format chooser": different parts of one matrix in different formats) and is
// cut into tiles, the work unit of one workgroup. All blocks land in one set
// of device arrays, so one kernel launch covers the whole matrix.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "host.h"

namespace ffx {

Modulus make_modulus(uint32_t m) {
  Modulus md;
  md.m = m;
  md.mu = UINT64_MAX / m;
  md.inv_m = 1.0 / (double)m;
  return md;
}

void Encoded::release() {
  for (void* p : allocs) (void)hipFree(p);
  allocs.clear();
  dm = DevMat{};
}

static inline uint32_t tag_of(uint32_t v, uint32_t m, bool split) {
  if (!split) return TAG_GEN;
  if (v == 1) return TAG_PLUS;  // for m = 2, 1 = -1 is counted as +1
  if (v == m - 1) return TAG_MINUS;
  return TAG_GEN;
}

// ---------------------------------------------------------------------------
// Statistics and features of rows [r0, r1).
// ---------------------------------------------------------------------------
constexpr int BAND_WINDOW = 128;  // dense diagonals are searched in [-128, 127]

BlockStats block_stats(const RCsr& A, int64_t r0, int64_t r1, uint32_t m, const PlanOpts& o) {
  BlockStats b;
  b.row0 = r0;
  b.nrows = r1 - r0;
  b.nnz = A.rp[r1] - A.rp[r0];
  std::vector<int64_t> diag(2 * BAND_WINDOW, 0);
  int64_t pm1 = 0, near[4] = {0, 0, 0, 0};
  double s = 0, s2 = 0, spread = 0;
  b.minlen = INT64_MAX;
  int hist[12] = {0};
  for (int64_t i = r0; i < r1; ++i) {
    int64_t len = A.rp[i + 1] - A.rp[i];
    s += (double)len;
    s2 += (double)len * (double)len;
    b.maxlen = std::max(b.maxlen, len);
    b.minlen = std::min(b.minlen, len);
    if (len == 0) b.empty++;
    else {
      int h = std::min(11, (int)std::floor(std::log2((double)len)));
      hist[h]++;
      spread += (double)(A.col[A.rp[i + 1] - 1] - A.col[A.rp[i]]) / (double)std::max<int64_t>(1, A.ncols);
    }
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      int64_t d = (int64_t)A.col[k] - i;
      uint32_t v = A.val[k];
      if (v == 1 || v == m - 1) pm1++;
      int64_t ad = d < 0 ? -d : d;
      if (ad <= 2) near[0]++;
      if (ad <= 8) near[1]++;
      if (ad <= 32) near[2]++;
      if (ad <= 64) near[3]++;
      if (d >= -BAND_WINDOW && d < BAND_WINDOW) diag[d + BAND_WINDOW]++;
    }
  }
  if (b.nrows == 0) b.minlen = 0;
  b.mean = b.nrows ? s / (double)b.nrows : 0;
  b.sd = b.nrows ? std::sqrt(std::max(0.0, s2 / (double)b.nrows - b.mean * b.mean)) : 0;
  b.pm1_frac = b.nnz ? (double)pm1 / (double)b.nnz : 0;

  // dense diagonals: at least 60% of the rows that can hold them
  std::vector<std::pair<int64_t, int32_t>> cand;
  for (int d = -BAND_WINDOW; d < BAND_WINDOW; ++d) {
    int64_t lo = std::max<int64_t>(r0, -(int64_t)d), hi = std::min<int64_t>(r1, A.ncols - d);
    int64_t possible = hi - lo;
    int64_t c = diag[d + BAND_WINDOW];
    if (possible > 0 && c > 0 && (double)c >= 0.6 * (double)possible) cand.push_back({c, d});
  }
  std::sort(cand.begin(), cand.end(), [](auto& x, auto& y) { return x.first > y.first; });
  if ((int)cand.size() > MAX_BAND) cand.resize(MAX_BAND);
  for (auto& c : cand) {
    b.band_offsets.push_back(c.second);
    b.band_nnz += c.first;
  }
  std::sort(b.band_offsets.begin(), b.band_offsets.end());

  // residual row lengths (without the band) for the ELL padding estimates
  std::vector<int64_t> rlen(b.nrows);
  for (int64_t i = r0; i < r1; ++i) {
    int64_t len = A.rp[i + 1] - A.rp[i];
    if (!b.band_offsets.empty())
      for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
        int64_t d = (int64_t)A.col[k] - i;
        if (std::binary_search(b.band_offsets.begin(), b.band_offsets.end(), (int32_t)d)) len--;
      }
    rlen[i - r0] = len;
    if (len > o.tile_entries) b.long_rows++;
  }
  for (int64_t s0 = 0; s0 < b.nrows; s0 += WAVE) {
    int64_t w = 0;
    for (int64_t t = s0; t < std::min(b.nrows, s0 + WAVE); ++t) w = std::max(w, rlen[t]);
    b.sell_width_sum += w;
  }
  std::sort(rlen.begin(), rlen.end(), std::greater<int64_t>());
  for (int64_t s0 = 0; s0 < b.nrows; s0 += WAVE) b.sell_sorted_width_sum += rlen[s0];

  // the 32 features of the learned selector
  int64_t resid = b.nnz - b.band_nnz;
  float* f = b.feat;
  f[0] = (float)std::log2(1.0 + b.nrows);
  f[1] = (float)std::log2(1.0 + b.mean);
  f[2] = (float)std::log2(1.0 + b.sd);
  f[3] = (float)std::log2(1.0 + b.maxlen);
  f[4] = (float)std::log2(1.0 + b.minlen);
  f[5] = b.nrows ? (float)b.empty / (float)b.nrows : 0.f;
  f[6] = (float)b.pm1_frac;
  f[7] = b.nnz ? (float)b.band_nnz / (float)b.nnz : 0.f;
  f[8] = (float)b.band_offsets.size() / (float)MAX_BAND;
  f[9] = (float)std::log2(1.0 + (double)b.sell_width_sum * WAVE / std::max<int64_t>(1, resid));
  f[10] = (float)std::log2(1.0 + (double)b.sell_sorted_width_sum * WAVE / std::max<int64_t>(1, resid));
  f[11] = b.nrows ? (float)b.long_rows / (float)b.nrows * 100.f : 0.f;
  for (int h = 0; h < 12; ++h) f[12 + h] = b.nrows ? (float)hist[h] / (float)b.nrows : 0.f;
  f[24] = (b.nrows - b.empty) ? (float)(spread / (double)(b.nrows - b.empty)) : 0.f;
  for (int q = 0; q < 4; ++q) f[25 + q] = b.nnz ? (float)near[q] / (float)b.nnz : 0.f;
  f[29] = (float)std::log2(1.0 + (double)A.ncols);
  f[30] = b.mean > 0 ? (float)(b.sd / b.mean) : 0.f;
  f[31] = resid > 0 ? (float)std::log2(1.0 + (double)resid / std::max<int64_t>(1, b.nrows)) : 0.f;
  return b;
}

// The plain heuristic, after the paper's chooser (Section 2.4): an ELL-like
// part when rows are filled evenly (the "c + r" distribution), the rest in a
// CSR-like format; dense diagonals go to a DIA-like part. Thresholds are
// starting points for the autotuner, not tuned constants.
int heuristic_format(const BlockStats& b, const PlanOpts& o) {
  int64_t resid = b.nnz - b.band_nnz;
  bool band = !b.band_offsets.empty() && b.band_nnz >= 0.2 * (double)std::max<int64_t>(1, b.nnz);
  double pad = (double)b.sell_width_sum * WAVE / (double)std::max<int64_t>(1, resid);
  double pad_sorted = (double)b.sell_sorted_width_sum * WAVE / (double)std::max<int64_t>(1, resid);
  int64_t rmax = b.maxlen;  // upper bound of the residual maximum
  int base;
  if (resid == 0 || (pad <= 1.3 && rmax <= 1024)) base = FFX_FMT_SELL;
  else if (pad_sorted <= 1.3 && rmax <= 256) base = FFX_FMT_SELL_SORTED;
  else base = FFX_FMT_STREAM;
  (void)o;
  if (!band) return base;
  return base == FFX_FMT_STREAM ? FFX_FMT_BAND_STREAM : base == FFX_FMT_SELL ? FFX_FMT_BAND_SELL : FFX_FMT_BAND_SELL_SORTED;
}

// ---------------------------------------------------------------------------
// Encoding
// ---------------------------------------------------------------------------
namespace {

struct HostEnc {
  std::vector<Tile> tiles;
  std::vector<uint32_t> ent, val, choff, rowp, perm, swidth, bval;
  std::vector<int32_t> boffs;
  int64_t max_tile_entries = 0;
  int64_t n_plus = 0, n_minus = 0, n_band = 0, nnz = 0, max_row_terms = 0;

  // pads the entry stream to a 16-byte boundary with padding words
  void align_ent() {
    while (ent.size() % WIDE) ent.push_back(PAD_WORD);
  }
  // appends n words (64 for SELL, up to 256 for STREAM/LONG) as one value chunk
  void push_chunk(const uint32_t* w, const uint32_t* v, int n) {
    choff.push_back((uint32_t)val.size());
    for (int i = 0; i < n; ++i) {
      ent.push_back(w[i]);
      if ((w[i] >> TAG_SHIFT) == TAG_GEN) val.push_back(v[i]);
    }
  }
};

struct BlockRows {  // residual entries and band values of one block
  std::vector<int64_t> rp;        // residual row pointers (block-local)
  std::vector<uint32_t> word, v;  // residual entries
  std::vector<uint32_t> band;     // nrows x nd band values (0 = absent)
  int nd = 0;
};

BlockRows split_block(const RCsr& A, int64_t r0, int64_t r1, const std::vector<int32_t>& offs, uint32_t m,
                      bool split, HostEnc& H) {
  BlockRows R;
  R.nd = (int)offs.size();
  int64_t nr = r1 - r0;
  R.rp.assign(nr + 1, 0);
  R.band.assign((size_t)nr * R.nd, 0);
  for (int64_t i = r0; i < r1; ++i) {
    H.max_row_terms = std::max<int64_t>(H.max_row_terms, A.rp[i + 1] - A.rp[i]);
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      uint32_t c = A.col[k], v = A.val[k];
      H.nnz++;
      if (R.nd) {
        int64_t d = (int64_t)c - i;
        auto it = std::lower_bound(offs.begin(), offs.end(), (int32_t)std::max<int64_t>(INT32_MIN, std::min<int64_t>(INT32_MAX, d)));
        if (it != offs.end() && *it == d) {
          R.band[(size_t)(i - r0) * R.nd + (it - offs.begin())] = v;
          H.n_band++;
          continue;
        }
      }
      uint32_t t = tag_of(v, m, split);
      if (t == TAG_PLUS) H.n_plus++;
      if (t == TAG_MINUS) H.n_minus++;
      R.word.push_back((t << TAG_SHIFT) | c);
      R.v.push_back(v);
    }
    R.rp[i - r0 + 1] = (int64_t)R.word.size();
  }
  return R;
}

// One row (block-local index t) as a LONG tile: all lanes of a workgroup sweep it.
void encode_long(const BlockRows& R, int64_t r0, int64_t t, uint32_t boff, HostEnc& H) {
  Tile T{};
  T.kind = TK_LONG | ((uint32_t)R.nd << 8) | (1u << 16);
  T.row0 = (uint32_t)(r0 + t);
  H.align_ent();
  T.e0 = (uint32_t)H.ent.size();
  T.ne = (uint32_t)(R.rp[t + 1] - R.rp[t]);
  T.c0 = (uint32_t)H.choff.size();
  T.boff = boff;
  for (int64_t k = R.rp[t]; k < R.rp[t + 1]; k += WCHUNK) {
    int n = (int)std::min<int64_t>(WCHUNK, R.rp[t + 1] - k);
    H.push_chunk(&R.word[k], &R.v[k], n);
  }
  H.align_ent();
  T.b0 = (uint32_t)H.bval.size();
  for (int d = 0; d < R.nd; ++d) H.bval.push_back(R.band[(size_t)t * R.nd + d]);
  H.tiles.push_back(T);
}

void encode_stream(const BlockRows& R, int64_t r0, int64_t nr, uint32_t boff, int NE, HostEnc& H) {
  auto rlen = [&](int64_t t) { return R.rp[t + 1] - R.rp[t]; };
  auto push_band = [&](int64_t t0, int64_t cnt, Tile& T) {
    T.b0 = (uint32_t)H.bval.size();
    for (int d = 0; d < R.nd; ++d)
      for (int64_t t = t0; t < t0 + cnt; ++t) H.bval.push_back(R.band[(size_t)t * R.nd + d]);
  };
  int64_t t = 0;
  while (t < nr) {
    if (rlen(t) > NE) {  // one long row
      encode_long(R, r0, t, boff, H);
      ++t;
      continue;
    }
    int64_t t0 = t, ne = 0;
    while (t < nr && t - t0 < TILE_THREADS && rlen(t) <= NE && ne + rlen(t) <= NE) ne += rlen(t++);
    Tile T{};
    int64_t rows = t - t0;
    T.kind = TK_STREAM | ((uint32_t)R.nd << 8) | ((uint32_t)rows << 16);
    int64_t longest = 0;
    for (int64_t q = t0; q < t; ++q) longest = std::max<int64_t>(longest, rlen(q));
    if (longest > (int64_t)STREAM_LONG_ROW) T.kind |= TF_LONGROWS;
    T.row0 = (uint32_t)(r0 + t0);
    H.align_ent();
    T.e0 = (uint32_t)H.ent.size();
    T.ne = (uint32_t)ne;
    T.c0 = (uint32_t)H.choff.size();
    T.aux = (uint32_t)H.rowp.size();
    T.boff = boff;
    for (int64_t q = t0; q <= t; ++q) H.rowp.push_back((uint32_t)(T.e0 + (R.rp[q] - R.rp[t0])));
    for (int64_t k = R.rp[t0]; k < R.rp[t]; k += WCHUNK) {
      int n = (int)std::min<int64_t>(WCHUNK, R.rp[t] - k);
      H.push_chunk(&R.word[k], &R.v[k], n);
    }
    H.align_ent();
    push_band(t0, rows, T);
    H.max_tile_entries = std::max<int64_t>(H.max_tile_entries, ne);
    H.tiles.push_back(T);
  }
}

// SELL rows longer than this become LONG tiles of their own (the hybrid split
// of Section 2.4): no slice then waits on one long row.
constexpr int64_t SELL_ROW_CAP = 256;

void encode_sell(const BlockRows& R, int64_t r0, int64_t nr, bool sorted, uint32_t boff, HostEnc& H) {
  auto rlen = [&](int64_t t) { return R.rp[t + 1] - R.rp[t]; };
  // slot order: rows by decreasing residual length when sorted, else natural; long rows leave the slices,
  // and then the slots name their rows through perm[] in either order
  std::vector<int64_t> order, longrows;
  for (int64_t t = 0; t < nr; ++t) (rlen(t) > SELL_ROW_CAP ? longrows : order).push_back(t);
  const bool explicit_rows = sorted || !longrows.empty();
  if (sorted)
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return rlen(a) > rlen(b); });
  const int64_t nslots = ((int64_t)order.size() + WAVE - 1) / WAVE * WAVE;
  order.resize(nslots, -1);
  uint32_t words[SELL_GROUP], vals[SELL_GROUP];
  for (int64_t s0 = 0; s0 < nslots; s0 += WAVE * SELL_SLICES) {
    int nsl = (int)std::min<int64_t>(SELL_SLICES, (nslots - s0) / WAVE);
    Tile T{};
    T.kind = TK_SELL | (explicit_rows ? TF_SORTED : 0) | ((uint32_t)R.nd << 8) | ((uint32_t)(nsl * WAVE) << 16);
    H.align_ent();
    T.e0 = (uint32_t)H.ent.size();
    T.ne = (uint32_t)nsl;
    T.c0 = (uint32_t)H.choff.size();
    T.aux = (uint32_t)H.swidth.size();
    T.boff = boff;
    if (explicit_rows) {
      T.row0 = (uint32_t)H.perm.size();
      for (int64_t q = s0; q < s0 + nsl * WAVE; ++q) H.perm.push_back(order[q] < 0 ? 0xFFFFFFFFu : (uint32_t)(r0 + order[q]));
    } else {
      T.row0 = (uint32_t)(r0 + s0);
    }
    for (int sl = 0; sl < nsl; ++sl) {
      int64_t w = 0;
      for (int l = 0; l < WAVE; ++l) {
        int64_t t = order[s0 + sl * WAVE + l];
        if (t >= 0) w = std::max<int64_t>(w, rlen(t));
      }
      const int64_t groups = (w + WIDE - 1) / WIDE;
      H.swidth.push_back((uint32_t)groups);
      for (int64_t g = 0; g < groups; ++g) {  // word 4*lane + k: entry 4g + k of the lane's row
        for (int l = 0; l < WAVE; ++l) {
          int64_t t = order[s0 + sl * WAVE + l];
          for (int k = 0; k < WIDE; ++k) {
            int64_t j = g * WIDE + k;
            bool in = t >= 0 && j < rlen(t);
            words[l * WIDE + k] = in ? R.word[R.rp[t] + j] : PAD_WORD;
            vals[l * WIDE + k] = in ? R.v[R.rp[t] + j] : 0u;
          }
        }
        H.push_chunk(words, vals, SELL_GROUP);
      }
    }
    T.b0 = (uint32_t)H.bval.size();
    for (int d = 0; d < R.nd; ++d)
      for (int64_t q = s0; q < s0 + nsl * WAVE; ++q) {
        int64_t t = order[q];
        H.bval.push_back(t >= 0 ? R.band[(size_t)t * R.nd + d] : 0u);
      }
    H.tiles.push_back(T);
  }
  for (int64_t t : longrows) encode_long(R, r0, t, boff, H);
}

template <typename T>
size_t add_part(std::vector<size_t>& offs, size_t& total, size_t n) {
  size_t off = total;
  offs.push_back(off);
  total += (n * sizeof(T) + 255) / 256 * 256;
  return off;
}

}  // namespace

// Appends part P (one block encoded from offset 0) to G, moving its offsets.
static void merge_part(HostEnc& G, const HostEnc& P) {
  const uint32_t o_ent = (uint32_t)G.ent.size(), o_val = (uint32_t)G.val.size(), o_choff = (uint32_t)G.choff.size(),
                 o_rowp = (uint32_t)G.rowp.size(), o_perm = (uint32_t)G.perm.size(),
                 o_sw = (uint32_t)G.swidth.size(), o_bval = (uint32_t)G.bval.size(),
                 o_boffs = (uint32_t)G.boffs.size();
  for (Tile T : P.tiles) {
    T.e0 += o_ent;
    T.c0 += o_choff;
    T.b0 += o_bval;
    T.boff += o_boffs;
    if (tile_kind(T.kind) == TK_STREAM) T.aux += o_rowp;
    if (tile_kind(T.kind) == TK_SELL) {
      T.aux += o_sw;
      if (T.kind & TF_SORTED) T.row0 += o_perm;
    }
    G.tiles.push_back(T);
  }
  G.ent.insert(G.ent.end(), P.ent.begin(), P.ent.end());
  G.val.insert(G.val.end(), P.val.begin(), P.val.end());
  for (uint32_t c : P.choff) G.choff.push_back(c + o_val);
  for (uint32_t r : P.rowp) G.rowp.push_back(r + o_ent);
  G.perm.insert(G.perm.end(), P.perm.begin(), P.perm.end());
  G.swidth.insert(G.swidth.end(), P.swidth.begin(), P.swidth.end());
  G.bval.insert(G.bval.end(), P.bval.begin(), P.bval.end());
  G.boffs.insert(G.boffs.end(), P.boffs.begin(), P.boffs.end());
  G.max_tile_entries = std::max(G.max_tile_entries, P.max_tile_entries);
  G.max_row_terms = std::max(G.max_row_terms, P.max_row_terms);
  G.n_plus += P.n_plus;
  G.n_minus += P.n_minus;
  G.n_band += P.n_band;
  G.nnz += P.nnz;
}

void encode(const RCsr& A, const Modulus& md, const PlanOpts& o, hipStream_t stream, Encoded* out,
            const std::vector<int32_t>* forced) {
  const int64_t BR = o.block_rows;
  int64_t nblocks = (A.nrows + BR - 1) / BR;
  std::vector<BlockStats> stats(nblocks);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t b = 0; b < nblocks; ++b) stats[b] = block_stats(A, b * BR, std::min(A.nrows, (b + 1) * BR), md.m, o);
  std::vector<int32_t> fmt(nblocks, FFX_FMT_STREAM);
  bool chosen = false;
  if (forced) {
    if ((int64_t)forced->size() != nblocks) fail(FFX_EINVAL, "forced format list has %zu entries, matrix has %lld blocks", forced->size(), (long long)nblocks);
    fmt = *forced;
    chosen = true;
  } else if (o.selector == FFX_SEL_FIXED) {
    std::fill(fmt.begin(), fmt.end(), o.fixed_format);
    chosen = true;
  } else if (o.selector == FFX_SEL_LEARNED) {
    chosen = learned_formats(o.model_path, stats, fmt, stream);
  }
  if (!chosen)
    for (int64_t b = 0; b < nblocks; ++b) fmt[b] = heuristic_format(stats[b], o);
  for (int64_t b = 0; b < nblocks; ++b)
    if (fmt[b] < 0 || fmt[b] >= FFX_NUM_FORMATS) fail(FFX_EINVAL, "format %d for block %lld", fmt[b], (long long)b);

  out->block_fmt = fmt;
  std::fill(out->format_blocks, out->format_blocks + FFX_NUM_FORMATS, 0);
  for (int64_t b = 0; b < nblocks; ++b) out->format_blocks[fmt[b]]++;
  // every block is encoded on its own (in parallel), then the parts are merged in order
  std::vector<HostEnc> parts(nblocks);
  static const std::vector<int32_t> no_band;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t b = 0; b < nblocks; ++b) {
    const int f = fmt[b];
    HostEnc& P = parts[b];
    int64_t r0 = b * BR, r1 = std::min(A.nrows, (b + 1) * BR);
    bool band = f >= FFX_FMT_BAND_STREAM;
    const std::vector<int32_t>& offs = band ? stats[b].band_offsets : no_band;
    P.boffs.assign(offs.begin(), offs.end());
    BlockRows R = split_block(A, r0, r1, offs, md.m, o.split_pm1, P);
    int base = band ? f - FFX_FMT_BAND_STREAM : f;
    if (base == FFX_FMT_STREAM) encode_stream(R, r0, r1 - r0, 0, o.tile_entries, P);
    else encode_sell(R, r0, r1 - r0, base == FFX_FMT_SELL_SORTED, 0, P);
  }
  HostEnc H;
  out->block_tile0.assign(nblocks + 1, 0);
  for (int64_t b = 0; b < nblocks; ++b) {
    out->block_tile0[b] = (uint32_t)H.tiles.size();
    merge_part(H, parts[b]);
    HostEnc().tiles.swap(parts[b].tiles);  // free as we go
    parts[b] = HostEnc();
  }
  out->block_tile0[nblocks] = (uint32_t)H.tiles.size();
  if (H.ent.size() >= UINT32_MAX || H.val.size() >= UINT32_MAX || H.bval.size() >= UINT32_MAX)
    fail(FFX_EUNSUPPORTED, "encoded matrix exceeds 2^32 words in one array");
  // a last value offset after the last chunk: chunk c's values end at choff[c + 1] for every c
  H.choff.push_back((uint32_t)H.val.size());

  // one device allocation, 256-byte aligned parts
  const bool small = md.small();
  const size_t vb = small ? 2 : 4;
  std::vector<size_t> offs;
  size_t total = 0;
  add_part<Tile>(offs, total, H.tiles.size());
  add_part<uint32_t>(offs, total, H.ent.size());
  // 16 spare bytes: a lane reads its values with one 12- or 16-byte load
  size_t o_val = total; offs.push_back(o_val); total += (H.val.size() * vb + 16 + 255) / 256 * 256;
  add_part<uint32_t>(offs, total, H.choff.size());
  add_part<uint32_t>(offs, total, H.rowp.size());
  add_part<uint32_t>(offs, total, H.perm.size());
  add_part<uint32_t>(offs, total, H.swidth.size());
  size_t o_bval = total; offs.push_back(o_bval); total += (H.bval.size() * vb + 255) / 256 * 256;
  add_part<int32_t>(offs, total, H.boffs.size());
  std::vector<uint32_t> ltiles;  // STREAM tiles with long rows, for the s > 1 long-row kernel
  for (size_t t = 0; t < H.tiles.size(); ++t)
    if (tile_kind(H.tiles[t].kind) == TK_STREAM && (H.tiles[t].kind & TF_LONGROWS)) ltiles.push_back((uint32_t)t);
  add_part<uint32_t>(offs, total, ltiles.size());
  if (total == 0) total = 256;
  std::vector<unsigned char> host(total, 0);
  auto put = [&](size_t off, const void* src, size_t bytes) { if (bytes) std::memcpy(host.data() + off, src, bytes); };
  put(offs[0], H.tiles.data(), H.tiles.size() * sizeof(Tile));
  put(offs[1], H.ent.data(), H.ent.size() * 4);
  if (small) {
    uint16_t* p = (uint16_t*)(host.data() + offs[2]);
    for (size_t i = 0; i < H.val.size(); ++i) p[i] = (uint16_t)H.val[i];
    uint16_t* q = (uint16_t*)(host.data() + offs[7]);
    for (size_t i = 0; i < H.bval.size(); ++i) q[i] = (uint16_t)H.bval[i];
  } else {
    put(offs[2], H.val.data(), H.val.size() * 4);
    put(offs[7], H.bval.data(), H.bval.size() * 4);
  }
  put(offs[3], H.choff.data(), H.choff.size() * 4);
  put(offs[4], H.rowp.data(), H.rowp.size() * 4);
  put(offs[5], H.perm.data(), H.perm.size() * 4);
  put(offs[6], H.swidth.data(), H.swidth.size() * 4);
  put(offs[9], ltiles.data(), ltiles.size() * 4);
  put(offs[8], H.boffs.data(), H.boffs.size() * 4);

  void* dev = nullptr;
  if (hipMalloc(&dev, total) != hipSuccess) fail(FFX_ENOMEM, "hipMalloc of %zu bytes for the encoded matrix failed", total);
  out->allocs.push_back(dev);
  FFX_HIP(hipMemcpyAsync(dev, host.data(), total, hipMemcpyHostToDevice, stream));
  FFX_HIP(hipStreamSynchronize(stream));
  unsigned char* d = (unsigned char*)dev;
  DevMat& dm = out->dm;
  dm.tiles = (const Tile*)(d + offs[0]);
  dm.ent = (const uint32_t*)(d + offs[1]);
  dm.val = (const void*)(d + offs[2]);
  dm.choff = (const uint32_t*)(d + offs[3]);
  dm.rowp = (const uint32_t*)(d + offs[4]);
  dm.perm = (const uint32_t*)(d + offs[5]);
  dm.swidth = (const uint32_t*)(d + offs[6]);
  dm.bval = (const void*)(d + offs[7]);
  dm.boffs = (const int32_t*)(d + offs[8]);
  dm.ltiles = (const uint32_t*)(d + offs[9]);
  dm.nltiles = (uint32_t)ltiles.size();
  dm.ntiles = (uint32_t)H.tiles.size();
  dm.nrows = (uint32_t)A.nrows;
  dm.ncols = (uint32_t)A.ncols;
  dm.m = md.m;
  dm.mu = md.mu;
  dm.inv_m = md.inv_m;
  dm.inv_mf = 1.0f / (float)md.m;

  out->nrows = A.nrows;
  out->ncols = A.ncols;
  out->ntiles = (int64_t)H.tiles.size();
  out->max_row_terms = H.max_row_terms;
  out->n_band = H.n_band;
  out->n_plus = H.n_plus;
  out->n_minus = H.n_minus;
  out->nnz = H.nnz;
  out->device_bytes = (int64_t)total;
  out->stream_bytes = (int64_t)(H.tiles.size() * sizeof(Tile) + H.ent.size() * 4 + H.val.size() * vb +
                                H.choff.size() * 4 + H.rowp.size() * 4 + H.perm.size() * 4 + H.swidth.size() * 4 +
                                H.bval.size() * vb + H.boffs.size() * 4);
  out->max_tile_entries = H.max_tile_entries;
  std::fill(out->kind_tiles, out->kind_tiles + 3, 0);
  for (const Tile& T : H.tiles) out->kind_tiles[tile_kind(T.kind) == TK_SELL ? 2 : tile_kind(T.kind) == TK_LONG ? 1 : 0]++;
  out->tile_cost.resize(H.tiles.size());
  for (size_t t = 0; t < H.tiles.size(); ++t) {
    const Tile& T = H.tiles[t];
    uint64_t words = 0;
    if (tile_kind(T.kind) == TK_SELL)
      for (uint32_t k = 0; k < T.ne; ++k) words += (uint64_t)H.swidth[T.aux + k] * SELL_GROUP;
    else
      words = T.ne;
    uint64_t rows = tile_kind(T.kind) == TK_LONG ? 1 : tile_rows(T.kind);
    out->tile_cost[t] = (uint32_t)std::min<uint64_t>(UINT32_MAX, words + rows * tile_nd(T.kind) + rows);
  }
  out->n_ent = (int64_t)H.ent.size();
  out->n_val = (int64_t)H.val.size();
  out->n_choff = (int64_t)H.choff.size();
  out->n_rowp = (int64_t)H.rowp.size();
  out->n_perm = (int64_t)H.perm.size();
  out->n_swidth = (int64_t)H.swidth.size();
  out->n_bval = (int64_t)H.bval.size();
  out->n_boffs = (int64_t)H.boffs.size();
}

}  // namespace ffx
