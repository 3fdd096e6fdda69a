// Column-sorted row groups (layout in sg.h): the host encoder.
#include <algorithm>
#include <cstring>

#include "host.h"

namespace ffx {

void SgEncoded::release() {
  if (alloc) (void)hipFree(alloc);
  alloc = nullptr;
  dm = SgMat{};
  ngroups = 0;
}

namespace {

struct SgPart {  // one group, encoded from offset 0
  std::vector<uint32_t> ent, choff, cbase;
  std::vector<uint16_t> val;
};

inline uint32_t sg_tag(uint32_t v, uint32_t m, bool split) {
  if (!split) return TAG_GEN;
  if (v == 1) return TAG_PLUS;  // m = 2: 1 = -1 counts as +1
  if (v == m - 1) return TAG_MINUS;
  return TAG_GEN;
}

// rows [r0, r1) of A: entries sorted by (column, row), cut into chunks within 65,536-column panels
void encode_group(const RCsr& A, int64_t r0, int64_t r1, uint32_t m, bool split, SgPart& P) {
  const int64_t k0 = A.rp[r0], k1 = A.rp[r1];
  // key: column (bits 30..59) | row in the group (bits 16..29) | value (bits 0..15)
  std::vector<uint64_t> key((size_t)(k1 - k0));
  for (int64_t i = r0; i < r1; ++i)
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
      key[k - k0] = ((uint64_t)A.col[k] << 30) | ((uint64_t)(i - r0) << SG_ROW_SHIFT) | A.val[k];
  std::sort(key.begin(), key.end());
  size_t q = 0;
  uint32_t w[SG_CHUNK];
  while (q < key.size()) {
    const uint32_t panel = (uint32_t)(key[q] >> 30) >> 16;
    size_t q1 = q;
    while (q1 < key.size() && ((uint32_t)(key[q1] >> 30) >> 16) == panel) ++q1;
    for (size_t c = q; c < q1; c += SG_CHUNK) {
      P.choff.push_back((uint32_t)P.val.size());
      P.cbase.push_back(panel << 16);
      uint16_t vv[SG_CHUNK];
      for (int t = 0; t < SG_CHUNK; ++t) {
        if (c + t < q1) {
          const uint64_t kk = key[c + t];
          const uint32_t col = (uint32_t)(kk >> 30), lr = (uint32_t)(kk >> SG_ROW_SHIFT) & (SG_MAX_ROWS - 1);
          const uint32_t v = (uint32_t)(kk & 0xFFFFu);
          const uint32_t tag = sg_tag(v, m, split);
          w[t] = (tag << TAG_SHIFT) | (lr << SG_ROW_SHIFT) | (col & SG_COL_MASK);
          vv[t] = (uint16_t)v;
        } else {
          w[t] = PAD_WORD;
        }
      }
      // entry 64k + l at word 4l + k: one 16-byte load per lane; the general values in the same
      // lane-major order, so a lane's values are consecutive
      for (int l = 0; l < 64; ++l)
        for (int k = 0; k < 4; ++k) {
          const uint32_t word = w[64 * k + l];
          P.ent.push_back(word);
          if ((word >> TAG_SHIFT) == TAG_GEN) P.val.push_back(vv[64 * k + l]);
        }
    }
    q = q1;
  }
}

}  // namespace

void encode_sg(const RCsr& A, const Modulus& md, bool split_pm1, int target_groups, hipStream_t st, SgEncoded* out) {
  out->release();
  if (!md.small()) fail(FFX_EUNSUPPORTED, "column-sorted groups need m <= 65536");
  const int64_t n = A.nrows, nnz = A.nnz();
  if (n == 0) return;
  // groups of consecutive rows, about nnz / target entries each, at most SG_MAX_ROWS rows
  const int64_t want = std::max<int64_t>({(int64_t)std::max(1, target_groups), (n + SG_MAX_ROWS - 1) / SG_MAX_ROWS});
  std::vector<std::pair<int64_t, int64_t>> ranges;
  for (int64_t r = 0; r < n;) {
    const int64_t left = std::max<int64_t>(1, want - (int64_t)ranges.size());
    const int64_t target = (nnz - A.rp[r] + left - 1) / left;
    const int64_t r0 = r;
    ++r;
    while (r < n && r - r0 < (int64_t)SG_MAX_ROWS && A.rp[r + 1] - A.rp[r0] <= target) ++r;
    ranges.push_back({r0, r});
  }
  const int64_t G = (int64_t)ranges.size();
  std::vector<SgPart> parts(G);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t g = 0; g < G; ++g) encode_group(A, ranges[g].first, ranges[g].second, md.m, split_pm1, parts[g]);
  std::vector<SgGroup> groups(G);
  size_t nent = 0, nval = 0, nch = 0;
  uint32_t max_rows = 0;
  for (int64_t g = 0; g < G; ++g) {
    groups[g] = SgGroup{(uint32_t)ranges[g].first, (uint32_t)(ranges[g].second - ranges[g].first), (uint32_t)nch,
                        (uint32_t)parts[g].choff.size()};
    max_rows = std::max(max_rows, groups[g].nrows);
    nent += parts[g].ent.size();
    nval += parts[g].val.size();
    nch += parts[g].choff.size();
  }
  if (nent >= UINT32_MAX || nval >= UINT32_MAX) fail(FFX_EUNSUPPORTED, "column-sorted encoding exceeds 2^32 words");
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t o_g = 0, o_e = o_g + al(G * sizeof(SgGroup)), o_v = o_e + al(nent * 4),
               o_c = o_v + al(nval * 2 + 16), o_b = o_c + al(nch * 4), total = std::max<size_t>(256, o_b + al(nch * 4));
  std::vector<unsigned char> host(total, 0);
  std::memcpy(host.data() + o_g, groups.data(), G * sizeof(SgGroup));
  size_t e = 0, v = 0, c = 0;
  for (int64_t g = 0; g < G; ++g) {
    const SgPart& P = parts[g];
    std::memcpy(host.data() + o_e + e * 4, P.ent.data(), P.ent.size() * 4);
    std::memcpy(host.data() + o_v + v * 2, P.val.data(), P.val.size() * 2);
    uint32_t* ch = (uint32_t*)(host.data() + o_c) + c;
    for (size_t k = 0; k < P.choff.size(); ++k) ch[k] = P.choff[k] + (uint32_t)v;
    std::memcpy(host.data() + o_b + c * 4, P.cbase.data(), P.cbase.size() * 4);
    e += P.ent.size();
    v += P.val.size();
    c += P.choff.size();
  }
  if (hipMalloc(&out->alloc, total) != hipSuccess)
    fail(FFX_ENOMEM, "hipMalloc of %zu bytes for the column-sorted groups failed", total);
  if (hipMemcpyAsync(out->alloc, host.data(), total, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    out->release();
    fail(FFX_EDEVICE, "upload of the column-sorted groups failed");
  }
  unsigned char* d = (unsigned char*)out->alloc;
  SgMat& M = out->dm;
  M.groups = (const SgGroup*)(d + o_g);
  M.ent = (const uint32_t*)(d + o_e);
  M.val = (const uint16_t*)(d + o_v);
  M.choff = (const uint32_t*)(d + o_c);
  M.cbase = (const uint32_t*)(d + o_b);
  M.rowmap = nullptr;
  M.ngroups = (uint32_t)G;
  M.max_rows = max_rows;
  M.nrows = (uint32_t)n;
  M.m = md.m;
  M.mu = md.mu;
  out->ngroups = G;
  out->device_bytes = (int64_t)total;
  out->stream_bytes = (int64_t)(G * sizeof(SgGroup) + nent * 4 + nval * 2 + nch * 8);
}

}  // namespace ffx
