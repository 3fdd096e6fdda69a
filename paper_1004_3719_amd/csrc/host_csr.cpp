// Input validation and reduction modulo m of the caller's CSR/COO arrays.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "host.h"

namespace ffx {

static inline uint32_t canon_i64(int64_t v, uint32_t m) {
  int64_t r = v % (int64_t)m;
  return (uint32_t)(r < 0 ? r + (int64_t)m : r);
}

static inline int64_t raw_value(const void* vals, ffx_dtype vt, int64_t k) {
  return vt == FFX_I32 ? (int64_t)((const int32_t*)vals)[k] : ((const int64_t*)vals)[k];
}

static void check_common(int64_t nrows, int64_t ncols, const void* vals, ffx_dtype vt, uint32_t m) {
  if (m < 2 || m > 2147483647u) fail(FFX_EINVAL, "modulus %u outside [2, 2^31-1]", m);
  if (nrows < 0 || ncols < 0 || nrows > MAX_DIM || ncols > MAX_DIM)
    fail(FFX_EINVAL, "dimensions %lld x %lld outside [0, 2^30]", (long long)nrows, (long long)ncols);
  if (vt != FFX_I32 && vt != FFX_I64) fail(FFX_EINVAL, "value type %d is neither FFX_I32 nor FFX_I64", (int)vt);
  (void)vals;
}

// Appends row entries (col, residue) after sorting by column, adding
// duplicates modulo m and dropping zero residues.
static void finish_row(std::vector<std::pair<uint32_t, uint32_t>>& tmp, uint32_t m, RCsr& out) {
  std::sort(tmp.begin(), tmp.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
  size_t i = 0;
  while (i < tmp.size()) {
    uint32_t c = tmp[i].first;
    uint64_t s = 0;
    while (i < tmp.size() && tmp[i].first == c) s += tmp[i++].second;  // < 2^31 * count
    uint32_t r = (uint32_t)(s % m);
    if (r) {
      out.col.push_back(c);
      out.val.push_back(r);
    }
  }
}

RCsr reduce_csr(int64_t nrows, int64_t ncols, const int64_t* rowptr, const int32_t* colidx, const void* vals,
                ffx_dtype vt, uint32_t m) {
  check_common(nrows, ncols, vals, vt, m);
  if (!rowptr) fail(FFX_EINVAL, "rowptr is NULL");
  if (rowptr[0] != 0) fail(FFX_EINVAL, "rowptr[0] = %lld, expected 0", (long long)rowptr[0]);
  for (int64_t i = 0; i < nrows; ++i)
    if (rowptr[i + 1] < rowptr[i]) fail(FFX_EINVAL, "rowptr decreases at row %lld", (long long)i);
  int64_t nnz = rowptr[nrows];
  if (nnz >= (int64_t)UINT32_MAX) fail(FFX_EINVAL, "%lld entries, at most 2^32-2 supported", (long long)nnz);
  if (nnz > 0 && (!colidx || !vals)) fail(FFX_EINVAL, "colidx or vals is NULL");
  for (int64_t k = 0; k < nnz; ++k)
    if (colidx[k] < 0 || colidx[k] >= ncols)
      fail(FFX_EINVAL, "column index %d at entry %lld outside [0, %lld)", colidx[k], (long long)k, (long long)ncols);

  // two passes over the rows, both in parallel: kept entries per row, then the entries
  RCsr out;
  out.nrows = nrows;
  out.ncols = ncols;
  out.rp.assign(nrows + 1, 0);
  auto row_entries = [&](int64_t i, std::vector<std::pair<uint32_t, uint32_t>>& tmp) {
    int64_t a = rowptr[i], b = rowptr[i + 1];
    tmp.clear();
    bool sorted = true;
    for (int64_t k = a + 1; k < b; ++k)
      if (colidx[k] <= colidx[k - 1]) { sorted = false; break; }
    if (sorted) {
      for (int64_t k = a; k < b; ++k) {
        uint32_t r = canon_i64(raw_value(vals, vt, k), m);
        if (r) tmp.emplace_back((uint32_t)colidx[k], r);
      }
    } else {
      std::vector<std::pair<uint32_t, uint32_t>> raw;
      for (int64_t k = a; k < b; ++k) raw.emplace_back((uint32_t)colidx[k], canon_i64(raw_value(vals, vt, k), m));
      RCsr one;
      finish_row(raw, m, one);
      for (size_t q = 0; q < one.col.size(); ++q) tmp.emplace_back(one.col[q], one.val[q]);
    }
  };
#pragma omp parallel
  {
    std::vector<std::pair<uint32_t, uint32_t>> tmp;
#pragma omp for schedule(dynamic, 4096)
    for (int64_t i = 0; i < nrows; ++i) {
      row_entries(i, tmp);
      out.rp[i + 1] = (int64_t)tmp.size();
    }
  }
  for (int64_t i = 0; i < nrows; ++i) out.rp[i + 1] += out.rp[i];
  out.col.resize(out.rp[nrows]);
  out.val.resize(out.rp[nrows]);
#pragma omp parallel
  {
    std::vector<std::pair<uint32_t, uint32_t>> tmp;
#pragma omp for schedule(dynamic, 4096)
    for (int64_t i = 0; i < nrows; ++i) {
      row_entries(i, tmp);
      for (size_t q = 0; q < tmp.size(); ++q) {
        out.col[out.rp[i] + q] = tmp[q].first;
        out.val[out.rp[i] + q] = tmp[q].second;
      }
    }
  }
  return out;
}

RCsr reduce_coo(int64_t nrows, int64_t ncols, int64_t nnz, const int32_t* rowidx, const int32_t* colidx,
                const void* vals, ffx_dtype vt, uint32_t m) {
  check_common(nrows, ncols, vals, vt, m);
  if (nnz < 0 || nnz >= (int64_t)UINT32_MAX) fail(FFX_EINVAL, "nnz %lld outside [0, 2^32-2]", (long long)nnz);
  if (nnz > 0 && (!rowidx || !colidx || !vals)) fail(FFX_EINVAL, "rowidx, colidx or vals is NULL");
  std::vector<int64_t> cnt(nrows + 1, 0);
  for (int64_t k = 0; k < nnz; ++k) {
    if (rowidx[k] < 0 || rowidx[k] >= nrows)
      fail(FFX_EINVAL, "row index %d at entry %lld outside [0, %lld)", rowidx[k], (long long)k, (long long)nrows);
    if (colidx[k] < 0 || colidx[k] >= ncols)
      fail(FFX_EINVAL, "column index %d at entry %lld outside [0, %lld)", colidx[k], (long long)k, (long long)ncols);
    cnt[rowidx[k] + 1]++;
  }
  for (int64_t i = 0; i < nrows; ++i) cnt[i + 1] += cnt[i];
  std::vector<std::pair<uint32_t, uint32_t>> ent(nnz);
  std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
  for (int64_t k = 0; k < nnz; ++k) ent[pos[rowidx[k]]++] = {(uint32_t)colidx[k], canon_i64(raw_value(vals, vt, k), m)};
  RCsr out;
  out.nrows = nrows;
  out.ncols = ncols;
  out.rp.resize(nrows + 1);
  out.rp[0] = 0;
  std::vector<std::pair<uint32_t, uint32_t>> tmp;
  for (int64_t i = 0; i < nrows; ++i) {
    tmp.assign(ent.begin() + cnt[i], ent.begin() + cnt[i + 1]);
    finish_row(tmp, m, out);
    out.rp[i + 1] = (int64_t)out.col.size();
  }
  return out;
}

RCsr transpose(const RCsr& A) {
  RCsr T;
  T.nrows = A.ncols;
  T.ncols = A.nrows;
  T.rp.assign(A.ncols + 1, 0);
  for (uint32_t c : A.col) T.rp[c + 1]++;
  for (int64_t j = 0; j < A.ncols; ++j) T.rp[j + 1] += T.rp[j];
  T.col.resize(A.col.size());
  T.val.resize(A.val.size());
  std::vector<int64_t> pos(T.rp.begin(), T.rp.end() - 1);
  for (int64_t i = 0; i < A.nrows; ++i)
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      int64_t p = pos[A.col[k]]++;
      T.col[p] = (uint32_t)i;  // rows visited in increasing order: columns of T sorted
      T.val[p] = A.val[k];
    }
  return T;
}

}  // namespace ffx
