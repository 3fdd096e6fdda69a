// Symmetric reordering of a square matrix before it is encoded (the
// reordering of A that Section 4 (the conclusion) expects to improve the products): reverse
// Cuthill-McKee (Cuthill and McKee 1969, with the reversal of George 1971) on
// the pattern of A + A^T, started from a pseudo-peripheral node (George and
// Liu 1979). Rows that are coupled end up close together, so the x entries a
// tile gathers come from a narrow window that stays in L2.
#include <algorithm>
#include <numeric>

#include "host.h"

namespace ffx {

// Pattern of A + A^T without the diagonal, rows sorted and free of repeats.
static void sym_pattern(const RCsr& A, std::vector<int64_t>& rp, std::vector<uint32_t>& adj) {
  const int64_t n = A.nrows;
  std::vector<int64_t> cnt(n + 1, 0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      uint32_t j = A.col[k];
      if (j != (uint32_t)i) {
        cnt[i + 1]++;
        cnt[j + 1]++;
      }
    }
  std::partial_sum(cnt.begin(), cnt.end(), cnt.begin());
  std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
  std::vector<uint32_t> raw(cnt[n]);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      uint32_t j = A.col[k];
      if (j != (uint32_t)i) {
        raw[fill[i]++] = j;
        raw[fill[j]++] = (uint32_t)i;
      }
    }
  std::vector<int64_t> len(n);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < n; ++i) {
    auto b = raw.begin() + cnt[i], e = raw.begin() + cnt[i + 1];
    std::sort(b, e);
    len[i] = std::unique(b, e) - b;
  }
  rp.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) rp[i + 1] = rp[i] + len[i];
  adj.resize(rp[n]);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < n; ++i) std::copy_n(raw.begin() + cnt[i], len[i], adj.begin() + rp[i]);
}

std::vector<uint32_t> rcm_order(const RCsr& A) {
  const int64_t n = A.nrows;
  std::vector<int64_t> rp;
  std::vector<uint32_t> adj;
  sym_pattern(A, rp, adj);
  auto deg = [&](uint32_t v) { return rp[v + 1] - rp[v]; };
  std::vector<uint32_t> by_degree(n);
  std::iota(by_degree.begin(), by_degree.end(), 0u);
  std::stable_sort(by_degree.begin(), by_degree.end(), [&](uint32_t a, uint32_t b) { return deg(a) < deg(b); });

  std::vector<uint32_t> order;
  order.reserve(n);
  std::vector<char> placed(n, 0);
  std::vector<uint32_t> stamp(n, 0), queue;
  queue.reserve(n);
  uint32_t cur_stamp = 0;
  // breadth-first levels from s over the component of s: returns the number
  // of levels and leaves the last level at the tail of queue from `last`
  auto bfs = [&](uint32_t s, size_t& last) {
    ++cur_stamp;
    queue.clear();
    queue.push_back(s);
    stamp[s] = cur_stamp;
    size_t head = 0;
    int64_t levels = 0;
    last = 0;
    while (head < queue.size()) {
      size_t end = queue.size();
      last = head;
      ++levels;
      for (; head < end; ++head) {
        uint32_t u = queue[head];
        for (int64_t k = rp[u]; k < rp[u + 1]; ++k) {
          uint32_t v = adj[k];
          if (stamp[v] != cur_stamp) {
            stamp[v] = cur_stamp;
            queue.push_back(v);
          }
        }
      }
    }
    return levels;
  };
  std::vector<std::pair<int64_t, uint32_t>> nb;
  for (uint32_t first : by_degree) {
    if (placed[first]) continue;
    // pseudo-peripheral start: move to a smallest-degree node of the last
    // level while that lengthens the level structure
    uint32_t s = first;
    size_t last = 0;
    int64_t ecc = bfs(s, last);
    for (int iter = 0; iter < 16; ++iter) {
      uint32_t best = queue[last];
      for (size_t q = last; q < queue.size(); ++q)
        if (deg(queue[q]) < deg(best)) best = queue[q];
      size_t last2 = 0;
      int64_t e2 = bfs(best, last2);
      if (e2 <= ecc) break;
      s = best;
      ecc = e2;
      last = last2;
    }
    // Cuthill-McKee: breadth first, neighbours taken by increasing degree
    size_t head = order.size();
    order.push_back(s);
    placed[s] = 1;
    while (head < order.size()) {
      uint32_t u = order[head++];
      nb.clear();
      for (int64_t k = rp[u]; k < rp[u + 1]; ++k) {
        uint32_t v = adj[k];
        if (!placed[v]) {
          placed[v] = 1;
          nb.emplace_back(deg(v), v);
        }
      }
      std::sort(nb.begin(), nb.end());
      for (auto& p : nb) order.push_back(p.second);
    }
  }
  std::reverse(order.begin(), order.end());
  return order;
}

RCsr permute_sym(const RCsr& A, const std::vector<uint32_t>& perm) {
  const int64_t n = A.nrows;
  std::vector<uint32_t> inv(n);
  for (int64_t i = 0; i < n; ++i) inv[perm[i]] = (uint32_t)i;
  RCsr B;
  B.nrows = n;
  B.ncols = A.ncols;
  B.rp.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) B.rp[i + 1] = B.rp[i] + (A.rp[perm[i] + 1] - A.rp[perm[i]]);
  B.col.resize(A.col.size());
  B.val.resize(A.val.size());
#pragma omp parallel
  {
    std::vector<std::pair<uint32_t, uint32_t>> row;
#pragma omp for schedule(dynamic, 4096)
    for (int64_t i = 0; i < n; ++i) {
      const uint32_t o = perm[i];
      row.clear();
      for (int64_t k = A.rp[o]; k < A.rp[o + 1]; ++k) row.emplace_back(inv[A.col[k]], A.val[k]);
      std::sort(row.begin(), row.end());
      int64_t d = B.rp[i];
      for (auto& e : row) {
        B.col[d] = e.first;
        B.val[d++] = e.second;
      }
    }
  }
  return B;
}

int64_t bandwidth(const RCsr& A) {
  int64_t bw = 0;
#pragma omp parallel for reduction(max : bw) schedule(static, 65536)
  for (int64_t i = 0; i < A.nrows; ++i)
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) bw = std::max<int64_t>(bw, std::abs((int64_t)A.col[k] - i));
  return bw;
}

}  // namespace ffx
