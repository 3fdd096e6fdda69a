// Batched products Y_k = A_k X_k over many matrices in one persistent launch.
//
// A work item is (matrix k, tile t, a group of at most 8 right-hand-side
// columns). Persistent workgroups take items from a device counter in the
// order of a list sorted by decreasing estimated cost (longest-processing-
// time first), so large tiles start early and small ones fill the tail. The
// counter is cleared by a one-thread kernel before the launch (no memset), and
// both launches can be captured into a hipGraph and replayed.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <type_traits>

#include "host.h"
#include "launch.h"
#include "tiles.h"

namespace ffx {

struct BatchItem {
  uint32_t k;   // matrix
  uint32_t t;   // tile of that matrix
  uint16_t c0;  // first right-hand side of the group
  uint16_t sc;  // right-hand sides in the group
  uint32_t pad;
};
static_assert(sizeof(BatchItem) == 16, "item layout");

struct BatchOperand {
  const void* X;
  void* Y;
  int64_t ldx, ldy;
};

// Right-hand-side column chunks fall in four classes (1, 2, 3..4, 5..8
// columns), each with its own persistent kernel: a kernel holding every class's
// tile paths would take the registers of the largest and run at 3 waves per
// SIMD.
constexpr int NCLS = 4;
inline int chunk_class(int sc) { return sc <= 1 ? 0 : sc <= 2 ? 1 : sc <= 4 ? 2 : 3; }

// 4 workgroups (4 waves per SIMD) for the m <= 65536 kernels: they fit 128
// registers without spilling
template <class AR>
constexpr int batch_min_blocks() { return std::is_same<AR, ArSmall>::value ? 4 : 1; }

template <class AR, typename Tv, int SC>
__global__ __launch_bounds__(TILE_THREADS, batch_min_blocks<AR>()) void k_batch(const DevMat* __restrict__ mats,
                                                        const BatchOperand* __restrict__ ops,
                                                        const BatchItem* __restrict__ items, uint32_t nitems,
                                                        uint32_t* counter) {
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ uint32_t next;
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(counter, 1u);
    __syncthreads();
    const uint32_t it = next;
    __syncthreads();  // every lane has read `next` before thread 0 may overwrite it
    if (it >= nitems) break;
    const BatchItem I = items[it];
    const DevMat A = mats[I.k];
    const BatchOperand O = ops[I.k];
    const Tile T = A.tiles[I.t];
    const Tv* X = (const Tv*)O.X + I.c0;
    Tv* Y = (Tv*)O.Y + I.c0;
    const int sc = I.sc;
    const uint32_t kind = tile_kind(T.kind);
    if constexpr (SC == 1) {
      if (kind == TK_SELL) sell_tile<AR, Tv, Tv, 1, 2>(A, T, X, O.ldx, Y, O.ldy, 1, 1, 0);
      else if (kind == TK_LONG) long_tile<AR, Tv, Tv, 1, 2>(A, T, X, O.ldx, Y, O.ldy, 1, 1, 0, lds);
      else stream_tile_1<AR, Tv, Tv, 2>(A, T, X, O.ldx, Y, O.ldy, 1, 0, lds);
    } else {
      if (kind == TK_SELL) sell_tile_rc<AR, Tv, Tv, SC>(A, T, X, O.ldx, Y, O.ldy, sc, 1, 0);
      else if (kind == TK_LONG) long_tile<AR, Tv, Tv, SC, 1>(A, T, X, O.ldx, Y, O.ldy, sc, 1, 0, lds);
      else stream_tile_s<AR, Tv, Tv, SC>(A, T, X, O.ldx, Y, O.ldy, sc, 1, 0, lds);
    }
    __syncthreads();  // LDS is reused by the next item
  }
}

__global__ void k_batch_reset(uint32_t* counter, int n) {
  if (blockIdx.x == 0 && (int)threadIdx.x < n) counter[threadIdx.x] = 0;
}

template <class AR>
static size_t batch_lds(int64_t mte, int sc) {
  size_t a = tiles_lds_bytes<AR>(mte, sc);
  return a < 16 ? 16 : a;
}

// One class's persistent launch over items [first, first + n).
static hipError_t batch_launch_class(int ak, ffx_dtype dt, int cls, const DevMat* mats, const BatchOperand* ops,
                                     const BatchItem* items, uint32_t n, uint32_t* counter, int grid, int64_t mte,
                                     hipStream_t st) {
  auto go = [&](auto ar) {
    using AR = decltype(ar);
    auto launch = [&](auto tv, auto scv) {
      using Tv = decltype(tv);
      constexpr int SC = decltype(scv)::value;
      hipLaunchKernelGGL((k_batch<AR, Tv, SC>), dim3(grid), dim3(TILE_THREADS), batch_lds<AR>(mte, SC), st, mats, ops,
                         items, n, counter);
    };
    auto by_dt = [&](auto scv) {
      if (dt == FFX_I32) launch(int32_t{}, scv);
      else launch(int64_t{}, scv);
    };
    switch (cls) {
      case 0: by_dt(std::integral_constant<int, 1>{}); break;
      case 1: by_dt(std::integral_constant<int, 2>{}); break;
      case 2: by_dt(std::integral_constant<int, 4>{}); break;
      default: by_dt(std::integral_constant<int, 8>{}); break;
    }
  };
  switch (ak) {
    case AK_SMALL: go(ArSmall{}); break;
    case AK_BIG: go(ArBig<false>{}); break;
    case AK_BIG_CH: go(ArBig<true>{}); break;
    case AK_M31: go(ArM31{}); break;
    case AK_F64_16: go(ArF64<uint16_t, false>{}); break;
    case AK_F64_16_CH: go(ArF64<uint16_t, true>{}); break;
    case AK_F64_32: go(ArF64<uint32_t, false>{}); break;
    case AK_F64_32_CH: go(ArF64<uint32_t, true>{}); break;
    case AK_F32: go(ArF32<false>{}); break;
    case AK_F32_CH: go(ArF32<true>{}); break;
    case AK_F32C: go(ArCentered<float, uint16_t, false>{}); break;
    case AK_F32C_CH: go(ArCentered<float, uint16_t, true>{}); break;
    case AK_F64C_16: go(ArCentered<double, uint16_t, false>{}); break;
    case AK_F64C_16_CH: go(ArCentered<double, uint16_t, true>{}); break;
    case AK_F64C_32: go(ArCentered<double, uint32_t, false>{}); break;
    default: go(ArCentered<double, uint32_t, true>{}); break;
  }
  return hipGetLastError();
}

}  // namespace ffx

// ----------------------------------------------------------------- host ----
using namespace ffx;

struct ffx_batch_s {
  int count = 0;
  std::vector<ffx_matrix> mats;
  std::vector<int32_t> s;
  int ak = 0;
  int64_t mte = 0;
  int ncu = 0;
  ffx_batch_params params{};
  DevMat* d_mats = nullptr;
  BatchOperand* d_ops = nullptr;
  BatchItem* d_items = nullptr;
  uint32_t* d_counter = nullptr;  // one per chunk class
  uint32_t nitems = 0;
  uint32_t cls_first[NCLS] = {0, 0, 0, 0}, cls_n[NCLS] = {0, 0, 0, 0};
  std::vector<BatchOperand> h_ops;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  int graph_dt = -1;
  std::string signature;
  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
};

namespace ffx {
int matrix_arith_kind(const ffx_matrix_s& M);
const std::vector<uint32_t>& matrix_tile_cost(const ffx_matrix_s& M);
void set_last_error(const std::string& s);
}  // namespace ffx

static void batch_items(ffx_batch_s* B) {
  std::vector<BatchItem> items;
  std::vector<uint64_t> cost;
  const int chunk = B->params.max_chunk == 4 ? 4 : 8;
  for (int k = 0; k < B->count; ++k) {
    const auto& tc = matrix_tile_cost(*B->mats[k]);
    for (uint32_t t = 0; t < (uint32_t)tc.size(); ++t)
      for (int c0 = 0; c0 < B->s[k]; c0 += chunk) {
        int sc = std::min(chunk, B->s[k] - c0);
        items.push_back(BatchItem{(uint32_t)k, t, (uint16_t)c0, (uint16_t)sc, 0});
        cost.push_back((uint64_t)tc[t] * (uint64_t)(sc + 3));
      }
  }
  // by chunk class (each class is one kernel), then by decreasing cost when order == 0
  std::vector<size_t> idx(items.size());
  for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
  const bool by_cost = B->params.order == 0;
  std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) {
    int ca = chunk_class(items[a].sc), cb = chunk_class(items[b].sc);
    if (ca != cb) return ca < cb;
    return by_cost && cost[a] > cost[b];
  });
  std::vector<BatchItem> sorted(items.size());
  for (size_t i = 0; i < idx.size(); ++i) sorted[i] = items[idx[i]];
  items.swap(sorted);
  for (int c = 0; c < NCLS; ++c) B->cls_first[c] = B->cls_n[c] = 0;
  for (size_t i = 0; i < items.size(); ++i) {
    int c = chunk_class(items[i].sc);
    if (B->cls_n[c]++ == 0) B->cls_first[c] = (uint32_t)i;
  }
  if (B->d_items) (void)hipFree(B->d_items);
  B->d_items = nullptr;
  B->nitems = (uint32_t)items.size();
  if (items.empty()) return;
  FFX_HIP(hipMalloc(&B->d_items, items.size() * sizeof(BatchItem)));
  FFX_HIP(hipMemcpy(B->d_items, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice));
}

static void check_params(const ffx_batch_params& p) {
  if (p.wg_per_cu < 0 || p.wg_per_cu > 8) fail(FFX_EINVAL, "wg_per_cu %d outside [0, 8]", p.wg_per_cu);
  if (p.order != 0 && p.order != 1) fail(FFX_EINVAL, "order %d", p.order);
  if (p.max_chunk != 4 && p.max_chunk != 8) fail(FFX_EINVAL, "max_chunk %d (4 or 8)", p.max_chunk);
}

static void batch_run(ffx_batch_s* B, const void* const* X, const int64_t* ldx, void* const* Y, const int64_t* ldy,
                      ffx_dtype dt, hipStream_t st) {
  if (dt != FFX_I32 && dt != FFX_I64) fail(FFX_EINVAL, "dtype %d", (int)dt);
  if (!X || !Y || !ldx || !ldy) fail(FFX_EINVAL, "NULL operand array");
  const size_t es = dt == FFX_I32 ? 4 : 8;
  for (int k = 0; k < B->count; ++k) {
    const auto& I = B->mats[k]->info;
    if (ldx[k] < B->s[k] || ldy[k] < B->s[k]) fail(FFX_EINVAL, "matrix %d: leading dimension below s", k);
    if ((I.ncols > 0 && !X[k]) || (I.nrows > 0 && !Y[k])) fail(FFX_EINVAL, "matrix %d: NULL operand", k);
    uintptr_t x0 = (uintptr_t)X[k], x1 = x0 + (uintptr_t)(((I.ncols > 0 ? I.ncols - 1 : 0) * ldx[k] + B->s[k]) * es);
    uintptr_t y0 = (uintptr_t)Y[k], y1 = y0 + (uintptr_t)(((I.nrows > 0 ? I.nrows - 1 : 0) * ldy[k] + B->s[k]) * es);
    if (I.ncols > 0 && I.nrows > 0 && x0 < y1 && y0 < x1) fail(FFX_EINVAL, "matrix %d: X and Y overlap", k);
    B->h_ops[k] = BatchOperand{X[k], Y[k], ldx[k], ldy[k]};
  }
  if (B->nitems == 0) return;
  // operand table: pageable host memory, so the copy is staged before the call returns
  FFX_HIP(hipMemcpyAsync(B->d_ops, B->h_ops.data(), B->h_ops.size() * sizeof(BatchOperand), hipMemcpyHostToDevice, st));
  const int wpc = B->params.wg_per_cu ? B->params.wg_per_cu : 4;
  auto grid_of = [&](int c) { return (int)std::min<int64_t>((int64_t)B->ncu * wpc, B->cls_n[c]); };
  auto launch_class = [&](int c, hipStream_t s) {
    return batch_launch_class(B->ak, dt, c, B->d_mats, B->d_ops, B->d_items + B->cls_first[c], B->cls_n[c],
                              B->d_counter + c, grid_of(c), B->mte, s);
  };
  if (B->params.use_graph) {
    if (B->exec && B->graph_dt != (int)dt) B->drop_graph();
    if (!B->exec) {
      // the classes are independent branches of one graph: their kernels share the GPU and their
      // tails overlap
      B->graph_dt = (int)dt;
      hipStream_t cs, br[NCLS] = {};
      hipEvent_t ev0 = nullptr, evc[NCLS] = {};
      FFX_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      hipError_t e = hipSuccess;
      for (int c = 0; c < NCLS && e == hipSuccess; ++c) {
        e = hipStreamCreateWithFlags(&br[c], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&evc[c], hipEventDisableTiming);
      }
      if (e == hipSuccess) e = hipEventCreateWithFlags(&ev0, hipEventDisableTiming);
      if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, cs, B->d_counter, NCLS);
        hipError_t le = hipEventRecord(ev0, cs);
        for (int c = 0; c < NCLS && le == hipSuccess; ++c) {
          if (!B->cls_n[c]) continue;
          le = hipStreamWaitEvent(br[c], ev0, 0);
          if (le == hipSuccess) le = launch_class(c, br[c]);
          if (le == hipSuccess) le = hipEventRecord(evc[c], br[c]);
          if (le == hipSuccess) le = hipStreamWaitEvent(cs, evc[c], 0);
        }
        e = hipStreamEndCapture(cs, &B->graph);
        if (e == hipSuccess) e = le;
      }
      if (e == hipSuccess) e = hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0);
      for (int c = 0; c < NCLS; ++c) {
        if (evc[c]) (void)hipEventDestroy(evc[c]);
        if (br[c]) (void)hipStreamDestroy(br[c]);
      }
      if (ev0) (void)hipEventDestroy(ev0);
      (void)hipStreamDestroy(cs);
      if (e != hipSuccess) {
        B->drop_graph();
        FFX_HIP(e);
      }
    }
    FFX_HIP(hipGraphLaunch(B->exec, st));
    return;
  }
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, st, B->d_counter, NCLS);
  for (int c = 0; c < NCLS; ++c)
    if (B->cls_n[c]) FFX_HIP(launch_class(c, st));
}


static std::string device_name() {
  int dev = 0;
  hipDeviceProp_t p;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
  return std::string(p.gcnArchName) + ":" + std::to_string(p.multiProcessorCount);
}

// tiny JSON cache: one line per entry, "key": {"wg_per_cu": a, "order": b, "max_chunk": c}
static bool cache_lookup(const char* path, const std::string& key, ffx_batch_params& p) {
  if (!path) return false;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    size_t q = line.find("\"" + key + "\"");
    if (q == std::string::npos) continue;
    int a, b, c;
    const char* s = line.c_str() + q + key.size() + 2;
    if (sscanf(s, " : {\"wg_per_cu\": %d, \"order\": %d, \"max_chunk\": %d", &a, &b, &c) == 3) {
      p.wg_per_cu = a;
      p.order = b;
      p.max_chunk = c;
      return true;
    }
  }
  return false;
}

static void cache_store(const char* path, const std::string& key, const ffx_batch_params& p) {
  if (!path) return;
  std::vector<std::string> lines;
  {
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line))
      if (line.find("\"" + key + "\"") == std::string::npos && line.find("\":") != std::string::npos) {
        while (!line.empty() && (line.back() == ',' || line.back() == ' ')) line.pop_back();
        lines.push_back(line);
      }
  }
  char buf[512];
  snprintf(buf, sizeof buf, "  \"%s\": {\"wg_per_cu\": %d, \"order\": %d, \"max_chunk\": %d}", key.c_str(),
           p.wg_per_cu, p.order, p.max_chunk);
  lines.push_back(buf);
  std::ofstream f(path);
  f << "{\n";
  for (size_t i = 0; i < lines.size(); ++i) f << lines[i] << (i + 1 < lines.size() ? ",\n" : "\n");
  f << "}\n";
}

extern "C" {

ffx_status ffx_batch_create(int32_t count, const ffx_matrix* mats, const int32_t* s, const ffx_batch_params* params,
                            void* stream, ffx_batch* out) {
  return guard([&] {
    if (!out) fail(FFX_EINVAL, "out is NULL");
    *out = nullptr;
    if (count < 1 || !mats || !s) fail(FFX_EINVAL, "empty batch");
    ffx_batch_s* B = new ffx_batch_s();
    try {
      B->count = count;
      B->mats.assign(mats, mats + count);
      B->s.assign(s, s + count);
      B->params = ffx_batch_params{0, 0, 8, 1};
      if (params) {
        check_params(*params);
        B->params = *params;
      }
      std::vector<DevMat> dm(count);
      std::ostringstream sig;
      sig << count;
      for (int k = 0; k < count; ++k) {
        if (!mats[k]) fail(FFX_EINVAL, "matrix %d is NULL", k);
        if (s[k] < 1 || s[k] > MAX_S) fail(FFX_EINVAL, "matrix %d: s = %d outside [1, 16]", k, s[k]);
        if (mats[k]->perm)
          fail(FFX_EINVAL, "matrix %d is reordered: a batch takes matrices stored in the caller's order", k);
        int ak = matrix_arith_kind(*mats[k]);
        if (k == 0) B->ak = ak;
        else if (ak != B->ak || mats[k]->md.m != mats[0]->md.m)
          fail(FFX_EINVAL, "matrix %d: all matrices of a batch need the same modulus and accumulator", k);
        dm[k] = mats[k]->A.dm;
        B->mte = std::max(B->mte, mats[k]->A.max_tile_entries);
        sig << "|" << mats[k]->info.nrows << "x" << mats[k]->info.nnz << "s" << s[k];
      }
      B->signature = sig.str();
      int dev = 0;
      FFX_HIP(hipGetDevice(&dev));
      FFX_HIP(hipDeviceGetAttribute(&B->ncu, hipDeviceAttributeMultiprocessorCount, dev));
      FFX_HIP(hipMalloc(&B->d_mats, sizeof(DevMat) * count));
      FFX_HIP(hipMemcpy(B->d_mats, dm.data(), sizeof(DevMat) * count, hipMemcpyHostToDevice));
      FFX_HIP(hipMalloc(&B->d_ops, sizeof(BatchOperand) * count));
      FFX_HIP(hipMalloc(&B->d_counter, NCLS * sizeof(uint32_t)));
      B->h_ops.resize(count);
      batch_items(B);
      (void)stream;
    } catch (...) {
      if (B->d_mats) (void)hipFree(B->d_mats);
      if (B->d_ops) (void)hipFree(B->d_ops);
      if (B->d_items) (void)hipFree(B->d_items);
      if (B->d_counter) (void)hipFree(B->d_counter);
      delete B;
      throw;
    }
    *out = B;
  });
}

ffx_status ffx_batch_spmm(ffx_batch B, const void* const* X, const int64_t* ldx, void* const* Y, const int64_t* ldy,
                          ffx_dtype dtype, void* stream) {
  return guard([&] {
    if (!B) fail(FFX_EINVAL, "batch is NULL");
    batch_run(B, X, ldx, Y, ldy, dtype, (hipStream_t)stream);
  });
}

ffx_status ffx_batch_get_params(ffx_batch B, ffx_batch_params* p) {
  return guard([&] {
    if (!B || !p) fail(FFX_EINVAL, "NULL argument");
    *p = B->params;
  });
}

ffx_status ffx_batch_set_params(ffx_batch B, const ffx_batch_params* p) {
  return guard([&] {
    if (!B || !p) fail(FFX_EINVAL, "NULL argument");
    check_params(*p);
    bool relist = p->order != B->params.order || p->max_chunk != B->params.max_chunk;
    B->params = *p;
    B->drop_graph();
    if (relist) batch_items(B);
  });
}

ffx_status ffx_batch_tune(ffx_batch B, const void* const* X, const int64_t* ldx, void* const* Y, const int64_t* ldy,
                          ffx_dtype dtype, int32_t reps, const char* cache_path, void* stream, ffx_batch_params* best) {
  return guard([&] {
    if (!B) fail(FFX_EINVAL, "batch is NULL");
    hipStream_t st = (hipStream_t)stream;
    const std::string key = device_name() + "|" + B->signature;
    ffx_batch_params p = B->params;
    if (cache_lookup(cache_path, key, p)) {
      check_params(p);
      bool relist = p.order != B->params.order || p.max_chunk != B->params.max_chunk;
      B->params.wg_per_cu = p.wg_per_cu;
      B->params.order = p.order;
      B->params.max_chunk = p.max_chunk;
      B->drop_graph();
      if (relist) batch_items(B);
      if (best) *best = B->params;
      return;
    }
    if (reps < 1) reps = 3;
    hipEvent_t e0, e1;
    FFX_HIP(hipEventCreate(&e0));
    FFX_HIP(hipEventCreate(&e1));
    float best_ms = 1e30f;
    ffx_batch_params bp = B->params;
    const int wpcs[] = {1, 2, 4, 8};
    for (int chunk : {8, 4})
      for (int order : {0, 1})
        for (int wpc : wpcs) {
          ffx_batch_params c{wpc, order, chunk, 0};
          bool relist = c.order != B->params.order || c.max_chunk != B->params.max_chunk;
          B->params = c;
          B->drop_graph();
          if (relist) batch_items(B);
          batch_run(B, X, ldx, Y, ldy, dtype, st);  // warm
          FFX_HIP(hipEventRecord(e0, st));
          for (int r = 0; r < reps; ++r) batch_run(B, X, ldx, Y, ldy, dtype, st);
          FFX_HIP(hipEventRecord(e1, st));
          FFX_HIP(hipEventSynchronize(e1));
          float ms = 0;
          FFX_HIP(hipEventElapsedTime(&ms, e0, e1));
          if (ms < best_ms) {
            best_ms = ms;
            bp = c;
          }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    bp.use_graph = 1;
    bool relist = bp.order != B->params.order || bp.max_chunk != B->params.max_chunk;
    B->params = bp;
    B->drop_graph();
    if (relist) batch_items(B);
    cache_store(cache_path, key, bp);
    if (best) *best = bp;
  });
}

ffx_status ffx_batch_destroy(ffx_batch B) {
  return guard([&] {
    if (!B) return;
    B->drop_graph();
    if (B->d_mats) (void)hipFree(B->d_mats);
    if (B->d_ops) (void)hipFree(B->d_ops);
    if (B->d_items) (void)hipFree(B->d_items);
    if (B->d_counter) (void)hipFree(B->d_counter);
    delete B;
  });
}

}  // extern "C"
