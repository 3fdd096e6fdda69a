// Batched products Y_k = A_k X_k over many matrices in one persistent launch.
//
// A work item is (matrix k, tile t, a group of at most 8 right-hand-side
// columns). Persistent workgroups take items from device counters in the
// order of lists sorted by decreasing estimated cost (longest-processing-
// time first), so large tiles start early and small ones fill the tail. The
// counters are cleared by a one-thread kernel before the launch (no memset),
// and the launches can be captured into a hipGraph and replayed.
//
// XCD-affine queues: MI355X has 8 XCDs, each with its own L2, and hands out
// consecutive workgroups to the XCDs in turn. With `xcd` set, the matrices are
// split over 8 queues by estimated cost (longest first, to the least loaded
// queue) and workgroup g works on queue g mod 8 first, so one matrix's X is
// gathered through one L2 instead of all eight; a workgroup whose queue is
// empty helps the others in turn. Results never depend on which workgroup
// takes an item.
//
// 16-bit X: for m <= 65536 every residue fits 16 bits; with `compact_x` the
// launch first copies each X_k to 16 bits (one kernel over the whole batch)
// and the tiles gather half the bytes (off by default: a row gather costs a
// cache line whatever its width, so the copy has not paid for itself).
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
  uint16_t* X16;   // 16-bit copy of X (leading dimension s), or null
  int64_t ncols;   // rows of X
  int32_t s, pad;
};

constexpr int NQ = 8;  // work queues per chunk class: one per XCD

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

// One class's items: queue q holds items [qfirst[q], qfirst[q] + qn[q]) of `items`; counter[q]
// hands them out. Every workgroup sweeps all NQ queues, its own first, until each is exhausted.
template <class AR, typename Tx, typename Tv, int SC>
__global__ __launch_bounds__(TILE_THREADS, batch_min_blocks<AR>()) void k_batch(const DevMat* __restrict__ mats,
                                                        const BatchOperand* __restrict__ ops,
                                                        const BatchItem* __restrict__ items,
                                                        const uint32_t* __restrict__ qinfo, uint32_t* counter) {
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ uint32_t next;
  const uint32_t home = blockIdx.x % NQ;
  for (uint32_t j = 0; j < NQ; ++j) {
    const uint32_t q = (home + j) % NQ;
    const uint32_t qf = qinfo[q], qn = qinfo[NQ + q];
    for (;;) {
      if (threadIdx.x == 0) next = atomicAdd(&counter[q], 1u);
      __syncthreads();
      const uint32_t it = next;
      __syncthreads();  // every lane has read `next` before thread 0 may overwrite it
      if (it >= qn) break;
      const BatchItem I = items[qf + it];
      const DevMat A = mats[I.k];
      const BatchOperand O = ops[I.k];
      const Tile T = A.tiles[I.t];
      const bool x16 = sizeof(Tx) == 2;
      const Tx* X = x16 ? (const Tx*)O.X16 + I.c0 : (const Tx*)O.X + I.c0;
      const int64_t ldx = x16 ? (int64_t)O.s : O.ldx;
      Tv* Y = (Tv*)O.Y + I.c0;
      const int sc = I.sc;
      const uint32_t kind = tile_kind(T.kind);
      if constexpr (SC == 1) {
        if (kind == TK_SELL) sell_tile<AR, Tx, Tv, 1, 2>(A, T, X, ldx, Y, O.ldy, 1, 1, 0);
        else if (kind == TK_LONG) long_tile<AR, Tx, Tv, 1, 2>(A, T, X, ldx, Y, O.ldy, 1, 1, 0, lds);
        else stream_tile_1<AR, Tx, Tv, 2>(A, T, X, ldx, Y, O.ldy, 1, 0, lds);
      } else {
        if (kind == TK_SELL) sell_tile_rc<AR, Tx, Tv, SC>(A, T, X, ldx, Y, O.ldy, sc, 1, 0);
        else if (kind == TK_LONG) long_tile<AR, Tx, Tv, SC, 1>(A, T, X, ldx, Y, O.ldy, sc, 1, 0, lds);
        else stream_tile_s<AR, Tx, Tv, SC>(A, T, X, ldx, Y, O.ldy, sc, 1, 0, lds);
      }
      __syncthreads();  // LDS is reused by the next item
    }
  }
}

// X16 of every operand with one: element e = row * s + c of X_k, row-major with leading dimension s.
// blockIdx.y is the matrix; blocks stride over its elements.
template <typename Tv>
__global__ void k_batch_x16(const BatchOperand* __restrict__ ops) {
  const BatchOperand O = ops[blockIdx.y];
  if (!O.X16) return;
  const int64_t total = O.ncols * O.s;
  const Tv* X = (const Tv*)O.X;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t first = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (O.ldx == O.s) {  // contiguous rows: a plain converting copy
    for (int64_t e = first; e < total; e += stride) O.X16[e] = (uint16_t)X[e];
    return;
  }
  // strided rows: walk (row, column) without dividing (a 64-bit division per element is slow)
  const int64_t s = O.s;
  int64_t row = first / s, c = first - row * s;
  const int64_t drow = stride / s, dc = stride - drow * s;
  for (int64_t e = first; e < total; e += stride) {
    O.X16[e] = (uint16_t)X[row * O.ldx + c];
    row += drow;
    c += dc;
    if (c >= s) {
      c -= s;
      ++row;
    }
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

// One class's persistent launch over its items (qinfo: the class's queue table, counter: its NQ counters).
static hipError_t batch_launch_class(int ak, ffx_dtype dt, bool x16, int cls, const DevMat* mats,
                                     const BatchOperand* ops, const BatchItem* items, const uint32_t* qinfo,
                                     uint32_t* counter, int grid, int64_t mte, hipStream_t st) {
  auto go = [&](auto ar) {
    using AR = decltype(ar);
    auto launch = [&](auto tx, auto tv, auto scv) {
      using Tx = decltype(tx);
      using Tv = decltype(tv);
      constexpr int SC = decltype(scv)::value;
      hipLaunchKernelGGL((k_batch<AR, Tx, Tv, SC>), dim3(grid), dim3(TILE_THREADS), batch_lds<AR>(mte, SC), st, mats,
                         ops, items, qinfo, counter);
    };
    auto by_dt = [&](auto scv) {
      // the 16-bit gathers are built for the integer class of m <= 65536 only
      if constexpr (std::is_same<AR, ArSmall>::value) {
        if (x16) {
          if (dt == FFX_I32) launch(uint16_t{}, int32_t{}, scv);
          else launch(uint16_t{}, int64_t{}, scv);
          return;
        }
      }
      if (dt == FFX_I32) launch(int32_t{}, int32_t{}, scv);
      else launch(int64_t{}, int64_t{}, scv);
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
  uint32_t* d_counter = nullptr;  // NQ per chunk class
  uint32_t* d_qinfo = nullptr;    // per chunk class: NQ queue starts, then NQ queue lengths (items of the class)
  uint16_t* d_x16 = nullptr;      // 16-bit copies of every X_k (compact_x)
  std::vector<int64_t> x16_off;   // element offset of each X_k's copy
  uint32_t nitems = 0;
  uint32_t cls_first[NCLS] = {0, 0, 0, 0}, cls_n[NCLS] = {0, 0, 0, 0};
  bool small = false;             // m <= 65536 on the integer class: 16-bit X is available
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
  std::vector<uint64_t> mcost(B->count, 0);
  for (int k = 0; k < B->count; ++k) {
    const auto& tc = matrix_tile_cost(*B->mats[k]);
    for (uint32_t t = 0; t < (uint32_t)tc.size(); ++t)
      for (int c0 = 0; c0 < B->s[k]; c0 += chunk) {
        int sc = std::min(chunk, B->s[k] - c0);
        items.push_back(BatchItem{(uint32_t)k, t, (uint16_t)c0, (uint16_t)sc, 0});
        cost.push_back((uint64_t)tc[t] * (uint64_t)(sc + 3));
        mcost[k] += cost.back();
      }
  }
  // queue of each matrix: all in queue 0, or (xcd) longest matrix first to the least loaded queue
  std::vector<int> mq(B->count, 0);
  if (B->params.xcd) {
    std::vector<int> order(B->count);
    for (int k = 0; k < B->count; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return mcost[a] > mcost[b]; });
    uint64_t load[NQ] = {0};
    for (int k : order) {
      int q = (int)(std::min_element(load, load + NQ) - load);
      mq[k] = q;
      load[q] += mcost[k];
    }
  }
  // by chunk class (each class is one kernel), then queue, then by decreasing cost when order == 0
  std::vector<size_t> idx(items.size());
  for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
  const bool by_cost = B->params.order == 0;
  std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) {
    int ca = chunk_class(items[a].sc), cb = chunk_class(items[b].sc);
    if (ca != cb) return ca < cb;
    int qa = mq[items[a].k], qb = mq[items[b].k];
    if (qa != qb) return qa < qb;
    return by_cost && cost[a] > cost[b];
  });
  std::vector<BatchItem> sorted(items.size());
  for (size_t i = 0; i < idx.size(); ++i) sorted[i] = items[idx[i]];
  items.swap(sorted);
  std::vector<uint32_t> qinfo(NCLS * 2 * NQ, 0);
  for (int c = 0; c < NCLS; ++c) B->cls_first[c] = B->cls_n[c] = 0;
  for (size_t i = 0; i < items.size(); ++i) {
    int c = chunk_class(items[i].sc);
    if (B->cls_n[c]++ == 0) B->cls_first[c] = (uint32_t)i;
  }
  for (size_t i = 0; i < items.size(); ++i) {  // queue starts relative to the class's first item
    int c = chunk_class(items[i].sc), q = mq[items[i].k];
    uint32_t* qi = &qinfo[c * 2 * NQ];
    if (qi[NQ + q]++ == 0) qi[q] = (uint32_t)i - B->cls_first[c];
  }
  if (B->d_items) (void)hipFree(B->d_items);
  B->d_items = nullptr;
  B->nitems = (uint32_t)items.size();
  FFX_HIP(hipMemcpy(B->d_qinfo, qinfo.data(), qinfo.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
  if (items.empty()) return;
  FFX_HIP(hipMalloc(&B->d_items, items.size() * sizeof(BatchItem)));
  FFX_HIP(hipMemcpy(B->d_items, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice));
}

static void check_params(const ffx_batch_params& p) {
  if (p.wg_per_cu < 0 || p.wg_per_cu > 8) fail(FFX_EINVAL, "wg_per_cu %d outside [0, 8]", p.wg_per_cu);
  if (p.order != 0 && p.order != 1) fail(FFX_EINVAL, "order %d", p.order);
  if (p.max_chunk != 4 && p.max_chunk != 8) fail(FFX_EINVAL, "max_chunk %d (4 or 8)", p.max_chunk);
  if (p.xcd != 0 && p.xcd != 1) fail(FFX_EINVAL, "xcd %d (0 or 1)", p.xcd);
  if (p.compact_x < -1 || p.compact_x > 1) fail(FFX_EINVAL, "compact_x %d (-1, 0 or 1)", p.compact_x);
}

// whether this batch's launches gather from 16-bit copies of X
static bool use_x16(const ffx_batch_s* B) { return B->small && B->params.compact_x == 1; }

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
  const bool x16 = use_x16(B);
  if (x16 && !B->d_x16) {
    int64_t total = 0;
    B->x16_off.assign(B->count, 0);
    for (int k = 0; k < B->count; ++k) {
      B->x16_off[k] = total;
      total += (B->mats[k]->info.ncols * B->s[k] + 127) / 128 * 128;  // 256-byte aligned copies
    }
    FFX_HIP(hipMalloc((void**)&B->d_x16, (size_t)std::max<int64_t>(total, 1) * 2));
  }
  for (int k = 0; k < B->count; ++k) {
    BatchOperand& o = B->h_ops[k];
    o.X16 = x16 ? B->d_x16 + B->x16_off[k] : nullptr;
    o.ncols = B->mats[k]->info.ncols;
    o.s = B->s[k];
  }
  // operand table: pageable host memory, so the copy is staged before the call returns
  FFX_HIP(hipMemcpyAsync(B->d_ops, B->h_ops.data(), B->h_ops.size() * sizeof(BatchOperand), hipMemcpyHostToDevice, st));
  const int wpc = B->params.wg_per_cu ? B->params.wg_per_cu : 4;
  auto grid_of = [&](int c) { return (int)std::min<int64_t>((int64_t)B->ncu * wpc, B->cls_n[c]); };
  auto launch_class = [&](int c, hipStream_t s) {
    return batch_launch_class(B->ak, dt, x16, c, B->d_mats, B->d_ops, B->d_items + B->cls_first[c],
                              B->d_qinfo + c * 2 * NQ, B->d_counter + c * NQ, grid_of(c), B->mte, s);
  };
  auto launch_x16 = [&](hipStream_t s) -> hipError_t {
    if (!x16) return hipSuccess;
    if (dt == FFX_I32) hipLaunchKernelGGL(k_batch_x16<int32_t>, dim3(64, B->count), dim3(256), 0, s, B->d_ops);
    else hipLaunchKernelGGL(k_batch_x16<int64_t>, dim3(64, B->count), dim3(256), 0, s, B->d_ops);
    return hipGetLastError();
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
        hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, cs, B->d_counter, NCLS * NQ);
        hipError_t le = launch_x16(cs);
        if (le == hipSuccess) le = hipEventRecord(ev0, cs);
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
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, st, B->d_counter, NCLS * NQ);
  FFX_HIP(launch_x16(st));
  for (int c = 0; c < NCLS; ++c)
    if (B->cls_n[c]) FFX_HIP(launch_class(c, st));
}


static std::string device_name() {
  int dev = 0;
  hipDeviceProp_t p;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
  return std::string(p.gcnArchName) + ":" + std::to_string(p.multiProcessorCount);
}

// tiny JSON cache: one line per entry, "key": {"wg_per_cu": a, "order": b, "max_chunk": c, "xcd": d,
// "compact_x": e}
static bool cache_lookup(const char* path, const std::string& key, ffx_batch_params& p) {
  if (!path) return false;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    size_t q = line.find("\"" + key + "\"");
    if (q == std::string::npos) continue;
    int a, b, c, d, e;
    const char* s = line.c_str() + q + key.size() + 2;
    if (sscanf(s, " : {\"wg_per_cu\": %d, \"order\": %d, \"max_chunk\": %d, \"xcd\": %d, \"compact_x\": %d", &a, &b, &c,
               &d, &e) == 5) {
      p.wg_per_cu = a;
      p.order = b;
      p.max_chunk = c;
      p.xcd = d;
      p.compact_x = e;
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
  // the key can be long (one term per matrix): the line is built without a fixed-size buffer
  char buf[160];
  snprintf(buf, sizeof buf, "{\"wg_per_cu\": %d, \"order\": %d, \"max_chunk\": %d, \"xcd\": %d, \"compact_x\": %d}",
           p.wg_per_cu, p.order, p.max_chunk, p.xcd, p.compact_x);
  lines.push_back("  \"" + key + "\": " + buf);
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
      B->params = ffx_batch_params{0, 0, 8, 1, 1, -1};
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
      FFX_HIP(hipMalloc(&B->d_counter, NCLS * NQ * sizeof(uint32_t)));
      FFX_HIP(hipMalloc(&B->d_qinfo, NCLS * 2 * NQ * sizeof(uint32_t)));
      B->small = B->ak == AK_SMALL;
      B->h_ops.resize(count);
      batch_items(B);
      (void)stream;
    } catch (...) {
      if (B->d_mats) (void)hipFree(B->d_mats);
      if (B->d_ops) (void)hipFree(B->d_ops);
      if (B->d_items) (void)hipFree(B->d_items);
      if (B->d_counter) (void)hipFree(B->d_counter);
      if (B->d_qinfo) (void)hipFree(B->d_qinfo);
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
    bool relist = p->order != B->params.order || p->max_chunk != B->params.max_chunk || p->xcd != B->params.xcd;
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
    auto apply = [&](const ffx_batch_params& c) {
      bool relist = c.order != B->params.order || c.max_chunk != B->params.max_chunk || c.xcd != B->params.xcd;
      B->params = c;
      B->drop_graph();
      if (relist) batch_items(B);
    };
    if (cache_lookup(cache_path, key, p)) {
      check_params(p);
      p.use_graph = B->params.use_graph;
      apply(p);
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
    const int x16s[] = {0, 1};
    for (int x16 : x16s) {
      if (x16 && !B->small) continue;
      for (int xcd : {1, 0})
        for (int chunk : {8, 4})
          for (int order : {0, 1})
            for (int wpc : wpcs) {
              ffx_batch_params c{wpc, order, chunk, 0, xcd, x16};
              apply(c);
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
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    bp.use_graph = 1;
    apply(bp);
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
    if (B->d_qinfo) (void)hipFree(B->d_qinfo);
    if (B->d_x16) (void)hipFree(B->d_x16);
    delete B;
  });
}

}  // extern "C"
