// The C ABI: argument checks, matrix construction and product dispatch.
#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "host.h"
#include "launch.h"

namespace ffx {

static thread_local std::string g_last_error;

void set_last_error(const std::string& s) { g_last_error = s; }

void fail(ffx_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  throw Error{st, buf};
}

// iterations per hipGraph replay of ffx_sequence (0: direct launches)
static std::atomic<int> g_seq_graph_batch{64};

static int arith_kind(const ffx_matrix_s& M) {
  bool small = M.md.small();
  if (M.acc == FFX_ACC_FP64) {
    if (small) return M.chunk ? AK_F64_16_CH : AK_F64_16;
    return M.chunk ? AK_F64_32_CH : AK_F64_32;
  }
  if (M.acc == FFX_ACC_FP64_CENTERED) {
    if (small) return M.chunk ? AK_F64C_16_CH : AK_F64C_16;
    return M.chunk ? AK_F64C_32_CH : AK_F64C_32;
  }
  if (M.acc == FFX_ACC_FP32) return M.chunk ? AK_F32_CH : AK_F32;
  if (M.acc == FFX_ACC_FP32_CENTERED) return M.chunk ? AK_F32C_CH : AK_F32C;
  if (small) return AK_SMALL;
  if (M.md.m == 2147483647u) return AK_M31;
  return M.chunk ? AK_BIG_CH : AK_BIG;
}

// Integer class of the sequence, whatever the product path of the matrix. The
// projection U^T W adds products of two residues over many rows, so for m >
// 65536 it always needs the reductions of the chunked class (or the folding
// class of 2^31 - 1), even where no matrix row does.
static bool only_sell(const Encoded& E) { return E.kind_tiles[0] == 0 && E.kind_tiles[1] == 0; }

static int seq_kind(const ffx_matrix_s& M) {
  if (M.md.small()) return AK_SMALL;
  if (M.md.m == 2147483647u) return AK_M31;
  return AK_BIG_CH;
}

int matrix_arith_kind(const ffx_matrix_s& M) { return arith_kind(M); }
const std::vector<uint32_t>& matrix_tile_cost(const ffx_matrix_s& M) { return M.A.tile_cost; }

static PlanOpts plan_opts(const ffx_build_opts* o) {
  ffx_build_opts d;
  ffx_build_opts_default(&d);
  if (o) {
    if (o->size < sizeof(uint32_t) || o->size > sizeof(ffx_build_opts))
      fail(FFX_EINVAL, "ffx_build_opts.size = %u (expected %zu)", o->size, sizeof(ffx_build_opts));
    std::memcpy(&d, o, o->size);
    d.size = sizeof(ffx_build_opts);
  }
  PlanOpts p;
  if (d.acc < FFX_ACC_AUTO || d.acc > FFX_ACC_FP32_CENTERED) fail(FFX_EINVAL, "accumulator %d", d.acc);
  p.acc = d.acc == FFX_ACC_AUTO ? FFX_ACC_INT64 : d.acc;
  if (d.selector < FFX_SEL_HEURISTIC || d.selector > FFX_SEL_FIXED) fail(FFX_EINVAL, "selector %d", d.selector);
  p.selector = d.selector;
  if (d.selector == FFX_SEL_FIXED && (d.fixed_format < 0 || d.fixed_format >= FFX_NUM_FORMATS))
    fail(FFX_EINVAL, "fixed format %d", d.fixed_format);
  p.fixed_format = d.fixed_format;
  p.split_pm1 = d.split_pm1 != 0;
  if (d.block_rows < 64 || d.block_rows > 65536 || d.block_rows % 64)
    fail(FFX_EINVAL, "block_rows %d is not a multiple of 64 in [64, 65536]", d.block_rows);
  p.block_rows = d.block_rows;
  int te = d.tile_entries ? d.tile_entries : 2048;
  if (te < 256 || te > 4096) fail(FFX_EINVAL, "tile_entries %d outside [256, 4096]", te);
  p.tile_entries = te;
  if (d.compact_x < -1 || d.compact_x > 1) fail(FFX_EINVAL, "compact_x %d not in {-1, 0, 1}", d.compact_x);
  p.compact_x = d.compact_x;
  if (d.model_path) p.model_path = d.model_path;
  if (d.reorder < 0 || d.reorder > 1) fail(FFX_EINVAL, "reorder %d not in {0, 1}", d.reorder);
  p.reorder = d.reorder != 0;
  if (d.col_sorted < -1 || d.col_sorted > 1) fail(FFX_EINVAL, "col_sorted %d not in {-1, 0, 1}", d.col_sorted);
  p.col_sorted = d.col_sorted;
  return p;
}

// Keeps freed stream-ordered allocations in the device pool, so the per-call
// workspaces of products do not return to the driver between calls.
static void warm_pool(hipStream_t st) {
  static std::once_flag once;
  std::call_once(once, [&] {
    int dev = 0;
    hipMemPool_t pool;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
      uint64_t thr = UINT64_MAX;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
  });
  (void)st;
}

// Delayed-reduction bound (Section 2.2): the number of terms that can be
// added to a reduced accumulator while every partial sum stays exact.
// Canonical operands lie in [0, m-1]: a term is at most (m-1)^2 (or m, the
// term m - 0 of an entry of residue m-1), a reduced accumulator at most m-1,
// and sums must stay at most 2^63 - 1 (int64) or 2^p - 1 (p = 53 for doubles,
// 24 for floats: every integer up to 2^p is exact). Centered operands lie in
// [-h, h], h = floor(m/2): a term is at most h^2 in magnitude and sums of both
// signs stay exact while their magnitude is at most 2^p - 1. Partial sums of
// up to 257 reduced lanes also meet before the final reduction; the bound
// covers them whenever it is at least 1 (257 * rmax <= rmax + tmax for rmax
// >= 256, and 257 * 255 < 2^24 otherwise).
static int64_t reduce_bound(int acc, uint32_t m) {
  const bool centered = acc == FFX_ACC_FP64_CENTERED || acc == FFX_ACC_FP32_CENTERED;
  const uint64_t rmax = centered ? m >> 1 : (uint64_t)m - 1;
  const uint64_t tmax = std::max<uint64_t>(rmax * rmax, centered ? rmax : m);
  uint64_t limit = (uint64_t)INT64_MAX;
  if (acc == FFX_ACC_FP64 || acc == FFX_ACC_FP64_CENTERED) limit = ((uint64_t)1 << 53) - 1;
  if (acc == FFX_ACC_FP32 || acc == FFX_ACC_FP32_CENTERED) limit = ((uint64_t)1 << 24) - 1;
  return terms_before_reduce(limit, rmax, tmax);
}

static const char* acc_name(int acc) {
  switch (acc) {
    case FFX_ACC_INT64: return "INT64";
    case FFX_ACC_FP64: return "FP64";
    case FFX_ACC_FP32: return "FP32";
    case FFX_ACC_FP64_CENTERED: return "centered FP64";
    default: return "centered FP32";
  }
}

static ffx_matrix_s* build(const RCsr& A, uint32_t m, const ffx_build_opts* opts, int build_t, hipStream_t st) {
  PlanOpts po = plan_opts(opts);
  ffx_matrix_s* M = new ffx_matrix_s();
  try {
    M->md = make_modulus(m);
    M->acc = po.acc;
    const int64_t b = reduce_bound(po.acc, m);
    if (b < 1)
      fail(FFX_EBOUND, "the %s accumulator cannot hold one product of residues modulo %u exactly",
           acc_name(po.acc), m);
    // reordering (Section 4, the conclusion): the handle stores B = P A P^T and keeps perm
    RCsr B;
    if (po.reorder) {
      if (A.nrows != A.ncols)
        fail(FFX_EINVAL, "reordering needs a square matrix (%lld x %lld)", (long long)A.nrows, (long long)A.ncols);
      std::vector<uint32_t> perm = rcm_order(A);
      B = permute_sym(A, perm);
      if (A.nrows > 0) {
        FFX_HIP(hipMalloc((void**)&M->perm, perm.size() * sizeof(uint32_t)));
        FFX_HIP(hipMemcpy(M->perm, perm.data(), perm.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
      }
    }
    const RCsr& S = po.reorder ? B : A;
    encode(S, M->md, po, st, &M->A);
    int64_t maxterms = M->A.max_row_terms;
    if (build_t) {
      RCsr T = transpose(S);
      encode(T, M->md, po, st, &M->AT);
      M->has_t = true;
      maxterms = std::max(maxterms, M->AT.max_row_terms);
    } else {
      // the scatter form of A^T sums one column per output: bound by the longest column
      std::vector<int64_t> cnt(S.ncols, 0);
      for (uint32_t c : S.col) cnt[c]++;
      for (int64_t v : cnt) maxterms = std::max(maxterms, v);
    }
    M->chunk = maxterms > b;
    M->compact_x = M->md.small() && (po.compact_x == 1 || (po.compact_x == -1 && A.ncols * 4 > (1 << 20)));
    // column-sorted groups for one-vector products: integer sums of terms below 2^32
    const bool sg_ok = M->md.small() && M->acc == FFX_ACC_INT64 && S.nrows > 0;
    const bool sg_auto = S.nnz() >= ((int64_t)1 << 22) && S.ncols >= ((int64_t)1 << 18);
    if (sg_ok && (po.col_sorted == 1 || (po.col_sorted == -1 && sg_auto))) {
      int dev = 0, ncu = 0;
      FFX_HIP(hipGetDevice(&dev));
      FFX_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
      encode_sg(S, M->md, po.split_pm1, ncu, st, &M->sg);
      M->sg.dm.rowmap = M->perm;
    }
    M->A.dm.reduce_every = b;
    M->AT.dm.reduce_every = b;
    ffx_matrix_info& I = M->info;
    I.nrows = A.nrows;
    I.ncols = A.ncols;
    I.m = m;
    I.acc = M->acc;
    I.nnz = M->A.nnz;
    I.n_plus = M->A.n_plus;
    I.n_minus = M->A.n_minus;
    I.n_band = M->A.n_band;
    I.nblocks = (int64_t)M->A.block_fmt.size();
    I.ntiles = M->A.ntiles;
    I.max_row_terms = maxterms;
    I.reduce_every = b;
    I.device_bytes = M->A.device_bytes + (M->has_t ? M->AT.device_bytes : 0);
    I.stream_bytes = M->A.stream_bytes;
    I.has_transpose = M->has_t;
    I.value_bytes = M->md.small() ? 2 : 4;
    for (int f = 0; f < FFX_NUM_FORMATS; ++f) I.format_blocks[f] = M->A.format_blocks[f];
    I.reordered = po.reorder;
    I.bandwidth_input = bandwidth(A);
    I.bandwidth_stored = po.reorder ? bandwidth(B) : I.bandwidth_input;
    I.device_bytes += po.reorder ? A.nrows * (int64_t)sizeof(uint32_t) : 0;
    I.sg_groups = M->sg.ngroups;
    I.sg_stream_bytes = M->sg.stream_bytes;
    I.device_bytes += M->sg.device_bytes;
  } catch (...) {
    M->A.release();
    M->AT.release();
    M->sg.release();
    if (M->perm) (void)hipFree(M->perm);
    delete M;
    throw;
  }
  return M;
}

static size_t esize(ffx_dtype dt) { return dt == FFX_I32 ? 4 : 8; }

static void check_dtype(ffx_dtype dt) {
  if (dt != FFX_I32 && dt != FFX_I64) fail(FFX_EINVAL, "dtype %d is neither FFX_I32 nor FFX_I64", (int)dt);
}

// byte range [lo, hi) covered by an n x s block with leading dimension ld
static void span(const void* p, int64_t n, int s, int64_t ld, ffx_dtype dt, uintptr_t& lo, uintptr_t& hi) {
  lo = (uintptr_t)p;
  hi = n > 0 ? lo + (uintptr_t)(((n - 1) * ld + s) * (int64_t)esize(dt)) : lo;
}

static void check_block(const char* what, const void* p, int64_t n, int s, int64_t ld) {
  if (ld < s) fail(FFX_EINVAL, "%s: leading dimension %lld < s = %d", what, (long long)ld, s);
  if (n > 0 && !p) fail(FFX_EINVAL, "%s is NULL", what);
}

static void check_disjoint(const char* a, const void* pa, int64_t na, int64_t lda, const char* b, const void* pb,
                           int64_t nb, int64_t ldb, int s, ffx_dtype dt) {
  uintptr_t a0, a1, b0, b1;
  span(pa, na, s, lda, dt, a0, a1);
  span(pb, nb, s, ldb, dt, b0, b1);
  if (a0 < b1 && b0 < a1) fail(FFX_EINVAL, "%s and %s overlap", a, b);
}


// For a reordered handle: gathers the caller's n x s block X (and Y when
// y_in) into compact copies in the stored order, runs f(xp, yp), which leaves
// its result in yp, and scatters yp back into Y.
template <class F>
static void permuted(const ffx_matrix_s& M, int64_t n, int s, size_t esz, const void* X, int64_t ldx, void* Y,
                     int64_t ldy, bool y_in, hipStream_t st, F&& f) {
  warm_pool(st);
  void* buf[2] = {nullptr, nullptr};
  const size_t bytes = (size_t)n * s * esz;
  for (int q = 0; q < 2; ++q)
    if (hipMallocAsync(&buf[q], bytes, st) != hipSuccess) {
      for (void* p : buf) if (p) (void)hipFreeAsync(p, st);
      fail(FFX_ENOMEM, "hipMallocAsync of %zu bytes failed", bytes);
    }
  hipError_t e = launch_permute_rows(esz, X, ldx, buf[0], s, M.perm, n, s, false, st);
  if (e == hipSuccess && y_in) e = launch_permute_rows(esz, Y, ldy, buf[1], s, M.perm, n, s, false, st);
  if (e == hipSuccess) {
    try {
      f(buf[0], buf[1]);
    } catch (...) {
      for (void* p : buf) (void)hipFreeAsync(p, st);
      throw;
    }
    e = launch_permute_rows(esz, buf[1], s, Y, ldy, M.perm, n, s, true, st);
  }
  for (void* p : buf) (void)hipFreeAsync(p, st);
  FFX_HIP(e);
}

// Checks the arguments of a product; returns false when there is nothing to compute.
static bool check_product(ffx_matrix M, bool trans, int s, uint32_t alpha, const void* X, int64_t ldx,
                          uint32_t beta, const void* Y, int64_t ldy, ffx_dtype dt) {
  if (!M) fail(FFX_EINVAL, "matrix handle is NULL");
  check_dtype(dt);
  if (s < 1 || s > MAX_S) fail(FFX_EINVAL, "s = %d outside [1, %d]", s, MAX_S);
  if (alpha >= M->md.m || beta >= M->md.m) fail(FFX_EINVAL, "alpha or beta not in [0, m-1]");
  const int64_t nin = trans ? M->info.nrows : M->info.ncols;
  const int64_t nout = trans ? M->info.ncols : M->info.nrows;
  check_block("x", X, nin, s, ldx);
  check_block("y", Y, nout, s, ldy);
  check_disjoint("x", X, nin, ldx, "y", Y, nout, ldy, s, dt);
  return nout > 0;
}

// A row product runs the tiles of an encoded operator: A, or the stored A^T.
// The other transposed product scatters the entries of A.
static bool row_product(const ffx_matrix_s& M, bool trans) { return !trans || M.has_t; }

// Device bytes of the temporary a row product with s vectors needs: the
// 16-bit copy of x (one vector, m <= 65536, compact_x), or x gathered into the
// stored order of a reordered handle (into that 16-bit copy when there is one).
static size_t row_scratch_bytes(const ffx_matrix_s& M, bool trans, int s, ffx_dtype dt) {
  const int64_t nin = trans ? M.info.nrows : M.info.ncols;
  const bool c16 = s == 1 && M.compact_x;
  if (nin == 0) return 0;
  if (c16) return (size_t)nin * 2;
  return M.perm ? (size_t)nin * s * esize(dt) : 0;
}

// The row product with its temporary in `scratch` (row_scratch_bytes of device
// memory, or null when that is 0). Allocates nothing.
static hipError_t row_product_in(const ffx_matrix_s& M, bool trans, int s, uint32_t alpha, const void* X,
                                 int64_t ldx, uint32_t beta, void* Y, int64_t ldy, ffx_dtype dt, hipStream_t st,
                                 void* scratch) {
  const Encoded& E = trans ? M.AT : M.A;
  const int64_t nin = trans ? M.info.nrows : M.info.ncols;
  const int ak = arith_kind(M);
  const bool c16 = s == 1 && M.compact_x && nin > 0;
  if (!trans && s == 1 && M.sg.ngroups) {
    // column-sorted groups: x (its 16-bit copy when the product takes one) in the stored order, and
    // y written through the row map of a reordered handle (set in the groups' descriptor)
    const void* xs = X;
    if (M.perm) {
      hipError_t e = c16 ? launch_permute_to_u16(dt, X, ldx, (uint16_t*)scratch, M.perm, nin, st)
                         : launch_permute_rows(esize(dt), X, ldx, scratch, 1, M.perm, nin, 1, false, st);
      if (e != hipSuccess) return e;
      xs = scratch;
    } else if (c16) {
      hipError_t e = launch_compact_x(dt, X, ldx, (uint16_t*)scratch, nin, st);
      if (e != hipSuccess) return e;
    }
    return launch_sg(M.sg.dm, dt, xs, c16 ? (const uint16_t*)scratch : nullptr, Y, alpha, beta, st);
  }
  DevMat dm = E.dm;
  if (M.perm) {
    // stored as P A P^T: gather x into the stored order (into the 16-bit copy when the product takes
    // one) and let the tiles write each row of y to its caller's row
    dm.rowmap = M.perm;
    hipError_t e = c16 ? launch_permute_to_u16(dt, X, ldx, (uint16_t*)scratch, M.perm, nin, st)
                       : launch_permute_rows(esize(dt), X, ldx, scratch, s, M.perm, nin, s, false, st);
    if (e != hipSuccess) return e;
    return launch_tiles(ak, dm, E.max_tile_entries, dt, c16 ? nullptr : scratch, s, Y, ldy, s, alpha, beta, st,
                        c16 ? (const uint16_t*)scratch : nullptr);
  }
  if (c16) {
    hipError_t e = launch_compact_x(dt, X, ldx, (uint16_t*)scratch, nin, st);
    if (e != hipSuccess) return e;
    return launch_tiles(ak, dm, E.max_tile_entries, dt, X, ldx, Y, ldy, s, alpha, beta, st,
                        (const uint16_t*)scratch);
  }
  return launch_tiles(ak, dm, E.max_tile_entries, dt, X, ldx, Y, ldy, s, alpha, beta, st);
}

// The temporary of ffx_spmv_noalloc: a static device array, one copy per GPU.
// Host code never passes its name to a kernel (that is a host-side stand-in);
// it takes the device address from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char noalloc_scratch[FFX_NOALLOC_SCRATCH_BYTES];
constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_noalloc_mu;
static void* g_noalloc_ptr[NOALLOC_MAX_DEVICES];

// Device address of the current device's copy of noalloc_scratch.
static void* noalloc_scratch_ptr() {
  int dev = 0;
  FFX_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) fail(FFX_EUNSUPPORTED, "device ordinal %d", dev);
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
    if (e != hipSuccess || !p)
      fail(FFX_EDEVICE, "hipGetSymbolAddress of the static scratch failed: %s", hipGetErrorString(e));
    g_noalloc_ptr[dev] = p;
  }
  return g_noalloc_ptr[dev];
}

static void product(ffx_matrix M, bool trans, int s, uint32_t alpha, const void* X, int64_t ldx, uint32_t beta,
                    void* Y, int64_t ldy, ffx_dtype dt, hipStream_t st) {
  if (!check_product(M, trans, s, alpha, X, ldx, beta, Y, ldy, dt)) return;
  const int64_t nin = trans ? M->info.nrows : M->info.ncols;
  const int64_t nout = trans ? M->info.ncols : M->info.nrows;
  if (row_product(*M, trans)) {
    const size_t bytes = row_scratch_bytes(*M, trans, s, dt);
    if (!bytes) {
      FFX_HIP(row_product_in(*M, trans, s, alpha, X, ldx, beta, Y, ldy, dt, st, nullptr));
      return;
    }
    auto& C = M->scr;
    std::lock_guard<std::mutex> lock(C.mu);
    if (C.bytes < bytes) {  // grow: the previous temporary is freed once every product is done
      if (C.p) {
        FFX_HIP(hipDeviceSynchronize());
        (void)hipFree(C.p);
        C.p = nullptr;
        C.bytes = 0;
      }
      if (hipMalloc(&C.p, bytes) != hipSuccess) fail(FFX_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
      C.bytes = bytes;
    } else if (C.used && C.last != st) {
      if (!C.multi) {  // the products so far recorded nothing: wait for all of them, once
        FFX_HIP(hipDeviceSynchronize());
        FFX_HIP(hipEventCreateWithFlags(&C.done, hipEventDisableTiming));
        C.multi = true;
      } else {
        FFX_HIP(hipStreamWaitEvent(st, C.done, 0));
      }
    }
    hipError_t e = row_product_in(*M, trans, s, alpha, X, ldx, beta, Y, ldy, dt, st, C.p);
    if (e == hipSuccess && C.multi) e = hipEventRecord(C.done, st);
    C.last = st;
    C.used = true;
    FFX_HIP(e);
    return;
  }
  // the scatter form of A^T, with 64-bit integer atomics into a temporary
  auto scatter = [&](const void* xs, int64_t ldxs, void* ys, int64_t ldys) {
    warm_pool(st);
    unsigned long long* acc = nullptr;
    size_t bytes = (size_t)nout * s * sizeof(uint64_t);
    if (hipMallocAsync((void**)&acc, bytes, st) != hipSuccess) fail(FFX_ENOMEM, "hipMallocAsync of %zu bytes", bytes);
    hipError_t e = launch_transpose_scatter(M->md.small(), M->A.dm, dt, xs, ldxs, ys, ldys, s, alpha, beta, acc, st);
    (void)hipFreeAsync(acc, st);
    FFX_HIP(e);
  };
  if (M->perm) {  // gather x (and y when beta != 0) into the stored order, scatter y back
    permuted(*M, nin, s, esize(dt), X, ldx, Y, ldy, beta != 0, st,
             [&](void* xp, void* yp) { scatter(xp, s, yp, s); });
    return;
  }
  scatter(X, ldx, Y, ldy);
}

// W = A^k V for k >= 1 on the stored operator; the last product writes its
// row r to row rowmap[r] of W when rowmap is not null.
static void power_iter(const ffx_matrix_s& M, int64_t k, int s, const void* V, int64_t ldv, void* W, int64_t ldw,
                       ffx_dtype dtype, hipStream_t st, const uint32_t* rowmap) {
  {
    const int64_t n = M.info.nrows;
    const int ak = arith_kind(M);
    const Encoded& E = M.A;
    void* tmp[2] = {nullptr, nullptr};
    size_t bytes = (size_t)n * s * esize(dtype);
    if (k >= 2) {
      for (int q = 0; q < (k >= 3 ? 2 : 1); ++q)
        if (hipMallocAsync(&tmp[q], bytes, st) != hipSuccess) {
          for (void* p : tmp) if (p) (void)hipFreeAsync(p, st);
          fail(FFX_ENOMEM, "hipMallocAsync of %zu bytes failed", bytes);
        }
    }
    // one vector on a handle with column-sorted groups: every product on the groups (through a
    // 16-bit copy of the current vector when the handle takes one); they write y with unit stride
    // Each product but the last also writes its result as the next one's 16-bit x (two buffers in turn),
    // so only V is copied to 16 bits.
    const bool sg = s == 1 && M.sg.ngroups && ldw == 1;
    uint16_t* x16[2] = {nullptr, nullptr};
    if (sg && M.compact_x && n > 0) {
      for (int q = 0; q < (k >= 2 ? 2 : 1); ++q)
        if (hipMallocAsync((void**)&x16[q], (size_t)n * 2, st) != hipSuccess) {
          for (void* p : tmp) if (p) (void)hipFreeAsync(p, st);
          for (void* p : x16) if (p) (void)hipFreeAsync(p, st);
          fail(FFX_ENOMEM, "hipMallocAsync of %zu bytes failed", (size_t)n * 2);
        }
    }
    const void* cur = V;
    int64_t ldc = ldv;
    hipError_t e = hipSuccess;
    for (int64_t it = 0; it < k && e == hipSuccess; ++it) {
      bool last = it == k - 1;
      void* dst = last ? W : tmp[it & 1];
      int64_t ldd = last ? ldw : s;
      if (sg && (x16[0] || ldc == 1)) {
        SgMat g = M.sg.dm;
        g.rowmap = last ? rowmap : nullptr;
        uint16_t* xin = x16[it & 1];
        if (xin && it == 0) e = launch_compact_x(dtype, cur, ldc, xin, n, st);
        if (e == hipSuccess) e = launch_sg(g, dtype, cur, xin, dst, 1, 0, st, last ? nullptr : x16[(it + 1) & 1]);
      } else {
        DevMat dm = E.dm;
        if (last) dm.rowmap = rowmap;
        e = launch_tiles(ak, dm, E.max_tile_entries, dtype, cur, ldc, dst, ldd, s, 1, 0, st);
      }
      cur = dst;
      ldc = ldd;
    }
    for (void* p : tmp) if (p) (void)hipFreeAsync(p, st);
    for (void* p : x16) if (p) (void)hipFreeAsync(p, st);
    FFX_HIP(e);
  }
}

}  // namespace ffx

using namespace ffx;

extern "C" {

void ffx_build_opts_default(ffx_build_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->size = sizeof *o;
  o->acc = FFX_ACC_AUTO;
  o->selector = FFX_SEL_HEURISTIC;
  o->fixed_format = FFX_FMT_STREAM;
  o->split_pm1 = 1;
  o->block_rows = 4096;
  o->build_transpose = 0;
  o->tile_entries = 0;
  o->compact_x = -1;
  o->model_path = nullptr;
  o->reorder = 0;
  o->col_sorted = -1;
}

ffx_status ffx_matrix_create_csr(int64_t nrows, int64_t ncols, const int64_t* rowptr, const int32_t* colidx,
                                 const void* vals, ffx_dtype val_type, uint32_t m, const ffx_build_opts* opts,
                                 void* stream, ffx_matrix* out) {
  return guard([&] {
    if (!out) fail(FFX_EINVAL, "out is NULL");
    *out = nullptr;
    RCsr A = reduce_csr(nrows, ncols, rowptr, colidx, vals, val_type, m);
    A.nrows = nrows;
    int bt = opts && opts->size >= offsetof(ffx_build_opts, build_transpose) + sizeof(int32_t) ? opts->build_transpose : 0;
    ffx_matrix M = build(A, m, opts, bt, (hipStream_t)stream);
    M->info.nnz_input = rowptr ? rowptr[nrows] : 0;
    *out = M;
  });
}

ffx_status ffx_matrix_create_coo(int64_t nrows, int64_t ncols, int64_t nnz, const int32_t* rowidx,
                                 const int32_t* colidx, const void* vals, ffx_dtype val_type, uint32_t m,
                                 const ffx_build_opts* opts, void* stream, ffx_matrix* out) {
  return guard([&] {
    if (!out) fail(FFX_EINVAL, "out is NULL");
    *out = nullptr;
    RCsr A = reduce_coo(nrows, ncols, nnz, rowidx, colidx, vals, val_type, m);
    int bt = opts && opts->size >= offsetof(ffx_build_opts, build_transpose) + sizeof(int32_t) ? opts->build_transpose : 0;
    ffx_matrix M = build(A, m, opts, bt, (hipStream_t)stream);
    M->info.nnz_input = nnz;
    *out = M;
  });
}

ffx_status ffx_matrix_info_get(ffx_matrix A, ffx_matrix_info* info) {
  return guard([&] {
    if (!A || !info) fail(FFX_EINVAL, "NULL argument");
    *info = A->info;
  });
}

ffx_status ffx_matrix_block_formats(ffx_matrix A, int32_t transpose, int32_t* out, int64_t cap) {
  return guard([&] {
    if (!A || (cap > 0 && !out)) fail(FFX_EINVAL, "NULL argument");
    if (transpose && !A->has_t) fail(FFX_EINVAL, "the handle holds no A^T");
    const auto& f = transpose ? A->AT.block_fmt : A->A.block_fmt;
    int64_t n = std::min<int64_t>(cap, (int64_t)f.size());
    for (int64_t i = 0; i < n; ++i) out[i] = f[i];
  });
}

ffx_status ffx_matrix_destroy(ffx_matrix A) {
  return guard([&] {
    if (!A) return;
    if (A->scr.p) {  // every product that used the temporary is done before it is freed
      (void)hipDeviceSynchronize();
      (void)hipFree(A->scr.p);
    }
    if (A->scr.done) (void)hipEventDestroy(A->scr.done);
    A->A.release();
    A->AT.release();
    A->sg.release();
    if (A->perm) (void)hipFree(A->perm);
    delete A;
  });
}

ffx_status ffx_spmv(ffx_matrix A, uint32_t alpha, const void* x, uint32_t beta, void* y, ffx_dtype dtype,
                    void* stream) {
  return guard([&] { product(A, false, 1, alpha, x, 1, beta, y, 1, dtype, (hipStream_t)stream); });
}

ffx_status ffx_spmv_noalloc(ffx_matrix A, uint32_t alpha, const void* x, uint32_t beta, void* y, ffx_dtype dtype,
                            void* stream) {
  return guard([&] {
    if (!check_product(A, false, 1, alpha, x, 1, beta, y, 1, dtype)) return;
    const size_t bytes = row_scratch_bytes(*A, false, 1, dtype);
    if (bytes > (size_t)FFX_NOALLOC_SCRATCH_BYTES)
      fail(FFX_EINVAL, "this product needs %zu bytes of temporary; the static scratch holds %zu", bytes,
           (size_t)FFX_NOALLOC_SCRATCH_BYTES);
    void* tmp = bytes ? noalloc_scratch_ptr() : nullptr;
    FFX_HIP(row_product_in(*A, false, 1, alpha, x, 1, beta, y, 1, dtype, (hipStream_t)stream, tmp));
  });
}

ffx_status ffx_spmv_t(ffx_matrix A, uint32_t alpha, const void* x, uint32_t beta, void* y, ffx_dtype dtype,
                      void* stream) {
  return guard([&] { product(A, true, 1, alpha, x, 1, beta, y, 1, dtype, (hipStream_t)stream); });
}

ffx_status ffx_spmm(ffx_matrix A, int32_t s, uint32_t alpha, const void* X, int64_t ldx, uint32_t beta, void* Y,
                    int64_t ldy, ffx_dtype dtype, void* stream) {
  return guard([&] { product(A, false, s, alpha, X, ldx, beta, Y, ldy, dtype, (hipStream_t)stream); });
}

ffx_status ffx_spmm_t(ffx_matrix A, int32_t s, uint32_t alpha, const void* X, int64_t ldx, uint32_t beta, void* Y,
                      int64_t ldy, ffx_dtype dtype, void* stream) {
  return guard([&] { product(A, true, s, alpha, X, ldx, beta, Y, ldy, dtype, (hipStream_t)stream); });
}

ffx_status ffx_power(ffx_matrix A, int64_t k, int32_t s, const void* V, int64_t ldv, void* W, int64_t ldw,
                     ffx_dtype dtype, void* stream) {
  return guard([&] {
    if (!A) fail(FFX_EINVAL, "matrix handle is NULL");
    check_dtype(dtype);
    if (A->info.nrows != A->info.ncols) fail(FFX_EINVAL, "power needs a square matrix");
    if (k < 0) fail(FFX_EINVAL, "k = %lld < 0", (long long)k);
    if (s < 1 || s > MAX_S) fail(FFX_EINVAL, "s = %d outside [1, %d]", s, MAX_S);
    const int64_t n = A->info.nrows;
    check_block("V", V, n, s, ldv);
    check_block("W", W, n, s, ldw);
    check_disjoint("V", V, n, ldv, "W", W, n, ldw, s, dtype);
    hipStream_t st = (hipStream_t)stream;
    if (n == 0) return;
    if (k == 0) {
      FFX_HIP(launch_copy_block(dtype, V, ldv, W, ldw, n, s, st));
      return;
    }
    if (A->perm) {  // V gathered once into the stored order; the last product writes W in the caller's order
      warm_pool(st);
      void* vp = nullptr;
      const size_t bytes = (size_t)n * s * esize(dtype);
      if (hipMallocAsync(&vp, bytes, st) != hipSuccess) fail(FFX_ENOMEM, "hipMallocAsync of %zu bytes failed", bytes);
      hipError_t e = launch_permute_rows(esize(dtype), V, ldv, vp, s, A->perm, n, s, false, st);
      if (e == hipSuccess) {
        try {
          power_iter(*A, k, s, vp, s, W, ldw, dtype, st, A->perm);
        } catch (...) {
          (void)hipFreeAsync(vp, st);
          throw;
        }
      }
      (void)hipFreeAsync(vp, st);
      FFX_HIP(e);
      return;
    }
    power_iter(*A, k, s, V, ldv, W, ldw, dtype, st, nullptr);
  });
}

ffx_status ffx_sequence(ffx_matrix A, int32_t s, const void* U, int64_t ldu, const void* V, int64_t ldv, int64_t L,
                        void* S, void* Wlast, ffx_dtype dtype, void* stream) {
  return guard([&] {
    if (!A) fail(FFX_EINVAL, "matrix handle is NULL");
    check_dtype(dtype);
    if (A->info.nrows != A->info.ncols) fail(FFX_EINVAL, "sequence needs a square matrix");
    if (L < 0) fail(FFX_EINVAL, "L = %lld < 0", (long long)L);
    if (s < 1 || s > MAX_S) fail(FFX_EINVAL, "s = %d outside [1, %d]", s, MAX_S);
    const int64_t n = A->info.nrows;
    check_block("U", U, n, s, ldu);
    check_block("V", V, n, s, ldv);
    if (L > 0 && !S) fail(FFX_EINVAL, "S is NULL");
    if (Wlast) {
      check_disjoint("V", V, n, ldv, "Wlast", Wlast, n, s, s, dtype);
      check_disjoint("U", U, n, ldu, "Wlast", Wlast, n, s, s, dtype);
      check_disjoint("S", S, L * s, s, "Wlast", Wlast, n, s, s, dtype);
    }
    if (L > 0) {
      check_disjoint("U", U, n, ldu, "S", S, L * s, s, s, dtype);
      check_disjoint("V", V, n, ldv, "S", S, L * s, s, s, dtype);
    }
    hipStream_t st = (hipStream_t)stream;
    if (n == 0) return;
    if (L == 0) {
      if (Wlast) FFX_HIP(launch_copy_block(dtype, V, ldv, Wlast, s, n, s, st));
      return;
    }
    warm_pool(st);
    const Encoded& E = A->A;
    size_t wbytes = (size_t)n * s * sizeof(int32_t);  // W_i and U are kept as int32 residues
    size_t pbytes = ((size_t)std::max<int64_t>(E.ntiles, 1) * SELL_SLICES + 64) * s * s * sizeof(uint64_t);
    void* ws[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    size_t sizes[6] = {wbytes, wbytes, wbytes, pbytes, pbytes, sizeof(int64_t)};
    for (int q = 0; q < 6; ++q)
      if (hipMallocAsync(&ws[q], sizes[q], st) != hipSuccess) {
        for (void* p : ws) if (p) (void)hipFreeAsync(p, st);
        fail(FFX_ENOMEM, "sequence workspace allocation failed");
      }
    const int gb = g_seq_graph_batch.load();
    const int batch = (gb > 0 && L >= 2 * (int64_t)gb) ? gb : 0;
    // reordered: S_i = (P U)^T B^i (P V) with B = P A P^T, and A^L V = P^T B^L (P V)
    void* pw[3] = {nullptr, nullptr, nullptr};
    hipError_t e = hipSuccess;
    if (A->perm) {
      const size_t pb = (size_t)n * s * esize(dtype);
      for (int q = 0; q < (Wlast ? 3 : 2); ++q)
        if (hipMallocAsync(&pw[q], pb, st) != hipSuccess) {
          for (void* p : ws) (void)hipFreeAsync(p, st);
          for (void* p : pw) if (p) (void)hipFreeAsync(p, st);
          fail(FFX_ENOMEM, "sequence workspace allocation failed");
        }
      e = launch_permute_rows(esize(dtype), U, ldu, pw[0], s, A->perm, n, s, false, st);
      if (e == hipSuccess) e = launch_permute_rows(esize(dtype), V, ldv, pw[1], s, A->perm, n, s, false, st);
    }
    if (e == hipSuccess)
      e = launch_sequence(seq_kind(*A), only_sell(E), E.dm, E.max_tile_entries, dtype, A->perm ? pw[0] : U,
                          A->perm ? s : ldu, A->perm ? pw[1] : V, A->perm ? s : ldv, L, s, S,
                          A->perm ? pw[2] : Wlast, ws[0], ws[1], ws[2], (uint64_t*)ws[3], (uint64_t*)ws[4],
                          (int64_t*)ws[5], batch, st);
    if (e == hipSuccess && A->perm && Wlast)
      e = launch_permute_rows(esize(dtype), pw[2], s, Wlast, s, A->perm, n, s, true, st);
    for (void* p : ws) (void)hipFreeAsync(p, st);
    for (void* p : pw) if (p) (void)hipFreeAsync(p, st);
    FFX_HIP(e);
  });
}

ffx_status ffx_spmm_gf2(ffx_matrix A, int32_t w, const void* X, int64_t ldx, void* Y, int64_t ldy, void* stream) {
  return guard([&] {
    if (!A) fail(FFX_EINVAL, "matrix handle is NULL");
    if (A->md.m != 2) fail(FFX_EINVAL, "GF(2) product needs a matrix built with m = 2 (m = %u)", A->md.m);
    if (w < 1 || w > MAX_S) fail(FFX_EINVAL, "w = %d outside [1, %d]", w, MAX_S);
    const int64_t nin = A->info.ncols, nout = A->info.nrows;
    check_block("X", X, nin, w, ldx);
    check_block("Y", Y, nout, w, ldy);
    check_disjoint("X", X, nin, ldx, "Y", Y, nout, ldy, w, FFX_I32);
    if (nout == 0) return;
    const Encoded& E = A->A;
    hipStream_t st = (hipStream_t)stream;
    if (A->perm) {
      permuted(*A, nout, w, 4, X, ldx, Y, ldy, false, st, [&](void* xp, void* yp) {
        FFX_HIP(launch_tiles_gf2(E.dm, E.max_tile_entries, xp, w, yp, w, w, st));
      });
      return;
    }
    if (w == 1 && A->sg.ngroups) {  // one word per row: the column-sorted groups, summed by exclusive or
      FFX_HIP(launch_sg_gf2(A->sg.dm, (const uint32_t*)X, ldx, (uint32_t*)Y, ldy, st));
      return;
    }
    FFX_HIP(launch_tiles_gf2(E.dm, E.max_tile_entries, X, ldx, Y, ldy, w, st));
  });
}

ffx_status ffx_sequence_gf2(ffx_matrix A, int32_t w, const void* U, int64_t ldu, const void* V, int64_t ldv, int64_t L,
                            void* S, void* Wlast, void* stream) {
  return guard([&] {
    if (!A) fail(FFX_EINVAL, "matrix handle is NULL");
    if (A->md.m != 2) fail(FFX_EINVAL, "GF(2) sequence needs a matrix built with m = 2 (m = %u)", A->md.m);
    if (A->info.nrows != A->info.ncols) fail(FFX_EINVAL, "sequence needs a square matrix");
    if (w < 1 || w > MAX_S) fail(FFX_EINVAL, "w = %d outside [1, %d]", w, MAX_S);
    if (L < 0) fail(FFX_EINVAL, "L = %lld < 0", (long long)L);
    const int64_t n = A->info.nrows;
    const int npairs = 32 * w * w;
    check_block("U", U, n, w, ldu);
    check_block("V", V, n, w, ldv);
    if (L > 0 && !S) fail(FFX_EINVAL, "S is NULL");
    if (Wlast) {
      check_disjoint("V", V, n, ldv, "Wlast", Wlast, n, w, w, FFX_I32);
      check_disjoint("U", U, n, ldu, "Wlast", Wlast, n, w, w, FFX_I32);
      if (L > 0) check_disjoint("S", S, L * 32 * w, w, "Wlast", Wlast, n, w, w, FFX_I32);
    }
    if (L > 0) {
      check_disjoint("U", U, n, ldu, "S", S, L * 32 * w, w, w, FFX_I32);
      check_disjoint("V", V, n, ldv, "S", S, L * 32 * w, w, w, FFX_I32);
    }
    hipStream_t st = (hipStream_t)stream;
    if (n == 0) {  // empty sums
      if (L > 0) FFX_HIP(hipMemsetAsync(S, 0, (size_t)L * npairs * 4, st));
      return;
    }
    if (L == 0) {
      if (Wlast) FFX_HIP(launch_copy_block(FFX_I32, V, ldv, Wlast, w, n, w, st));
      return;
    }
    warm_pool(st);
    const Encoded& E = A->A;
    size_t wbytes = (size_t)n * w * 4;
    void* ws[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    size_t sizes[5] = {wbytes, wbytes, wbytes, gf2_sequence_part_words(E.dm, w) * 4, wbytes};
    const int nws = (A->perm && Wlast) ? 5 : 4;  // reordered: A^L V is scattered back from ws[4]
    for (int q = 0; q < nws; ++q)
      if (hipMallocAsync(&ws[q], sizes[q], st) != hipSuccess) {
        for (void* p : ws) if (p) (void)hipFreeAsync(p, st);
        fail(FFX_ENOMEM, "GF(2) sequence workspace allocation failed");
      }
    hipError_t e;
    if (A->perm) {  // the stored order of a reordered matrix
      e = launch_permute_rows(4, U, ldu, ws[0], w, A->perm, n, w, false, st);
      if (e == hipSuccess) e = launch_permute_rows(4, V, ldv, ws[1], w, A->perm, n, w, false, st);
    } else {
      e = launch_copy_block(FFX_I32, U, ldu, ws[0], w, n, w, st);
      if (e == hipSuccess) e = launch_copy_block(FFX_I32, V, ldv, ws[1], w, n, w, st);
    }
    if (e == hipSuccess)
      e = launch_sequence_gf2(E.dm, E.max_tile_entries, w, (const uint32_t*)ws[0], (const uint32_t*)ws[1], L,
                              (uint32_t*)S, (uint32_t*)ws[2], (uint32_t*)ws[3],
                              (uint32_t*)(A->perm && Wlast ? ws[4] : Wlast), st);
    if (e == hipSuccess && A->perm && Wlast) e = launch_permute_rows(4, ws[4], w, Wlast, w, A->perm, n, w, true, st);
    for (void* p : ws) if (p) (void)hipFreeAsync(p, st);
    FFX_HIP(e);
  });
}

ffx_status ffx_check_block(uint32_t m, const void* X, int64_t n, int32_t s, int64_t ldx, ffx_dtype dtype,
                           void* stream, int64_t* first_bad) {
  return guard([&] {
    if (first_bad) *first_bad = -1;
    if (m < 2 || m > 2147483647u) fail(FFX_EINVAL, "modulus %u outside [2, 2^31-1]", m);
    if (n < 0 || s < 1 || s > MAX_S) fail(FFX_EINVAL, "shape %lld x %d", (long long)n, s);
    check_dtype(dtype);
    check_block("X", X, n, s, ldx);
    if (n == 0) return;
    hipStream_t st = (hipStream_t)stream;
    unsigned long long* d = nullptr;
    if (hipMallocAsync((void**)&d, sizeof(unsigned long long), st) != hipSuccess)
      fail(FFX_ENOMEM, "hipMallocAsync of 8 bytes failed");
    unsigned long long h = ~0ull;
    hipError_t e = launch_check_block(dtype, X, n, s, ldx, m, d, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&h, d, sizeof h, hipMemcpyDeviceToHost, st);
    (void)hipFreeAsync(d, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    FFX_HIP(e);
    if (h != ~0ull) {
      if (first_bad) *first_bad = (int64_t)h;
      fail(FFX_EINVAL, "entry %llu of the block is not a residue in [0, %u]", h, m - 1);
    }
  });
}

ffx_status ffx_set_sequence_graph_batch(int32_t batch) {
  return guard([&] {
    if (batch < 0 || batch > 4096) fail(FFX_EINVAL, "graph batch %d outside [0, 4096]", batch);
    g_seq_graph_batch.store(batch);
  });
}

ffx_status ffx_block_features(int64_t nrows, int64_t ncols, const int64_t* rowptr, const int32_t* colidx,
                              const void* vals, ffx_dtype val_type, uint32_t m, const ffx_build_opts* opts, float* out,
                              int64_t cap, int64_t* nblocks) {
  return guard([&] {
    if (cap > 0 && !out) fail(FFX_EINVAL, "out is NULL");
    RCsr A = reduce_csr(nrows, ncols, rowptr, colidx, vals, val_type, m);
    PlanOpts po = plan_opts(opts);
    const int64_t BR = po.block_rows, nb = (nrows + BR - 1) / BR;
    for (int64_t b = 0; b < nb && b < cap; ++b) {
      BlockStats st = block_stats(A, b * BR, std::min(nrows, (b + 1) * BR), m, po);
      std::memcpy(out + b * NUM_FEATURES, st.feat, sizeof(float) * NUM_FEATURES);
    }
    if (nblocks) *nblocks = nb;
  });
}

ffx_status ffx_sigma_basis(uint32_t p, int32_t m, int32_t n, int64_t sigma, const uint32_t* G, int64_t ldg,
                           const int32_t* shift, uint32_t* M, int64_t ldm, int32_t* d_out, void* stream) {
  return guard([&] { sigma_basis(p, m, n, sigma, G, ldg, shift, M, ldm, d_out, (hipStream_t)stream); });
}

ffx_status ffx_sequence_rank(uint32_t p, int32_t s, int64_t L, const void* S, ffx_dtype dtype, int32_t* deg_out,
                             int64_t* rank, int64_t* deg_det, int64_t* codeg_det, void* stream) {
  return guard([&] {
    check_dtype(dtype);
    if (!deg_out || !rank || !deg_det || !codeg_det) fail(FFX_EINVAL, "NULL argument");
    sequence_rank(p, s, L, S, dtype, deg_out, rank, deg_det, codeg_det, (hipStream_t)stream);
  });
}

ffx_status ffx_reorder_rcm(int64_t n, const int64_t* rowptr, const int32_t* colidx, int32_t* perm) {
  return guard([&] {
    if (n < 0 || n > MAX_DIM) fail(FFX_EINVAL, "n = %lld outside [0, 2^30]", (long long)n);
    if (n > 0 && (!rowptr || !perm)) fail(FFX_EINVAL, "NULL argument");
    RCsr A;
    A.nrows = A.ncols = n;
    if (n == 0) return;
    if (rowptr[0] != 0) fail(FFX_EINVAL, "rowptr[0] = %lld, expected 0", (long long)rowptr[0]);
    A.rp.assign(rowptr, rowptr + n + 1);
    for (int64_t i = 0; i < n; ++i)
      if (rowptr[i + 1] < rowptr[i]) fail(FFX_EINVAL, "rowptr decreases at row %lld", (long long)i);
    const int64_t nnz = rowptr[n];
    if (nnz > 0 && !colidx) fail(FFX_EINVAL, "colidx is NULL");
    A.col.resize(nnz);
    for (int64_t k = 0; k < nnz; ++k) {
      if (colidx[k] < 0 || colidx[k] >= n)
        fail(FFX_EINVAL, "column index %d at entry %lld outside [0, %lld)", colidx[k], (long long)k, (long long)n);
      A.col[k] = (uint32_t)colidx[k];
    }
    std::vector<uint32_t> p = rcm_order(A);
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)p[i];
  });
}

ffx_status ffx_matrix_block_times(ffx_matrix M, const void* x, void* y, ffx_dtype dtype, int32_t reps, float* us_out,
                                  void* stream) {
  return guard([&] {
    if (!M || !us_out) fail(FFX_EINVAL, "NULL argument");
    check_dtype(dtype);
    const int64_t nin = M->info.ncols, nout = M->info.nrows;
    check_block("x", x, nin, 1, 1);
    check_block("y", y, nout, 1, 1);
    check_disjoint("x", x, nin, 1, "y", y, nout, 1, 1, dtype);
    hipStream_t st = (hipStream_t)stream;
    const Encoded& E = M->A;
    const int ak = arith_kind(*M);
    if (reps < 1) reps = 1;
    uint16_t* x16 = nullptr;
    if (M->compact_x && nin > 0) {
      warm_pool(st);
      if (hipMallocAsync((void**)&x16, (size_t)nin * 2, st) != hipSuccess) fail(FFX_ENOMEM, "x copy");
      FFX_HIP(launch_compact_x(dtype, x, 1, x16, nin, st));
    }
    hipEvent_t e0, e1;
    FFX_HIP(hipEventCreate(&e0));
    FFX_HIP(hipEventCreate(&e1));
    hipError_t e = hipSuccess;
    const int64_t nb = (int64_t)E.block_fmt.size();
    for (int64_t b = 0; b < nb && e == hipSuccess; ++b) {
      uint32_t t0 = E.block_tile0[b], nt = E.block_tile0[b + 1] - t0;
      if (nt == 0) {
        us_out[b] = 0.f;
        continue;
      }
      DevMat sub = E.dm;
      sub.tiles += t0;
      sub.ntiles = nt;
      // enough copies of the block to fill the GPU several times over
      uint32_t R = std::max<uint32_t>((uint32_t)reps, (8192 + nt - 1) / nt);
      uint32_t grid = std::min<uint64_t>((uint64_t)R * nt, 1u << 30) / nt * nt;
      R = grid / nt;
      e = launch_tiles(ak, sub, E.max_tile_entries, dtype, x, 1, y, 1, 1, 1, 0, st, x16, grid);  // warm
      if (e == hipSuccess) e = hipEventRecord(e0, st);
      if (e == hipSuccess) e = launch_tiles(ak, sub, E.max_tile_entries, dtype, x, 1, y, 1, 1, 1, 0, st, x16, grid);
      if (e == hipSuccess) e = hipEventRecord(e1, st);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      us_out[b] = ms * 1000.f / (float)R;
    }
    if (x16) (void)hipFreeAsync(x16, st);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    FFX_HIP(e);
  });
}

const char* ffx_status_str(ffx_status st) {
  switch (st) {
    case FFX_OK: return "FFX_OK";
    case FFX_EINVAL: return "FFX_EINVAL";
    case FFX_EBOUND: return "FFX_EBOUND";
    case FFX_ENOMEM: return "FFX_ENOMEM";
    case FFX_EDEVICE: return "FFX_EDEVICE";
    case FFX_EUNSUPPORTED: return "FFX_EUNSUPPORTED";
  }
  return "FFX_UNKNOWN";
}

const char* ffx_last_error(void) { return g_last_error.c_str(); }

const char* ffx_version(void) { return "ffx 0.1 (gfx950)"; }

}  // extern "C"
