// Host-side planner and runtime structures.
#pragma once

#include <stdint.h>

#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ffx_impl.h"
#include "sg.h"

namespace ffx {

// Error reporting: every C entry point converts a thrown Error into a status.
struct Error {
  ffx_status st;
  std::string msg;
};
[[noreturn]] void fail(ffx_status st, const char* fmt, ...);
void set_last_error(const std::string& s);
// Runs the body of a C entry point: a thrown Error becomes its status and the
// calling thread's last error; anything else thrown becomes FFX_ENOMEM (a host
// allocation) or FFX_EDEVICE.
template <class F>
ffx_status guard(F&& f) {
  try {
    f();
    set_last_error("");
    return FFX_OK;
  } catch (const Error& e) {
    set_last_error(e.msg);
    return e.st;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return FFX_ENOMEM;
  } catch (...) {
    set_last_error("unexpected internal error");
    return FFX_EDEVICE;
  }
}
#define FFX_HIP(call)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) ::ffx::fail(FFX_EDEVICE, "%s: %s", #call, hipGetErrorString(e_));   \
  } while (0)

// A matrix after reduction modulo m: rows sorted by column, duplicates merged,
// zero residues dropped; val[k] in [1, m-1].
struct RCsr {
  int64_t nrows = 0, ncols = 0;
  std::vector<int64_t> rp;
  std::vector<uint32_t> col;
  std::vector<uint32_t> val;
  int64_t nnz() const { return rp.empty() ? 0 : rp.back(); }
};

RCsr reduce_csr(int64_t nrows, int64_t ncols, const int64_t* rowptr, const int32_t* colidx, const void* vals,
                ffx_dtype vt, uint32_t m);
RCsr reduce_coo(int64_t nrows, int64_t ncols, int64_t nnz, const int32_t* rowidx, const int32_t* colidx,
                const void* vals, ffx_dtype vt, uint32_t m);
RCsr transpose(const RCsr& A);

// Reverse Cuthill-McKee order of a square matrix (pattern of A + A^T):
// perm[new] = old. permute_sym returns P A P^T, i.e. row i is row perm[i] of A
// with every column j renumbered to its new index. bandwidth: max |i - j|.
std::vector<uint32_t> rcm_order(const RCsr& A);
RCsr permute_sym(const RCsr& A, const std::vector<uint32_t>& perm);
int64_t bandwidth(const RCsr& A);

// Per-block statistics (also the features of the learned selector).
constexpr int NUM_FEATURES = 32;
struct BlockStats {
  int64_t row0 = 0, nrows = 0, nnz = 0;
  double mean = 0, sd = 0;
  int64_t maxlen = 0, minlen = 0, empty = 0;
  double pm1_frac = 0;
  std::vector<int32_t> band_offsets;  // chosen dense diagonals
  int64_t band_nnz = 0;
  int64_t sell_width_sum = 0;         // sum over 64-row slices of the longest residual row
  int64_t sell_sorted_width_sum = 0;  // same after sorting rows by residual length
  int64_t long_rows = 0;              // residual rows longer than one STREAM tile
  float feat[NUM_FEATURES];
};

struct PlanOpts {
  int acc = FFX_ACC_INT64;
  int selector = FFX_SEL_HEURISTIC;
  int fixed_format = FFX_FMT_STREAM;
  bool split_pm1 = true;
  int block_rows = 4096;
  int tile_entries = 1024;
  int compact_x = -1;
  std::string model_path;
  bool reorder = false;
  int col_sorted = -1;
};

BlockStats block_stats(const RCsr& A, int64_t r0, int64_t r1, uint32_t m, const PlanOpts& o);
int heuristic_format(const BlockStats& b, const PlanOpts& o);

// One encoded operator (A or A^T) on the device.
struct Encoded {
  DevMat dm{};
  std::vector<void*> allocs;
  int64_t nrows = 0, ncols = 0;
  int64_t ntiles = 0, max_row_terms = 0, n_band = 0, n_plus = 0, n_minus = 0, nnz = 0;
  int64_t device_bytes = 0, stream_bytes = 0;
  int64_t max_tile_entries = 0;  // largest STREAM tile (sizes the LDS of a launch)
  std::vector<int32_t> block_fmt;
  std::vector<uint32_t> tile_cost;  // per tile: entry words read (with padding) plus band slots
  std::vector<uint32_t> block_tile0;  // first tile of each block, plus the tile count at the end
  int64_t format_blocks[FFX_NUM_FORMATS] = {0, 0, 0, 0, 0, 0};
  int64_t kind_tiles[3] = {0, 0, 0};  // STREAM, LONG and SELL tiles
  // sizes (elements) of each device array, for the batched concatenation
  int64_t n_ent = 0, n_val = 0, n_choff = 0, n_rowp = 0, n_perm = 0, n_swidth = 0, n_bval = 0, n_boffs = 0;
  void release();
};

struct Modulus {
  uint32_t m = 0;
  uint64_t mu = 0;
  double inv_m = 0;
  bool small() const { return m <= 65536u; }  // (m-1)^2 < 2^32 and values fit 16 bits
};
Modulus make_modulus(uint32_t m);

// Encodes A (block formats chosen per opts) and uploads it.
void encode(const RCsr& A, const Modulus& md, const PlanOpts& o, hipStream_t stream, Encoded* out,
            const std::vector<int32_t>* forced_formats = nullptr);

// Column-sorted row groups of a matrix for the one-vector product (sg.h).
struct SgEncoded {
  SgMat dm{};
  void* alloc = nullptr;
  int64_t ngroups = 0, device_bytes = 0, stream_bytes = 0;
  void release();
};
// Encodes A (m <= 65536) in about target_groups groups and uploads it.
void encode_sg(const RCsr& A, const Modulus& md, bool split_pm1, int target_groups, hipStream_t st, SgEncoded* out);

// Learned selector hook: fills fmt for the blocks, returns false to fall back.
bool learned_formats(const std::string& model_path, const std::vector<BlockStats>& blocks, std::vector<int32_t>& fmt,
                     hipStream_t stream);
int matrix_arith_kind(const ffx_matrix_s& M);

// Order basis and block-Wiedemann rank (sigma.hip); arguments as ffx_sigma_basis and
// ffx_sequence_rank.
void sigma_basis(uint32_t p, int m, int n, int64_t sigma, const uint32_t* G, int64_t ldg, const int32_t* shift,
                 uint32_t* M, int64_t ldm, int32_t* d_out, hipStream_t st);
void sequence_rank(uint32_t p, int s, int64_t L, const void* S, ffx_dtype dt, int32_t* deg_out, int64_t* rank,
                   int64_t* deg_det, int64_t* codeg_det, hipStream_t st);

}  // namespace ffx

struct ffx_matrix_s {
  ffx::Modulus md;
  int acc = FFX_ACC_INT64;
  bool chunk = false;   // some row needs reductions inside the row
  bool compact_x = false;  // one-vector products gather x from a 16-bit copy
  ffx::Encoded A, AT;
  ffx::SgEncoded sg;  // column-sorted groups of A for one-vector products (when built)
  bool has_t = false;
  // reordered matrices: A and AT hold P A P^T; perm[new] = old on the device
  uint32_t* perm = nullptr;
  ffx_matrix_info info{};
  // The temporary of the row products (x in 16 bits and/or in the stored order), allocated on the
  // first product that needs one and kept until destroy: a stream-ordered allocation per product
  // cost the host ~75 us. While every product uses one stream, stream order protects it. The first
  // product on another stream synchronizes the device once; from then on (`multi`) `done` is
  // recorded after each product and a product on another stream than `last` waits for it, so
  // products on one handle stay correct on any streams (they serialize where they share the
  // temporary). An event per product costs the GPU a few microseconds, hence not before it is
  // needed. `mu` makes the wait, the launches and the record atomic.
  struct {
    std::mutex mu;
    void* p = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
    hipStream_t last = nullptr;
    bool used = false;
    bool multi = false;
  } scr;
};
