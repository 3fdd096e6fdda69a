/*
 * ffx -- exact sparse matrix products over Z/mZ on MI355X (gfx950).
 *
 * C ABI of the library libffx.so. Every call returns an ffx_status; nothing
 * throws across this boundary. After a failure, ffx_last_error() returns a
 * message for the calling thread.
 *
 * Operations (paper, Section 2 opening paragraph): y <- alpha*A*x + beta*y,
 * the apply y <- A*x (alpha = 1, beta = 0), and the block form
 * Y <- alpha*A*X + beta*Y; the transpose product (Section 1 and Section 4);
 * the power A^k*V and the projected sequence U^T A^i V of block Wiedemann's
 * first step (Section 2.5 "Performance issues", Section 3 step 1,
 * Section 3.1).
 *
 * Conventions shared by every call:
 *  - 2 <= m <= 2^31-1. m need not be prime; only ring operations are used.
 *  - Residues are represented on [0, m-1] (Section 2.2). Matrix values given
 *    to a create call may be any int32/int64 and are reduced there; every
 *    vector entry, alpha and beta passed to a product must already be in
 *    [0, m-1] (otherwise the result is unspecified). Outputs are always in
 *    [0, m-1].
 *  - Dense multi-vectors are n x s with row j's s residues contiguous,
 *    leading dimension ld >= s (the layout Section 2.5 "Using multi-vectors"
 *    describes as reading A once with x and y accessed contiguously).
 *  - Vector, multi-vector and sequence pointers are caller-owned DEVICE
 *    memory; calls are ordered on the given stream (a hipStream_t passed as
 *    void*, NULL for the null stream) and return before the kernels finish.
 *    The library never frees caller memory.
 *  - Input and output vectors must not overlap. With beta = 0 the output is
 *    write-only (its previous contents are ignored).
 *  - A matrix handle's matrix is read-only after creation, and products on
 *    one handle may be issued on different streams and from several host
 *    threads. The handle keeps one device temporary for its row products
 *    (the 16-bit copy of x, or x in the stored order of a reordered matrix;
 *    allocated by the first product that needs it, freed by destroy): the
 *    first product on a second stream synchronizes the device once, and from
 *    then on products on different streams are ordered on that temporary by
 *    an event (they serialize rather than overlap). Such products are not
 *    for HIP graph capture (the allocation and the synchronization are not
 *    stream operations); ffx_spmv_noalloc is.
 */
#ifndef FFX_H
#define FFX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FFX_OK = 0,
  FFX_EINVAL = 1,       /* bad argument: modulus, shape, index, pointer, overlap */
  FFX_EBOUND = 2,       /* requested accumulator cannot hold one product exactly */
  FFX_ENOMEM = 3,       /* host or device allocation failed */
  FFX_EDEVICE = 4,      /* a HIP runtime call failed */
  FFX_EUNSUPPORTED = 5  /* valid request outside what the library implements */
} ffx_status;

typedef enum { FFX_I32 = 0, FFX_I64 = 1 } ffx_dtype;

/* Accumulator of the delayed reduction (Section 2.2): products are summed in
 * a wide type and reduced modulo m only when the next term could exceed what
 * the type holds exactly. INT64: unsigned 64-bit integers, at most
 * 2^63 - 1 before a reduction. FP64: doubles, at most 2^53 - 1 (every
 * integer up to 2^53 is exact). FP32: floats, at most 2^24 - 1 (m <= 4096).
 * The CENTERED variants (Section 2.2, the ring represented on
 * [-floor((m-1)/2), ceil((m-1)/2)]) use every operand as a residue of
 * magnitude at most floor(m/2), so a product is about a quarter of (m-1)^2
 * and sums of both signs stay exact up to 2^53 - 1 (m <= 189,812,531) or
 * 2^24 - 1 (m <= 8191) in magnitude: about four times as many terms between
 * reductions. Inputs and results stay canonical residues in [0, m-1] for
 * every accumulator. A floating accumulator that cannot hold one product
 * exactly is refused with FFX_EBOUND. AUTO: INT64. */
typedef enum {
  FFX_ACC_AUTO = 0,
  FFX_ACC_INT64 = 1,
  FFX_ACC_FP64 = 2,
  FFX_ACC_FP32 = 3,
  FFX_ACC_FP64_CENTERED = 4,
  FFX_ACC_FP32_CENTERED = 5
} ffx_acc;

/* Who chooses each row block's storage format (Section 2.4 "Heuristic format
 * chooser"): the plain heuristic, the learned cost model (falls back to the
 * heuristic when no usable model is loaded), or one fixed format for all. */
typedef enum { FFX_SEL_HEURISTIC = 0, FFX_SEL_LEARNED = 1, FFX_SEL_FIXED = 2 } ffx_sel;

/* Per-block storage formats. A block is a run of block_rows consecutive
 * rows. Every format stores +-1 entries without a value when split_pm1 is
 * set (Section 2.4 "Taking into account the +-1"); the BAND_* formats move
 * the block's densest diagonals into a diagonal-major part whose values are
 * stored densely (the DIA idea of Section 2.1) and keep the rest in the
 * named residual format. The result never depends on the format. */
typedef enum {
  FFX_FMT_STREAM = 0,            /* CSR rows staged through LDS in balanced tiles */
  FFX_FMT_SELL = 1,              /* sliced ELL: 64-row slices, column-major, padded */
  FFX_FMT_SELL_SORTED = 2,       /* sliced ELL over rows sorted by length inside the block */
  FFX_FMT_BAND_STREAM = 3,
  FFX_FMT_BAND_SELL = 4,
  FFX_FMT_BAND_SELL_SORTED = 5,
  FFX_NUM_FORMATS = 6
} ffx_format;

typedef struct {
  uint32_t size;            /* sizeof(ffx_build_opts) */
  int32_t acc;              /* ffx_acc, default FFX_ACC_AUTO */
  int32_t selector;         /* ffx_sel, default FFX_SEL_HEURISTIC */
  int32_t fixed_format;     /* ffx_format used when selector == FFX_SEL_FIXED */
  int32_t split_pm1;        /* 1 (default): +-1 stored without values; 0: every entry has a value */
  int32_t block_rows;       /* rows per format block, a multiple of 64 in [64, 65536]; default 4096 */
  int32_t build_transpose;  /* 1: also encode A^T so ffx_spmv_t/ffx_spmm_t run as row products */
  int32_t tile_entries;     /* entries per STREAM tile, 256..4096, 0 = default (2048) */
  int32_t compact_x;        /* m <= 65536, one vector: gather x from a 16-bit copy made per product
                               (-1 = when x exceeds 1 MiB, 0 = never, 1 = always); never changes a result */
  const char* model_path;   /* learned selector weights; NULL = none */
  int32_t reorder;          /* square matrices: 1 = store P A P^T under the reverse Cuthill-McKee order
                               of the pattern of A + A^T (Section 4, reordering A), so the x entries
                               of a tile come from a narrow window; every entry point then takes and
                               returns vectors in the caller's order (one gather in, one scatter out
                               per call, once per call for ffx_power and ffx_sequence); never changes
                               a result. 0 (default): the caller's order. Batches refuse reordered
                               matrices. */
  int32_t col_sorted;       /* m <= 65536 with the int64 accumulator: 1 = also store A as column-sorted
                               row groups (about one per compute unit, entries sorted by column inside
                               a group) that ffx_spmv and ffx_spmv_noalloc use for y = alpha*A*x +
                               beta*y: the lanes of one gather then share cache lines of x. Costs a
                               second copy of A on the device. 0 = never; -1 (default) = when A has
                               at least 4 Mi entries and 256 Ki columns. Never changes a result. */
} ffx_build_opts;

typedef struct ffx_matrix_s* ffx_matrix;

typedef struct {
  int64_t nrows, ncols;
  uint32_t m;
  int32_t acc;              /* accumulator actually used (ffx_acc, never FFX_ACC_AUTO) */
  int64_t nnz_input;        /* entries given to the create call */
  int64_t nnz;              /* stored nonzero residues after merging duplicates and dropping zeros */
  int64_t n_plus, n_minus;  /* entries stored without a value (residue 1 and m-1) */
  int64_t n_band;           /* entries held in BAND diagonals */
  int64_t nblocks;
  int64_t ntiles;
  int64_t max_row_terms;    /* longest row, in terms */
  int64_t reduce_every;     /* bound b: terms summed between reductions (>= max_row_terms: never) */
  int64_t device_bytes;     /* device memory held by the handle (A, and A^T when built) */
  int64_t stream_bytes;     /* bytes one product streams from the encoded matrix (excluding x and y) */
  int32_t has_transpose;
  int32_t value_bytes;      /* 2 when m <= 65536, else 4 */
  int64_t format_blocks[FFX_NUM_FORMATS]; /* number of blocks in each format */
  int32_t reordered;        /* 1 when the handle stores P A P^T (ffx_build_opts.reorder) */
  int64_t bandwidth_input;  /* max |i - j| over the entries of A */
  int64_t bandwidth_stored; /* the same for the stored operator (P A P^T when reordered) */
  int64_t sg_groups;        /* column-sorted row groups (ffx_build_opts.col_sorted), 0 when not built */
  int64_t sg_stream_bytes;  /* bytes a one-vector product streams from them (excluding x and y) */
} ffx_matrix_info;

/* Fill *opts with the defaults. */
void ffx_build_opts_default(ffx_build_opts* opts);

/* Build a matrix from host CSR arrays (Section 2.1: start = rowptr,
 * colid = colidx, data = vals). rowptr has nrows+1 entries (rowptr[0] = 0,
 * nondecreasing); colidx[k] in [0, ncols); vals is int32 or int64 per
 * val_type. Columns need not be sorted; duplicates add. Values are reduced to
 * [0, m-1], zero residues dropped, residues 1 and m-1 classified as +-1 (for
 * m = 2, 1 = -1 counts as +1). Limits: nrows, ncols <= 2^30, nnz < 2^32.
 * The host arrays are copied; the caller keeps them. Device uploads are
 * issued on `stream` and complete before return. opts may be NULL. */
ffx_status ffx_matrix_create_csr(int64_t nrows, int64_t ncols, const int64_t* rowptr, const int32_t* colidx,
                                 const void* vals, ffx_dtype val_type, uint32_t m, const ffx_build_opts* opts,
                                 void* stream, ffx_matrix* out);

/* Same from coordinate triples (Section 2.1: data, colid, rowid), any order. */
ffx_status ffx_matrix_create_coo(int64_t nrows, int64_t ncols, int64_t nnz, const int32_t* rowidx,
                                 const int32_t* colidx, const void* vals, ffx_dtype val_type, uint32_t m,
                                 const ffx_build_opts* opts, void* stream, ffx_matrix* out);

ffx_status ffx_matrix_info_get(ffx_matrix A, ffx_matrix_info* info);

/* Format of each row block of A (transpose = 0) or of A^T (transpose = 1):
 * writes min(cap, nblocks) ffx_format values to out (host memory). */
ffx_status ffx_matrix_block_formats(ffx_matrix A, int32_t transpose, int32_t* out, int64_t cap);

/* Frees the handle and its device memory (NULL: nothing). When the handle
 * holds the temporary of its row products, the device is synchronized first,
 * so no product still running uses it. */
ffx_status ffx_matrix_destroy(ffx_matrix A);

/* Y <- A X over GF(2) with bit-packed blocks (Section 4 points to compressing
 * GF(2) vectors into machine words). A must have been built with m = 2, so
 * every stored entry is 1. X (ncols x w) and Y (nrows x w) are 32-bit words in
 * device memory with leading dimensions ldx, ldy >= w: bit b of word c of row
 * j is entry j of vector 32c + b, so one call multiplies A by 32w vectors.
 * Sums are exclusive ors; Y is overwritten. w in [1, 16]. FFX_EINVAL for
 * m != 2, a bad w or shape, NULL or overlapping blocks. */
ffx_status ffx_spmm_gf2(ffx_matrix A, int32_t w, const void* X, int64_t ldx, void* Y, int64_t ldy, void* stream);

/* The block-Wiedemann sequence over GF(2) with packed blocks (Section 3,
 * step 1, with the GF(2) compression of Section 4): S_i = U^T A^i V for
 * i = 0 .. L-1 and 32w vectors. A: built with m = 2, square. U, V: n x w
 * words (device, leading dimensions >= w), bit b of word c of row j being
 * entry j of vector 32c + b. S: L * 32w * w words (device); row a of S_i is
 * S[(i*32w + a)*w .. +w), bit b of its word c being the parity of the rows
 * where vector a of U and vector 32c + b of A^i V are both 1. Wlast (n x w,
 * leading dimension w, or NULL) receives A^L V. w in [1, 16]. Errors as for
 * ffx_sequence. */
ffx_status ffx_sequence_gf2(ffx_matrix A, int32_t w, const void* U, int64_t ldu, const void* V, int64_t ldv, int64_t L,
                            void* S, void* Wlast, void* stream);

/* Checked mode. Products take vector entries that are already residues in
 * [0, m-1] (Section 2.2) and do not look at them; this call checks an n x s
 * block X (device memory, element type dtype, leading dimension ldx >= s)
 * before use. FFX_OK when every entry is in [0, m-1]; FFX_EINVAL when one is
 * not, with *first_bad (when not NULL) the smallest flat index k*ldx + c of
 * such an entry, and -1 on FFX_OK. FFX_EINVAL also for a bad modulus, dtype or
 * shape. Runs on `stream` and waits for it. */
ffx_status ffx_check_block(uint32_t m, const void* X, int64_t n, int32_t s, int64_t ldx, ffx_dtype dtype,
                           void* stream, int64_t* first_bad);

/* y <- alpha*A*x + beta*y (mod m). x: ncols entries, y: nrows entries, both
 * of element type dtype. */
ffx_status ffx_spmv(ffx_matrix A, uint32_t alpha, const void* x, uint32_t beta, void* y, ffx_dtype dtype,
                    void* stream);

/* y <- alpha*A^T*x + beta*y (mod m). x: nrows entries, y: ncols entries.
 * Uses the stored A^T when the handle has one, else a scatter with 64-bit
 * integer atomics into a temporary, which is exact in any order. */
ffx_status ffx_spmv_t(ffx_matrix A, uint32_t alpha, const void* x, uint32_t beta, void* y, ffx_dtype dtype,
                      void* stream);

/* y <- alpha*A*x + beta*y (mod m), as ffx_spmv, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc): this call allocates nothing. The
 * temporary that ffx_spmv keeps in the handle (the 16-bit copy of x when
 * m <= 65536, or x gathered into the stored order of a reordered handle)
 * lives instead in a static device array of FFX_NOALLOC_SCRATCH_BYTES bytes,
 * one per GPU, held from the first call on that GPU until the process ends.
 * FFX_EINVAL when the product needs more than that (2 bytes per column of A
 * for the 16-bit copy; 4 or 8 bytes per column for a reordered handle whose
 * x is not copied to 16 bits), checked before anything is enqueued. Every
 * call on one GPU shares that GPU's array: calls on one stream are ordered,
 * but calls that overlap on different streams of the same GPU race. The
 * result is identical to ffx_spmv's. */
#define FFX_NOALLOC_SCRATCH_BYTES (32u << 20)
ffx_status ffx_spmv_noalloc(ffx_matrix A, uint32_t alpha, const void* x, uint32_t beta, void* y, ffx_dtype dtype,
                            void* stream);

/* Y <- alpha*A*X + beta*Y (mod m) for s in [1, 16] vectors. X: ncols x s
 * (ldx), Y: nrows x s (ldy). */
ffx_status ffx_spmm(ffx_matrix A, int32_t s, uint32_t alpha, const void* X, int64_t ldx, uint32_t beta, void* Y,
                    int64_t ldy, ffx_dtype dtype, void* stream);

/* Y <- alpha*A^T*X + beta*Y (mod m). X: nrows x s (ldx), Y: ncols x s (ldy). */
ffx_status ffx_spmm_t(ffx_matrix A, int32_t s, uint32_t alpha, const void* X, int64_t ldx, uint32_t beta,
                      void* Y, int64_t ldy, ffx_dtype dtype, void* stream);

/* W <- A^k V (mod m) for square A, k >= 0, s in [1, 16]; V and W: n x s
 * (ldv, ldw). The iterates stay on the device (Section 2.5 "Performance
 * issues", the smpv_n loop). V and W may not overlap. */
ffx_status ffx_power(ffx_matrix A, int64_t k, int32_t s, const void* V, int64_t ldv, void* W, int64_t ldw,
                     ffx_dtype dtype, void* stream);

/* S_i = U^T A^i V (mod m) for i = 0 .. L-1 (Section 3, step 1; Section 3.1),
 * square A, s in [1, 16]. U and V: n x s (ldu, ldv). S: L*s*s entries of
 * type dtype, S[(i*s + a)*s + b] = sum_k U[k][a] * (A^i V)[k][b] mod m.
 * If Wlast is not NULL it receives A^L V (n x s, leading dimension s).
 * The whole loop runs on the device; no data returns to the host. */
ffx_status ffx_sequence(ffx_matrix A, int32_t s, const void* U, int64_t ldu, const void* V, int64_t ldv, int64_t L,
                        void* S, void* Wlast, ffx_dtype dtype, void* stream);

/* Iterations per hipGraph replay in ffx_sequence: the steps of `batch`
 * iterations are captured once and the graph is replayed (Section 2.5: the
 * iterates stay on the device and the host only launches). Default 64; 0
 * launches every iteration directly. Process-wide, read at each
 * ffx_sequence call; a tuning knob only, results never depend on it.
 * FFX_EINVAL when batch is outside [0, 4096]. */
ffx_status ffx_set_sequence_graph_batch(int32_t batch);

/* ------------------------------------------------------------------------
 * Batched products: Y_k <- A_k X_k (mod m) for many matrices of uneven size,
 * each with its own number s_k of right-hand sides, in one persistent launch.
 * It generalises the paper's treatment of submatrices in parallel
 * (Section 2.4, "New formats": split A into submatrices treated in parallel)
 * to independent matrices; the launch parameters (workgroups per CU, item
 * order, column chunk, XCD queues, 16-bit X) come from a tuner that
 * times candidates on the batch itself, as the paper suggests tuning the
 * format parameters for the machine (Section 2.4, "Heuristic format chooser").
 * ------------------------------------------------------------------------ */
typedef struct ffx_batch_s* ffx_batch;

typedef struct {
  int32_t wg_per_cu;   /* persistent workgroups per compute unit (1..8); 0 = tuned or default 4 */
  int32_t order;       /* 0: work items by decreasing estimated cost, 1: matrix order */
  int32_t max_chunk;   /* right-hand sides per work item: 4 or 8 (wider blocks are split) */
  int32_t use_graph;   /* 1: replay a captured hipGraph of the launch */
  int32_t xcd;         /* 1: matrices split over 8 work queues, one per XCD (L2), workgroup g starting on
                          queue g mod 8 and helping the others when its own is empty; 0: one queue */
  int32_t compact_x;   /* m <= 65536, int64 accumulator: 1 gathers X from 16-bit copies made by the launch
                          (the batch keeps the copies' memory, 2 bytes per element of every X_k), 0 never,
                          -1 (default) as 0: a row gather costs a cache line either way, so on MI355X the
                          copy has not paid for itself on multi-vector batches; the tuner tries both */
} ffx_batch_params;

/* Group `count` matrices (all with the same modulus and accumulator) with
 * s[k] in [1, 16] right-hand sides each. The handles stay owned by the
 * caller and must outlive the batch. The batch copies their descriptors and
 * builds its work list on the device. params may be NULL (defaults). */
ffx_status ffx_batch_create(int32_t count, const ffx_matrix* mats, const int32_t* s, const ffx_batch_params* params,
                            void* stream, ffx_batch* out);

/* Y_k <- A_k X_k for all k, one launch. X and Y are HOST arrays of `count`
 * DEVICE pointers; ldx[k] >= s[k], ldy[k] >= s[k] (host arrays). X_k has
 * ncols_k rows, Y_k nrows_k rows, all of element type dtype.
 * Unlike a matrix handle, a batch handle holds per-call device state (the
 * operand table and the work counters that each call rewrites on its stream):
 * calls on one batch handle (ffx_batch_spmm, ffx_batch_tune) must not overlap,
 * so issue them on one stream, or order the streams, and from one host thread
 * at a time. Separate batch handles over the same matrices are independent. */
ffx_status ffx_batch_spmm(ffx_batch B, const void* const* X, const int64_t* ldx, void* const* Y, const int64_t* ldy,
                          ffx_dtype dtype, void* stream);

/* Times each candidate launch configuration `reps` times on the given
 * operands, keeps the fastest in the batch and writes it to *best (may be
 * NULL). When cache_path is not NULL the choice is also stored there (JSON,
 * keyed by device name and batch signature) and read back by later calls. */
ffx_status ffx_batch_tune(ffx_batch B, const void* const* X, const int64_t* ldx, void* const* Y, const int64_t* ldy,
                          ffx_dtype dtype, int32_t reps, const char* cache_path, void* stream, ffx_batch_params* best);

ffx_status ffx_batch_get_params(ffx_batch B, ffx_batch_params* params);
ffx_status ffx_batch_set_params(ffx_batch B, const ffx_batch_params* params);
ffx_status ffx_batch_destroy(ffx_batch B);

/* ------------------------------------------------------------------------
 * Learned format selection. The paper's chooser is a hand heuristic whose
 * thresholds "vary according to the architecture" and need tuning (Section
 * 2.4, "Heuristic format chooser"). Here a small network predicts, from 32
 * features of a row block, the log2 time of each of the FFX_NUM_FORMATS
 * formats, and the block takes the predicted fastest. It is trained on
 * timings the library measures (ffx_matrix_block_times) with the library's
 * own forward, backward and Adam kernels. It only chooses formats: results
 * never depend on it, and a build with FFX_SEL_LEARNED falls back to the
 * heuristic when the model file is missing, corrupt or predicts non-finite
 * values.
 * ------------------------------------------------------------------------ */
#define FFX_SELECTOR_FEATURES 32
#define FFX_SELECTOR_PARAMS 6662

typedef struct ffx_selector_s* ffx_selector;

/* A network with He-uniform weights drawn from `seed`, zero biases, and
 * identity input standardisation (mean 0, scale 1). */
ffx_status ffx_selector_create(uint64_t seed, ffx_selector* out);
/* Host copies of the 6,662 parameters (W1 64x32, b1, W2 64x64, b2, W3 6x64,
 * b3, row-major) and of the 32 input means and scales (x' = (x-mean)*scale).
 * Any pointer may be NULL to leave that part unchanged / unread. */
ffx_status ffx_selector_set_params(ffx_selector S, const float* theta, const float* mean, const float* scale);
ffx_status ffx_selector_get_params(ffx_selector S, float* theta, float* mean, float* scale);
/* out (device, n x 6) <- predictions for X (device, n x 32 raw features). */
ffx_status ffx_selector_predict(ffx_selector S, const float* X, int64_t n, float* out, void* stream);
/* grad (device, 6,662) <- gradient of loss = sum(M*(f(X)-T)^2)/(2n) over the n
 * samples; T and M are device n x 6 (M is 0/1). *loss (host) when not NULL;
 * the call then waits for the stream. */
ffx_status ffx_selector_gradient(ffx_selector S, const float* X, const float* T, const float* M, int64_t n,
                                 float* grad, double* loss, void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the gradient of that loss. */
ffx_status ffx_selector_train_step(ffx_selector S, const float* X, const float* T, const float* M, int64_t n, float lr,
                                   double* loss, void* stream);
/* A checksummed binary file of the parameters and standardisation. */
ffx_status ffx_selector_save(ffx_selector S, const char* path);
ffx_status ffx_selector_load(const char* path, ffx_selector* out);
ffx_status ffx_selector_destroy(ffx_selector S);

/* The 32 features of each row block of a host CSR matrix, as the builder
 * computes them (opts: block_rows, tile_entries, split_pm1); out (host)
 * receives min(cap, nblocks) rows of 32 floats. Returns the block count in
 * *nblocks when not NULL. */
ffx_status ffx_block_features(int64_t nrows, int64_t ncols, const int64_t* rowptr, const int32_t* colidx,
                              const void* vals, ffx_dtype val_type, uint32_t m, const ffx_build_opts* opts, float* out,
                              int64_t cap, int64_t* nblocks);

/* Labels for training the selector, measured by the library on this GPU
 * (Section 2.4, "Heuristic format chooser": the chooser's thresholds depend on
 * the machine, so they are replaced by measurement). The window is a host CSR
 * matrix given as to ffx_matrix_create_csr, m <= 65536. It is built once per
 * format with every block forced to that format (the rest of the build from
 * opts: block_rows, tile_entries, split_pm1, acc, compact_x; never with
 * column-sorted groups, which would bypass the formats), and its whole
 * product y = A x is timed in place on `stream` with HIP events: the median of
 * `reps` launches (1..10000) after two warm-ups, x int32 residues drawn from
 * `seed`. Timing the whole product keeps x at its real size, so the gathers
 * cost what they cost in use. Outputs (host, cap rows each; FFX_EINVAL when
 * cap is below the block count): feat, nblocks x 32 block features as the
 * builder computes them; labels, nblocks x FFX_NUM_FORMATS, log2 of the
 * window's product time per block in microseconds (every block of the window
 * gets the window's label); heur (or NULL), the heuristic's format of each
 * block. *nblocks (when not NULL) receives the block count. Waits for the
 * stream. */
ffx_status ffx_selector_label(int64_t nrows, int64_t ncols, const int64_t* rowptr, const int32_t* colidx,
                              const void* vals, ffx_dtype val_type, uint32_t m, const ffx_build_opts* opts,
                              int32_t reps, uint64_t seed, void* stream, int64_t cap, float* feat, float* labels,
                              int32_t* heur, int64_t* nblocks);

typedef struct {
  uint32_t size;         /* sizeof(ffx_train_opts) */
  int32_t epochs;        /* passes over the training samples; default 60 */
  int32_t batch;         /* samples per Adam step; default 512 */
  float lr;              /* peak rate, decayed as lr * (1 + cos(pi * epoch / epochs)) / 2; default 2e-3 */
  uint64_t seed;         /* initial weights (as ffx_selector_create) and sample order; default 0 */
  int64_t n_val;         /* the first n_val samples are held out; -1 (default): n / 10 */
  int32_t n_margins;     /* candidate decision margins in log2 units; 0 (default): 0, .05, .1, .2, .3, .5 */
  const float* margins;  /* n_margins values (host) */
} ffx_train_opts;

typedef struct {
  double train_loss, val_loss;  /* final masked half mean squared errors, targets relative to STREAM */
  float margin;                 /* the decision margin folded into the output biases */
  double val_cost;              /* held out: summed label time of the network's choices / of the best choices */
  double val_cost_stream;       /* the same for STREAM on every block */
  double val_cost_heuristic;    /* the same for heur (0 when heur is NULL) */
  int32_t steps;                /* Adam steps taken */
} ffx_train_report;

void ffx_train_opts_default(ffx_train_opts* opts);

/* Trains a selector from scratch on n labelled blocks (host arrays): X (n x 32
 * raw features), T (n x FFX_NUM_FORMATS, log2 microseconds as
 * ffx_selector_label writes them), mask (n x FFX_NUM_FORMATS of 0/1, or NULL:
 * every label present), heur (n heuristic formats, or NULL; only reported).
 * The steps, all in the library: input standardisation from the training
 * samples (mean and 1/sd of each feature, scale 1 where sd < 1e-6); targets
 * relative to STREAM (T[., f] - T[., 0]); minibatch Adam on the library's
 * forward/backward kernels with the samples reshuffled every epoch and a
 * cosine-decayed rate; then, on the held-out samples, the decision margin
 * with the least summed label time (a block leaves STREAM only when the
 * network predicts a gain above it), folded into the output biases. The model
 * is written to out_model (when not NULL) and returned in *out (when not
 * NULL; the caller destroys it). FFX_EINVAL for non-finite inputs or options
 * out of range. Waits for the stream. */
ffx_status ffx_selector_train(const float* X, const float* T, const float* mask, const int32_t* heur, int64_t n,
                              const ffx_train_opts* opts, const char* out_model, ffx_selector* out,
                              ffx_train_report* report, void* stream);

/* Install-time tuning of the tile size (Section 2.4, "Heuristic format
 * chooser": the parameters of the formats are tuned for the machine). The
 * matrix (host CSR as to ffx_matrix_create_csr, the rest of the build from
 * opts) is built with each candidate tile_entries (512, 1024, 2048, 4096),
 * and the product with s vectors (s in [1, 16]; int32 residues drawn from
 * seed) is timed on the tiles with HIP events, the median of `reps` launches
 * (1..10000) after two warm-ups. *best_tile_entries receives the fastest;
 * us_out (host, 4 floats, or NULL) the median microseconds of each candidate.
 * The rows per wave are fixed by the formats (one row per lane in SELL slices,
 * 64/s rows per wave in the multi-vector tiles), so the tile size is the
 * shape left to tune. Waits for the stream. */
ffx_status ffx_tune_tile_entries(int64_t nrows, int64_t ncols, const int64_t* rowptr, const int32_t* colidx,
                                 const void* vals, ffx_dtype val_type, uint32_t m, const ffx_build_opts* opts,
                                 int32_t s, int32_t reps, uint64_t seed, void* stream, int32_t* best_tile_entries,
                                 float* us_out);

/* Order basis (sigma-basis) of an m x n power series over the prime field
 * F_p, p < 2^31 (block Wiedemann step 2, Section 3.2; PM-Basis of Giorgi,
 * Jeannerod and Villard 2003 with one-order-at-a-time M-Basis below 32 orders):
 * M (m x m polynomial matrix, degree <= sigma) with M G = 0 mod x^sigma that
 * is reduced with respect to the shifted degrees. At each order the rows are
 * taken by increasing shifted degree (ties by index) and put in echelon form
 * of the residual coefficient; rows that keep a nonzero residual (pivot column:
 * their first nonzero entry) are multiplied by x. The result is exactly that
 * of this process run one order at a time.
 * G (device): entry (r, c) holds sigma coefficients at G + (r*n + c)*ldg,
 * residues in [0, p-1]; ldg >= sigma. shift (host, m): the initial shifted
 * degrees, in [0, 2^28]. M (device): entry (r, c) at M + (r*m + c)*ldm,
 * ldm >= sigma + 1, coefficients beyond the degree zeroed. d_out (host, m):
 * the final shifted degrees. Needs 1 <= n <= m <= 16, n <= 8, p prime
 * (FFX_EINVAL otherwise). Waits for the stream. */
ffx_status ffx_sigma_basis(uint32_t p, int32_t m, int32_t n, int64_t sigma, const uint32_t* G, int64_t ldg,
                           const int32_t* shift, uint32_t* M, int64_t ldm, int32_t* d_out, void* stream);

/* Polynomial matrix products of the order basis whose two operands both have
 * at least min_length coefficients go through number-theoretic transforms
 * over three primes below 2^31 and a CRT (the paper's DFT multiplication,
 * Section 3.2); smaller ones are schoolbook convolutions. Default 1024; 1
 * sends every product through the transforms, 0 none. Process-wide; a tuning
 * knob only: results never depend on it. FFX_EINVAL for a negative value. */
ffx_status ffx_set_ntt_threshold(int64_t min_length);

/* Block Wiedemann steps 2 and 3 (Section 3) on a sequence S_i = U^T A^i V,
 * i < L (as ffx_sequence writes it: device, L x s x s, residues mod the prime
 * p, dtype int32 or int64): the minimal left matrix generator F of the
 * sequence from the order basis of [S(x); -I] with shifts 0 on its first s
 * rows and 1 on the last s (the s rows of smallest shifted degree), and
 *   *rank = deg det F - codeg det F,
 * with deg det F = the sum of F's row degrees (deg_out, host, s entries) and
 * codeg det F its x-adic valuation. With L = 2n/s + O(1) terms, random U and V
 * and A meeting the preconditions of Kaltofen (1991), this is the rank of A.
 * FFX_EUNSUPPORTED when the generator is not row reduced or det F vanishes
 * (sequence too short or degenerate projections). s <= 8. Waits for the
 * stream. */
ffx_status ffx_sequence_rank(uint32_t p, int32_t s, int64_t L, const void* S, ffx_dtype dtype, int32_t* deg_out,
                             int64_t* rank, int64_t* deg_det, int64_t* codeg_det, void* stream);

/* The reordering used by ffx_build_opts.reorder, on the host alone (no GPU
 * call): reverse Cuthill-McKee (Cuthill and McKee 1969, reversed as George
 * 1971) on the pattern of A + A^T of the square n x n pattern (rowptr,
 * colidx), each connected part started from a pseudo-peripheral node (George
 * and Liu 1979), neighbours visited by increasing degree, ties by index.
 * perm (host, n entries) receives perm[new] = old. Section 4 names reordering
 * A as a way to faster products. */
ffx_status ffx_reorder_rcm(int64_t n, const int64_t* rowptr, const int32_t* colidx, int32_t* perm);

/* Time of each row block of A in its stored format, in microseconds per
 * product (host array, nblocks floats): the block's tiles are launched
 * `reps` times over in one grid large enough to fill the GPU, timed with HIP
 * events, and the time divided by the repetitions. x: ncols entries of
 * dtype (device). The outputs written meanwhile are the product's rows. */
ffx_status ffx_matrix_block_times(ffx_matrix A, const void* x, void* y, ffx_dtype dtype, int32_t reps, float* us_out,
                                  void* stream);

/* Calibration of the roofline of the products. A product streams its matrix
 * coalesced and gathers one element (or one row of s elements) of x per entry
 * at the entry's column; Section 2.5 ("Performance issues") names memory
 * access as what limits sparse products, and on MI355X the limit of the large
 * products is the rate at which random gathers are served by the vector L1/L2
 * caches, well before HBM bandwidth. This call measures that rate in the
 * products' pattern: count gathers of row_bytes-byte rows (2, 4, 8, 16, 32 or
 * 64) from a device table of table_bytes bytes, each lane reading a streamed
 * index word and gathering the row it names; indices are uniform over the
 * table (window 0) or uniform inside aligned windows of `window` rows visited
 * in order (the locality of a banded or reordered matrix). *rate (host)
 * receives gathers per second, the median of `reps` launches (1..1000) after
 * a warm-up launch. Allocates and frees its own buffers; waits for the
 * stream. */
ffx_status ffx_gather_rate(int64_t table_bytes, int32_t row_bytes, int64_t count, int64_t window, int32_t reps,
                           void* stream, double* rate);

/* Status name and the calling thread's last error message. */
const char* ffx_status_str(ffx_status st);
const char* ffx_last_error(void);

/* Library version string. */
const char* ffx_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FFX_H */
