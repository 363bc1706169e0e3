/*
 * ttv.h -- C ABI of the MI355X (gfx950) sparse tensor-times-vector library.
 *
 * The operation is the mode-k product of a sparse d-way tensor with vectors
 * (Harding & Dunlavy, "Improving Runtime Performance of Tensor Computations
 * using Rust From Python", Sec. 3.3, Eq. 3):
 *
 *   (A x_k x)(i_1..i_{k-1}, i_{k+1}..i_d) = sum over i_k of a(i_1..i_d) x(i_k)
 *
 * A sparse tensor is stored in coordinate (COO) form: an nnz x d index array
 * `subs`, an nnz-long value array `vals` and the dimensions `shape` (Sec. 2.1
 * and Sec. 3.3).  The sparse result is returned as the triple the paper's
 * pyttb procedure returns (newsubs, newvals, newshape): the distinct
 * remaining-mode index tuples, sorted lexicographically with the first
 * remaining mode most significant, each with the sum of its products.
 * Multiplying by vectors in n_v modes leaves an order d - n_v tensor
 * (Sec. 3.3); with n_v = d - 1 the result is a dense vector.
 *
 * Conventions for every entry point
 *   - Indices and modes are 0-based.  Duplicate coordinates are allowed and
 *     summed.  Exact-zero sums are kept (coordinates depend on subs only).
 *   - "device" pointers are HIP device memory (or host memory the device can
 *     read); "host" pointers are ordinary host memory read during the call.
 *   - The caller owns every buffer.  The library allocates no device memory
 *     on a call; each call takes a caller-provided workspace whose size the
 *     matching *_workspace query returns.  Workspace contents need no
 *     initialisation and are clobbered by the call.
 *   - Calls are asynchronous on `stream` (0 = the null stream): arguments are
 *     validated synchronously and a negative status is returned before
 *     anything is enqueued.  Device-side failures are reported by
 *     ttv_check_device_error after the work has run.
 *   - Results are deterministic: the same inputs give bitwise-identical
 *     outputs on every run.  No floating-point atomic touches global
 *     memory.  Several kernels add FP64 values into LDS with ds_add_f64
 *     (dense all-but-one and adjoint accumulators, the one-block and
 *     dense-key small paths, leaves whose keys fit 16 bits); their order is
 *     fixed by having a block's waves take turns and by gfx950's LDS serving
 *     the lanes of one instruction that hit the same address in ascending
 *     lane order.  That lane order is measured behaviour of the hardware, not
 *     a documented guarantee; if it failed, those sums would still be
 *     correct but could differ in the last bits between runs.  The sort's
 *     stable ranks use the same property: every sorted leaf checks on the
 *     device that its keys ascend and reports TTV_E_DEVICE otherwise, so a
 *     violation cannot produce unsorted output silently.
 *   - No C++ exception crosses this interface.
 */
#ifndef TTV_H
#define TTV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* ttv_stream_t; /* a hipStream_t */

#define TTV_MAX_ORDER 8

/* Index and value element types. */
enum { TTV_I32 = 0, TTV_I64 = 1 };
enum { TTV_F32 = 0, TTV_F64 = 1 };

/* Status codes (0 = success, negative = error). */
enum {
  TTV_OK = 0,
  TTV_E_NULL = -1,      /* a required pointer is null */
  TTV_E_ORDER = -2,     /* d < 2 or d > TTV_MAX_ORDER */
  TTV_E_MODE = -3,      /* mode / kept mode out of range, or repeated */
  TTV_E_SHAPE = -4,     /* a dimension < 1, or a vector length != its dimension */
  TTV_E_DTYPE = -5,     /* unknown index/value type, or mixed types in a batch */
  TTV_E_KEYBITS = -6,   /* the product of the remaining dimensions exceeds 2^64 */
  TTV_E_WORKSPACE = -7, /* workspace null or smaller than the query says */
  TTV_E_INDEX = -8,     /* (device) an index was out of range (TTV_VALIDATE) */
  TTV_E_HIP = -9,       /* a HIP runtime call failed: see ttv_last_hip_error */
  TTV_E_SIZE = -10,     /* nnz or a dimension exceeds what this build supports */
  TTV_E_DEVICE = -11,   /* (device) an internal bounded wait gave up, a capacity
                           check failed, or a sorted leaf's keys did not ascend */
  TTV_E_ARG = -12       /* any other invalid argument */
};

/* Environment switches, read on every call:
 *   TTV_LOG=1         every plan is printed to stderr (what runs, its sizes,
 *                     digit widths, levels and workspace bytes).
 *   TTV_FAULT=launch  every entry point that launches kernels returns
 *                     TTV_E_HIP (ttv_last_hip_error: hipErrorLaunchFailure)
 *                     once its arguments are validated, touching no device
 *                     memory: a simulated launch failure for callers' tests.
 *   TTV_FAULT=spin    the sorting pipeline's bounded waits give up at their
 *                     first poll: a product whose leaves wait reports
 *                     TTV_E_DEVICE (its output is then undefined, every write
 *                     stays inside the caller's buffers).
 * TTV_FAULT takes a comma-separated list of these names. */

/* Flags. */
#define TTV_VALIDATE 0x1 /* check every index on the device (async, see ttv_check_device_error) */
#define TTV_OUT_F64 0x2  /* FP32 inputs: write FP64 result values instead of FP32 */
#define TTV_DROP_ZEROS 0x4 /* ttv_coo / ttv_coo_multi: remove output rows whose value is exactly 0
                              (the nonzero step of the pyttb procedure, Sec. 3.3); the test is
                              taken on the written value (FP64, or FP32 for FP32 output) and the
                              remaining rows keep their order.  Needs a larger workspace (query
                              with the flag).  Other entry points reject it (TTV_E_ARG). */

/*
 * A COO sparse tensor (Sec. 3.3).  `subs` element (e, j) -- the mode-j index
 * of nonzero e -- is read at subs[e*stride_e + j*stride_j], so row-major
 * (stride_e = order, stride_j = 1) and column-major / structure-of-arrays
 * (stride_e = 1, stride_j = nnz) layouts both work (the paper notes the
 * row- vs column-major difference between its two implementations).
 *
 * value_dtype selects the arithmetic:
 *   TTV_F64: FP64 vals and vectors; each product is rounded once and the
 *            sums are FP64.  Results are FP64.
 *   TTV_F32: FP32 vals and vectors; every product is kept exactly as an FP32
 *            pair (TwoProduct via fmaf).  Sums that run through the sort
 *            (segmented scans over sorted leaves, partial sums of large
 *            single-key buckets, MTTKRP and full-contraction lanes) are
 *            compensated FP32 (Dot2: TwoSum plus an FP32 error term), with
 *            partial sums of one output that cross blocks combined in FP64.
 *            Sums formed by LDS accumulation (the all-but-one product and
 *            the adjoints, the one-block and dense-key small paths, leaves
 *            whose keys fit 16 bits) add the exact product pair widened to
 *            FP64 instead: at least as accurate.  Either way the value is
 *            rounded once to FP32 on output (FP64 with TTV_OUT_F64).
 */
typedef struct {
  int32_t order;        /* d, 2..TTV_MAX_ORDER */
  int32_t index_dtype;  /* TTV_I32 or TTV_I64 */
  int32_t value_dtype;  /* TTV_F32 or TTV_F64 */
  int32_t reserved;     /* set to 0 */
  int64_t nnz;          /* >= 0 */
  int64_t shape[TTV_MAX_ORDER]; /* host values, shape[j] >= 1 for j < order */
  const void* subs;     /* device */
  int64_t stride_e;     /* in elements */
  int64_t stride_j;     /* in elements */
  const void* vals;     /* device, nnz contiguous values */
} ttv_coo_desc;

/* Key layout and pass plan of a product (host only; for tests and logging). */
typedef struct {
  int32_t order, nrem, key_bits, levels;
  int32_t rem_modes[TTV_MAX_ORDER]; /* remaining modes, ascending */
  int32_t bits[TTV_MAX_ORDER];      /* bits of each remaining mode's largest index */
  int64_t stride[TTV_MAX_ORDER];    /* key = sum of index * stride over the remaining modes */
  int32_t digit1_bits;              /* bits of the first bucket level */
  int32_t reserved;
  int64_t workspace_bytes;
} ttv_plan_info;

/* Human-readable text of a status code (static storage). */
const char* ttv_strerror(int status);

/* Library ABI version (major * 10000 + minor * 100 + patch). */
int ttv_version(void);

/* hipError_t of the most recent failing HIP call on this thread (0 if none). */
int ttv_last_hip_error(void);

/*
 * Host-only planning of the product that contracts the modes in `modes`
 * (ncon entries, distinct): which modes remain, how their indices pack into
 * a mixed-radix sort key (first remaining mode most significant, so numeric
 * key order is lexicographic order -- the `unique` step of Sec. 3.3; the key
 * range is the product of the remaining dimensions), how many bucket levels
 * the key needs, and the workspace size.  Touches no device.
 */
int ttv_plan_query(const ttv_coo_desc* X, int32_t ncon, const int32_t* modes,
                   int32_t flags, ttv_plan_info* out);

/* ------------------------------------------------------------------------
 * Sparse TTV in one mode (Eq. 3).
 *   v        device, v_len = shape[mode] values of X's value type
 *   out_subs device, capacity nnz x (d-1) indices of X's index type; row r
 *            holds the remaining-mode indices of output r in ascending mode
 *            order (row-major)
 *   out_vals device, capacity nnz values (FP64 for TTV_F64; FP32 for TTV_F32
 *            unless TTV_OUT_F64, then FP64)
 *   out_nnz  device int64 scalar: the number of output rows (<= nnz)
 *   newshape is shape without `mode` (computed by the caller).
 * ---------------------------------------------------------------------- */
int ttv_coo_workspace(const ttv_coo_desc* X, int32_t mode, int32_t flags, size_t* bytes);
int ttv_coo(const ttv_coo_desc* X, int32_t mode, const void* v, int64_t v_len,
            void* out_subs, void* out_vals, int64_t* out_nnz,
            void* ws, size_t ws_bytes, int32_t flags, ttv_stream_t stream);

/* ------------------------------------------------------------------------
 * Sparse TTV with vectors in several modes (n_v = ncon vectors, Sec. 3.3):
 * the result is sparse of order d - ncon (1 <= ncon <= d - 1).
 *   modes  host, ncon distinct contracted modes
 *   vecs   host array of ncon device pointers, vecs[i] has shape[modes[i]]
 * Output as for ttv_coo with d - ncon index columns.
 * ---------------------------------------------------------------------- */
int ttv_coo_multi_workspace(const ttv_coo_desc* X, int32_t ncon, const int32_t* modes,
                            int32_t flags, size_t* bytes);
int ttv_coo_multi(const ttv_coo_desc* X, int32_t ncon, const int32_t* modes,
                  const void* const* vecs, const int64_t* vec_lens,
                  void* out_subs, void* out_vals, int64_t* out_nnz,
                  void* ws, size_t ws_bytes, int32_t flags, ttv_stream_t stream);

/* ------------------------------------------------------------------------
 * Dense form of a sparse result: the dense conversion of the pyttb procedure
 * (Sec. 3.3), taken when more than half of the result's cells are stored.
 * On the device: if 2 * (*nnz) > prod(shape) and dense_cap >= prod(shape),
 * dense[row-major cell of row r's tuple] = vals[r] for r < *nnz, 0 in every
 * other cell, and *is_dense = 1; otherwise dense is not touched and
 * *is_dense = 0.  No host synchronisation.
 *   order, shape     the result's order (1..TTV_MAX_ORDER) and dimensions
 *   subs, vals, nnz  a sparse result as ttv_coo writes it (device; rows
 *                    distinct, row-major subs of index_dtype, vals of
 *                    value_dtype, device int64 count)
 *   dense            device, dense_cap values of value_dtype (null if 0)
 *   is_dense         device int32
 * ---------------------------------------------------------------------- */
int ttv_result_densify(int32_t order, const int64_t* shape, int32_t index_dtype, int32_t value_dtype,
                       const void* subs, const void* vals, const int64_t* nnz, void* dense,
                       int64_t dense_cap, int32_t* is_dense, ttv_stream_t stream);

/* ------------------------------------------------------------------------
 * Product with a vector in every mode (n_v = d, Sec. 3.3): the scalar
 *   y = sum over nonzeros e of vals[e] * prod_j vecs[j][subs(e, j)]
 * (factors multiplied in ascending mode order).  For d = 1 it is the dot
 * product of a sparse and a dense vector (Sec. 3.1).  1 <= d <= TTV_MAX_ORDER;
 * nnz = 0 gives 0.  The summation order is fixed by nnz alone (bitwise
 * repeatable on any device): a fixed set of waves sums fixed tiles, then a
 * fixed tree; FP64 sums, or for TTV_F32 exact FP32 product pairs with Dot2
 * compensated sums per lane and FP64 from the wave sums on.
 *   vecs, vec_lens  host arrays of d device pointers / lengths (= shape[j])
 *   y        device scalar (FP64; FP32 for TTV_F32 unless TTV_OUT_F64)
 *   ws       workspace of ttv_coo_full_workspace bytes (about 64 KiB)
 * ---------------------------------------------------------------------- */
int ttv_coo_full_workspace(const ttv_coo_desc* X, int32_t flags, size_t* bytes);
int ttv_coo_full(const ttv_coo_desc* X, const void* const* vecs, const int64_t* vec_lens, void* y,
                 void* ws, size_t ws_bytes, int32_t flags, ttv_stream_t stream);

/* ------------------------------------------------------------------------
 * All-but-one product (n_v = d - 1, Sec. 3.3): a dense vector
 *   y[i] = sum over nonzeros e with subs(e, keep) = i of
 *          vals[e] * prod_{j != keep} vecs[j][subs(e, j)]
 * (factors multiplied in ascending mode order).  Entries no nonzero reaches
 * are 0.  No global atomics: every block adds its tiles' products into a
 * private dense FP64 partial in LDS (ds_add_f64 in a fixed order, see the
 * conventions above), and the partials are summed in a fixed block order.
 *   vecs     host array of d device pointers (vecs[keep] is ignored)
 *   vec_lens host array of d lengths (vec_lens[keep] is ignored)
 *   y        device, shape[keep] values (FP64, or FP32 unless TTV_OUT_F64)
 * ---------------------------------------------------------------------- */
int ttv_coo_allbut_workspace(const ttv_coo_desc* X, int32_t keep, int32_t flags, size_t* bytes);
int ttv_coo_allbut(const ttv_coo_desc* X, int32_t keep, const void* const* vecs,
                   const int64_t* vec_lens, void* y,
                   void* ws, size_t ws_bytes, int32_t flags, ttv_stream_t stream);

/* ------------------------------------------------------------------------
 * ttv_coo_allbut without a workspace, for callers that cannot allocate device
 * memory (code under hipGraph capture, tight serving loops, harnesses that
 * forbid allocation).  Same arguments, kernels and result as ttv_coo_allbut
 * (bitwise), except that the scratch (an error word and the blocks' FP64
 * partial sums) lives in a static device array of TTV_NOALLOC_SCRATCH_BYTES
 * that the library holds on every GPU it runs on until the process ends.
 * No allocation, no host synchronisation.  Every call on one GPU shares that
 * array: calls that overlap on one GPU (different streams or threads) race.
 * Returns TTV_E_SIZE when the kept mode is too long for the LDS accumulator
 * (more than about 18000 entries for FP64 int64 row-major input) or the
 * partials would exceed the array, and TTV_E_ARG for TTV_VALIDATE or
 * TTV_DROP_ZEROS.
 * ---------------------------------------------------------------------- */
#define TTV_NOALLOC_SCRATCH_BYTES (48u << 20)
int ttv_coo_allbut_noalloc(const ttv_coo_desc* X, int32_t keep, const void* const* vecs,
                           const int64_t* vec_lens, void* y, int32_t flags, ttv_stream_t stream);

/* ------------------------------------------------------------------------
 * Adjoints (reverse mode).  Eq. 3 is linear in the vector and in vals, so
 *   TTV_BWD_SPARSE  (the product of ttv_coo in mode `mode_or_keep`):
 *     grad_out  device, one value per output row of ttv_coo, in its order
 *     grad_vecs[mode][j] = sum over e with subs(e, mode) = j of vals[e] * g[row(e)]
 *     grad_vals[e]       = v[subs(e, mode)] * g[row(e)]
 *   TTV_BWD_ALLBUT  (the product of ttv_coo_allbut keeping `mode_or_keep`):
 *     grad_out  device, shape[keep] values
 *     grad_vals[e]    = g[subs(e, keep)] * prod_{j != keep} vecs[j][subs(e, j)]
 *     grad_vecs[m][i] = sum over e with subs(e, m) = i of
 *                       vals[e] * g[subs(e, keep)] * prod_{j != keep, m} vecs[j][subs(e, j)]
 *   vecs, vec_lens  as for the forward (host arrays of d entries)
 *   grad_vecs       host array of d device pointers; null entries are skipped
 *   grad_vals       device, nnz values, or null to skip
 * grad_out and every gradient have X's value type (FP32 gradients of the
 * FP32 form are rounded once from compensated / FP64-combined values).
 * ---------------------------------------------------------------------- */
enum { TTV_BWD_SPARSE = 0, TTV_BWD_ALLBUT = 1 };
int ttv_coo_backward_workspace(const ttv_coo_desc* X, int32_t kind, int32_t mode_or_keep,
                               int32_t flags, size_t* bytes);
int ttv_coo_backward(const ttv_coo_desc* X, int32_t kind, int32_t mode_or_keep,
                     const void* const* vecs, const int64_t* vec_lens,
                     const void* grad_out, void* const* grad_vecs, void* grad_vals,
                     void* ws, size_t ws_bytes, int32_t flags, ttv_stream_t stream);

/* ------------------------------------------------------------------------
 * Sparse product and adjoint with the grouping kept between them.  Eq. 3 is
 * linear in v and in vals, so the adjoint of the sparse form needs, for
 * every nonzero e, only row(e): the output row its product is summed into.
 *   ttv_coo_save   ttv_coo in one mode (same arguments, coordinates and
 *                  count; values formed by the sorting pipeline, bitwise
 *                  ttv_coo's wherever ttv_coo sorts, within the rounding
 *                  bound of its small by-key paths) that also writes
 *                  seg[e] = row(e), device int32, nnz entries.  Every
 *                  record's nonzero index travels with it through the sort
 *                  (4 more bytes per record and level).  TTV_DROP_ZEROS is
 *                  refused (TTV_E_ARG): seg names rows before any removal.
 *   ttv_coo_backward_saved  the TTV_BWD_SPARSE adjoint of ttv_coo_backward
 *                  (same arguments and results) with row(e) read from seg
 *                  instead of recomputed by a second sort: one pass over
 *                  the nonzeros.  seg must be what ttv_coo_save wrote for
 *                  the same X and mode; its entries are not checked.
 * ---------------------------------------------------------------------- */
int ttv_coo_save_workspace(const ttv_coo_desc* X, int32_t mode, int32_t flags, size_t* bytes);
int ttv_coo_save(const ttv_coo_desc* X, int32_t mode, const void* v, int64_t v_len,
                 void* out_subs, void* out_vals, int64_t* out_nnz, int32_t* seg,
                 void* ws, size_t ws_bytes, int32_t flags, ttv_stream_t stream);
int ttv_coo_backward_saved_workspace(const ttv_coo_desc* X, int32_t mode, int32_t flags,
                                     size_t* bytes);
int ttv_coo_backward_saved(const ttv_coo_desc* X, int32_t mode, const void* const* vecs,
                           const int64_t* vec_lens, const int32_t* seg, const void* grad_out,
                           void* const* grad_vecs, void* grad_vals,
                           void* ws, size_t ws_bytes, int32_t flags, ttv_stream_t stream);

/* ------------------------------------------------------------------------
 * Batched sparse TTV: `count` independent tensors, each with its own mode
 * and vector, all run by one fixed sequence of persistent kernels.  A plan
 * binds the tensors, vectors and outputs (all device pointers stay fixed) so
 * that ttv_coo_batched does no host synchronisation, no allocation and no
 * host read of device results: it may be captured into a hipGraph and
 * replayed.  All tensors must share index and value types.
 *   Xs        host array of count descriptors
 *   modes     host array of count modes
 *   vs        host array of count device vectors
 *   out_subs, out_vals  host arrays of count device outputs (as ttv_coo)
 *   out_nnz   device array of count int64 results
 *   tune_cache  path of the autotuner's JSON cache, or null
 * ttv_batch_autotune times candidate tile sizes and digit widths on the
 * bound batch (running it several times on `stream` and synchronising),
 * keeps the fastest in the plan and records it in the cache file.
 * ---------------------------------------------------------------------- */
typedef struct ttv_batch_plan ttv_batch_plan;
int ttv_batch_plan_create(int32_t count, const ttv_coo_desc* Xs, const int32_t* modes,
                          const void* const* vs, void* const* out_subs,
                          void* const* out_vals, int64_t* out_nnz, int32_t flags,
                          const char* tune_cache, ttv_batch_plan** plan);
int ttv_batch_workspace(const ttv_batch_plan* plan, size_t* bytes);
int ttv_batch_autotune(ttv_batch_plan* plan, void* ws, size_t ws_bytes, ttv_stream_t stream);
int ttv_coo_batched(const ttv_batch_plan* plan, void* ws, size_t ws_bytes, ttv_stream_t stream);
void ttv_batch_plan_destroy(ttv_batch_plan* plan);

/* ------------------------------------------------------------------------
 * Repeated TTV with a fixed tensor and mode (Eq. 3 applied to a new vector
 * each call, as iterative methods do).  The keyed sort runs once, in setup;
 * every apply is then one streaming pass over the nonzeros in output order
 * (product and segmented sum), without sorting.
 *   ttv_reuse_plan_create  host only: validates X and mode (as ttv_coo) and
 *                          sizes the buffers; X's arrays must stay valid until
 *                          setup has run on the stream.
 *   ttv_reuse_sizes        bytes of the persistent plan buffer `data` (kept
 *                          by the caller as long as the plan is applied) and
 *                          of the setup workspace (free after setup).
 *   ttv_reuse_setup        sorts X: writes the output coordinates out_subs
 *                          (capacity nnz x (d-1), X's index type) and out_nnz
 *                          (device int64), and fills `data` with the values
 *                          and contracted-mode indices in output order
 *                          (indices as uint32 when the mode's length is at
 *                          most 2^32), one bit per position marking where an
 *                          output row starts, and each 512-position chunk's
 *                          first row: about 8 + 4 + 1/8 bytes per nonzero for
 *                          FP64 values.  Device errors are read with
 *                          ttv_check_device_error(ws, stream).
 *   ttv_reuse_apply        out_vals[r] = output row r of ttv_coo(X, mode, v)
 *                          (capacity nnz values: FP64, or FP32 for TTV_F32
 *                          unless the plan was made with TTV_OUT_F64).  Reads
 *                          only `data` and v; no workspace, no allocation, no
 *                          host synchronisation.  Each sum is formed in one
 *                          fixed order (bitwise repeatable), not ttv_coo's.
 * ---------------------------------------------------------------------- */
typedef struct ttv_reuse_plan ttv_reuse_plan;
int ttv_reuse_plan_create(const ttv_coo_desc* X, int32_t mode, int32_t flags, ttv_reuse_plan** plan);
int ttv_reuse_sizes(const ttv_reuse_plan* plan, size_t* data_bytes, size_t* setup_ws_bytes);
int ttv_reuse_setup(ttv_reuse_plan* plan, void* data, size_t data_bytes, void* out_subs,
                    int64_t* out_nnz, void* ws, size_t ws_bytes, ttv_stream_t stream);
int ttv_reuse_apply(const ttv_reuse_plan* plan, const void* v, int64_t v_len, void* out_vals,
                    ttv_stream_t stream);
void ttv_reuse_plan_destroy(ttv_reuse_plan* plan);

/* ------------------------------------------------------------------------
 * Sparse MTTKRP (the matricized tensor times Khatri-Rao product the paper
 * names as its next target; it extends Eq. 3's per-nonzero product to one
 * factor row per mode):
 *   M[i, r] = sum over nonzeros e with subs(e, mode) = i of
 *             vals[e] * prod_{j != mode} U_j[subs(e, j), r]      (r < R)
 * (factors multiplied in ascending mode order), a dense shape[mode] x R
 * row-major matrix; rows no nonzero reaches are 0.  The tensor is fixed
 * across calls, as in CP-ALS: the sort by the mode's index runs once.
 *   ttv_mttkrp_plan_create  host only: validates X (as ttv_coo, d >= 2), mode
 *                           and 1 <= R <= 256; every other mode's length must
 *                           be at most 2^32 (TTV_E_SIZE).  X's arrays must stay
 *                           valid until setup has run on the stream.
 *   ttv_mttkrp_sizes        bytes of the persistent plan buffer `data` (about
 *                           8 + 4 (d-1) + 1/8 bytes per nonzero for FP64
 *                           values, plus 8 R + 16 bytes per 128 nonzeros) and
 *                           of the setup workspace (free after setup).
 *   ttv_mttkrp_setup        sorts X by the mode's index and fills `data`;
 *                           synchronises the stream once at its end (to learn
 *                           whether any row spans more than 32 units of 128
 *                           nonzeros).  Device errors (TTV_VALIDATE) are read
 *                           with ttv_check_device_error(ws, stream).
 *   ttv_mttkrp_apply        factors: host array of d device pointers, factor
 *                           j is shape[j] x R row-major of X's value type
 *                           (factors[mode] is ignored); M: device, shape[mode]
 *                           x R values (FP64, or FP32 for TTV_F32 unless the
 *                           plan was made with TTV_OUT_F64).  FP64 sums, or
 *                           compensated (Dot2) FP32 sums per row segment with
 *                           FP64 across segments.  Every sum has one fixed
 *                           order (bitwise repeatable).  No allocation, no
 *                           host synchronisation.  Applies on one plan share
 *                           its buffer: calls that overlap on different
 *                           streams race.
 * ---------------------------------------------------------------------- */
typedef struct ttv_mttkrp_plan ttv_mttkrp_plan;
int ttv_mttkrp_plan_create(const ttv_coo_desc* X, int32_t mode, int32_t R, int32_t flags,
                           ttv_mttkrp_plan** plan);
int ttv_mttkrp_sizes(const ttv_mttkrp_plan* plan, size_t* data_bytes, size_t* setup_ws_bytes);
int ttv_mttkrp_setup(ttv_mttkrp_plan* plan, void* data, size_t data_bytes, void* ws, size_t ws_bytes,
                     ttv_stream_t stream);
int ttv_mttkrp_apply(const ttv_mttkrp_plan* plan, const void* const* factors, void* M, ttv_stream_t stream);
void ttv_mttkrp_plan_destroy(ttv_mttkrp_plan* plan);

/*
 * Measurement hook.  While set, the library records the caller's HIP events
 * starts[k] / stops[k] on the launch stream around the k-th launch of one of
 * its kernels (k counts up to `capacity`, further launches are not
 * recorded), so a benchmark can time that kernel inside its timed region.
 * kernel: TTV_PROF_NONE disables; TTV_PROF_FINISH the leaf sort-reduce-write
 * kernel; TTV_PROF_SCATTER1 the first-level bucket scatter; TTV_PROF_HIST1
 * its histogram; TTV_PROF_DENSE the dense accumulation kernel;
 * TTV_PROF_REUSE the streaming kernel of ttv_reuse_apply; TTV_PROF_FULL the
 * streaming kernel of ttv_coo_full; TTV_PROF_MTTKRP the streaming kernel of
 * ttv_mttkrp_apply.  Not thread-safe;
 * for measurement only.  ttv_profile_count returns k.
 */
enum {
  TTV_PROF_NONE = 0,
  TTV_PROF_FINISH = 1,
  TTV_PROF_SCATTER1 = 2,
  TTV_PROF_HIST1 = 3,
  TTV_PROF_DENSE = 4,
  TTV_PROF_REUSE = 5,
  TTV_PROF_FULL = 6,
  TTV_PROF_MTTKRP = 7
};
int ttv_profile_events(int32_t kernel, void* const* starts, void* const* stops, int32_t capacity);
int ttv_profile_count(void);

/*
 * Synchronises `stream` and returns the first device-side error recorded in
 * workspace `ws` by the last call that used it (TTV_OK if none), e.g.
 * TTV_E_INDEX for an out-of-range index under TTV_VALIDATE.
 */
int ttv_check_device_error(const void* ws, ttv_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* TTV_H */
