// Internal layout shared by the host planner and the gfx950 kernels.
//
// The sparse TTV of Eq. 3 (Sec. 3.3) is computed as a keyed reduction: every
// nonzero becomes a 16-byte record (key, payload) whose key packs the indices
// of the modes that survive the product and whose payload is the product of
// the value with the vector entries of the contracted modes.  Records are
// bucketed by the key's most significant bits (one or more scatter levels),
// every bucket that fits in LDS is sorted there and reduced, and the unique
// keys are unpacked into the output coordinates in lexicographic order.
#pragma once

#include <stdint.h>

#include "ttv.h"

namespace ttv {

constexpr int kWave = 64;
constexpr int kMaxOrder = TTV_MAX_ORDER;
constexpr int kRMax = 12;                // digit bits per bucket level
constexpr int kNDig = 1 << kRMax;        // row stride of the per-tile digit tables
constexpr int kCap = 4096;               // most records an LDS leaf holds
constexpr int kSmall = kCap / 2;         // buckets up to this size are merged into chunks
constexpr int kMaxLevels = 8;            // 64-bit keys with 12-bit digits need at most 6
constexpr int kPureTile = 16384;         // records per block when reducing a single-key bucket
constexpr int kScatterThreads = 256;     // 4 waves
constexpr int kHistThreads = 1024;       // 16 waves
constexpr int kBitmapWordsPerBlock = 2048;  // leaf-start bitmap words per block: 256 threads x 8
constexpr int kHistIPT = 4;
constexpr int kFewTiles = 16;            // deeper-level jobs of at most this many tiles: column scan per thread
constexpr int kScatterIPT = 8;           // records per thread per round
constexpr int kFinishThreads = 512;     // 8 waves
constexpr int kFinishIPT = kCap / kFinishThreads;
constexpr int kSortDigit = 8;            // LDS radix digit width
constexpr int kDenseBits = 12;           // a bucket whose keys span at most this many bits is summed by key
                                         // in LDS (a dense leaf), whatever its size
constexpr int kDenseTile = 16384;        // records of a dense leaf per block of partial sums (larger leaves)
constexpr int kDenseSlotWords = (1 << kDenseBits) + (1 << kDenseBits) / 64;  // sums + presence bits

// Value forms.
enum Form : int32_t {
  kF64 = 0,  // FP64 inputs, FP64 products and sums
  kC32 = 1,  // FP32 inputs, exact FP32 product pairs, Dot2 compensated sums
};

// Where the records of a job or leaf live.
enum Src : int32_t { kSrcRaw = 0, kSrcA = 1, kSrcB = 2 };

// Output / operation modes of the keyed-reduction pipeline.
enum PipeMode : int32_t {
  kPipeTTV = 0,     // sparse output: coordinates + summed values
  kPipeSegMap = 1,  // no values: for every input nonzero, the output row it lands in
  kPipePerm = 2,    // no values: output coordinates, and for every sorted position the
                    // nonzero there (perm_out) and its output row (seg_out)
  kPipeTTVSeg = 3,  // kPipeTTV, and for every input nonzero the output row it lands in
                    // (seg_out): each record's nonzero index travels in a parallel
                    // 4-byte array beside the record buffers
};

// Modes whose records carry products and whose leaves sum them.
__host__ __device__ constexpr bool pm_values(int pm) { return pm == kPipeTTV || pm == kPipeTTVSeg; }

struct Rec {
  uint64_t key;
  uint64_t pay;
};

// Per-tensor description, resident in the workspace.
struct TDesc {
  const void* subs;
  const void* vals;
  const void* vec[kMaxOrder];   // vector of every contracted mode (null elsewhere)
  void* out_subs;               // (nnz_out, nrem) row-major, index dtype of the input
  void* out_vals;               // nnz_out values
  long long* out_nnz;           // device scalar
  int32_t* seg_out;             // output row per nonzero (kPipeSegMap, kPipeTTVSeg); per sorted
                                // position (kPipePerm)
  int32_t* perm_out;            // nonzero per sorted position (kPipePerm)
  const void* segfac;           // optional factor of every payload, gathered through segidx
  const int32_t* segidx;
  long long nnz;
  long long base;               // first record of this tensor in the record buffers
  long long stride_e, stride_j; // subs element (e, j) at subs[e*stride_e + j*stride_j]
  long long dims[kMaxOrder];
  int32_t order;
  int32_t nrem;                 // remaining (kept) modes
  int32_t ncon;                 // contracted modes
  int32_t keybits;
  int32_t rem[kMaxOrder];       // remaining modes, ascending; rem[0] is most significant
  int32_t con[kMaxOrder];       // contracted modes, ascending
  // Keys are mixed-radix: key = sum_i idx(rem[i]) * kstride[i], kstride[nrem-1] = 1,
  // kstride[i] = kstride[i+1] * dims[rem[i+1]] -- dense, and ordered like the tuples.
  unsigned long long kstride[kMaxOrder];
  unsigned long long kmagic[kMaxOrder];  // key / kstride[i] by multiply-high (invariant divisor)
  int32_t ksh1[kMaxOrder];
  int32_t ksh2[kMaxOrder];
  unsigned long long mstride[kMaxOrder];  // per mode: key stride of a remaining mode
  int32_t mrem[kMaxOrder];                // per mode: 1 if the mode remains in the key
  int32_t r1;                   // digit bits of the first level
  int32_t pad0;
  int32_t out_f64;              // compensated form writes FP64 values
  int32_t validate;             // check every index against dims
};

// A bucket that is split by the next digit.
struct Job {
  long long start;        // global record position
  long long size;
  unsigned long long prefix;  // key bits above this job's digit
  long long tile0;        // first tile of this job in the level's tile list
  int32_t ntiles;
  int32_t tensor;
  int32_t shift;          // lowest bit of this job's digit
  int32_t r;              // digit bits
  int32_t src;            // where the records are read from
  int32_t pad;
};

// A range of records reduced by one finishing block.
//   kLeafSort   at most kCap records: LDS radix sort (or sort-free ranks) and segmented sums
//   kLeafPure   one key, more than kCap records: partial sums of kPureTile records, combined
//   kLeafDense  relative keys of 1..kDenseBits bits, more than kCap records: sums by key in LDS;
//               larger than kDenseTile records: per-block partial sums by key, combined
enum LeafKind : int32_t { kLeafSort = 0, kLeafPure = 1, kLeafDense = 2 };
struct Leaf {
  long long start;
  long long size;
  unsigned long long base;  // smallest key of the leaf: relative keys are key - base
  long long ptile0;         // pure / dense leaves: first partial tile
  long long pslot;          // dense leaves: first word of the partial slots in the dense pool
  int32_t nptiles;
  int32_t tensor;
  int32_t kind;
  int32_t src;
  int32_t bits;             // bits of the relative keys
  int32_t pad;
};

// Words of one dense-leaf partial slot: 2^bits FP64 sums, then the presence
// bits of the keys (one u32 per 32 keys, rounded up to whole u64 words).
__host__ __device__ inline long long dense_slot_words(int bits) {
  const long long nk = 1ll << bits;
  return nk + (nk + 63) / 64;
}

// Device-side counters, zeroed by the init kernel of every call.
struct Ctrl {
  int32_t njobs[kMaxLevels + 1];
  int32_t ntiles[kMaxLevels + 1];
  int32_t nleaves;
  int32_t npure;
  int32_t ticket;
  int32_t error;          // first device-side error (TTV_E_* code), 0 if none
  long long total;        // records over all tensors
  int32_t bm_done;        // reserved (zeroed by the init kernel)
  int32_t pad;
  unsigned long long dwords;  // words of the dense pool handed out
};

// Byte offsets of every region inside the caller's workspace.
struct Layout {
  size_t ctrl, desc, jobs, tiles, table, starts, leaves, ordered, status;
  size_t bitmap, wordpre, blockpre, partials, ptile_leaf, dpool, recA, recB, auxA, auxB, end;
  long long jcap, tcap, lcap, pcap, words, wblocks, dpcap;
  int32_t count, levels;
};

// Row class of an index layout: rows of se <= 8 consecutive indices are read
// whole (row-major), anything else column by column.
__host__ __device__ inline bool rows_coalesced(int order, long long se, long long sj) {
  return (order == 1 || sj == 1) && se >= order && se <= kMaxOrder;
}
__host__ __device__ inline int row_width_class(int order, long long se, long long sj) {
  const int need = rows_coalesced(order, se, sj) ? (int)se : order;
  return need <= 3 ? 3 : (need <= 5 ? 5 : kMaxOrder);
}

}  // namespace ttv
