// Keyed-reduction pipeline for sparse TTV on gfx950 (Eq. 3, Sec. 3.3).
//
// The pyttb procedure the paper times finds the modes left after the
// product (a set difference), gathers the unique tuples of their indices,
// accumulates the products onto those tuples and returns the triple
// (newsubs, newvals, newshape).  Here the same result is built from:
//
//   level l = 1..L      hist -> colscan -> classify -> scatter
//       Records (key, payload) are scattered into buckets by the next
//       kRMax-bit digit of the key (level 1 reads the COO input directly and
//       forms key and payload on the fly).  Buckets that fit in LDS become
//       leaves (small neighbours are merged into chunks); larger ones are
//       split again at the next level; a bucket whose key is fully fixed is
//       a single output row (a "pure" leaf).
//   pure reduce         multi-block partial sums of the large single-key leaves
//   bitmap scan + rank  leaves are numbered in key order (their start offsets)
//   finish              one block per leaf, taken in key order: LDS radix sort
//                       of the relative keys, segmented reduction, decoupled
//                       look-back over the leaves for the output offsets, and
//                       the unpacked coordinates and values are written.
//
// Every placement is computed from integer counts and a fixed block order,
// so the result is bitwise deterministic.
#include <hip/hip_runtime.h>

#include "ttv_device.hpp"
#include "ttv_host.h"

namespace ttv {

struct WsView {
  char* b;
  Layout L;
  __device__ __forceinline__ Ctrl* ctrl() const { return reinterpret_cast<Ctrl*>(b + L.ctrl); }
  __device__ __forceinline__ TDesc* desc() const { return reinterpret_cast<TDesc*>(b + L.desc); }
  __device__ __forceinline__ Job* jobs(int level) const {
    return reinterpret_cast<Job*>(b + L.jobs) + (size_t)(level - 1) * L.jcap;
  }
  __device__ __forceinline__ int* tiles(int level) const {
    return reinterpret_cast<int*>(b + L.tiles) + (size_t)(level - 1) * L.tcap;
  }
  __device__ __forceinline__ unsigned* table() const { return reinterpret_cast<unsigned*>(b + L.table); }
  __device__ __forceinline__ unsigned* starts() const { return reinterpret_cast<unsigned*>(b + L.starts); }
  __device__ __forceinline__ Leaf* leaves() const { return reinterpret_cast<Leaf*>(b + L.leaves); }
  __device__ __forceinline__ Leaf* ordered() const { return reinterpret_cast<Leaf*>(b + L.ordered); }
  __device__ __forceinline__ unsigned long long* status() const {
    return reinterpret_cast<unsigned long long*>(b + L.status);
  }
  __device__ __forceinline__ unsigned* bitmap() const { return reinterpret_cast<unsigned*>(b + L.bitmap); }
  __device__ __forceinline__ unsigned* wordpre() const { return reinterpret_cast<unsigned*>(b + L.wordpre); }
  __device__ __forceinline__ unsigned* blockpre() const { return reinterpret_cast<unsigned*>(b + L.blockpre); }
  __device__ __forceinline__ double* partials() const { return reinterpret_cast<double*>(b + L.partials); }
  __device__ __forceinline__ int* ptile_leaf() const { return reinterpret_cast<int*>(b + L.ptile_leaf); }
  __device__ __forceinline__ unsigned long long* dpool() const {
    return reinterpret_cast<unsigned long long*>(b + L.dpool);
  }
  __device__ __forceinline__ Rec* rec(int src) const {
    return reinterpret_cast<Rec*>(b + (src == kSrcA ? L.recA : L.recB));
  }
  // nonzero index of every record, beside rec(src) (kPipeTTVSeg)
  __device__ __forceinline__ int32_t* aux(int src) const {
    return reinterpret_cast<int32_t*>(b + (src == kSrcA ? L.auxA : L.auxB));
  }
};

__device__ __forceinline__ int dst_of(int level) { return (level & 1) ? kSrcA : kSrcB; }

// A capacity violation (which the workspace bounds rule out) stops all later
// kernels of the call instead of letting them read unwritten records.
__device__ __forceinline__ bool aborted(const Ctrl* C) { return C->error == TTV_E_DEVICE; }
__device__ __forceinline__ int clampi(long long v, long long cap) { return (int)(v < cap ? v : cap); }


#ifdef TTV_PHASE_PROFILE
// Build-time option for kernel phase timing (wall clock, 100 MHz ticks).
__device__ unsigned long long g_phase[16];
#define TTV_PHASE_DECL unsigned long long ph_t = wall_clock64();
#define TTV_PHASE(i)                                             \
  if (threadIdx.x == 0) {                                        \
    const unsigned long long ph_n = wall_clock64();              \
    atomicAdd(&g_phase[i], ph_n - ph_t);                         \
    ph_t = ph_n;                                                 \
  }
extern "C" int ttv_debug_phases(unsigned long long* out) {
  return (int)hipMemcpyFromSymbol(out, HIP_SYMBOL(g_phase), sizeof(g_phase));
}
extern "C" int ttv_debug_phases_reset() {
  unsigned long long z[16] = {0};
  return (int)hipMemcpyToSymbol(HIP_SYMBOL(g_phase), z, sizeof(z));
}
#define TTV_COUNT(i) \
  if (threadIdx.x == 0) atomicAdd(&g_phase[i], 1ull);
__device__ unsigned long long g_phase2[16];
#define TTV_PHASE2(i)                                            \
  if (threadIdx.x == 0) {                                        \
    const unsigned long long ph_n = wall_clock64();              \
    atomicAdd(&g_phase2[i], ph_n - ph_t);                        \
    ph_t = ph_n;                                                 \
  }
extern "C" int ttv_debug_phases2(unsigned long long* out) {
  return (int)hipMemcpyFromSymbol(out, HIP_SYMBOL(g_phase2), sizeof(g_phase2));
}
extern "C" int ttv_debug_phases2_reset() {
  unsigned long long z[16] = {0};
  return (int)hipMemcpyToSymbol(HIP_SYMBOL(g_phase2), z, sizeof(z));
}
// look-back statistics per leaf kind k (0 dense, 1 pure, 2 sort-free, 3
// sorted): wall time at slot 5 + k, polling rounds at 9 + k; steps at 13,
// look-backs at 14, look-backs that polled at 15
#define TTV_LB_DECL                                 \
  const unsigned long long lb_t0 = wall_clock64(); \
  unsigned lb_steps = 0, lb_waits = 0;
#define TTV_LB_STEP ++lb_steps;
#define TTV_LB_WAIT ++lb_waits;
#define TTV_LB_END(k)                                                  \
  if (lane_id() == 0) {                                                \
    atomicAdd(&g_phase2[5 + (k)], wall_clock64() - lb_t0);            \
    atomicAdd(&g_phase2[9 + (k)], (unsigned long long)lb_waits);      \
    atomicAdd(&g_phase2[13], (unsigned long long)lb_steps);           \
    atomicAdd(&g_phase2[14], 1ull);                                    \
    if (lb_waits) atomicAdd(&g_phase2[15], 1ull);                      \
  }
#else
#define TTV_PHASE_DECL
#define TTV_PHASE(i)
#define TTV_COUNT(i)
#define TTV_PHASE2(i)
#define TTV_LB_DECL
#define TTV_LB_STEP
#define TTV_LB_WAIT
#define TTV_LB_END(k)
#endif

constexpr unsigned long long kFlagAgg = 1ull << 62;
constexpr unsigned long long kFlagInc = 2ull << 62;
constexpr unsigned long long kValMask = (1ull << 62) - 1;
constexpr int kClassifySlices = 16;           // blocks per level-1 job in classify

// ---------------------------------------------------------------------------
// Records from the COO input: key = remaining-mode indices packed with the
// first remaining mode most significant; payload = value times the vector
// entries of the contracted modes (ascending), or the nonzero's index.
// ---------------------------------------------------------------------------
// What a tile needs to read nonzeros of one tensor, staged in LDS once per
// tile (descriptor fields read from global memory would be fetched again
// after every store).
template <typename IdxT, int F, int MO>
struct RawSrc {
  using In = typename FormOps<F>::In;
  const IdxT* subs;
  const In* vals;
  long long se;
  long long sj;        // stride between the indices of one nonzero
  int order;
  int validate;
  int rowmajor;        // rows of se <= kMaxOrder consecutive indices: read whole rows, coalesced
  unsigned remmask;    // bit m: mode m remains in the key
  const In* vec[MO];
  long long dim[MO];
  unsigned long long kst[MO];  // key stride of a remaining mode
  const In* segfac;
  const int32_t* segidx;
  __device__ __forceinline__ bool rem(int m) const { return (remmask >> m) & 1u; }
  __device__ __forceinline__ void set(const TDesc& D) {
    subs = static_cast<const IdxT*>(D.subs);
    vals = static_cast<const In*>(D.vals);
    segfac = static_cast<const In*>(D.segfac);
    segidx = D.segidx;
    se = D.stride_e;
    sj = D.stride_j;
    order = D.order;
    validate = D.validate;
    rowmajor = rows_coalesced(D.order, D.stride_e, D.stride_j);
    remmask = 0;
#pragma unroll
    for (int m = 0; m < MO; ++m) {
      vec[m] = static_cast<const In*>(D.vec[m]);
      dim[m] = D.dims[m];
      kst[m] = D.mstride[m];
      remmask |= (D.mrem[m] ? 1u : 0u) << m;
    }
  }
};

// The index columns of one round: item j of this lane is nonzero
// r0 + j*64 + lane, valid while j*64 + lane < nrec (r0 is the first nonzero of
// the wave's slice).  x[m][j] holds mode m's index (0 for m >= order or an
// invalid item).
//   Row-major rows (se consecutive indices per nonzero): the wave reads its
//   slice as consecutive words (every lane one word per load, so a load covers
//   whole cache lines) and transposes 64 rows at a time through its LDS stage
//   (64*MO words).  A lane reading its own row directly would touch 64 rows'
//   worth of lines per load for one index each, which caps the read rate well
//   below HBM bandwidth.
//   Other strides (structure of arrays): one load per mode, lane-consecutive.
template <typename IdxT, int F, int IPT, int MO, typename Fn>
__device__ __forceinline__ void for_cols(const RawSrc<IdxT, F, MO>& S, long long r0, long long nrec, IdxT* stage,
                                         Fn&& f) {
  for_rows<IdxT, IPT, MO>(S.subs, S.se, S.sj, S.order, S.rowmajor != 0, r0, nrec, stage, f);
}

template <typename IdxT, int F, int IPT, int MO>
__device__ __forceinline__ void fetch_cols(const RawSrc<IdxT, F, MO>& S, long long r0, long long nrec, IdxT* stage,
                                           long long (&x)[MO][IPT]) {
#pragma unroll
  for (int m = 0; m < MO; ++m)
#pragma unroll
    for (int j = 0; j < IPT; ++j) x[m][j] = 0;
  for_cols<IdxT, F, IPT, MO>(S, r0, nrec, stage, [&](int m, int j, long long v) { x[m][j] = v; });
}

// One round of IPT records per lane (as fetch_cols): key and payload.  The
// index columns come in first, then the vector entries of the contracted modes
// are gathered together (a second memory round trip).
template <typename IdxT, int F, int PM, int IPT, int MO>
__device__ __forceinline__ void load_round(const RawSrc<IdxT, F, MO>& S, long long r0, long long nrec, IdxT* stage,
                                           Ctrl* C, uint64_t (&key)[IPT], uint64_t (&pay)[IPT]) {
  using FO = FormOps<F>;
  using In = typename FO::In;
  const gptr<const In> vals = to_global(S.vals);
  const unsigned ln = lane_id();
  const int order = S.order;
  In a[IPT];
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const long long i = (long long)j * 64 + ln;
    a[j] = (pm_values(PM) && i < nrec) ? vals[r0 + i] : (In)0;
  }
  long long x[MO][IPT];
  fetch_cols<IdxT, F, IPT, MO>(S, r0, nrec, stage, x);
  if (S.validate) {
#pragma unroll
    for (int m = 0; m < MO; ++m)
#pragma unroll
      for (int j = 0; j < IPT; ++j)
        if (m < order && (long long)j * 64 + ln < nrec && (x[m][j] < 0 || x[m][j] >= S.dim[m])) {
          set_error(C, TTV_E_INDEX);
          x[m][j] = 0;
        }
  }
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    key[j] = 0;
    pay[j] = !pm_values(PM) ? (uint64_t)(r0 + (long long)j * 64 + ln) : FO::start_prod(a[j]);
  }
#pragma unroll
  for (int m = 0; m < MO; ++m) {
    if (m >= order) break;
    if (S.rem(m)) {
      const unsigned long long st = S.kst[m];
#pragma unroll
      for (int j = 0; j < IPT; ++j) key[j] += (uint64_t)x[m][j] * st;
    }
  }
  if (!pm_values(PM)) return;
  In g[MO][IPT];
#pragma unroll
  for (int m = 0; m < MO; ++m) {
    const bool use = m < order && !S.rem(m) && S.vec[m] != nullptr;
    const gptr<const In> vec = to_global(S.vec[m]);
#pragma unroll
    for (int j = 0; j < IPT; ++j) g[m][j] = (use && (long long)j * 64 + ln < nrec) ? vec[x[m][j]] : (In)1;
  }
#pragma unroll
  for (int m = 0; m < MO; ++m) {
    if (m >= order) break;
    if (!S.rem(m) && S.vec[m]) {
#pragma unroll
      for (int j = 0; j < IPT; ++j) pay[j] = FO::mul_prod(pay[j], g[m][j]);
    }
  }
  if (S.segfac) {
    const gptr<const In> sf = to_global(S.segfac);
    const gptr<const int32_t> sx = to_global(S.segidx);
    In h[IPT];
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      const long long i = (long long)j * 64 + ln;
      h[j] = i < nrec ? sf[sx[r0 + i]] : (In)0;
    }
#pragma unroll
    for (int j = 0; j < IPT; ++j) pay[j] = FO::mul_prod(pay[j], h[j]);
  }
}

// ---------------------------------------------------------------------------
// init: descriptors, counters, level-1 jobs and tiles, zeroed leaf bitmap
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_init(WsView W, TDesc d0, const TDesc* descs_in, int count,
                                              int T1) {
  const long long words = W.L.words;
  unsigned* bm = W.bitmap();
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < words;
       i += (long long)gridDim.x * blockDim.x)
    bm[i] = 0u;
  if (blockIdx.x != 0) return;
  TDesc* D = W.desc();
  Ctrl* C = W.ctrl();
  if (descs_in == nullptr) {
    if (threadIdx.x == 0) D[0] = d0;
  } else {
    for (int t = threadIdx.x; t < count; t += blockDim.x) D[t] = descs_in[t];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < count; t += blockDim.x)
    if (D[t].out_nnz) *D[t].out_nnz = 0;
  if (threadIdx.x == 0) {
    for (int l = 0; l <= kMaxLevels; ++l) {
      C->njobs[l] = 0;
      C->ntiles[l] = 0;
    }
    C->nleaves = 0;
    C->npure = 0;
    C->ticket = 0;
    C->bm_done = 0;
    C->error = 0;
    C->dwords = 0;
  }
  // level-1 jobs (one per nonempty tensor) and their tiles, in tensor order:
  // job and first-tile offsets from block scans over chunks of 256 tensors
  __shared__ unsigned wsum[256 / 64];
  __shared__ unsigned s_tex[256 + 1];  // first tile of every tensor of the chunk (chunk-relative)
  __shared__ int s_job[256];           // its job (-1: empty tensor)
  __shared__ long long s_tile;
  __shared__ int s_nj;
  __shared__ unsigned long long s_total;
  if (threadIdx.x == 0) {
    s_tile = 0;
    s_nj = 0;
    s_total = 0;
  }
  __syncthreads();
  Job* J1 = W.jobs(1);
  for (int c0 = 0; c0 < count; c0 += 256) {
    const int t = c0 + (int)threadIdx.x;
    const long long nnz = t < count ? D[t].nnz : 0;
    const bool ok = nnz > 0;
    const unsigned nt = ok ? (unsigned)((nnz + T1 - 1) / T1) : 0u;
    unsigned ntot, jtot;
    const unsigned tex = block_excl_scan<256>(nt, wsum, ntot);
    const unsigned jex = block_excl_scan<256>(ok ? 1u : 0u, wsum, jtot);
    if (nnz > 0) atomicAdd(&s_total, (unsigned long long)nnz);
    if (ok) {
      Job J;
      J.start = D[t].base;
      J.size = nnz;
      J.prefix = 0;
      J.tile0 = s_tile + tex;
      J.ntiles = (int)nt;
      J.tensor = t;
      J.shift = D[t].keybits - D[t].r1;
      J.r = D[t].r1;
      J.src = kSrcRaw;
      J.pad = 0;
      J1[s_nj + (int)jex] = J;
    }
    s_tex[threadIdx.x] = tex;
    s_job[threadIdx.x] = ok ? s_nj + (int)jex : -1;
    if (threadIdx.x == 0) s_tex[256] = ntot;
    __syncthreads();
    // the chunk's tiles, one per thread: its tensor by binary search on the
    // first tiles (empty tensors own no tile)
    int* T = W.tiles(1);
    for (unsigned k = threadIdx.x; k < ntot; k += 256) {
      int lo = 0, hi = 255;  // last tensor whose first tile is <= k and that owns tiles
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_tex[mid] <= k)
          lo = mid;
        else
          hi = mid - 1;
      }
      // (the largest such tensor owns tile k: an empty one would share its
      // first tile with the next, so it cannot be the largest)
      T[s_tile + k] = s_job[lo];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      s_tile += ntot;
      s_nj += (int)jtot;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    C->njobs[1] = s_nj;
    C->ntiles[1] = (int)s_tile;
    C->total = (long long)s_total;
  }
}

// LDS histogram add; a wave whose valid lanes share one digit adds once.
__device__ __forceinline__ void hist_add(unsigned* hist, unsigned d, bool valid) {
  const uint64_t vm = ballot(valid);
  if (vm == 0) return;
  const int first = __ffsll((long long)vm) - 1;
  const unsigned d0 = __shfl(d, first, 64);
  const uint64_t same = ballot(valid && d == d0);
  if (same == vm) {
    if ((int)lane_id() == first) atomicAdd(&hist[d0], (unsigned)__popcll(vm));
  } else if (valid) {
    atomicAdd(&hist[d], 1u);
  }
}

// ---------------------------------------------------------------------------
// hist: per-tile digit counts -> table[tile][digit]
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// hist: per-tile digit counts -> table[tile][digit]
// ---------------------------------------------------------------------------
template <typename IdxT, int MO>
__global__ __launch_bounds__(kHistThreads) void k_hist(WsView W, int level, int T) {
  constexpr int NT = kHistThreads;
  constexpr int IPT = MO <= 3 ? kHistIPT : (MO <= 5 ? 3 : 2);  // rows per lane per round within 128 VGPRs
  __shared__ unsigned hist[kNDig];
  __shared__ IdxT stage[NT / 64][64 * MO];
  __shared__ RawSrc<IdxT, kF64, MO> rsrc;
  Ctrl* C = W.ctrl();
  if (aborted(C)) return;
  const int ntiles = clampi(C->ntiles[level], W.L.tcap);
  const Job* jobs = W.jobs(level);
  const int* tj = W.tiles(level);
  unsigned* table = W.table();
  const int w = threadIdx.x >> 6;
  const unsigned ln = lane_id();
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const Job J = jobs[tj[t]];
    const int nd = 1 << J.r;
    const unsigned mask = (unsigned)nd - 1u;
    for (int i = threadIdx.x; i < nd; i += NT) hist[i] = 0u;
    const TDesc* Dp = W.desc() + J.tensor;
    if (threadIdx.x == 0 && J.src == kSrcRaw) rsrc.set(*Dp);
    __syncthreads();
    const RawSrc<IdxT, kF64, MO>& S = rsrc;
    const long long b = (long long)(t - J.tile0) * T;
    const long long n = (J.size - b < (long long)T) ? J.size - b : (long long)T;
    const long long roff = J.start - Dp->base + b;
    // keys of bucketed records: the first word of each 16-byte record
    const gptr<const uint64_t> srcK = (J.src == kSrcRaw)
                                          ? (gptr<const uint64_t>)nullptr
                                          : to_global((const uint64_t*)W.rec(J.src)) + 2 * (J.start + b);
    // rounds of NT*IPT records; wave w takes a contiguous 64*IPT slice
    for (long long rb = 0; rb < n; rb += NT * IPT) {
      const long long s0 = rb + (long long)w * 64 * IPT;
      const long long i0 = s0 + ln;
      uint64_t key[IPT];
      if (srcK) {
#pragma unroll
        for (int j = 0; j < IPT; ++j) key[j] = (i0 + j * 64 < n) ? srcK[2 * (i0 + j * 64)] : 0;
      } else {
#pragma unroll
        for (int j = 0; j < IPT; ++j) key[j] = 0;
        for_cols<IdxT, kF64, IPT, MO>(S, roff + s0, n - s0, stage[w], [&](int m, int j, long long v) {
          if (!S.rem(m)) return;
          // out-of-range indices count as 0 here; the scatter reports them
          if (S.validate && (v < 0 || v >= S.dim[m])) v = 0;
          key[j] += (uint64_t)v * S.kst[m];
        });
      }
#pragma unroll
      for (int j = 0; j < IPT; ++j) {
        const bool valid = i0 + j * 64 < n;
        hist_add(hist, (unsigned)(key[j] >> J.shift) & mask, valid);
      }
    }
    __syncthreads();
    unsigned* row = table + (size_t)t * kNDig;
    for (int i = threadIdx.x; i < nd; i += NT) row[i] = hist[i];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// colscan: for every (job, digit) the exclusive prefix of the counts over the
// job's tiles, in tile order (in place); digit totals go to starts[job].
// Block = 64 digits x 16 tile groups.
// ---------------------------------------------------------------------------
// Column scan of one 64-digit chunk of job j: the tiles split in 16 groups,
// each group sums its tiles' counts, then every group rewrites its tiles'
// counts as running offsets (exclusive, in tile order); starts gets the
// digit totals.
__device__ __forceinline__ void colscan_chunk(WsView W, const Job& J, int j, int ch, unsigned (&part)[16][64]) {
  unsigned* table = W.table();
  const int dd = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int nd = 1 << J.r;
  const int d = ch * 64 + dd;
  const bool act = d < nd;
  const int per = (J.ntiles + 15) / 16;
  const long long t0 = J.tile0 + (long long)g * per;
  long long t1 = t0 + per;
  if (t1 > J.tile0 + J.ntiles) t1 = J.tile0 + J.ntiles;
  unsigned s = 0;
  if (act) {
#pragma unroll 8
    for (long long t = t0; t < t1; ++t) s += table[(size_t)t * kNDig + d];
  }
  part[g][dd] = s;
  __syncthreads();
  unsigned off = 0, tot = 0;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const unsigned v = part[q][dd];
    off += (q < g) ? v : 0u;
    tot += v;
  }
  if (act) {
    unsigned run = off;
    for (long long t = t0; t < t1; ++t) {
      unsigned* p = &table[(size_t)t * kNDig + d];
      const unsigned c = *p;
      *p = run;
      run += c;
    }
    if (g == 0) W.starts()[(size_t)j * kNDig + d] = tot;
  }
  __syncthreads();
}

// Column scan of one job of at most kFewTiles tiles: one digit column per
// thread, its tiles in order.
__device__ __forceinline__ void colscan_serial(WsView W, const Job& J, int j) {
  unsigned* table = W.table();
  const int nd = 1 << J.r;
  for (int d = threadIdx.x; d < nd; d += blockDim.x) {
    unsigned c[kFewTiles];
#pragma unroll
    for (int k = 0; k < kFewTiles; ++k) c[k] = k < J.ntiles ? table[(size_t)(J.tile0 + k) * kNDig + d] : 0u;
    unsigned run = 0;
#pragma unroll
    for (int k = 0; k < kFewTiles; ++k)
      if (k < J.ntiles) {
        table[(size_t)(J.tile0 + k) * kNDig + d] = run;
        run += c[k];
      }
    W.starts()[(size_t)j * kNDig + d] = run;
  }
}

// Per-(tile, digit) bucket offsets and per-job digit totals.  A single
// tensor's first level is one job of many tiles: items are its 64-digit
// chunks.  Otherwise (deeper levels, and the first level of a batch) jobs of
// few tiles take one block each; the jobs with more tiles are listed per
// batch of 1024 jobs and their (job, chunk) items spread over the blocks.
__global__ __launch_bounds__(1024) void k_colscan(WsView W, int level) {
  __shared__ unsigned part[16][64];
  __shared__ int bigs[1024];
  __shared__ unsigned wsum[1024 / 64];
  Ctrl* C = W.ctrl();
  if (aborted(C)) return;
  const int njobs = clampi(C->njobs[level], W.L.jcap);
  const Job* jobs = W.jobs(level);
  if (level == 1 && njobs == 1) {  // one tensor: its many tiles in (64-digit chunk) items
    const Job J = jobs[0];
    for (int ch = blockIdx.x; ch < 64; ch += gridDim.x)
      if (ch * 64 < (1 << J.r)) colscan_chunk(W, J, 0, ch, part);  // uniform over the block
    return;
  }
  for (int j = blockIdx.x; j < njobs; j += gridDim.x) {
    const Job J = jobs[j];
    if (J.ntiles <= kFewTiles) colscan_serial(W, J, j);
  }
  for (int jb = 0; jb < njobs; jb += 1024) {
    const int j = jb + (int)threadIdx.x;
    const bool big = j < njobs && jobs[j].ntiles > kFewTiles;
    unsigned nbig;
    const unsigned pos = block_excl_scan<1024>(big ? 1u : 0u, wsum, nbig);
    if (big) bigs[pos] = j;
    __syncthreads();
    for (long long it = blockIdx.x; it < (long long)nbig * 64; it += gridDim.x) {
      const int jj = bigs[it >> 6], ch = (int)(it & 63);
      const Job J = jobs[jj];
      if (ch * 64 >= (1 << J.r)) continue;  // uniform over the block
      colscan_chunk(W, J, jj, ch, part);
    }
    __syncthreads();
  }
}

// Block scans (1024 threads) of ints with max / min; exclusive.
template <bool IsMax>
__device__ __forceinline__ int block_excl_mm(int v, int ident, int* wsum) {
  const unsigned ln = lane_id();
  int inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(inc, o, 64);
    if ((int)ln >= o) inc = IsMax ? max(inc, y) : min(inc, y);
  }
  int ex = __shfl_up(inc, 1, 64);
  if (ln == 0) ex = ident;
  const int w = threadIdx.x >> 6;
  if (ln == 63) wsum[w] = inc;
  __syncthreads();
  int carry = ident;
  for (int i = 0; i < w; ++i) carry = IsMax ? max(carry, wsum[i]) : min(carry, wsum[i]);
  __syncthreads();
  return IsMax ? max(carry, ex) : min(carry, ex);
}

// ---------------------------------------------------------------------------
// classify: per job, bucket starts and the fate of every bucket.
// ---------------------------------------------------------------------------
// Shared memory of one classify item.
struct ClassifySmem {
  unsigned s_start[kNDig + 1];
  int s_nb[kNDig];             // the digit if it starts a bucket group (else nd), then the next start after it
  unsigned char s_cls[kNDig];  // 0 empty, 1 small, 2 medium, 3 large; +4: starts a group
  unsigned wsum[16];
  int wsi[16];
};

// One classify item: digits [dlo, dhi) of job j at this level (a job's 2^r
// digits are split over `slices` items; each recomputes the job-wide scans
// from the digit totals, which stay in place -- the scatter derives the
// bucket starts itself).  NT threads, kNDig/NT digits per thread.
template <int NT>
__device__ __forceinline__ void classify_item(WsView W, Ctrl* C, int level, int Tnext, int maxlevel, int j, int slice, int slices,
                              int dense_bits, ClassifySmem& sm) {
  constexpr int DPT = kNDig / NT;
  unsigned* s_start = sm.s_start;
  int* s_nb = sm.s_nb;
  unsigned char* s_cls = sm.s_cls;
  unsigned* wsum = sm.wsum;
  int* wsi = sm.wsi;
  const int tid = threadIdx.x;
  {
    const Job J = W.jobs(level)[j];
    if (J.size == 0) return;  // uniform over the block
    const int nd = 1 << J.r;
    const int dlo = (int)((long long)nd * slice / slices), dhi = (int)((long long)nd * (slice + 1) / slices);
    const unsigned* tot = W.starts() + (size_t)j * kNDig;
    // per-thread digit runs are kept in LDS, not in (dynamically indexed) arrays
    unsigned s = 0;
#pragma unroll 4
    for (int q = 0; q < DPT; ++q) {
      const int d = tid * DPT + q;
      const unsigned v = d < nd ? tot[d] : 0u;
      if (d < nd) s_start[d] = v;
      s += v;
    }
    unsigned total;
    unsigned ex = block_excl_scan<NT>(s, wsum, total);
#pragma unroll 4
    for (int q = 0; q < DPT; ++q) {
      const int d = tid * DPT + q;
      if (d < nd) {
        const unsigned v = s_start[d];
        s_start[d] = ex;
        s_cls[d] = v == 0 ? 0 : (v <= (unsigned)kSmall ? 1 : (v <= (unsigned)kCap ? 2 : 3));
        ex += v;
      }
    }
    if (tid == 0) s_start[nd] = total;
    __syncthreads();
    // previous non-empty digit (exclusive max-scan)
    int lm = -1;
    for (int q = 0; q < DPT; ++q) {
      const int d = tid * DPT + q;
      if (d < nd && s_cls[d] != 0) lm = d;
    }
    int prev = block_excl_mm<true>(lm, -1, wsi);
    // bucket-group starts: every non-small bucket, and a small bucket after a
    // non-small one or in a new kSmall window
    for (int q = 0; q < DPT; ++q) {
      const int d = tid * DPT + q;
      if (d >= nd) break;
      bool bnd = false;
      if (s_cls[d] != 0) {
        if (s_cls[d] != 1) {
          bnd = true;
        } else {
          bnd = prev < 0 || s_cls[prev] != 1 ||
                (J.start + s_start[prev]) / kSmall != (J.start + s_start[d]) / kSmall;
        }
        prev = d;
      }
      s_nb[d] = bnd ? d : nd;
    }
    __syncthreads();
    for (int q = 0; q < DPT; ++q) {
      const int d = tid * DPT + q;
      if (d < nd && s_nb[d] == d) s_cls[d] |= 4;
    }
    // next group start after each digit (suffix min-scan, done on reversed order)
    const int rt = NT - 1 - tid;  // this thread scans the digits of thread rt, reversed
    int rv = nd;
    for (int q = 0; q < DPT; ++q) {
      const int d = rt * DPT + q;
      if (d < nd) rv = min(rv, s_nb[d]);
    }
    int nxt = block_excl_mm<false>(rv, nd, wsi);  // min over digits of threads > rt
    for (int q = DPT - 1; q >= 0; --q) {
      const int d = rt * DPT + q;
      if (d < nd) {
        const int here = s_nb[d];
        s_nb[d] = nxt;  // first group start strictly after digit d
        nxt = min(nxt, here);
      }
    }
    __syncthreads();
    // emit jobs and leaves; slots come from one block-wide reservation per
    // counter (a per-bucket atomic on one address serialises thousands of
    // buckets), handed out in digit order.
    const int dstb = dst_of(level);
    const bool deeper = J.shift > 0 && level + 1 <= maxlevel;
    // a bucket too large for a leaf is split again at the next level unless
    // its keys span at most dense_bits bits: then it is one dense leaf
    // (kLeafPure when the key is fully fixed)
    const bool split = J.shift > dense_bits;
    const int dslot = (J.shift > 0 && !split) ? (int)dense_slot_words(J.shift) : 0;
    unsigned c_lj = 0, c_tile = 0, c_pure = 0, c_dw = 0;  // c_lj: leaves (low 16 bits), jobs (high 16 bits)
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
      const int d = tid * DPT + q;
      if (d < dlo || d >= dhi || !(s_cls[d] & 4)) continue;
      const unsigned szd = s_start[d + 1] - s_start[d];
      if ((s_cls[d] & 3) == 3 && split) {
        if (deeper) {
          c_lj += 1u << 16;
          c_tile += (unsigned)(((unsigned long long)szd + Tnext - 1) / Tnext);
        }
      } else {
        c_lj += 1u;
        if ((s_cls[d] & 3) == 3) {
          if (J.shift == 0) {
            c_pure += (unsigned)(((unsigned long long)szd + kPureTile - 1) / kPureTile);
          } else {
            const unsigned nt = (unsigned)(((unsigned long long)szd + kDenseTile - 1) / kDenseTile);
            c_pure += nt;
            c_dw += nt * (unsigned)dslot;
          }
        }
      }
    }
    __shared__ long long s_base[5];
    unsigned t_lj, t_tile, t_pure, t_dw;
    unsigned o_lj = block_excl_scan<NT>(c_lj, wsum, t_lj);
    unsigned o_tile = block_excl_scan<NT>(c_tile, wsum, t_tile);
    unsigned o_pure = block_excl_scan<NT>(c_pure, wsum, t_pure);
    unsigned o_dw = block_excl_scan<NT>(c_dw, wsum, t_dw);
    if (tid == 0) {
      s_base[0] = (t_lj & 0xffffu) ? atomicAdd(&C->nleaves, (int)(t_lj & 0xffffu)) : 0;
      s_base[1] = (t_lj >> 16) ? atomicAdd(&C->njobs[level + 1], (int)(t_lj >> 16)) : 0;
      s_base[2] = t_tile ? atomicAdd(&C->ntiles[level + 1], (int)t_tile) : 0;
      s_base[3] = t_pure ? atomicAdd(&C->npure, (int)t_pure) : 0;
      s_base[4] = t_dw ? (long long)atomicAdd(&C->dwords, (unsigned long long)t_dw) : 0;
    }
    __syncthreads();
    long long nlid = s_base[0] + (o_lj & 0xffffu);
    long long njid = s_base[1] + (o_lj >> 16);
    long long nt0 = s_base[2] + o_tile;
    long long np0 = s_base[3] + o_pure;
    long long ndw = s_base[4] + o_dw;
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
      const int d = tid * DPT + q;
      if (d < dlo || d >= dhi || !(s_cls[d] & 4)) continue;
      const long long gstart = J.start + s_start[d];
      const unsigned long long dbase = J.prefix | ((unsigned long long)d << J.shift);
      const int cls = s_cls[d] & 3;
      const unsigned szd = s_start[d + 1] - s_start[d];
      if (cls == 3 && split) {
        const long long size = szd;
        if (!deeper) {
          set_error(C, TTV_E_DEVICE);
          continue;
        }
        const long long jid = njid++;
        int nt = (int)((size + Tnext - 1) / Tnext);
        const long long t0 = nt0;
        nt0 += nt;
        if (jid >= W.L.jcap) {
          set_error(C, TTV_E_DEVICE);
          continue;
        }
        Job N;
        N.start = gstart;
        N.size = size;
        if (t0 + nt > W.L.tcap) {  // keep a valid, empty job in the slot
          set_error(C, TTV_E_DEVICE);
          nt = 0;
          N.size = 0;
        }
        // digit bits of the new job: enough for sub-buckets of about kSmall
        // records, but at least what the levels after it (and a dense
        // leaf) cannot take
        {
          const int after = maxlevel - (level + 1);
          const int need = J.shift - kRMax * after - dense_bits;
          int rs = 1;
          while (rs < kRMax && (size >> rs) > kSmall) ++rs;
          int r = rs > need ? rs : need;
          if (r > kRMax) r = kRMax;
          if (r > J.shift) r = J.shift;
          N.r = r;
        }
        N.shift = J.shift - N.r;
        N.prefix = dbase;
        N.tile0 = t0;
        N.ntiles = nt;
        N.tensor = J.tensor;
        N.src = dstb;
        N.pad = 0;
        W.jobs(level + 1)[jid] = N;
        int* T = W.tiles(level + 1);
        for (int k = 0; k < nt; ++k) T[t0 + k] = (int)jid;
        continue;
      }
      const long long lid = nlid++;
      Leaf Lf;
      Lf.start = gstart;
      Lf.base = dbase;
      Lf.tensor = J.tensor;
      Lf.src = dstb;
      Lf.ptile0 = 0;
      Lf.nptiles = 0;
      Lf.pslot = 0;
      Lf.pad = 0;
      Lf.kind = kLeafSort;
      if (cls == 3 && J.shift == 0) {  // single key, too large for one block: pure leaf
        Lf.size = szd;
        Lf.kind = kLeafPure;
        Lf.bits = 0;
        const int np = (int)((Lf.size + kPureTile - 1) / kPureTile);
        const long long p0 = np0;
        np0 += np;
        if (p0 + np > W.L.pcap) {
          set_error(C, TTV_E_DEVICE);
          continue;
        }
        Lf.ptile0 = p0;
        Lf.nptiles = np;
      } else if (cls == 3) {  // at most dense_bits key bits: summed by key
        Lf.size = szd;
        Lf.kind = kLeafDense;
        Lf.bits = J.shift;
        // partial sums by key per kDenseTile records, formed before the
        // finishing pass (which then knows the leaf's distinct keys at once)
        const int np = (int)((Lf.size + kDenseTile - 1) / kDenseTile);
        const long long p0 = np0, w0 = ndw;
        np0 += np;
        ndw += (long long)np * dslot;
        if (p0 + np > W.L.pcap || w0 + (long long)np * dslot > W.L.dpcap) {
          set_error(C, TTV_E_DEVICE);
          continue;
        }
        Lf.ptile0 = p0;
        Lf.nptiles = np;
        Lf.pslot = w0;
      } else if (cls == 2) {
        Lf.size = szd;
        Lf.bits = J.shift;
      } else {
        const int nb = s_nb[d];
        Lf.size = (long long)s_start[nb] - s_start[d];
        Lf.bits = J.shift + bitlen64((unsigned long long)(nb - d - 1));
      }
      if (lid >= W.L.lcap) {
        set_error(C, TTV_E_DEVICE);
        continue;
      }
      W.leaves()[lid] = Lf;
      if (Lf.nptiles > 0) {
        int* pl = W.ptile_leaf();
        for (int k = 0; k < Lf.nptiles; ++k) pl[Lf.ptile0 + k] = (int)lid;
      }
      atomicOr(&W.bitmap()[gstart >> 5], 1u << (gstart & 31));
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// scatter: move every record of a tile to its bucket.  Within a tile the
// records keep their order (rounds of 2048; inside a round wave-major, then
// item, then lane), so bucket contents are in input order.
// ---------------------------------------------------------------------------
// Jobs of few digits write each round through an LDS stage in destination
// order: a round's records of one bucket leave as one run of consecutive
// addresses instead of one scattered 16-byte store each.  The counters fit
// jobs of up to kSortedDig digits; measured, the extra barriers and LDS
// passes cost more than the runs save from 512 digits on (about 4 records
// per bucket and round), so only jobs of at most kSortedRounds digits (8 or
// more records per bucket and round) take them.
constexpr int kSortedDig = 1024;
constexpr int kSortedRounds = 256;
template <typename IdxT, int MO>
struct ScatterSmem {
  // next position of every bucket; with at most kSortedDig digits the upper
  // three quarters hold the round's digit counts, their exclusive scan and
  // the position of round slot 0 per digit
  unsigned cursor[kNDig];
  union {
    IdxT stage[kScatterThreads / 64][64 * MO];      // level-1 index rows (load_round)
    u64x2 stg[kScatterThreads * kScatterIPT];       // a round's records by rank
  };
  unsigned wsum[kScatterThreads / 64];
};
static_assert(4 * kSortedDig <= kNDig, "sorted rounds keep their counters in the cursor array");

// The first `gc` blocks classify this level's buckets (classify_item over
// njobs*slices items); the others scatter its tiles.  Neither role reads what
// the other writes in this launch.
// REC: a deeper level's kernel, whose jobs all read the records of the level
// before (loaded one round ahead); otherwise each job reads COO rows (the
// first level) or records.
template <typename IdxT, int F, int PM, int MO, bool REC>
__global__ __launch_bounds__(kScatterThreads, MO <= 3 ? 3 : 2) void k_scatter(WsView W, int level, int T, int Tnext, int maxlevel,
                                                             int slices, int gc, int smax) {
  constexpr int IPT = kScatterIPT;
  constexpr int RW = 64 * IPT;            // records per wave per round
  constexpr int RN = kScatterThreads * IPT;
  union Smem {
    ScatterSmem<IdxT, MO> sc;
    ClassifySmem cl;
  };
  __shared__ Smem smem;  // the two roles share the block's LDS
  __shared__ RawSrc<IdxT, F, MO> rsrc;
  Ctrl* C = W.ctrl();
  if (aborted(C)) return;
  if ((int)blockIdx.x < gc) {
    ClassifySmem& cs = smem.cl;
    const int njobs = clampi(C->njobs[level], W.L.jcap);
    for (long long it = blockIdx.x; it < (long long)njobs * slices; it += gc) {
      classify_item<kScatterThreads>(W, C, level, Tnext, maxlevel, (int)(it / slices), (int)(it % slices), slices,
                                     PM == kPipePerm ? 0 : kDenseBits, cs);
      __syncthreads();
    }
    return;
  }
  ScatterSmem<IdxT, MO>& ss = smem.sc;
  unsigned* cursor = ss.cursor;
  unsigned* const ls = cursor + kSortedDig;      // round: exclusive scan of the digit counts
  unsigned* const ob = cursor + 2 * kSortedDig;  // round: cursor before the round minus ls
  unsigned* const lc = cursor + 3 * kSortedDig;  // round: digit counts
  u64x2* const stg = ss.stg;
  auto& stage = ss.stage;
  unsigned* wsum_s = ss.wsum;
  const int ntiles = clampi(C->ntiles[level], W.L.tcap);
  const Job* jobs = W.jobs(level);
  const int* tj = W.tiles(level);
  const int w = threadIdx.x >> 6;
  const unsigned ln = lane_id();
  const int bid = (int)blockIdx.x - gc, nsb = (int)gridDim.x - gc;
  for (int t = bid; t < ntiles; t += nsb) {
    const int jid = tj[t];
    const Job J = jobs[jid];
    if (REC && J.src == kSrcRaw) {  // only first-level jobs read rows (uniform over the block)
      if (threadIdx.x == 0) set_error(C, TTV_E_DEVICE);
      continue;
    }
    const int nd = 1 << J.r;
    const unsigned mask = (unsigned)nd - 1u;
    const unsigned* row = W.table() + (size_t)t * kNDig;
    const unsigned* tot = W.starts() + (size_t)jid * kNDig;
    {  // bucket starts: exclusive scan of the job's digit totals, plus this tile's offsets
      constexpr int DPT = kNDig / kScatterThreads;
      const int d0 = threadIdx.x * DPT;
      unsigned v[DPT], sum = 0;
#pragma unroll
      for (int q = 0; q < DPT; ++q) {
        v[q] = d0 + q < nd ? tot[d0 + q] : 0u;
        sum += v[q];
      }
      unsigned all;
      unsigned ex = block_excl_scan<kScatterThreads>(sum, wsum_s, all);
#pragma unroll
      for (int q = 0; q < DPT; ++q) {
        if (d0 + q < nd) cursor[d0 + q] = ex + row[d0 + q];
        ex += v[q];
      }
    }
    if (threadIdx.x == 0 && J.src == kSrcRaw) rsrc.set(W.desc()[J.tensor]);
    __syncthreads();
    const long long b = (long long)(t - J.tile0) * T;
    const long long n = (J.size - b < (long long)T) ? J.size - b : (long long)T;
    Rec* dst = W.rec(dst_of(level)) + J.start;
    const gptr<const u64x2> srcR = (J.src == kSrcRaw)
                                       ? (gptr<const u64x2>)nullptr
                                       : to_global((const u64x2*)W.rec(J.src)) + J.start + b;
    const TDesc* Dp = W.desc() + J.tensor;
    const long long roff = J.start - Dp->base + b;
    const RawSrc<IdxT, F, MO>& S = rsrc;
    gptr<u64x2> gdst = to_global((u64x2*)dst);
    // kPipeTTVSeg: the records' nonzero indices move alongside them
    const gptr<const int32_t> srcX =
        (PM == kPipeTTVSeg && srcR) ? to_global((const int32_t*)W.aux(J.src)) + J.start + b : (gptr<const int32_t>)nullptr;
    const gptr<int32_t> gaux =
        PM == kPipeTTVSeg ? to_global(W.aux(dst_of(level))) + J.start : (gptr<int32_t>)nullptr;
    // Records of deeper levels: the next round's are loaded during this
    // round's turns (issued after this round's loads; the turns' barriers
    // wait only for LDS).  Segment-map-carrying records load as they come.
    constexpr bool kPre = REC && PM != kPipeTTVSeg;
    u64x2 nxr[IPT];
    auto prefetch = [&](long long rb) {
      const long long i0 = rb + (long long)w * RW + ln;
#pragma unroll
      for (int j = 0; j < IPT; ++j)
        if (i0 + j * 64 < n) nxr[j] = srcR[i0 + j * 64];
    };
    if (kPre) prefetch(0);
    for (long long rb = 0; rb < n; rb += RN) {
      uint64_t key[IPT], pay[IPT];
      unsigned dg[IPT];
      int32_t ax[IPT];
      {
        const long long i0 = rb + (long long)w * RW + ln;
        if (REC || srcR) {
#pragma unroll
          for (int j = 0; j < IPT; ++j) {
            key[j] = 0;
            pay[j] = 0;
            ax[j] = 0;
            if (i0 + j * 64 < n) {
              const u64x2 r = kPre ? nxr[j] : srcR[i0 + j * 64];
              key[j] = r.x;
              pay[j] = r.y;
              if (PM == kPipeTTVSeg) ax[j] = srcX[i0 + j * 64];
            }
          }
          if (kPre && rb + RN < n) prefetch(rb + RN);
        } else {
          const long long s0 = rb + (long long)w * RW;
          load_round<IdxT, F, PM, IPT, MO>(S, roff + s0, n - s0, stage[w], C, key, pay);
#pragma unroll
          for (int j = 0; j < IPT; ++j) ax[j] = (int32_t)(roff + i0 + j * 64);  // the nonzero's index in its tensor
        }
      }
#pragma unroll
      for (int j = 0; j < IPT; ++j) dg[j] = (unsigned)(key[j] >> J.shift) & mask;
      if (PM != kPipeTTVSeg && nd <= smax) {  // uniform over the block (smax <= kSortedDig)
        // ranks within the round by (digit, input order): the waves take
        // turns on the round's digit counters (lanes of one LDS atomic on
        // one counter served in lane order), so each record's position is
        // the one the direct path below gives it
        for (int q = threadIdx.x; q < nd; q += kScatterThreads) lc[q] = 0u;
        __syncthreads();
        unsigned lpos[IPT];
        for (int turn = 0; turn < kScatterThreads / 64; ++turn) {
          if (w == turn) {
#pragma unroll
            for (int j = 0; j < IPT; ++j) {
              const long long i = rb + (long long)w * RW + j * 64 + ln;
              lpos[j] = i < n ? atomicAdd(&lc[dg[j]], 1u) : 0u;
            }
          }
          __syncthreads();
        }
        {
          constexpr int DPS = kSortedDig / kScatterThreads;
          const int d0 = threadIdx.x * DPS;
          unsigned v[DPS], sum = 0;
#pragma unroll
          for (int q = 0; q < DPS; ++q) {
            v[q] = d0 + q < nd ? lc[d0 + q] : 0u;
            sum += v[q];
          }
          unsigned all;
          unsigned ex = block_excl_scan<kScatterThreads>(sum, wsum_s, all);
#pragma unroll
          for (int q = 0; q < DPS; ++q) {
            if (d0 + q < nd) {
              ls[d0 + q] = ex;
              ob[d0 + q] = cursor[d0 + q] - ex;  // modulo 2^32: ob + rank is the position
              cursor[d0 + q] += v[q];
            }
            ex += v[q];
          }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
          const long long i = rb + (long long)w * RW + j * 64 + ln;
          if (i < n) {
            const unsigned rk = ls[dg[j]] + lpos[j];
            if (rk < (unsigned)RN) {  // always, unless the counters are corrupt: then report, never write outside
              u64x2 r;
              r.x = key[j];
              r.y = pay[j];
              stg[rk] = r;
            } else {
              set_error(C, TTV_E_DEVICE);
            }
          }
        }
        __syncthreads();
        // consecutive lanes take consecutive ranks: runs of one bucket go
        // out as consecutive addresses
        const int cnt = (int)((n - rb) < (long long)RN ? (n - rb) : (long long)RN);
        for (int q = threadIdx.x; q < cnt; q += kScatterThreads) {
          const u64x2 r = stg[q];
          gdst[ob[(unsigned)(r.x >> J.shift) & mask] + (unsigned)q] = r;
        }
        __syncthreads();  // the stage and the round counters are reused by the next round
        continue;
      }
      // positions: the waves take turns adding to the bucket cursors; in a
      // wave, items in order, and the lanes of one LDS atomic that hit the
      // same cursor are served in lane order, so every bucket receives the
      // round's records in input order (wave, item, lane)
      unsigned pos[IPT];
      for (int turn = 0; turn < kScatterThreads / 64; ++turn) {
        if (w == turn) {
#pragma unroll
          for (int j = 0; j < IPT; ++j) {
            const long long i = rb + (long long)w * RW + j * 64 + ln;
            pos[j] = i < n ? atomicAdd(&cursor[dg[j]], 1u) : 0u;
          }
        }
        __syncthreads();
      }
#pragma unroll
      for (int j = 0; j < IPT; ++j) {
        const long long i = rb + (long long)w * RW + j * 64 + ln;
        if (i < n) {
          u64x2 r;
          r.x = key[j];
          r.y = pay[j];
          gdst[pos[j]] = r;
          if (PM == kPipeTTVSeg) gaux[pos[j]] = ax[j];
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// pure reduce: partial sums of single-key leaves, kPureTile records per block
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// leaf numbering: popcount prefix of the leaf-start bitmap.  Every block
// prefixes its words and stores its sum; a one-block kernel then scans the
// block sums (the kernel boundary orders the two: no device-scope atomic per
// block, whose release would write back the L2 on every block).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bitmap(WsView W) {
  constexpr int WPT = kBitmapWordsPerBlock / 256;
  __shared__ unsigned wsum[4];
  const long long w0 = (long long)blockIdx.x * kBitmapWordsPerBlock + threadIdx.x * WPT;
  const gptr<const unsigned> bm = to_global((const unsigned*)W.bitmap());
  unsigned c[WPT];
  unsigned s = 0;
#pragma unroll
  for (int q = 0; q < WPT; ++q) {
    const long long wi = w0 + q;
    c[q] = wi < W.L.words ? (unsigned)__popc(bm[wi]) : 0u;
    s += c[q];
  }
  unsigned tot;
  unsigned ex = block_excl_scan<256>(s, wsum, tot);
  unsigned* wp = W.wordpre();
#pragma unroll
  for (int q = 0; q < WPT; ++q) {
    const long long wi = w0 + q;
    if (wi < W.L.words) wp[wi] = ex;
    ex += c[q];
  }
  if (threadIdx.x == 0) W.blockpre()[blockIdx.x] = tot;
}

// Exclusive scan of k_bitmap's block sums, in place (one block).
__global__ __launch_bounds__(1024) void k_bitmap_scan(WsView W) {
  __shared__ unsigned wsum[1024 / 64];
  unsigned* bp = W.blockpre();
  const long long n = W.L.wblocks;
  unsigned carry = 0;
  for (long long b0 = 0; b0 < n; b0 += 1024) {
    const long long i = b0 + threadIdx.x;
    const unsigned v = i < n ? bp[i] : 0u;
    unsigned t;
    const unsigned e = block_excl_scan<1024>(v, wsum, t);
    if (i < n) bp[i] = carry + e;
    carry += t;
  }
}

// One partial tile of a dense leaf: the FP64 sums by relative key of up to
// kDenseTile records (FP32 payloads: the exact pair, widened) and the
// presence bits of the keys, written to the tile's slot in the dense pool.
// Records are added in order: waves take turns over contiguous slices, a
// wave's items in order, and same-entry lanes of one ds_add_f64 in lane
// order (as in the sort-free leaves).  Without values (segment maps) only
// the presence bits are formed.
constexpr int kLeavesThreads = 256;
constexpr int kLeavesIPT = 8;
template <int F, int PM>
__device__ __forceinline__ void dense_tile(WsView W, const Leaf& Lf, int p, double* sums, unsigned* pres) {
  using FO = FormOps<F>;
  constexpr int NW = kLeavesThreads / 64;
  constexpr int RN = kLeavesThreads * kLeavesIPT;
  const int tid = threadIdx.x, w = tid >> 6;
  const unsigned ln = lane_id();
  const int nk = 1 << Lf.bits, words = (nk + 31) >> 5;
  if (pm_values(PM))
    for (int q = tid; q < nk; q += kLeavesThreads) sums[q] = 0.0;
  for (int q = tid; q < words; q += kLeavesThreads) pres[q] = 0u;
  __syncthreads();
  const long long b = (long long)(p - Lf.ptile0) * kDenseTile;
  const long long e = (Lf.size - b < (long long)kDenseTile) ? Lf.size : b + kDenseTile;
  const gptr<const u64x2> R = to_global(reinterpret_cast<const u64x2*>(W.rec(Lf.src))) + Lf.start;
  const unsigned kmask = (unsigned)nk - 1u;
  // the next round's records are loaded while this round is added (no global
  // store is pending, so the turns' barriers do not wait for those loads)
  u64x2 nx[kLeavesIPT];
  auto fetch = [&](long long rb) {
#pragma unroll
    for (int j = 0; j < kLeavesIPT; ++j) {
      const long long i = rb + (long long)w * 64 * kLeavesIPT + j * 64 + ln;
      if (i < e) nx[j] = R[i];
    }
  };
  fetch(b);
  for (long long rb = b; rb < e; rb += RN) {
    u64x2 cur[kLeavesIPT];
#pragma unroll
    for (int j = 0; j < kLeavesIPT; ++j) cur[j] = nx[j];
    if (rb + RN < e) fetch(rb + RN);
    unsigned k[kLeavesIPT];
    double v[kLeavesIPT];
#pragma unroll
    for (int j = 0; j < kLeavesIPT; ++j) {
      const long long i = rb + (long long)w * 64 * kLeavesIPT + j * 64 + ln;
      k[j] = 0xffffffffu;
      v[j] = 0.0;
      if (i < e) {
        const u64x2 rc = cur[j];
        k[j] = (unsigned)(rc.x - Lf.base) & kmask;
        if (pm_values(PM)) v[j] = FO::to_f64(FO::from_pay(rc.y));
        atomicOr(&pres[k[j] >> 5], 1u << (k[j] & 31u));
      }
    }
    if (pm_values(PM)) {
      for (int turn = 0; turn < NW; ++turn) {
        if (w == turn) {
#pragma unroll
          for (int j = 0; j < kLeavesIPT; ++j)
            if (k[j] != 0xffffffffu) atomicAdd(&sums[k[j]], v[j]);
        }
        __syncthreads();
      }
    }
  }
  __syncthreads();
  gptr<unsigned long long> slot =
      to_global(W.dpool()) + Lf.pslot + (long long)(p - Lf.ptile0) * dense_slot_words(Lf.bits);
  if (pm_values(PM))
    for (int q = tid; q < nk; q += kLeavesThreads) slot[q] = (unsigned long long)__double_as_longlong(sums[q]);
  gptr<unsigned> sp = (gptr<unsigned>)(slot + nk);
  for (int q = tid; q < words; q += kLeavesThreads) sp[q] = pres[q];
  __syncthreads();
}

// Pure leaves: partial sums of kPureTile records each; dense leaves larger
// than kDenseTile records: partial sums by key per kDenseTile records (both
// combined in FP64 by the finishing pass).  Then every leaf is placed at its
// rank (key order).
template <int F, int PM>
__global__ __launch_bounds__(kLeavesThreads) void k_leaves(WsView W) {
  using FO = FormOps<F>;
  using Acc = typename FO::Acc;
  __shared__ Acc red[256];
  __shared__ double s_sums[1 << kDenseBits];
  __shared__ unsigned s_pres[(1 << kDenseBits) / 32];
  Ctrl* C = W.ctrl();
  if (aborted(C)) return;
  const int np = clampi(C->npure, W.L.pcap);
  for (int p = blockIdx.x; p < np; p += gridDim.x) {
    const Leaf Lf = W.leaves()[W.ptile_leaf()[p]];
    if (Lf.kind == kLeafDense) {
      if (PM == kPipePerm || Lf.bits < 1 || Lf.bits > kDenseBits) {  // excluded by classification
        if (threadIdx.x == 0) set_error(C, TTV_E_DEVICE);
        continue;
      }
      dense_tile<F, PM>(W, Lf, p, s_sums, s_pres);
      continue;
    }
    const long long b = (long long)(p - Lf.ptile0) * kPureTile;
    const long long e = (Lf.size - b < (long long)kPureTile) ? Lf.size : b + kPureTile;
    const Rec* R = W.rec(Lf.src) + Lf.start;
    Acc a = FO::zero();
    for (long long i = b + threadIdx.x; i < e; i += 256) a = FO::add(a, FO::from_pay(R[i].pay));
    red[threadIdx.x] = a;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) red[threadIdx.x] = FO::add(red[threadIdx.x], red[threadIdx.x + h]);
      __syncthreads();
    }
    if (threadIdx.x == 0) W.partials()[p] = FO::to_f64(red[0]);
    __syncthreads();
  }
  const int nl = clampi(C->nleaves, W.L.lcap);
  const Leaf* Ls = W.leaves();
  Leaf* O = W.ordered();
  unsigned long long* S = W.status();
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nl; i += gridDim.x * blockDim.x) {
    const Leaf Lf = Ls[i];
    const long long wi = Lf.start >> 5;
    const unsigned below = (unsigned)__popc(W.bitmap()[wi] & ((1u << (Lf.start & 31)) - 1u));
    const long long r = (long long)W.blockpre()[wi / kBitmapWordsPerBlock] + W.wordpre()[wi] + below;
    if (r < 0 || r >= nl) {
      set_error(C, TTV_E_DEVICE);
      continue;
    }
    O[r] = Lf;
    S[r] = 0ull;
  }
}

// ---------------------------------------------------------------------------
// finish
// ---------------------------------------------------------------------------
__device__ __forceinline__ void publish(unsigned long long* S, int r, unsigned long long v) {
  __hip_atomic_store(&S[r], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Decoupled look-back by one wave: 64 predecessors per step; the nearest
// inclusive prefix ends the walk, the aggregates after it are added.
// `early` is this lane's status word of the first window (predecessor
// r-1-lane) read some time before, or 0: published words never change
// meaning (an aggregate stays the leaf's count), so only the words still 0
// are read again.
__device__ long long lookback_wave(unsigned long long* S, int r, int spin_limit, Ctrl* C,
                                   unsigned long long early = 0, int kind = 0) {
  // Each step reads kLookG groups of 64 predecessors, their loads in flight
  // together (lane l of group g reads predecessor base - 64 g - l).  The
  // groups are then resolved nearest first: a lane waits only while its
  // status is unpublished and no inclusive prefix lies between it and this
  // leaf, and the walk stops at the group holding the nearest inclusive
  // prefix (the first leaf of a tensor of a batch publishes one at once, so
  // statuses beyond it may still be unpublished and are never waited for).
  constexpr int kLookG = 4;
  const unsigned ln = lane_id();
  long long prefix = 0;
  TTV_LB_DECL
  for (int base = r - 1;; base -= 64 * kLookG) {
    TTV_LB_STEP
    unsigned long long s[kLookG];
#pragma unroll
    for (int g = 0; g < kLookG; ++g) {
      const int j = base - 64 * g - (int)ln;
      s[g] = kFlagInc;  // before the first leaf: an inclusive prefix of 0
      if (j >= 0) {
        s[g] = (base == r - 1 && g == 0) ? early : 0ull;
        if (!(s[g] >> 62)) s[g] = __hip_atomic_load(&S[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    long long v = 0;
    bool found = false;
#pragma unroll
    for (int g = 0; g < kLookG; ++g) {
      const int j = base - 64 * g - (int)ln;
      int spins = 0;
      uint64_t pm;
      int stop;
      for (;;) {
        pm = ballot((s[g] >> 62) == 2);
        stop = pm ? __ffsll((long long)pm) - 1 : 63;
        const bool need = (int)ln <= stop && j >= 0 && !(s[g] >> 62);
        if (!ballot(need)) break;
        TTV_LB_WAIT
        if (need) {
          if (++spins > spin_limit) {
            set_error(C, TTV_E_DEVICE);
            s[g] = kFlagInc;
          } else {
            __builtin_amdgcn_s_sleep(1);
            s[g] = __hip_atomic_load(&S[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
        }
      }
      v += ((int)ln <= stop) ? (long long)(s[g] & kValMask) : 0;
      if (pm) {
        found = true;
        break;  // wave-uniform
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    prefix += v;
    if (found) break;
  }
  TTV_LB_END(kind)
  (void)kind;
  return prefix;
}

// Output pointers and key layout of one tensor, held in registers while a
// leaf is written (the descriptor itself lives in global memory).
template <typename IdxT, int F>
struct OutInfo {
  gptr<IdxT> subs;
  gptr<double> v64;
  gptr<float> v32;
  int nrem;
  int f64out;
  unsigned long long kst[kMaxOrder];
  unsigned long long mag[kMaxOrder];
  int sh1[kMaxOrder];
  int sh2[kMaxOrder];
  __device__ __forceinline__ void load(const TDesc& D) {
    subs = to_global(static_cast<IdxT*>(D.out_subs));
    v64 = to_global(static_cast<double*>(D.out_vals));
    v32 = to_global(static_cast<float*>(D.out_vals));
    nrem = D.nrem;
    f64out = (F == kF64) || D.out_f64;
#pragma unroll
    for (int i = 0; i < kMaxOrder; ++i) {
      kst[i] = D.kstride[i];
      mag[i] = D.kmagic[i];
      sh1[i] = D.ksh1[i];
      sh2[i] = D.ksh2[i];
    }
  }
  // unpack the mixed-radix key into the remaining indices, then the value
  __device__ __forceinline__ void write(long long row, uint64_t key, double v) const {
    write_subs(row, key);
    if (f64out)
      v64[row] = v;
    else
      v32[row] = (float)v;
  }
  __device__ __forceinline__ void write_subs(long long row, uint64_t key) const {
    gptr<IdxT> o = subs + row * nrem;
    unsigned long long k = key;
    // kept rolled: the constants stay in LDS instead of pinning registers
#pragma unroll 1
    for (int i = 0; i < nrem - 1; ++i) {
      const unsigned long long q = udiv_magic(k, mag[i], sh1[i], sh2[i]);
      o[i] = (IdxT)q;
      k -= q * kst[i];
    }
    o[nrem - 1] = (IdxT)k;  // the last stride is 1
  }
};

template <typename IdxT, int F, int PM>
__global__ __launch_bounds__(kFinishThreads, 4) void k_finish(WsView W, int spin_limit) {
  using FO = FormOps<F>;
  using Acc = typename FO::Acc;
  constexpr int NT = kFinishThreads;
  constexpr int IPT = kFinishIPT;
  constexpr int NW = NT / 64;
  constexpr int MAXD = 8;  // widest LDS digit
  // Region A holds, by leaf kind: the sort's relative keys and positions
  // (sk, si); a sort-free leaf's row sums and row keys (acc, rkey); a dense
  // leaf's sums by key (acc).  With the digit counters (cnt) the block
  // needs about 49 KB of LDS, room for three blocks per CU; at 128 VGPRs per
  // lane (four waves per SIMD) two of them run per CU.  Bounds that force six
  // waves per SIMD spill about 160 bytes per lane and measured slower.
  __shared__ __attribute__((aligned(16))) unsigned char smA[kCap * 8 + kCap * 2];
  unsigned* const sk = reinterpret_cast<unsigned*>(smA);
  unsigned short* const si = reinterpret_cast<unsigned short*>(smA + kCap * 4);
  double* const acc = reinterpret_cast<double*>(smA);
  unsigned short* const rkey = reinterpret_cast<unsigned short*>(smA + kCap * 8);
  __shared__ unsigned cnt[NW << MAXD];
  __shared__ unsigned wsum[NW];
  __shared__ Seg<F> wagg[NW];
  __shared__ int s_ticket;
  __shared__ long long s_prefix;
  __shared__ OutInfo<IdxT, F> sO;
  // the tensor whose output layout sO holds, with its record range and
  // output pointers (reloaded only when a leaf of another tensor comes)
  struct TensorOut {
    long long base, nnz;
    long long* out_nnz;
    int32_t* seg_out;
    int tensor;
  };
  __shared__ TensorOut sT;
  Ctrl* C = W.ctrl();
  if (aborted(C)) return;
  const int nleaves = clampi(C->nleaves, W.L.lcap);
  unsigned long long* S = W.status();
  const int tid = threadIdx.x, w = tid >> 6;
  const unsigned ln = lane_id();
  TTV_PHASE_DECL
  // Tickets hand out the leaves in key order, each when a block is free to
  // start it (a leaf ticketed ahead of time would hold up the look-backs of
  // every later leaf until its block got to it).
  if (tid == 0) sT.tensor = -1;
  for (;;) {
    if (tid == 0) s_ticket = atomicAdd(&C->ticket, 1);
    __syncthreads();
    const int r = s_ticket;
    if (r >= nleaves) break;
    TTV_PHASE(0)
    const Leaf Lf = W.ordered()[r];
    const TDesc& D = W.desc()[Lf.tensor];
    if (tid == 0 && Lf.tensor != sT.tensor) {
      sO.load(D);
      sT.base = D.base;
      sT.nnz = D.nnz;
      sT.out_nnz = D.out_nnz;
      sT.seg_out = D.seg_out;
      sT.tensor = Lf.tensor;
    }
    __syncthreads();
    const bool first = Lf.start == sT.base;
    const bool last = Lf.start + Lf.size == sT.base + sT.nnz;
    gptr<long long> out_nnz = to_global(sT.out_nnz);
    gptr<int32_t> seg_out = to_global(sT.seg_out);
    const OutInfo<IdxT, F>& O = sO;
    const gptr<const Rec> R = to_global(static_cast<const Rec*>(W.rec(Lf.src))) + Lf.start;
    const gptr<const u64x2> Rv = to_global(reinterpret_cast<const u64x2*>(W.rec(Lf.src))) + Lf.start;
    const int n = (int)(Lf.size < (long long)kCap ? Lf.size : (long long)kCap);
    if (Lf.kind == kLeafDense) {
      // ---- dense leaf: the partial slots of k_leaves (sums by relative key,
      // at most kDenseBits bits, and presence bits) added up in tile order;
      // the distinct keys are known before any sum, so the leaf's count is
      // published at once; present keys written in key order ----
      const int nk = 1 << Lf.bits, words = (nk + 31) >> 5;
      const unsigned kmask = (unsigned)nk - 1u;
      double* sums = acc;  // kCap >= 2^kDenseBits entries
      unsigned* pres = cnt;
      unsigned* wpre = cnt + (1 << kDenseBits) / 32;
      if (PM == kPipePerm || Lf.bits < 1 || Lf.bits > kDenseBits || Lf.size <= 0 || Lf.nptiles < 1) {
        // excluded by classification
        if (tid == 0) {
          set_error(C, TTV_E_DEVICE);
          publish(S, r, kFlagInc);
        }
        __syncthreads();
        continue;
      }
      const long long slotw = dense_slot_words(Lf.bits);
      const gptr<const unsigned long long> slots = to_global((const unsigned long long*)W.dpool()) + Lf.pslot;
      {  // every (tile, word) pair by its own thread: the loads are all in flight at once
        for (int q = tid; q < words; q += NT) pres[q] = 0u;
        __syncthreads();
        const int wsh = Lf.bits > 5 ? Lf.bits - 5 : 0;  // words = 2^wsh
        const int tot = Lf.nptiles << wsh;
        for (int e = tid; e < tot; e += NT) {
          const int t = e >> wsh, q = e & (words - 1);
          const unsigned m = ((const gptr<const unsigned>)(slots + t * slotw + nk))[q];
          if (m) atomicOr(&pres[q], m);
        }
        __syncthreads();
      }
      // distinct keys: popcount prefix of the presence words (at most NT words)
      unsigned u = 0;
      {
        const unsigned c = tid < words ? (unsigned)__popc(pres[tid]) : 0u;
        const unsigned ex = block_excl_scan<NT>(c, wsum, u);
        if (tid < words) wpre[tid] = ex;
      }
      if (tid == 0) publish(S, r, (first ? kFlagInc : kFlagAgg) | (unsigned long long)u);
      if (pm_values(PM) && Lf.nptiles > 0) {  // the slots' sums, tile by tile (8 loads in flight)
        for (int q = tid; q < nk; q += NT) {
          double a = 0.0;
          int t = 0;
          for (; t + 8 <= Lf.nptiles; t += 8) {
            double x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) x[u] = __longlong_as_double((long long)slots[(t + u) * slotw + q]);
#pragma unroll
            for (int u = 0; u < 8; ++u) a += x[u];
          }
          for (; t < Lf.nptiles; ++t) a += __longlong_as_double((long long)slots[t * slotw + q]);
          sums[q] = a;
        }
      }
      if (w == 0) {
        const long long prefix = first ? 0 : lookback_wave(S, r, spin_limit, C, 0ull, 0);
        if (ln == 0) {
          if (!first) publish(S, r, kFlagInc | (unsigned long long)(prefix + u));
          s_prefix = prefix;
          if (last && out_nnz) *out_nnz = prefix + u;
        }
      }
      __syncthreads();
      const long long prefix = s_prefix;
      if (pm_values(PM)) {
        for (int q = tid; q < nk; q += NT) {
          const unsigned pw = pres[q >> 5], bit = 1u << (q & 31);
          if (pw & bit) O.write(prefix + wpre[q >> 5] + (unsigned)__popc(pw & (bit - 1u)), Lf.base + q, sums[q]);
        }
      }
      if (PM == kPipeSegMap || PM == kPipeTTVSeg) {  // every record's row: the rank of its key
        const gptr<const int32_t> Xa = to_global((const int32_t*)W.aux(Lf.src)) + Lf.start;
        for (long long i = tid; i < Lf.size; i += NT) {
          const u64x2 rc = Rv[i];
          const unsigned kk = (unsigned)(rc.x - Lf.base) & kmask;
          const unsigned pw = pres[kk >> 5];
          const long long e = PM == kPipeSegMap ? (long long)rc.y : (long long)Xa[i];
          seg_out[e] = (int32_t)(prefix + wpre[kk >> 5] + (unsigned)__popc(pw & ((1u << (kk & 31)) - 1u)));
        }
      }
      __syncthreads();
      TTV_PHASE(10)
      TTV_COUNT(13)
      continue;
    }
    if (Lf.kind != kLeafPure && (Lf.size > kCap || Lf.size <= 0)) {  // excluded by classification
      if (tid == 0) {
        set_error(C, TTV_E_DEVICE);
        publish(S, r, kFlagInc);
      }
      __syncthreads();
      continue;
    }
    if (Lf.kind == kLeafPure) {
      if (tid == 0) publish(S, r, (first ? kFlagInc : kFlagAgg) | 1ull);
      if (w == 0) {
        const long long prefix = first ? 0 : lookback_wave(S, r, spin_limit, C, 0ull, 1);
        if (ln == 0) {
          if (!first) publish(S, r, kFlagInc | (unsigned long long)(prefix + 1));
          s_prefix = prefix;
          double v = 0.0;
          const double* P = W.partials() + Lf.ptile0;
          for (int k = 0; k < Lf.nptiles; ++k) v += P[k];
          if (pm_values(PM)) O.write(prefix, Lf.base, v);
          if (PM == kPipePerm) O.write_subs(prefix, Lf.base);
          if (last && out_nnz) *out_nnz = prefix + 1;
        }
      }
      if (PM == kPipeSegMap) {
        __syncthreads();
        const long long row = s_prefix;
        for (long long i = tid; i < Lf.size; i += NT) seg_out[(long long)R[i].pay] = (int32_t)row;
      }
      if (PM == kPipeTTVSeg) {
        __syncthreads();
        const long long row = s_prefix;
        const gptr<const int32_t> Xa = to_global((const int32_t*)W.aux(Lf.src)) + Lf.start;
        for (long long i = tid; i < Lf.size; i += NT) seg_out[(long long)Xa[i]] = (int32_t)row;
      }
      if (PM == kPipePerm) {  // every record of the run, in record order
        __syncthreads();
        const long long row = s_prefix;
        const long long pos0 = Lf.start - D.base;
        gptr<int32_t> perm_out = to_global(D.perm_out);
        for (long long i = tid; i < Lf.size; i += NT) {
          perm_out[pos0 + i] = (int32_t)R[i].pay;
          seg_out[pos0 + i] = (int32_t)row;
        }
      }
      __syncthreads();
      TTV_PHASE(11)
      TTV_COUNT(14)
      continue;
    }
    // ---- LDS radix sort of the relative keys.  Wave w holds the contiguous
    // positions [w*64*nj, (w+1)*64*nj), item j of a lane is position
    // w*64*nj + j*64 + lane: ranking in (wave, item, lane) order is ranking
    // in position order, which keeps every pass stable. ----
    const bool wide = Lf.bits > 32;
    const int nj = (n + 64 * NW - 1) / (64 * NW);
    unsigned k[IPT];
    unsigned ix[IPT];
    uint64_t pl[IPT];  // the items' payloads (sorted leaves read them again after the sort)
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      const int i = w * 64 * nj + j * 64 + (int)ln;
      ix[j] = (unsigned)i;
      k[j] = 0;
      pl[j] = 0;
      if (j < nj) {
        const u64x2 rc = Rv[i < n ? i : n - 1];  // whole records: one coalesced 16-byte read per item
        k[j] = (unsigned)(rc.x - Lf.base);
        pl[j] = rc.y;
      }
    }
    TTV_PHASE(1)
    // Distinct keys counted before the sort when the relative keys are narrow
    // enough for a presence bitmap in the counter space: the aggregate is
    // published this early, so the look-backs of later leaves rarely wait.
    constexpr int kEarlyBits = 5 + MAXD + (NW >= 8 ? 3 : (NW >= 4 ? 2 : (NW >= 2 ? 1 : 0)));  // bits in cnt
    static_assert((NW & (NW - 1)) == 0 && NW <= 8, "counter space is NW << MAXD words");
    const bool early = !wide && Lf.bits <= kEarlyBits;
    unsigned u_early = 0;
    unsigned long long lb_early = 0;
    if (early) {
      const int words = 1 << (Lf.bits > 5 ? Lf.bits - 5 : 0);
      for (int q = tid; q < words; q += NT) cnt[q] = 0u;
      __syncthreads();
#pragma unroll
      for (int j = 0; j < IPT; ++j) {
        const int i = w * 64 * nj + j * 64 + (int)ln;
        if (j < nj && i < n) atomicOr(&cnt[k[j] >> 5], 1u << (k[j] & 31u));
      }
      __syncthreads();
      // popcount prefix of the bitmap words (each thread a contiguous run);
      // with room for it (words <= half the counter space) it is kept after
      // the bitmap: the rank of a key among the distinct keys is then
      // wordpre[key / 32] + popcount of the lower bits of its word
      const bool keep_pre = 2 * words <= (NW << MAXD);
      const int wpt = (words + NT - 1) / NT;
      unsigned c = 0;
      for (int q = tid * wpt; q < words && q < (tid + 1) * wpt; ++q) c += (unsigned)__popc(cnt[q]);
      unsigned ex = block_excl_scan<NT>(c, wsum, u_early);  // its barriers also end the bitmap's use
      if (keep_pre) {
        for (int q = tid * wpt; q < words && q < (tid + 1) * wpt; ++q) {
          cnt[words + q] = ex;
          ex += (unsigned)__popc(cnt[q]);
        }
        // the prefix words are written, and the bitmap read, by every thread
        // before any reuses the counter space (the sort clears it)
        __syncthreads();
      }
      if (tid == 0) publish(S, r, (first ? kFlagInc : kFlagAgg) | (unsigned long long)u_early);
      // the look-back's first window is read now and used after the sort
      if (w == 0 && !first) {
        const int jp = r - 1 - (int)ln;
        lb_early = jp >= 0 ? __hip_atomic_load(&S[jp], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : kFlagInc;
      }
      if constexpr (pm_values(PM)) {
        // (a leaf of few distinct keys is sorted instead: its in-order adds
        // would pile many lanes of one atomic onto one row)
        if (keep_pre && u_early >= 64u) {
          // ---- sort-free leaf: every record knows its output row (the rank
          // of its key on the bitmap); each row's sum is built in FP64 from
          // 0, its records adding in leaf order (waves in turn, items in
          // order, same-entry lanes of one ds_add_f64 in lane order), so the
          // sum is the in-order sum, bitwise repeatable.  A leaf whose keys
          // are all distinct stores each product directly.  An FP32 record's
          // payload is its exact product pair, widened to FP64 (no rounding
          // before the sum).  Every record writes its row's key (the same
          // value for all records of a row). ----
          TTV_PHASE2(0)
          const bool dups = u_early < (unsigned)n;
          if (dups)
            for (int q = tid; q < (int)u_early; q += NT) acc[q] = 0.0;
          __syncthreads();  // also orders the prefix words before their reads
          unsigned row[IPT];
          double pv[IPT];  // the record's product in FP64
#pragma unroll
          for (int j = 0; j < IPT; ++j) {
            const int i = w * 64 * nj + j * 64 + (int)ln;
            row[j] = 0xffffffffu;
            pv[j] = 0.0;
            if (j < nj && i < n) {
              const unsigned kk = k[j], wi = kk >> 5;
              row[j] = cnt[words + wi] + (unsigned)__popc(cnt[wi] & ((1u << (kk & 31u)) - 1u));
              pv[j] = FO::to_f64(FO::from_pay(pl[j]));
              if (row[j] < u_early) {  // always: the rank of a present key
                rkey[row[j]] = (unsigned short)kk;
                if (!dups) acc[row[j]] = pv[j];
              } else {
                set_error(C, TTV_E_DEVICE);
                row[j] = 0xffffffffu;
              }
            }
          }
          TTV_PHASE2(1)
          if (dups) {  // some key repeats: in-order adds
            for (int turn = 0; turn < NW; ++turn) {
              if (w == turn) {
#pragma unroll
                for (int j = 0; j < IPT; ++j)
                  if (row[j] != 0xffffffffu) atomicAdd(&acc[row[j]], pv[j]);
              }
              __syncthreads();
            }
          } else {
            __syncthreads();
          }
          TTV_PHASE2(2)
          if (w == 0) {
            const long long prefix = first ? 0 : lookback_wave(S, r, spin_limit, C, lb_early, 2);
            if (ln == 0) {
              if (!first) publish(S, r, kFlagInc | (unsigned long long)(prefix + u_early));
              s_prefix = prefix;
              if (last && out_nnz) *out_nnz = prefix + u_early;
            }
          }
          __syncthreads();
          TTV_PHASE2(3)
          const long long prefix = s_prefix;
          for (int q = tid; q < (int)u_early; q += NT) O.write(prefix + q, Lf.base + rkey[q], acc[q]);
          if constexpr (PM == kPipeTTVSeg) {
            const gptr<const int32_t> Xa = to_global((const int32_t*)W.aux(Lf.src)) + Lf.start;
#pragma unroll
            for (int j = 0; j < IPT; ++j) {
              const int i = w * 64 * nj + j * 64 + (int)ln;
              if (j < nj && i < n && row[j] != 0xffffffffu) seg_out[(long long)Xa[i]] = (int32_t)(prefix + row[j]);
            }
          }
          __syncthreads();
          TTV_PHASE2(4)
          TTV_PHASE(7)
          TTV_COUNT(12)
          continue;
        }
      }
    }
    // Wider relative keys (up to 31 bits): the distinct keys are counted
    // before the sort as well, by inserting them into an LDS hash set (twice
    // as many slots as a leaf has records, linear probing), so such a leaf
    // publishes its count as early as a bitmap-counted one and later leaves
    // do not wait for its sort in their look-backs.
    const bool hashed = !wide && !early && Lf.bits <= 31;
    if (hashed) {
      constexpr int kSlotBits = 13;
      constexpr int kSlots = 1 << kSlotBits;
      constexpr unsigned kEmpty = 0xffffffffu;  // no key of at most 31 bits
      static_assert(kSlots >= 2 * kCap && kSlots * 4 <= (int)sizeof(smA), "hash set of the leaf's keys in region A");
      unsigned* const tab = reinterpret_cast<unsigned*>(smA);
      for (int q = tid; q < kSlots; q += NT) tab[q] = kEmpty;
      __syncthreads();
      unsigned mine = 0;
#pragma unroll
      for (int j = 0; j < IPT; ++j) {
        const int i = w * 64 * nj + j * 64 + (int)ln;
        if (j < nj && i < n) {
          unsigned h = (k[j] * 2654435761u) >> (32 - kSlotBits);
          for (int probe = 0; probe < kSlots; ++probe) {  // the set never fills: it ends at an empty slot
            const unsigned old = atomicCAS(&tab[h], kEmpty, k[j]);
            if (old == kEmpty) {
              ++mine;
              break;
            }
            if (old == k[j]) break;
            h = (h + 1) & (unsigned)(kSlots - 1);
          }
        }
      }
      block_excl_scan<NT>(mine, wsum, u_early);  // its barriers end the set's use before the sort reuses region A
      if (tid == 0) publish(S, r, (first ? kFlagInc : kFlagAgg) | (unsigned long long)u_early);
      if (w == 0 && !first) {
        const int jp = r - 1 - (int)ln;
        lb_early = jp >= 0 ? __hip_atomic_load(&S[jp], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : kFlagInc;
      }
    }
    const int npass = (Lf.bits + MAXD - 1) / MAXD;
    const int dw = npass ? (Lf.bits + npass - 1) / npass : 0;
    const int nb = 1 << dw;
    const unsigned dmask = (unsigned)nb - 1u;
    for (int pass = 0; pass < npass; ++pass) {
      const int sh = pass * dw;
      for (int q = tid; q < NW * nb; q += NT) cnt[q] = 0u;
      __syncthreads();
      unsigned rk[IPT];
#pragma unroll
      for (int j = 0; j < IPT; ++j) {
        const int i = w * 64 * nj + j * 64 + (int)ln;
        // stable rank: one LDS atomic per item on the wave's own counters
        // (same-address lanes of one instruction are served in lane order)
        rk[j] = 0;
        if (j < nj && i < n) {
          const unsigned d = wide ? (unsigned)(((R[ix[j]].key - Lf.base) >> sh) & dmask) : (k[j] >> sh) & dmask;
          rk[j] = atomicAdd(&cnt[w * nb + d], 1u);
        }
      }
      __syncthreads();
      {  // exclusive scan of the counters in (digit, wave) order
        const int E = NW * nb;
        const int ept = (E + NT - 1) / NT;
        unsigned v[8], s = 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int e = tid * ept + q;
          v[q] = (q < ept && e < E) ? cnt[(e % NW) * nb + e / NW] : 0u;
          s += v[q];
        }
        unsigned tot;
        unsigned ex = block_excl_scan<NT>(s, wsum, tot);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int e = tid * ept + q;
          if (q < ept && e < E) cnt[(e % NW) * nb + e / NW] = ex;
          ex += v[q];
        }
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < IPT; ++j) {
        const int i = w * 64 * nj + j * 64 + (int)ln;
        if (j < nj && i < n) {
          const unsigned d = wide ? (unsigned)(((R[ix[j]].key - Lf.base) >> sh) & dmask) : (k[j] >> sh) & dmask;
          const unsigned dest = cnt[w * nb + d] + rk[j];
          if (dest < (unsigned)n) {  // always, unless the counters are corrupt: then report, never write outside
            sk[dest] = k[j];
            si[dest] = (unsigned short)ix[j];
          } else {
            set_error(C, TTV_E_DEVICE);
          }
        }
      }
      __syncthreads();
      if (pass + 1 < npass) {
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
          const int i = w * 64 * nj + j * 64 + (int)ln;
          if (j < nj && i < n) {
            k[j] = sk[i];
            ix[j] = si[i];
          }
        }
        __syncthreads();
      }
    }
    if (npass == 0) {
#pragma unroll
      for (int j = 0; j < IPT; ++j) {
        const int i = w * 64 * nj + j * 64 + (int)ln;
        if (j < nj && i < n) {
          sk[i] = k[j];
          si[i] = (unsigned short)ix[j];
        }
      }
      __syncthreads();
    }
    TTV_PHASE(2)
    // ---- heads over the sorted order.  Wave w owns positions
    // [w*64*IPT, (w+1)*64*IPT) in IPT rounds of 64 consecutive positions
    // (lane-striped), so the output rows a round writes are contiguous. ----
    const int pw = w * 64 * nj;
    uint64_t hm[IPT];
    unsigned whc = 0;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      const int p = pw + j * 64 + (int)ln;
      bool hd = false;
      if (j < nj && p < n) {
        if (p == 0) {
          hd = true;
        } else {
          // the sort's ranks rely on LDS serving same-address lanes in lane
          // order; keys that do not ascend are reported, never written
          bool desc;
          if (wide) {
            const uint64_t a = R[si[p - 1]].key, b = R[si[p]].key;
            hd = b != a;
            desc = b < a;
          } else {
            hd = sk[p] != sk[p - 1];
            desc = sk[p] < sk[p - 1];
          }
          if (desc) set_error(C, TTV_E_DEVICE);
        }
      }
      hm[j] = ballot(hd);
      whc += (unsigned)__popcll(hm[j]);
    }
    if (ln == 0) wsum[w] = whc;
    __syncthreads();
    unsigned hbw = 0, u = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      const unsigned c = wsum[q];
      hbw += (q < w) ? c : 0u;
      u += c;
    }
    if (early || hashed) {
      if (tid == 0 && u != u_early) set_error(C, TTV_E_DEVICE);  // the two counts agree by construction
    } else if (tid == 0) {
      publish(S, r, (first ? kFlagInc : kFlagAgg) | (unsigned long long)u);
    }
    // wave 0 resolves this leaf's output offset while the others gather payloads
    if (w == 0) {
      const long long prefix = first ? 0 : lookback_wave(S, r, spin_limit, C, lb_early, 3);
      if (ln == 0) {
        if (!first) publish(S, r, kFlagInc | (unsigned long long)(prefix + u));
        s_prefix = prefix;
        if (last && out_nnz) *out_nnz = prefix + u;
      }
    }
    TTV_PHASE(3)
    // ---- payloads and the segmented scan (rounds within the wave) ----
    Acc val[IPT];
    if (pm_values(PM)) {
      uint64_t pay[IPT];
#pragma unroll
      for (int j = 0; j < IPT; ++j) {
        const int p = pw + j * 64 + (int)ln;
        pay[j] = 0;
        if (j < nj) pay[j] = Rv[si[p < n ? p : n - 1]].y;  // records are L2-resident: read at the start of the leaf
      }
      Acc c = FO::zero();  // value of the segment open at the end of the previous round
#pragma unroll
      for (int j = 0; j < IPT; ++j) {
        if (j >= nj) continue;
        const bool hd = (hm[j] >> ln) & 1ull;
        Seg<F> e;
        e.f = hd ? 1 : 0;
        e.v = FO::from_pay(pay[j]);
        e = wave_seg_scan<F>(e);
        // lanes before the round's first head continue the open segment
        val[j] = e.f ? e.v : FO::add(c, e.v);
        c = FO::shfl_last(val[j]);
      }
      if (ln == 0) {
        bool any = false;
#pragma unroll
        for (int j = 0; j < IPT; ++j) any = any || hm[j] != 0;
        wagg[w].f = any ? 1 : 0;
        wagg[w].v = c;
      }
    }
    __syncthreads();
    if (pm_values(PM)) {
      // the segment open at the start of this wave continues from earlier waves
      Seg<F> cw;
      cw.f = 0;
      cw.v = FO::zero();
      for (int q = 0; q < w; ++q) cw = seg_combine<F>(cw, wagg[q]);
      bool lead = true;
#pragma unroll
      for (int j = 0; j < IPT; ++j) {
        if (j >= nj) continue;
        const uint64_t upto = hm[j] & (~0ull >> (63 - ln));  // heads at lanes <= this one
        const bool my_lead = lead && upto == 0;
        if (my_lead) val[j] = FO::add(cw.v, val[j]);
        lead = lead && hm[j] == 0;
      }
    }
    TTV_PHASE(4)
    __syncthreads();
    TTV_PHASE(5)
    const long long prefix = s_prefix;
    // ---- write (consecutive lanes -> consecutive output rows) ----
    unsigned hrun = hbw;  // heads before this round
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      if (j >= nj) continue;
      const int p = pw + j * 64 + (int)ln;
      const unsigned upto = (unsigned)__popcll(hm[j] & (~0ull >> (63 - ln)));
      if (p < n) {
        const long long rowi = prefix + hrun + upto - 1;
        if (PM == kPipeSegMap) {
          seg_out[(long long)Rv[si[p]].y] = (int32_t)rowi;
        } else if (PM == kPipePerm) {
          // sorted position -> nonzero and output row; the run's last record
          // writes the row's coordinates
          const long long pos = Lf.start - D.base + p;
          to_global(D.perm_out)[pos] = (int32_t)Rv[si[p]].y;
          seg_out[pos] = (int32_t)rowi;
          const bool end = p == n - 1 || (wide ? R[si[p + 1]].key != R[si[p]].key : sk[p + 1] != sk[p]);
          if (end) O.write_subs(rowi, wide ? R[si[p]].key : Lf.base + sk[p]);
        } else {
          bool end;
          if (p == n - 1)
            end = true;
          else if (wide)
            end = R[si[p + 1]].key != R[si[p]].key;
          else
            end = sk[p + 1] != sk[p];
          if (end) {
            const uint64_t key = wide ? R[si[p]].key : Lf.base + sk[p];
            O.write(rowi, key, FO::to_f64(val[j]));
          }
          if (PM == kPipeTTVSeg) seg_out[(long long)to_global((const int32_t*)W.aux(Lf.src))[Lf.start + si[p]]] = (int32_t)rowi;
        }
      }
      hrun += (unsigned)__popcll(hm[j]);
    }
    __syncthreads();
    TTV_PHASE(6)
    TTV_COUNT(15)
  }
}

// ---------------------------------------------------------------------------
// host launcher
// ---------------------------------------------------------------------------
template <typename IdxT, int F, int PM, int MO>
static int launch_impl(const PipePlan& P, void* ws, hipStream_t s) {
  (void)hipGetLastError();  // errors left by earlier, unrelated runtime calls are not ours
  WsView W;
  W.b = static_cast<char*>(ws);
  W.L = P.L;
  const int cus = P.cus;
  const int g_init = (int)std::min<long long>(std::max<long long>(1, (P.L.words + 255) / 256), 4LL * cus);
  hipLaunchKernelGGL(k_init, dim3(g_init), dim3(256), 0, s, W, P.d0, P.descs_dev, P.count, P.T1);
  for (int l = 1; l <= P.levels; ++l) {
    const int T = l == 1 ? P.T1 : P.T2;
    const int Tn = P.T2;
    // deeper levels: grids sized for the chip, not for the (unknown) work --
    // every kernel strides over its items, and an empty level then costs
    // little more than its launches
    const int gt = l == 1 ? (int)std::max<long long>(1, std::min<long long>(P.tiles1, 8LL * cus)) : 2 * cus;
    const int gj = l == 1 ? std::max(1, P.count) : cus;
    if (l == 1) prof_begin(TTV_PROF_HIST1, s);
    hipLaunchKernelGGL((k_hist<IdxT, MO>), dim3(l == 1 ? gt : cus), dim3(kHistThreads), 0, s, W, l, T);
    if (l == 1) prof_end(TTV_PROF_HIST1, s);
    hipLaunchKernelGGL(k_colscan, dim3(l == 1 && P.count == 1 ? 64 : 2 * cus), dim3(1024), 0, s, W, l);
    // classify blocks first (short), then the scatter's tiles
    const int slices = l == 1 ? kClassifySlices : 1;
    const int gc = std::min(gj * slices, 4 * cus);
    if (l == 1) prof_begin(TTV_PROF_SCATTER1, s);
    if (l == 1)
      hipLaunchKernelGGL((k_scatter<IdxT, F, PM, MO, false>), dim3(gc + gt), dim3(kScatterThreads), 0, s, W, l, T,
                         Tn, P.levels, slices, gc, kSortedRounds);
    else  // records only: the narrowest row class keeps the block's LDS small
      hipLaunchKernelGGL((k_scatter<IdxT, F, PM, 3, true>), dim3(gc + gt), dim3(kScatterThreads), 0, s, W, l, T, Tn,
                         P.levels, slices, gc, kSortedRounds);
    if (l == 1) prof_end(TTV_PROF_SCATTER1, s);
  }
  hipLaunchKernelGGL(k_bitmap, dim3((unsigned)std::max<long long>(1, P.L.wblocks)), dim3(256), 0, s, W);
  hipLaunchKernelGGL(k_bitmap_scan, dim3(1), dim3(1024), 0, s, W);
  hipLaunchKernelGGL((k_leaves<F, PM>), dim3(4 * cus), dim3(kLeavesThreads), 0, s, W);
  prof_begin(TTV_PROF_FINISH, s);
  // three blocks per CU, as the LDS would allow; registers keep two resident
  // per CU, and a block that starts once one ends finds the tickets gone
  hipLaunchKernelGGL((k_finish<IdxT, F, PM>), dim3(3 * cus), dim3(kFinishThreads), 0, s, W,
                     fault_on("spin") ? 0 : P.spin_limit);
  prof_end(TTV_PROF_FINISH, s);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_last_hip_error((int)e);
    return TTV_E_HIP;
  }
  return TTV_OK;
}

// Register/LDS class of the raw-index loaders: the widest row (stride_e of a
// row-major tensor, else the order) over the tensors of the run.
static int row_class(const PipePlan& P) {
  int mo = 3;
  auto one = [&](const TDesc& D) { mo = std::max(mo, row_width_class(D.order, D.stride_e, D.stride_j)); };
  if (P.descs.empty())
    one(P.d0);
  else
    for (const TDesc& D : P.descs) one(D);
  return mo;
}

template <typename IdxT, int F, int PM>
static int launch_mo(const PipePlan& P, void* ws, hipStream_t s) {
  switch (row_class(P)) {
    case 3: return launch_impl<IdxT, F, PM, 3>(P, ws, s);
    case 5: return launch_impl<IdxT, F, PM, 5>(P, ws, s);
    default: return launch_impl<IdxT, F, PM, kMaxOrder>(P, ws, s);
  }
}

int launch_pipeline(const PipePlan& P, void* ws, hipStream_t s) {
  const bool i64 = P.idx64 != 0;
  if (P.pipe_mode == kPipePerm)  // records carry nonzero indices: the value form does not matter
    return i64 ? launch_mo<long long, kF64, kPipePerm>(P, ws, s) : launch_mo<int, kF64, kPipePerm>(P, ws, s);
  if (P.pipe_mode == kPipeSegMap) {
    if (P.form == kF64)
      return i64 ? launch_mo<long long, kF64, kPipeSegMap>(P, ws, s) : launch_mo<int, kF64, kPipeSegMap>(P, ws, s);
    return i64 ? launch_mo<long long, kC32, kPipeSegMap>(P, ws, s) : launch_mo<int, kC32, kPipeSegMap>(P, ws, s);
  }
  if (P.pipe_mode == kPipeTTVSeg) {
    if (P.form == kF64)
      return i64 ? launch_mo<long long, kF64, kPipeTTVSeg>(P, ws, s) : launch_mo<int, kF64, kPipeTTVSeg>(P, ws, s);
    return i64 ? launch_mo<long long, kC32, kPipeTTVSeg>(P, ws, s) : launch_mo<int, kC32, kPipeTTVSeg>(P, ws, s);
  }
  if (P.form == kF64)
    return i64 ? launch_mo<long long, kF64, kPipeTTV>(P, ws, s) : launch_mo<int, kF64, kPipeTTV>(P, ws, s);
  return i64 ? launch_mo<long long, kC32, kPipeTTV>(P, ws, s) : launch_mo<int, kC32, kPipeTTV>(P, ws, s);
}

}  // namespace ttv
