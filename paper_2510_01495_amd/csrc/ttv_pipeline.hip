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
  __device__ __forceinline__ Rec* rec(int src) const {
    return reinterpret_cast<Rec*>(b + (src == kSrcA ? L.recA : L.recB));
  }
};

__device__ __forceinline__ int dst_of(int level) { return (level & 1) ? kSrcA : kSrcB; }

// A capacity violation (which the workspace bounds rule out) stops all later
// kernels of the call instead of letting them read unwritten records.
__device__ __forceinline__ bool aborted(const Ctrl* C) { return C->error == TTV_E_DEVICE; }
__device__ __forceinline__ int clampi(long long v, long long cap) { return (int)(v < cap ? v : cap); }

__device__ __forceinline__ long long field(long long x, int width) {
  return x & (long long)((width >= 63) ? ~0ull >> 1 : ((1ull << width) - 1ull));
}

constexpr unsigned long long kFlagAgg = 1ull << 62;
constexpr unsigned long long kFlagInc = 2ull << 62;
constexpr unsigned long long kValMask = (1ull << 62) - 1;
constexpr int kBitmapWordsPerBlock = 8192;  // 256 threads x 32 words

// ---------------------------------------------------------------------------
// Records from the COO input: key = remaining-mode indices packed with the
// first remaining mode most significant; payload = value times the vector
// entries of the contracted modes (ascending), or the nonzero's index.
// ---------------------------------------------------------------------------
template <typename IdxT, int F, int PM>
__device__ __forceinline__ void make_record(const TDesc& D, long long e, Ctrl* C, uint64_t& key,
                                            uint64_t& pay) {
  using FO = FormOps<F>;
  using In = typename FO::In;
  uint64_t k = 0;
  for (int i = 0; i < D.nrem; ++i) {
    long long x = ld_idx<IdxT>(D, e, D.rem[i]);
    if (D.validate && (x < 0 || x >= D.dims[D.rem[i]])) {
      set_error(C, TTV_E_INDEX);
      x = 0;
    }
    k |= (uint64_t)field(x, D.width[i]) << D.shift[i];
  }
  key = k;
  if (PM == kPipeSegMap) {
    pay = (uint64_t)e;
    return;
  }
  uint64_t p = FO::start_prod(static_cast<const In*>(D.vals)[e]);
  for (int c = 0; c < D.ncon; ++c) {
    const int m = D.con[c];
    long long x = ld_idx<IdxT>(D, e, m);
    if (D.validate && (x < 0 || x >= D.dims[m])) {
      set_error(C, TTV_E_INDEX);
      x = 0;
    }
    p = FO::mul_prod(p, static_cast<const In*>(D.vec[m])[x]);
  }
  pay = p;
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
  __shared__ int s_nj;
  if (threadIdx.x == 0) {
    for (int l = 0; l <= kMaxLevels; ++l) {
      C->njobs[l] = 0;
      C->ntiles[l] = 0;
    }
    C->nleaves = 0;
    C->npure = 0;
    C->ticket = 0;
    C->error = 0;
    long long tile = 0, total = 0;
    int nj = 0;
    Job* J1 = W.jobs(1);
    for (int t = 0; t < count; ++t) {
      total += D[t].nnz;
      if (D[t].nnz == 0) continue;
      Job J;
      J.start = D[t].base;
      J.size = D[t].nnz;
      J.prefix = 0;
      J.tile0 = tile;
      J.ntiles = (int)((D[t].nnz + T1 - 1) / T1);
      J.tensor = t;
      J.shift = D[t].keybits - D[t].r1;
      J.r = D[t].r1;
      J.src = kSrcRaw;
      J.pad = 0;
      J1[nj++] = J;
      tile += J.ntiles;
    }
    C->njobs[1] = nj;
    C->ntiles[1] = (int)tile;
    C->total = total;
    s_nj = nj;
  }
  __syncthreads();
  const int nj = s_nj;
  const Job* J1 = W.jobs(1);
  int* T = W.tiles(1);
  for (int j = 0; j < nj; ++j) {
    const long long t0 = J1[j].tile0;
    const int nt = J1[j].ntiles;
    for (int k = threadIdx.x; k < nt; k += blockDim.x) T[t0 + k] = j;
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
template <typename IdxT>
__global__ __launch_bounds__(256) void k_hist(WsView W, int level, int T) {
  __shared__ unsigned hist[kNDig];
  Ctrl* C = W.ctrl();
  if (aborted(C)) return;
  const int ntiles = clampi(C->ntiles[level], W.L.tcap);
  const Job* jobs = W.jobs(level);
  const int* tj = W.tiles(level);
  unsigned* table = W.table();
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const Job J = jobs[tj[t]];
    const int nd = 1 << J.r;
    const unsigned mask = (unsigned)nd - 1u;
    for (int i = threadIdx.x; i < nd; i += 256) hist[i] = 0u;
    __syncthreads();
    const long long b = (long long)(t - J.tile0) * T;
    const long long n = (J.size - b < (long long)T) ? J.size - b : (long long)T;
    if (J.src == kSrcRaw) {
      const TDesc& D = W.desc()[J.tensor];
      const long long off = J.start - D.base + b;
      for (long long rb = 0; rb < n; rb += 256) {
        const long long i = rb + threadIdx.x;
        const bool valid = i < n;
        unsigned d = 0;
        if (valid) {
          uint64_t key = 0;
          for (int m = 0; m < D.ndig_modes; ++m) {
            long long x = ld_idx<IdxT>(D, off + i, D.rem[m]);
            if (D.validate && (x < 0 || x >= D.dims[D.rem[m]])) x = 0;
            key |= (uint64_t)field(x, D.width[m]) << D.shift[m];
          }
          d = (unsigned)(key >> J.shift) & mask;
        }
        hist_add(hist, d, valid);
      }
    } else {
      const Rec* R = W.rec(J.src) + J.start + b;
      for (long long rb = 0; rb < n; rb += 256) {
        const long long i = rb + threadIdx.x;
        const bool valid = i < n;
        const unsigned d = valid ? (unsigned)(R[i].key >> J.shift) & mask : 0u;
        hist_add(hist, d, valid);
      }
    }
    __syncthreads();
    unsigned* row = table + (size_t)t * kNDig;
    for (int i = threadIdx.x; i < nd; i += 256) row[i] = hist[i];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// colscan: for every (job, digit) the exclusive prefix of the counts over the
// job's tiles, in tile order (in place); digit totals go to starts[job].
// Block = 64 digits x 16 tile groups.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_colscan(WsView W, int level) {
  __shared__ unsigned part[16][64];
  Ctrl* C = W.ctrl();
  if (aborted(C)) return;
  const int njobs = clampi(C->njobs[level], W.L.jcap);
  const Job* jobs = W.jobs(level);
  unsigned* table = W.table();
  const int dd = threadIdx.x & 63, g = threadIdx.x >> 6;
  for (long long it = blockIdx.x; it < (long long)njobs * 64; it += gridDim.x) {
    const int j = (int)(it >> 6), ch = (int)(it & 63);
    const Job J = jobs[j];
    const int nd = 1 << J.r;
    if (ch * 64 >= nd) continue;  // uniform over the block
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
__global__ __launch_bounds__(1024) void k_classify(WsView W, int level, int Tnext, int maxlevel) {
  __shared__ unsigned s_start[kNDig + 1];
  __shared__ int s_nb[kNDig];
  __shared__ unsigned char s_cls[kNDig];  // 0 empty, 1 small, 2 medium, 3 large
  __shared__ unsigned wsum[16];
  __shared__ int wsi[16];
  Ctrl* C = W.ctrl();
  if (aborted(C)) return;
  const int njobs = clampi(C->njobs[level], W.L.jcap);
  const int tid = threadIdx.x;
  for (int j = blockIdx.x; j < njobs; j += gridDim.x) {
    const Job J = W.jobs(level)[j];
    if (J.size == 0) continue;  // uniform over the block
    const int nd = 1 << J.r;
    unsigned* tot = W.starts() + (size_t)j * kNDig;
    unsigned sz[4];
    unsigned s = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int d = tid * 4 + q;
      sz[q] = d < nd ? tot[d] : 0u;
      s += sz[q];
    }
    unsigned total;
    unsigned ex = block_excl_scan<1024>(s, wsum, total);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int d = tid * 4 + q;
      if (d < nd) {
        s_start[d] = ex;
        tot[d] = ex;
        s_cls[d] = sz[q] == 0 ? 0 : (sz[q] <= (unsigned)kSmall ? 1 : (sz[q] <= (unsigned)kCap ? 2 : 3));
      }
      ex += sz[q];
    }
    if (tid == 0) s_start[nd] = total;
    __syncthreads();
    // previous non-empty digit (exclusive max-scan)
    int lm = -1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int d = tid * 4 + q;
      if (d < nd && s_cls[d] != 0) lm = d;
    }
    int prev = block_excl_mm<true>(lm, -1, wsi);
    // chunk heads and boundaries
    bool bnd[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int d = tid * 4 + q;
      bnd[q] = false;
      if (d < nd && s_cls[d] != 0) {
        if (s_cls[d] != 1) {
          bnd[q] = true;
        } else {
          const bool head = prev < 0 || s_cls[prev] != 1 ||
                            (J.start + s_start[prev]) / kSmall != (J.start + s_start[d]) / kSmall;
          bnd[q] = head;
        }
        prev = d;
      }
    }
    // next boundary after each digit (suffix min-scan, done on reversed order)
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int d = tid * 4 + q;
      if (d < nd) s_nb[d] = bnd[q] ? d : nd;
    }
    __syncthreads();
    const int rt = 1023 - tid;  // this thread scans the digits of thread rt, reversed
    int rv = nd;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int d = rt * 4 + q;
      if (d < nd) rv = min(rv, s_nb[d]);
    }
    int nxt = block_excl_mm<false>(rv, nd, wsi);  // min over digits of threads > rt
    int nbq[4];
#pragma unroll
    for (int q = 3; q >= 0; --q) {
      const int d = rt * 4 + q;
      nbq[q] = nxt;  // first boundary strictly after digit d
      if (d < nd) nxt = min(nxt, s_nb[d]);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int d = rt * 4 + q;
      if (d < nd) s_nb[d] = nbq[q];
    }
    __syncthreads();
    // emit jobs and leaves
    const int dstb = dst_of(level);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int d = tid * 4 + q;
      if (d >= nd || !bnd[q]) continue;
      const long long gstart = J.start + s_start[d];
      const unsigned long long dbase = J.prefix | ((unsigned long long)d << J.shift);
      const int cls = s_cls[d];
      if (cls == 3 && J.shift > 0) {
        const long long size = sz[q];
        if (level + 1 > maxlevel) {
          set_error(C, TTV_E_DEVICE);
          continue;
        }
        const int jid = atomicAdd(&C->njobs[level + 1], 1);
        if (jid >= W.L.jcap) {
          set_error(C, TTV_E_DEVICE);
          continue;
        }
        int nt = (int)((size + Tnext - 1) / Tnext);
        const int t0 = atomicAdd(&C->ntiles[level + 1], nt);
        Job N;
        N.start = gstart;
        N.size = size;
        if ((long long)t0 + nt > W.L.tcap) {  // keep a valid, empty job in the slot
          set_error(C, TTV_E_DEVICE);
          nt = 0;
          N.size = 0;
        }
        N.r = J.shift < kRMax ? J.shift : kRMax;
        N.shift = J.shift - N.r;
        N.prefix = dbase;
        N.tile0 = t0;
        N.ntiles = nt;
        N.tensor = J.tensor;
        N.src = dstb;
        N.pad = 0;
        W.jobs(level + 1)[jid] = N;
        int* T = W.tiles(level + 1);
        for (int k = 0; k < nt; ++k) T[t0 + k] = jid;
        continue;
      }
      Leaf Lf;
      Lf.start = gstart;
      Lf.base = dbase;
      Lf.tensor = J.tensor;
      Lf.src = dstb;
      Lf.ptile0 = 0;
      Lf.nptiles = 0;
      Lf.pad = 0;
      Lf.kind = kLeafSort;
      if (cls == 3) {  // single key, too large for one block: pure leaf
        Lf.size = sz[q];
        Lf.kind = kLeafPure;
        Lf.bits = 0;
        const int np = (int)((Lf.size + kPureTile - 1) / kPureTile);
        const int p0 = atomicAdd(&C->npure, np);
        if ((long long)p0 + np > W.L.pcap) {
          set_error(C, TTV_E_DEVICE);
          continue;
        }
        Lf.ptile0 = p0;
        Lf.nptiles = np;
      } else if (cls == 2) {
        Lf.size = sz[q];
        Lf.bits = J.shift;
      } else {
        const int nb = s_nb[d];
        Lf.size = (long long)s_start[nb] - s_start[d];
        Lf.bits = J.shift + bitlen64((unsigned long long)(nb - d - 1));
      }
      const int lid = atomicAdd(&C->nleaves, 1);
      if (lid >= W.L.lcap) {
        set_error(C, TTV_E_DEVICE);
        continue;
      }
      W.leaves()[lid] = Lf;
      if (Lf.kind == kLeafPure) {
        int* pl = W.ptile_leaf();
        for (int k = 0; k < Lf.nptiles; ++k) pl[Lf.ptile0 + k] = lid;
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
template <typename IdxT, int F, int PM>
__global__ __launch_bounds__(kScatterThreads) void k_scatter(WsView W, int level, int T) {
  constexpr int IPT = kScatterIPT;
  constexpr int RW = 64 * IPT;            // records per wave per round
  constexpr int RN = kScatterThreads * IPT;
  __shared__ unsigned cursor[kNDig];
  __shared__ unsigned short wcnt[4][kNDig];
  Ctrl* C = W.ctrl();
  if (aborted(C)) return;
  const int ntiles = clampi(C->ntiles[level], W.L.tcap);
  const Job* jobs = W.jobs(level);
  const int* tj = W.tiles(level);
  const int w = threadIdx.x >> 6;
  const unsigned ln = lane_id();
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int jid = tj[t];
    const Job J = jobs[jid];
    const int nd = 1 << J.r;
    const unsigned mask = (unsigned)nd - 1u;
    const unsigned* row = W.table() + (size_t)t * kNDig;
    const unsigned* st = W.starts() + (size_t)jid * kNDig;
    for (int i = threadIdx.x; i < nd; i += kScatterThreads) {
      cursor[i] = st[i] + row[i];
      wcnt[0][i] = 0;
      wcnt[1][i] = 0;
      wcnt[2][i] = 0;
      wcnt[3][i] = 0;
    }
    __syncthreads();
    const long long b = (long long)(t - J.tile0) * T;
    const long long n = (J.size - b < (long long)T) ? J.size - b : (long long)T;
    Rec* dst = W.rec(dst_of(level)) + J.start;
    const Rec* srcR = (J.src == kSrcRaw) ? nullptr : W.rec(J.src) + J.start + b;
    const TDesc* Dp = W.desc() + J.tensor;
    const long long roff = J.start - Dp->base + b;
    for (long long rb = 0; rb < n; rb += RN) {
      uint64_t key[IPT], pay[IPT];
      unsigned dg[IPT], rk[IPT];
      bool first[IPT];
#pragma unroll
      for (int j = 0; j < IPT; ++j) {
        const long long i = rb + (long long)w * RW + j * 64 + ln;
        if (i < n) {
          if (srcR) {
            const Rec r = srcR[i];
            key[j] = r.key;
            pay[j] = r.pay;
          } else {
            make_record<IdxT, F, PM>(*Dp, roff + i, C, key[j], pay[j]);
          }
        }
      }
#pragma unroll
      for (int j = 0; j < IPT; ++j) {
        const long long i = rb + (long long)w * RW + j * 64 + ln;
        const bool valid = i < n;
        const uint64_t vm = ballot(valid);
        dg[j] = valid ? (unsigned)(key[j] >> J.shift) & mask : 0u;
        const uint64_t peers = match_digit(dg[j], J.r, vm);
        unsigned old = 0;
        if (valid) old = wcnt[w][dg[j]];
        const unsigned below = count_below(peers);
        rk[j] = old + below;
        first[j] = valid && old == 0 && below == 0;
        if (valid) wcnt[w][dg[j]] = (unsigned short)(old + (unsigned)__popcll(peers));
      }
      __syncthreads();
      bool up[IPT];
#pragma unroll
      for (int j = 0; j < IPT; ++j) {
        const long long i = rb + (long long)w * RW + j * 64 + ln;
        up[j] = false;
        if (i < n) {
          const unsigned d = dg[j];
          unsigned lower = 0;
          for (int q = 0; q < w; ++q) lower += wcnt[q][d];
          const unsigned pos = cursor[d] + lower + rk[j];
          Rec r;
          r.key = key[j];
          r.pay = pay[j];
          dst[pos] = r;
          up[j] = first[j] && lower == 0;
        }
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < IPT; ++j) {
        if (up[j]) {
          const unsigned d = dg[j];
          cursor[d] += (unsigned)wcnt[0][d] + wcnt[1][d] + wcnt[2][d] + wcnt[3][d];
        }
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < IPT; ++j)
        if (first[j]) wcnt[w][dg[j]] = 0;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// pure reduce: partial sums of single-key leaves, kPureTile records per block
// ---------------------------------------------------------------------------
template <int F>
__global__ __launch_bounds__(256) void k_pure(WsView W) {
  using FO = FormOps<F>;
  using Acc = typename FO::Acc;
  __shared__ Acc red[256];
  Ctrl* C = W.ctrl();
  if (aborted(C)) return;
  const int np = clampi(C->npure, W.L.pcap);
  for (int p = blockIdx.x; p < np; p += gridDim.x) {
    const Leaf Lf = W.leaves()[W.ptile_leaf()[p]];
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
}

// ---------------------------------------------------------------------------
// leaf numbering: popcount prefix of the leaf-start bitmap
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bm_a(WsView W) {
  __shared__ unsigned wsum[4];
  const long long w0 = (long long)blockIdx.x * kBitmapWordsPerBlock + threadIdx.x * 32;
  const unsigned* bm = W.bitmap();
  unsigned c[32];
  unsigned s = 0;
#pragma unroll
  for (int q = 0; q < 32; ++q) {
    const long long wi = w0 + q;
    c[q] = wi < W.L.words ? (unsigned)__popc(bm[wi]) : 0u;
    s += c[q];
  }
  unsigned tot;
  unsigned ex = block_excl_scan<256>(s, wsum, tot);
  unsigned* wp = W.wordpre();
#pragma unroll
  for (int q = 0; q < 32; ++q) {
    const long long wi = w0 + q;
    if (wi < W.L.words) wp[wi] = ex;
    ex += c[q];
  }
  if (threadIdx.x == 0) W.blockpre()[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_bm_b(WsView W) {
  __shared__ unsigned wsum[16];
  unsigned* bp = W.blockpre();
  const long long n = W.L.wblocks;
  unsigned carry = 0;
  for (long long b0 = 0; b0 < n; b0 += 1024) {
    const long long i = b0 + threadIdx.x;
    const unsigned v = i < n ? bp[i] : 0u;
    unsigned tot;
    const unsigned ex = block_excl_scan<1024>(v, wsum, tot);
    if (i < n) bp[i] = carry + ex;
    carry += tot;
  }
}

__global__ __launch_bounds__(256) void k_rank(WsView W) {
  Ctrl* C = W.ctrl();
  if (aborted(C)) return;
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
__device__ long long lookback(unsigned long long* S, int r, int spin_limit, Ctrl* C) {
  long long prefix = 0;
  for (int j = r - 1; j >= 0; --j) {
    unsigned long long s;
    int spins = 0;
    for (;;) {
      s = __hip_atomic_load(&S[j], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
      if (s >> 62) break;
      if (++spins > spin_limit) {
        set_error(C, TTV_E_DEVICE);
        return prefix;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    prefix += (long long)(s & kValMask);
    if ((s >> 62) == 2) break;
  }
  return prefix;
}

__device__ __forceinline__ void publish(unsigned long long* S, int r, unsigned long long v) {
  __hip_atomic_store(&S[r], v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename IdxT>
__device__ __forceinline__ void write_coords(const TDesc& D, long long row, uint64_t key) {
  IdxT* o = static_cast<IdxT*>(D.out_subs) + row * D.nrem;
  for (int i = 0; i < D.nrem; ++i) {
    const uint64_t m = D.width[i] >= 64 ? ~0ull : ((1ull << D.width[i]) - 1ull);
    o[i] = (IdxT)((key >> D.shift[i]) & m);
  }
}

template <int F>
__device__ __forceinline__ void write_value(const TDesc& D, long long row, double v64,
                                            const typename FormOps<F>::Acc& a) {
  if (F == kF64) {
    static_cast<double*>(D.out_vals)[row] = v64;
  } else if (D.out_f64) {
    static_cast<double*>(D.out_vals)[row] = v64;
  } else {
    static_cast<float*>(D.out_vals)[row] = (float)v64;
  }
}

template <typename IdxT, int F, int PM>
__global__ __launch_bounds__(kFinishThreads) void k_finish(WsView W, int spin_limit) {
  using FO = FormOps<F>;
  using Acc = typename FO::Acc;
  constexpr int NT = kFinishThreads;
  constexpr int IPT = kFinishIPT;
  constexpr int NW = NT / 64;
  __shared__ unsigned sk[kCap];
  __shared__ unsigned short si[kCap];
  __shared__ unsigned cnt[NW * 256];
  __shared__ unsigned wsum[NW];
  __shared__ Seg<F> wagg[NW];
  __shared__ int s_ticket;
  __shared__ long long s_prefix;
  Ctrl* C = W.ctrl();
  if (aborted(C)) return;
  const int nleaves = clampi(C->nleaves, W.L.lcap);
  unsigned long long* S = W.status();
  const int tid = threadIdx.x, w = tid >> 6;
  const unsigned ln = lane_id();
  for (;;) {
    if (tid == 0) s_ticket = atomicAdd(&C->ticket, 1);
    __syncthreads();
    const int r = s_ticket;
    if (r >= nleaves) break;
    const Leaf Lf = W.ordered()[r];
    const TDesc& D = W.desc()[Lf.tensor];
    const bool first = Lf.start == D.base;
    const bool last = Lf.start + Lf.size == D.base + D.nnz;
    const Rec* R = W.rec(Lf.src) + Lf.start;
    const long long n = Lf.size;
    if (Lf.kind != kLeafPure && (n > kCap || n <= 0)) {  // excluded by classification
      if (tid == 0) {
        set_error(C, TTV_E_DEVICE);
        publish(S, r, kFlagInc);
      }
      __syncthreads();
      continue;
    }
    if (Lf.kind == kLeafPure) {
      if (tid == 0) {
        publish(S, r, (first ? kFlagInc : kFlagAgg) | 1ull);
        double v = 0.0;
        const double* P = W.partials() + Lf.ptile0;
        for (int k = 0; k < Lf.nptiles; ++k) v += P[k];
        const long long prefix = first ? 0 : lookback(S, r, spin_limit, C);
        if (!first) publish(S, r, kFlagInc | (unsigned long long)(prefix + 1));
        s_prefix = prefix;
        if (PM == kPipeTTV) {
          write_coords<IdxT>(D, prefix, Lf.base);
          write_value<F>(D, prefix, v, FO::zero());
        }
        if (last && D.out_nnz) *D.out_nnz = prefix + 1;
      }
      if (PM == kPipeSegMap) {
        __syncthreads();
        const long long row = s_prefix;
        for (long long i = tid; i < n; i += NT) D.seg_out[(long long)R[i].pay] = (int32_t)row;
      }
      __syncthreads();
      continue;
    }
    // ---- load relative keys (wave-striped) ----
    const bool wide = Lf.bits > 32;
    unsigned k[IPT];
    unsigned short ix[IPT];
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      const int i = w * (64 * IPT) + j * 64 + (int)ln;
      k[j] = 0;
      ix[j] = (unsigned short)i;
      if (i < n) k[j] = (unsigned)(R[i].key - Lf.base);
    }
    const int npass = (Lf.bits + kSortDigit - 1) / kSortDigit;
    for (int pass = 0; pass < npass; ++pass) {
      const int sh = pass * kSortDigit;
      for (int q = tid; q < NW * 256; q += NT) cnt[q] = 0u;
      __syncthreads();
      unsigned dg[IPT], rk[IPT];
#pragma unroll
      for (int j = 0; j < IPT; ++j) {
        const int i = w * (64 * IPT) + j * 64 + (int)ln;
        const bool valid = i < n;
        const uint64_t vm = ballot(valid);
        unsigned d = 0;
        if (valid) {
          if (wide)
            d = (unsigned)(((R[ix[j]].key - Lf.base) >> sh) & 255u);
          else
            d = (k[j] >> sh) & 255u;
        }
        dg[j] = d;
        const uint64_t peers = match_digit(d, kSortDigit, vm);
        unsigned old = 0;
        if (valid) old = cnt[w * 256 + d];
        rk[j] = old + count_below(peers);
        if (valid) cnt[w * 256 + d] = old + (unsigned)__popcll(peers);
      }
      __syncthreads();
      {  // exclusive scan of the counters in (digit, wave) order
        unsigned v[4], s = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = tid * 4 + q;
          v[q] = cnt[(e & 7) * 256 + (e >> 3)];
          s += v[q];
        }
        unsigned tot;
        unsigned ex = block_excl_scan<NT>(s, wsum, tot);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = tid * 4 + q;
          cnt[(e & 7) * 256 + (e >> 3)] = ex;
          ex += v[q];
        }
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < IPT; ++j) {
        const int i = w * (64 * IPT) + j * 64 + (int)ln;
        if (i < n) {
          const unsigned dest = cnt[w * 256 + dg[j]] + rk[j];
          sk[dest] = k[j];
          si[dest] = ix[j];
        }
      }
      __syncthreads();
      if (pass + 1 < npass) {
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
          const int i = w * (64 * IPT) + j * 64 + (int)ln;
          if (i < n) {
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
        const int i = w * (64 * IPT) + j * 64 + (int)ln;
        if (i < n) {
          sk[i] = k[j];
          si[i] = ix[j];
        }
      }
      __syncthreads();
    }
    // ---- segmented reduction over the sorted order (blocked) ----
    const int p0 = tid * IPT;
    uint64_t fk[IPT];  // full keys (wide) or relative keys
    bool head[IPT];
    unsigned hc = 0;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      const int p = p0 + j;
      head[j] = false;
      fk[j] = 0;
      if (p < n) {
        fk[j] = wide ? R[si[p]].key : (uint64_t)sk[p];
        if (p == 0) {
          head[j] = true;
        } else {
          const uint64_t pk = (j > 0) ? fk[j - 1] : (wide ? R[si[p - 1]].key : (uint64_t)sk[p - 1]);
          head[j] = pk != fk[j];
        }
        hc += head[j] ? 1u : 0u;
      }
    }
    unsigned u;
    const unsigned hb = block_excl_scan<NT>(hc, wsum, u);
    if (tid == 0 && !first) publish(S, r, kFlagAgg | (unsigned long long)u);
    if (tid == 0 && first) publish(S, r, kFlagInc | (unsigned long long)u);
    Acc val[IPT];
    Seg<F> agg;
    agg.f = 0;
    agg.v = FO::zero();
    uint64_t pay[IPT];
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      const int p = p0 + j;
      pay[j] = 0;
      if (p < n) {
        pay[j] = R[si[p]].pay;
        if (PM == kPipeTTV) {
          const Acc x = FO::from_pay(pay[j]);
          if (head[j]) {
            agg.v = x;
            agg.f = 1;
          } else {
            agg.v = FO::add(agg.v, x);
          }
          val[j] = agg.v;
        }
      }
    }
    Seg<F> carry;
    carry.f = 0;
    carry.v = FO::zero();
    if (PM == kPipeTTV) {
      // exclusive segmented scan of the thread aggregates
      Seg<F> inc = agg;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        Seg<F> y;
        y.v = FO::shfl_up(inc.v, o);
        y.f = __shfl_up(inc.f, o, 64);
        if ((int)ln >= o) inc = seg_combine<F>(y, inc);
      }
      Seg<F> ex;
      ex.v = FO::shfl_up(inc.v, 1);
      ex.f = __shfl_up(inc.f, 1, 64);
      if (ln == 0) {
        ex.f = 0;
        ex.v = FO::zero();
      }
      if (ln == 63) wagg[w] = inc;
      __syncthreads();
      Seg<F> wc;
      wc.f = 0;
      wc.v = FO::zero();
      for (int q = 0; q < w; ++q) wc = seg_combine<F>(wc, wagg[q]);
      carry = seg_combine<F>(wc, ex);
    }
    if (tid == 0) {
      const long long prefix = first ? 0 : lookback(S, r, spin_limit, C);
      if (!first) publish(S, r, kFlagInc | (unsigned long long)(prefix + u));
      s_prefix = prefix;
      if (last && D.out_nnz) *D.out_nnz = prefix + u;
    }
    __syncthreads();
    const long long prefix = s_prefix;
    // ---- write ----
    unsigned lh = 0;
    bool seen = false;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      const int p = p0 + j;
      if (p >= n) continue;
      if (head[j]) {
        ++lh;
        seen = true;
      }
      const long long rowi = prefix + hb + lh - 1;
      if (PM == kPipeSegMap) {
        D.seg_out[(long long)pay[j]] = (int32_t)rowi;
        continue;
      }
      bool end;
      if (p == n - 1) {
        end = true;
      } else if (j + 1 < IPT) {
        end = head[j + 1];
      } else {
        const uint64_t nk = wide ? R[si[p + 1]].key : (uint64_t)sk[p + 1];
        end = nk != fk[j];
      }
      if (end) {
        const Acc a = seen ? val[j] : FO::add(carry.v, val[j]);
        const uint64_t key = wide ? fk[j] : Lf.base + fk[j];
        write_coords<IdxT>(D, rowi, key);
        write_value<F>(D, rowi, FO::to_f64(a), a);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// host launcher
// ---------------------------------------------------------------------------
template <typename IdxT, int F, int PM>
static int launch_impl(const PipePlan& P, void* ws, hipStream_t s) {
  WsView W;
  W.b = static_cast<char*>(ws);
  W.L = P.L;
  const int cus = P.cus;
  const int g_init = (int)std::min<long long>(std::max<long long>(1, (P.L.words + 255) / 256), 4LL * cus);
  hipLaunchKernelGGL(k_init, dim3(g_init), dim3(256), 0, s, W, P.d0, P.descs_dev, P.count, P.T1);
  for (int l = 1; l <= P.levels; ++l) {
    const int T = l == 1 ? P.T1 : P.T2;
    const int Tn = P.T2;
    const int gt = l == 1 ? (int)std::max<long long>(1, std::min<long long>(P.tiles1, 8LL * cus)) : 4 * cus;
    const int gj = l == 1 ? std::max(1, P.count) : 2 * cus;
    hipLaunchKernelGGL(k_hist<IdxT>, dim3(gt), dim3(256), 0, s, W, l, T);
    hipLaunchKernelGGL(k_colscan, dim3(l == 1 ? std::max(1, P.count * 64) : 4 * cus), dim3(1024), 0, s, W, l);
    hipLaunchKernelGGL(k_classify, dim3(std::min(gj, 4 * cus)), dim3(1024), 0, s, W, l, Tn, P.levels);
    hipLaunchKernelGGL((k_scatter<IdxT, F, PM>), dim3(gt), dim3(kScatterThreads), 0, s, W, l, T);
  }
  hipLaunchKernelGGL(k_pure<F>, dim3(2 * cus), dim3(256), 0, s, W);
  hipLaunchKernelGGL(k_bm_a, dim3((unsigned)std::max<long long>(1, P.L.wblocks)), dim3(256), 0, s, W);
  hipLaunchKernelGGL(k_bm_b, dim3(1), dim3(1024), 0, s, W);
  hipLaunchKernelGGL(k_rank, dim3(2 * cus), dim3(256), 0, s, W);
  hipLaunchKernelGGL((k_finish<IdxT, F, PM>), dim3(2 * cus), dim3(kFinishThreads), 0, s, W, P.spin_limit);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_last_hip_error((int)e);
    return TTV_E_HIP;
  }
  return TTV_OK;
}

int launch_pipeline(const PipePlan& P, void* ws, hipStream_t s) {
  const bool i64 = P.idx64 != 0;
  if (P.pipe_mode == kPipeSegMap) {
    if (P.form == kF64)
      return i64 ? launch_impl<long long, kF64, kPipeSegMap>(P, ws, s)
                 : launch_impl<int, kF64, kPipeSegMap>(P, ws, s);
    return i64 ? launch_impl<long long, kC32, kPipeSegMap>(P, ws, s)
               : launch_impl<int, kC32, kPipeSegMap>(P, ws, s);
  }
  if (P.form == kF64)
    return i64 ? launch_impl<long long, kF64, kPipeTTV>(P, ws, s) : launch_impl<int, kF64, kPipeTTV>(P, ws, s);
  return i64 ? launch_impl<long long, kC32, kPipeTTV>(P, ws, s) : launch_impl<int, kC32, kPipeTTV>(P, ws, s);
}

}  // namespace ttv
