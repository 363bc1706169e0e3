// Repeated sparse TTV with a fixed tensor and mode (the tensor is reused
// across calls with a new vector each time, as in the iterative methods of
// Sec. 3.3's motivation): the keyed sort of Eq. 3's index tuples runs once.
//
// Setup runs the sorting pipeline in its permutation mode: it writes the
// output coordinates (which do not depend on the vector) and, for every
// position of the sorted order, the nonzero there and its output row.  A
// gather then stores in the caller's plan buffer, in sorted order, the values
// and the contracted-mode indices (32-bit when the mode's length allows), one
// bit per position marking the first position of every output row, and the
// output row of every chunk's first position.
//
// Each apply is one streaming pass over that buffer: per sorted position the
// product value x v[index], and a segmented sum over runs of equal output
// row (a run starts at a marked position; a row's number is the chunk's first
// row plus the marks counted since).  Chunks of kReuseChunk positions are reduced by one block each
// (in-wave DPP segmented scans, carried across rounds and waves in order);
// rows inside a chunk are written directly, and the partial sums of a
// chunk's first and last rows are combined by a second kernel in chunk
// order, in FP64.  Every sum is formed in one fixed order (bitwise
// repeatable); the order differs from ttv_coo's, so the two agree within
// the rounding bound, not bitwise.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <type_traits>

#include "ttv.h"
#include "ttv_carry.hpp"
#include "ttv_device.hpp"
#include "ttv_host.h"

struct ttv_reuse_plan {
  ttv::PipePlan P;  // permutation-mode pipeline of the setup
  ttv_coo_desc X;   // descriptor (its arrays are read by setup only)
  int mode = 0;
  int nrem = 0;
  int idx64 = 1;
  int form = ttv::kF64;
  int out_f64 = 1;
  long long nnz = 0;
  long long nchunks = 0;
  int sidx32 = 1;  // contracted-mode indices stored as uint32 (the mode's length is at most 2^32)
  size_t off_sv = 0, off_sidx = 0, off_heads = 0, off_row0 = 0, off_groups = 0, off_carry = 0, data_bytes = 0;
  size_t off_perm = 0, off_rowid = 0, setup_bytes = 0;  // setup workspace: pipeline, permutation, rows
  void* data = nullptr;                  // bound by setup
  int cus = 0;                           // compute units of the setup's device
};

namespace ttv {
namespace {

constexpr int kReuseThreads = 256;                      // 4 waves, each with its own chunk
constexpr int kReuseLdsThreads = 1024;                  // v staged in LDS: 16 waves looping over chunks
constexpr int kReuseIPT = 8;
constexpr int kReuseChunk = 64 * kReuseIPT;             // sorted positions per wave
constexpr size_t kReuseHdr = 256;                       // int64 nnz_out at offset 0
constexpr size_t kReuseMaxVLds = 128 * 1024;            // largest vector staged in LDS

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// sv[k] = vals[perm[k]], sidx[k] = subs(perm[k], mode); heads bit k set when
// sorted position k starts an output row; row0[c] = output row of position
// c * kReuseChunk; the header gets nnz_out.  One wave per 64 positions.
template <typename IdxT, typename In, typename SIdx>
__global__ __launch_bounds__(256) void k_reuse_gather(const IdxT* subs, long long se, long long sjm, const In* vals,
                                                      const int32_t* perm, const int32_t* rowid, long long nnz,
                                                      In* sv, SIdx* sidx, unsigned long long* heads,
                                                      long long* row0, const long long* out_nnz, long long* hdr) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *hdr = *out_nnz;
  const gptr<const IdxT> gs = to_global(subs);
  const gptr<const In> gv = to_global(vals);
  const gptr<const int32_t> gp = to_global(perm);
  const gptr<const int32_t> gr = to_global(rowid);
  const unsigned ln = lane_id();
  const long long nw = (nnz + 63) / 64;
  const long long tw = (long long)gridDim.x * (blockDim.x / 64);
  for (long long q = (long long)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); q < nw; q += tw) {
    const long long k = q * 64 + ln;
    bool h = false;
    if (k < nnz) {
      const long long e = gp[k];
      sv[k] = gv[e];
      sidx[k] = (SIdx)gs[e * se + sjm];
      const int32_t r = gr[k];
      h = k == 0 || r != gr[k - 1];
      if (k % kReuseChunk == 0) row0[k / kReuseChunk] = r;
    }
    const uint64_t m = ballot(h);
    if (ln == 0) heads[q] = m;
  }
}

struct ReuseArgs {
  const void* sv;
  const void* sidx;
  const unsigned long long* heads;
  const long long* row0;
  const CarryGroup* groups;
  double* carry;
  const void* v;
  void* out;
  long long nnz;
  long long nchunks;
  long long vlen;
  int out_f64;
};

template <int F>
__device__ __forceinline__ void put(const ReuseArgs& A, long long row, double x) {
  if (A.out_f64)
    to_global(static_cast<double*>(A.out))[row] = x;
  else
    to_global(static_cast<float*>(A.out))[row] = (float)x;
}

// One chunk of one wave: products, heads and ends of runs of equal row, the
// segmented sums; rows inside the chunk are written, its first and last
// rows' partial sums go to the carries.  The chunk's first position always
// opens a run here (its row may continue from the previous chunk).  `vp`
// points to v in global memory or in LDS.
template <typename SIdx, int F, typename VP>
__device__ __forceinline__ void apply_chunk(const ReuseArgs& A, long long c, VP vp) {
  using FO = FormOps<F>;
  using Acc = typename FO::Acc;
  using In = typename FO::In;
  constexpr int IPT = kReuseIPT;
  const unsigned ln = lane_id();
  const gptr<const In> sv = to_global(static_cast<const In*>(A.sv));
  const gptr<const SIdx> sidx = to_global(static_cast<const SIdx*>(A.sidx));
  const long long k0 = c * kReuseChunk;
  const int n = (int)std::min<long long>(kReuseChunk, A.nnz - k0);
  uint64_t hm[IPT];  // run heads of every round of 64 positions
  bool end[IPT];
  Acc prod[IPT];
  {
    In a[IPT];
    SIdx ix[IPT];
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      const int p = j * 64 + (int)ln;
      const bool ok = p < n;
      a[j] = ok ? sv[k0 + p] : (In)0;
      ix[j] = ok ? sidx[k0 + p] : (SIdx)0;
    }
    uint64_t wd[IPT];
#pragma unroll
    for (int j = 0; j < IPT; ++j) wd[j] = uniform64(j * 64 < n ? A.heads[(k0 >> 6) + j] : 0ull);
    In g[IPT];
#pragma unroll
    for (int j = 0; j < IPT; ++j) g[j] = (j * 64 + (int)ln < n) ? vp[ix[j]] : (In)0;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      const int p = j * 64 + (int)ln;
      const int rem = n - j * 64;  // positions of this round inside the chunk
      const uint64_t vm = rem >= 64 ? ~0ull : (rem <= 0 ? 0ull : (~0ull >> (64 - rem)));
      hm[j] = (wd[j] | (j == 0 ? 1ull : 0ull)) & vm;
      // the last position of a round is followed by the next round's first
      // (or ends the chunk)
      const uint64_t nxt = ln < 63 ? (hm[j] >> (ln + 1)) : (j + 1 < IPT ? wd[j + 1] : 1ull);
      end[j] = p < n && (p == n - 1 || (nxt & 1ull));
      prod[j] = FO::from_pay(FO::mul_prod(FO::start_prod(a[j]), g[j]));
    }
  }
  // segmented scan in rounds of 64 consecutive positions, the running sum of
  // the open run carried from round to round; then the ends are written.
  // A run's row is the chunk's first row plus the heads after the first.
  const long long r0 = A.row0[c];
  Acc run = FO::zero();
  unsigned hrun = 0;
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const int p = j * 64 + (int)ln;
    Seg<F> e;
    e.f = (hm[j] >> ln) & 1ull ? 1 : 0;
    e.v = p < n ? prod[j] : FO::zero();
    e = wave_seg_scan<F>(e);
    const Acc val = e.f ? e.v : FO::add(run, e.v);
    run = FO::shfl_last(val);
    if (end[j]) {
      const unsigned heads = hrun + (unsigned)__popcll(hm[j] & (~0ull >> (63 - ln)));
      const bool firstrun = heads == 1, lastrun = p == n - 1;
      const double x = FO::to_f64(val);
      if (!firstrun && !lastrun)
        put<F>(A, r0 + (long long)heads - 1, x);
      else if (firstrun)
        to_global(A.carry)[2 * c] = x;
      else
        to_global(A.carry)[2 * c + 1] = x;
    }
    hrun += (unsigned)__popcll(hm[j]);
  }
}

// One chunk per wave, v gathered from global memory (no block-level
// synchronisation).
template <typename SIdx, int F>
__global__ __launch_bounds__(kReuseThreads) void k_reuse_apply(ReuseArgs A) {
  using In = typename FormOps<F>::In;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const long long c = (long long)blockIdx.x * (kReuseThreads / 64) + w;
  if (c >= A.nchunks) return;  // the whole wave
  apply_chunk<SIdx, F>(A, c, to_global(static_cast<const In*>(A.v)));
}

// v staged in LDS once per block (a gather from LDS instead of one cache
// line per lane); the block's waves then loop over chunks.
template <typename SIdx, int F>
__global__ __launch_bounds__(kReuseLdsThreads) void k_reuse_apply_lds(ReuseArgs A) {
  using In = typename FormOps<F>::In;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  In* vs = reinterpret_cast<In*>(smem);
  const gptr<const In> gv = to_global(static_cast<const In*>(A.v));
  // the copy: 16 loads per thread issued together, then their LDS stores
  for (long long b = 0; b < A.vlen; b += 16LL * kReuseLdsThreads) {
    In t[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const long long i = b + (long long)q * kReuseLdsThreads + threadIdx.x;
      t[q] = i < A.vlen ? gv[i] : (In)0;
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const long long i = b + (long long)q * kReuseLdsThreads + threadIdx.x;
      if (i < A.vlen) vs[i] = t[q];
    }
  }
  __syncthreads();
  constexpr int NW = kReuseLdsThreads / 64;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (long long c = (long long)blockIdx.x * NW + w; c < A.nchunks; c += (long long)gridDim.x * NW)
    apply_chunk<SIdx, F>(A, c, static_cast<const In*>(vs));
}

// Rows that touch a chunk boundary: the entry that opens a row adds the
// group's following entries in a fixed order that depends only on the plan
// (FP64): serially for up to kSerial entries, else the wave's 64 lanes sum
// strided subsets serially and a butterfly adds them.
template <int F>
__global__ __launch_bounds__(256) void k_reuse_combine(ReuseArgs A) {
  constexpr long long kSerial = 32;
  const long long E = 2 * A.nchunks;
  const gptr<const double> cv = to_global(static_cast<const double*>(A.carry));
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  CarryGroup g{-1, 0};
  double s = 0.0;
  if (e < E) {
    g.row = to_global(A.groups)[e].row;
    g.cnt = to_global(A.groups)[e].cnt;
    if (g.row >= 0) s = cv[e];
  }
  const long long c1 = e >> 1;
  if (g.row >= 0 && g.cnt <= kSerial) {
#pragma unroll 8
    for (long long k = 0; k < g.cnt; ++k) s += cv[2 * (c1 + 1 + k)];
    put<F>(A, g.row, s);
  }
  // long rows: the whole wave sums each one
  const unsigned ln = lane_id();
  uint64_t todo = ballot(g.row >= 0 && g.cnt > kSerial);
  while (todo) {
    const int L = __ffsll((long long)todo) - 1;
    todo &= todo - 1;
    const long long cL = __shfl(c1, L, 64), nL = __shfl(g.cnt, L, 64);
    double part = 0.0;
    for (long long k = ln; k < nL; k += 64) part += cv[2 * (cL + 1 + k)];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) part += __shfl_xor(part, d, 64);
    if ((int)ln == L) put<F>(A, g.row, s + part);
  }
}

int check_plan(const ttv_reuse_plan* p) { return p ? TTV_OK : TTV_E_NULL; }

}  // namespace
}  // namespace ttv

using namespace ttv;

extern "C" {

int ttv_reuse_plan_create(const ttv_coo_desc* X, int32_t mode, int32_t flags, ttv_reuse_plan** plan) {
  if (flags & TTV_DROP_ZEROS) return TTV_E_ARG;  // a plan keeps every row (which sums vanish depends on v)
  if (!plan) return TTV_E_NULL;
  *plan = nullptr;
  ttv_reuse_plan* p = new (std::nothrow) ttv_reuse_plan();
  if (!p) return TTV_E_ARG;
  int rc = plan_single(X, 1, &mode, flags, kPipePerm, p->P);
  if (rc) {
    delete p;
    return rc;
  }
  p->X = *X;
  p->mode = mode;
  p->nrem = X->order - 1;
  p->idx64 = X->index_dtype == TTV_I64 ? 1 : 0;
  p->form = X->value_dtype == TTV_F64 ? kF64 : kC32;
  p->out_f64 = (p->form == kF64 || (flags & TTV_OUT_F64)) ? 1 : 0;
  p->nnz = X->nnz;
  p->nchunks = (X->nnz + kReuseChunk - 1) / kReuseChunk;
  p->sidx32 = X->shape[mode] <= (1LL << 32) ? 1 : 0;
  const size_t isz = p->sidx32 ? 4 : 8, vsz = p->form == kF64 ? 8 : 4;
  size_t o = kReuseHdr;
  p->off_sv = o;
  o = align256(o + (size_t)p->nnz * vsz);
  p->off_sidx = o;
  o = align256(o + (size_t)p->nnz * isz);
  p->off_heads = o;
  o = align256(o + (size_t)((p->nnz + 63) / 64) * 8);
  p->off_row0 = o;
  o = align256(o + (size_t)p->nchunks * 8);
  p->off_groups = o;
  o = align256(o + (size_t)(2 * p->nchunks) * sizeof(CarryGroup));
  p->off_carry = o;
  o = align256(o + (size_t)(2 * p->nchunks) * sizeof(double));
  p->data_bytes = o;
  p->off_perm = align256(p->P.L.end);
  p->off_rowid = p->off_perm + align256((size_t)p->nnz * 4);
  p->setup_bytes = p->off_rowid + align256((size_t)p->nnz * 4);
  *plan = p;
  return TTV_OK;
}

int ttv_reuse_sizes(const ttv_reuse_plan* plan, size_t* data_bytes, size_t* setup_ws_bytes) {
  if (int rc = check_plan(plan)) return rc;
  if (!data_bytes || !setup_ws_bytes) return TTV_E_NULL;
  *data_bytes = plan->data_bytes;
  *setup_ws_bytes = plan->setup_bytes;
  return TTV_OK;
}

int ttv_reuse_setup(ttv_reuse_plan* plan, void* data, size_t data_bytes, void* out_subs, int64_t* out_nnz,
                    void* ws, size_t ws_bytes, ttv_stream_t stream) {
  if (int rc = check_plan(plan)) return rc;
  if (!out_nnz) return TTV_E_NULL;
  if (!data || data_bytes < plan->data_bytes || !ws || ws_bytes < plan->setup_bytes) return TTV_E_WORKSPACE;
  if (plan->nnz > 0 && !out_subs) return TTV_E_NULL;
  if (int f = fault_launch()) return f;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  (void)hipGetLastError();  // errors left by earlier, unrelated runtime calls are not ours
  char* d = static_cast<char*>(data);
  char* w = static_cast<char*>(ws);
  PipePlan P = plan->P;
  P.d0.out_subs = out_subs;
  P.d0.out_nnz = reinterpret_cast<long long*>(out_nnz);
  P.d0.seg_out = reinterpret_cast<int32_t*>(w + plan->off_rowid);
  P.d0.perm_out = reinterpret_cast<int32_t*>(w + plan->off_perm);
  P.cus = device_cus();
  int rc = launch_pipeline(P, ws, s);
  if (rc) return rc;
  const ttv_coo_desc& X = plan->X;
  const long long sjm = (long long)plan->mode * X.stride_j;
  const int g = (int)std::min<long long>(std::max<long long>(1, (plan->nnz + 255) / 256), 8LL * P.cus);
  const int32_t* perm = P.d0.perm_out;
  const int32_t* rowid = P.d0.seg_out;
  long long* hdr = reinterpret_cast<long long*>(d);
  const long long* onnz = reinterpret_cast<const long long*>(out_nnz);
  auto heads = reinterpret_cast<unsigned long long*>(d + plan->off_heads);
  auto row0 = reinterpret_cast<long long*>(d + plan->off_row0);
  auto run = [&](auto idx_tag, auto val_tag, auto sidx_tag) {
    using IdxT = decltype(idx_tag);
    using In = decltype(val_tag);
    using SIdx = decltype(sidx_tag);
    hipLaunchKernelGGL((k_reuse_gather<IdxT, In, SIdx>), dim3(g), dim3(256), 0, s, static_cast<const IdxT*>(X.subs),
                       X.stride_e, sjm, static_cast<const In*>(X.vals), perm, rowid, plan->nnz,
                       reinterpret_cast<In*>(d + plan->off_sv), reinterpret_cast<SIdx*>(d + plan->off_sidx), heads,
                       row0, onnz, hdr);
  };
  auto by_sidx = [&](auto idx_tag, auto val_tag) {
    if (plan->sidx32)
      run(idx_tag, val_tag, (uint32_t)0);
    else
      run(idx_tag, val_tag, (long long)0);
  };
  auto by_val = [&](auto idx_tag) {
    if (plan->form == kF64)
      by_sidx(idx_tag, 0.0);
    else
      by_sidx(idx_tag, 0.0f);
  };
  if (plan->idx64)
    by_val((long long)0);
  else
    by_val((int)0);
  if (plan->nnz > 0) {
    const long long ge = std::min<long long>((2 * plan->nchunks + 255) / 256, 4LL * P.cus);
    hipLaunchKernelGGL(k_carry_groups<kReuseChunk>, dim3((unsigned)ge), dim3(256), 0, s, rowid,
                       static_cast<const long long*>(row0), plan->nnz, plan->nchunks,
                       reinterpret_cast<CarryGroup*>(d + plan->off_groups));
  }
  plan->cus = P.cus;
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_last_hip_error((int)e);
    return TTV_E_HIP;
  }
  plan->data = data;
  return TTV_OK;
}

int ttv_reuse_apply(const ttv_reuse_plan* plan, const void* v, int64_t v_len, void* out_vals,
                    ttv_stream_t stream) {
  if (int rc = check_plan(plan)) return rc;
  if (!plan->data) return TTV_E_ARG;  // setup has not run
  if (v_len != plan->X.shape[plan->mode]) return TTV_E_SHAPE;
  if (plan->nnz == 0) return TTV_OK;
  if (!v || !out_vals) return TTV_E_NULL;
  if (int f = fault_launch()) return f;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  char* d = static_cast<char*>(plan->data);
  ReuseArgs A;
  A.sv = d + plan->off_sv;
  A.sidx = d + plan->off_sidx;
  A.heads = reinterpret_cast<const unsigned long long*>(d + plan->off_heads);
  A.row0 = reinterpret_cast<const long long*>(d + plan->off_row0);
  A.groups = reinterpret_cast<const CarryGroup*>(d + plan->off_groups);
  A.carry = reinterpret_cast<double*>(d + plan->off_carry);
  A.v = v;
  A.out = out_vals;
  A.nnz = plan->nnz;
  A.nchunks = plan->nchunks;
  A.out_f64 = plan->out_f64;
  A.vlen = v_len;
  // v is staged in LDS when it fits and the blocks' copies of it (from L2)
  // cost fewer bytes than the values they gather for
  const size_t vbytes = (size_t)v_len * (plan->form == kF64 ? 8 : 4);
  const size_t lds = align256(vbytes);
  const long long per_cu = lds <= 80 * 1024 ? 2 : 1;
  const long long gl = std::min<long long>(per_cu * plan->cus,
                                           (plan->nchunks + kReuseLdsThreads / 64 - 1) / (kReuseLdsThreads / 64));
  const bool use_lds = lds <= kReuseMaxVLds && (size_t)gl * vbytes <= (size_t)plan->nnz * (vbytes / v_len);
  const long long ga = (plan->nchunks + kReuseThreads / 64 - 1) / (kReuseThreads / 64);
  const long long gc = (2 * plan->nchunks + 255) / 256;
  auto launch = [&](auto sidx_tag, auto form_tag) {
    using SIdx = decltype(sidx_tag);
    constexpr int F = decltype(form_tag)::value;
    if (use_lds) {
      hipFuncSetAttribute((const void*)k_reuse_apply_lds<SIdx, F>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds);
      hipLaunchKernelGGL((k_reuse_apply_lds<SIdx, F>), dim3((unsigned)gl), dim3(kReuseLdsThreads), lds, s, A);
    } else {
      hipLaunchKernelGGL((k_reuse_apply<SIdx, F>), dim3((unsigned)ga), dim3(kReuseThreads), 0, s, A);
    }
  };
  prof_begin(TTV_PROF_REUSE, s);
  if (plan->form == kF64) {
    if (plan->sidx32)
      launch((uint32_t)0, std::integral_constant<int, kF64>());
    else
      launch((long long)0, std::integral_constant<int, kF64>());
  } else {
    if (plan->sidx32)
      launch((uint32_t)0, std::integral_constant<int, kC32>());
    else
      launch((long long)0, std::integral_constant<int, kC32>());
  }
  prof_end(TTV_PROF_REUSE, s);
  if (plan->form == kF64)
    hipLaunchKernelGGL(k_reuse_combine<kF64>, dim3((unsigned)gc), dim3(256), 0, s, A);
  else
    hipLaunchKernelGGL(k_reuse_combine<kC32>, dim3((unsigned)gc), dim3(256), 0, s, A);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_last_hip_error((int)e);
    return TTV_E_HIP;
  }
  return TTV_OK;
}

void ttv_reuse_plan_destroy(ttv_reuse_plan* plan) { delete plan; }

}  // extern "C"
