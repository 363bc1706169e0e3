// Repeated sparse TTV with a fixed tensor and mode (the tensor is reused
// across calls with a new vector each time, as in the iterative methods of
// Sec. 3.3's motivation): the keyed sort of Eq. 3's index tuples runs once.
//
// Setup runs the sorting pipeline in its permutation mode: it writes the
// output coordinates (which do not depend on the vector) and, for every
// position of the sorted order, the nonzero there and its output row.  A
// gather then stores the values and the contracted-mode indices in sorted
// order in the caller's plan buffer.
//
// Each apply is one streaming pass over that buffer: per sorted position the
// product value x v[index], and a segmented sum over runs of equal output
// row.  Chunks of kReuseChunk positions are reduced by one block each
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

#include "ttv.h"
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
  size_t off_sv = 0, off_sidx = 0, off_rowid = 0, off_carry = 0, data_bytes = 0;
  size_t off_perm = 0, setup_bytes = 0;  // setup workspace: pipeline, then the permutation
  void* data = nullptr;                  // bound by setup
};

namespace ttv {
namespace {

constexpr int kReuseThreads = 512;
constexpr int kReuseIPT = 8;
constexpr int kReuseChunk = kReuseThreads * kReuseIPT;  // sorted positions per block
constexpr size_t kReuseHdr = 256;                       // int64 nnz_out at offset 0

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Carry {
  long long row;  // -1: unused
  double val;
};

// sv[k] = vals[perm[k]], sidx[k] = subs(perm[k], mode); the header gets nnz_out.
template <typename IdxT, typename In>
__global__ __launch_bounds__(256) void k_reuse_gather(const IdxT* subs, long long se, long long sjm, const In* vals,
                                                      const int32_t* perm, long long nnz, In* sv, IdxT* sidx,
                                                      const long long* out_nnz, long long* hdr) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *hdr = *out_nnz;
  const gptr<const IdxT> gs = to_global(subs);
  const gptr<const In> gv = to_global(vals);
  const gptr<const int32_t> gp = to_global(perm);
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < nnz;
       k += (long long)gridDim.x * blockDim.x) {
    const long long e = gp[k];
    sv[k] = gv[e];
    sidx[k] = gs[e * se + sjm];
  }
}

struct ReuseArgs {
  const void* sv;
  const void* sidx;
  const int32_t* rowid;
  Carry* carry;
  const void* v;
  void* out;
  long long nnz;
  long long nchunks;
  int out_f64;
};

template <int F>
__device__ __forceinline__ void put(const ReuseArgs& A, long long row, double x) {
  if (A.out_f64)
    to_global(static_cast<double*>(A.out))[row] = x;
  else
    to_global(static_cast<float*>(A.out))[row] = (float)x;
}

// One chunk per block: products, heads and ends of runs of equal row, the
// segmented sums; rows inside the chunk are written, its first and last
// rows' partial sums go to the carries.
template <typename IdxT, int F>
__global__ __launch_bounds__(kReuseThreads) void k_reuse_apply(ReuseArgs A) {
  using FO = FormOps<F>;
  using Acc = typename FO::Acc;
  using In = typename FO::In;
  constexpr int NT = kReuseThreads, IPT = kReuseIPT, NW = NT / 64;
  __shared__ unsigned wsum[NW];
  __shared__ Seg<F> wagg[NW];
  const int tid = threadIdx.x, w = tid >> 6;
  const unsigned ln = lane_id();
  const gptr<const In> sv = to_global(static_cast<const In*>(A.sv));
  const gptr<const IdxT> sidx = to_global(static_cast<const IdxT*>(A.sidx));
  const gptr<const int32_t> rowid = to_global(A.rowid);
  const gptr<const In> v = to_global(static_cast<const In*>(A.v));
  for (long long b = blockIdx.x; b < A.nchunks; b += gridDim.x) {
    const long long k0 = b * kReuseChunk;
    const int n = (int)std::min<long long>(kReuseChunk, A.nnz - k0);
    const int pw = w * 64 * IPT;  // wave w: positions [pw, pw + 64*IPT), rounds of 64
    int row[IPT];
    bool hd[IPT], end[IPT];
    Acc prod[IPT];
    {
      int rprev[IPT], rnext[IPT];
      In a[IPT];
      IdxT ix[IPT];
#pragma unroll
      for (int j = 0; j < IPT; ++j) {
        const int p = pw + j * 64 + (int)ln;
        const bool ok = p < n;
        row[j] = ok ? rowid[k0 + p] : -1;
        rprev[j] = (ok && p > 0) ? rowid[k0 + p - 1] : -1;
        rnext[j] = (ok && p + 1 < n) ? rowid[k0 + p + 1] : -1;
        a[j] = ok ? sv[k0 + p] : (In)0;
        ix[j] = ok ? sidx[k0 + p] : (IdxT)0;
      }
      In g[IPT];
#pragma unroll
      for (int j = 0; j < IPT; ++j) g[j] = (pw + j * 64 + (int)ln < n) ? v[ix[j]] : (In)0;
#pragma unroll
      for (int j = 0; j < IPT; ++j) {
        const int p = pw + j * 64 + (int)ln;
        hd[j] = p < n && (p == 0 || row[j] != rprev[j]);
        end[j] = p < n && (p == n - 1 || row[j] != rnext[j]);
        prod[j] = FO::from_pay(FO::mul_prod(FO::start_prod(a[j]), g[j]));
      }
    }
    // segmented scan in rounds of 64 consecutive positions, then across waves
    uint64_t hm[IPT];
    Acc val[IPT];
    unsigned whc = 0;
    {
      Acc c = FO::zero();
#pragma unroll
      for (int j = 0; j < IPT; ++j) {
        hm[j] = ballot(hd[j]);
        whc += (unsigned)__popcll(hm[j]);
        Seg<F> e;
        e.f = hd[j] ? 1 : 0;
        e.v = (pw + j * 64 + (int)ln < n) ? prod[j] : FO::zero();
        e = wave_seg_scan<F>(e);
        val[j] = e.f ? e.v : FO::add(c, e.v);
        c = FO::shfl_last(val[j]);
      }
      if (ln == 0) {
        wsum[w] = whc;
        wagg[w].f = whc ? 1 : 0;
        wagg[w].v = c;
      }
    }
    __syncthreads();
    Seg<F> cw;
    cw.f = 0;
    cw.v = FO::zero();
    unsigned hbw = 0;
    for (int q = 0; q < w; ++q) {
      cw = seg_combine<F>(cw, wagg[q]);
      hbw += wsum[q];
    }
    {
      bool lead = true;
#pragma unroll
      for (int j = 0; j < IPT; ++j) {
        const uint64_t upto = hm[j] & (~0ull >> (63 - ln));
        if (lead && upto == 0) val[j] = FO::add(cw.v, val[j]);
        lead = lead && hm[j] == 0;
      }
    }
    // run ends: the chunk's first run (one head so far) and last run (ending
    // at the chunk's end) may continue in the neighbouring chunks
    unsigned hrun = hbw;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      const int p = pw + j * 64 + (int)ln;
      if (end[j]) {
        const unsigned heads = hrun + (unsigned)__popcll(hm[j] & (~0ull >> (63 - ln)));
        const bool firstrun = heads == 1, lastrun = p == n - 1;
        const double x = FO::to_f64(val[j]);
        if (!firstrun && !lastrun) {
          put<F>(A, row[j], x);
        } else {
          Carry* cb = A.carry + 2 * b;
          if (firstrun) cb[0] = Carry{row[j], x};
          if (lastrun) cb[1] = firstrun ? Carry{-1, 0.0} : Carry{row[j], x};
        }
      }
      hrun += (unsigned)__popcll(hm[j]);
    }
    __syncthreads();
  }
}

// Rows that touch a chunk boundary: the entry holding a row's first partial
// adds the following entries of the same row, in chunk order (FP64).
template <int F>
__global__ __launch_bounds__(256) void k_reuse_combine(ReuseArgs A) {
  const long long E = 2 * A.nchunks;
  const Carry* c = A.carry;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < E;
       e += (long long)gridDim.x * blockDim.x) {
    const long long r = c[e].row;
    if (r < 0) continue;
    long long q = e - 1;  // the previous used entry (at most one unused entry lies between)
    while (q >= 0 && c[q].row < 0) --q;
    if (q >= 0 && c[q].row == r) continue;  // not the row's first partial
    double s = c[e].val;
    for (long long f = e + 1; f < E; ++f) {
      const long long rf = c[f].row;
      if (rf < 0) continue;
      if (rf != r) break;
      s += c[f].val;
    }
    put<F>(A, r, s);
  }
}

int check_plan(const ttv_reuse_plan* p) { return p ? TTV_OK : TTV_E_NULL; }

}  // namespace
}  // namespace ttv

using namespace ttv;

extern "C" {

int ttv_reuse_plan_create(const ttv_coo_desc* X, int32_t mode, int32_t flags, ttv_reuse_plan** plan) {
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
  const size_t isz = p->idx64 ? 8 : 4, vsz = p->form == kF64 ? 8 : 4;
  size_t o = kReuseHdr;
  p->off_sv = o;
  o = align256(o + (size_t)p->nnz * vsz);
  p->off_sidx = o;
  o = align256(o + (size_t)p->nnz * isz);
  p->off_rowid = o;
  o = align256(o + (size_t)p->nnz * 4);
  p->off_carry = o;
  o = align256(o + (size_t)(2 * p->nchunks) * sizeof(Carry));
  p->data_bytes = o;
  p->off_perm = align256(p->P.L.end);
  p->setup_bytes = p->off_perm + align256((size_t)p->nnz * 4);
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
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  (void)hipGetLastError();  // errors left by earlier, unrelated runtime calls are not ours
  char* d = static_cast<char*>(data);
  char* w = static_cast<char*>(ws);
  PipePlan P = plan->P;
  P.d0.out_subs = out_subs;
  P.d0.out_nnz = reinterpret_cast<long long*>(out_nnz);
  P.d0.seg_out = reinterpret_cast<int32_t*>(d + plan->off_rowid);
  P.d0.perm_out = reinterpret_cast<int32_t*>(w + plan->off_perm);
  P.cus = device_cus();
  int rc = launch_pipeline(P, ws, s);
  if (rc) return rc;
  const ttv_coo_desc& X = plan->X;
  const long long sjm = (long long)plan->mode * X.stride_j;
  const int g = (int)std::min<long long>(std::max<long long>(1, (plan->nnz + 255) / 256), 8LL * P.cus);
  const int32_t* perm = P.d0.perm_out;
  long long* hdr = reinterpret_cast<long long*>(d);
  const long long* onnz = reinterpret_cast<const long long*>(out_nnz);
  if (plan->idx64) {
    if (plan->form == kF64)
      hipLaunchKernelGGL((k_reuse_gather<long long, double>), dim3(g), dim3(256), 0, s,
                         static_cast<const long long*>(X.subs), X.stride_e, sjm, static_cast<const double*>(X.vals),
                         perm, plan->nnz, reinterpret_cast<double*>(d + plan->off_sv),
                         reinterpret_cast<long long*>(d + plan->off_sidx), onnz, hdr);
    else
      hipLaunchKernelGGL((k_reuse_gather<long long, float>), dim3(g), dim3(256), 0, s,
                         static_cast<const long long*>(X.subs), X.stride_e, sjm, static_cast<const float*>(X.vals),
                         perm, plan->nnz, reinterpret_cast<float*>(d + plan->off_sv),
                         reinterpret_cast<long long*>(d + plan->off_sidx), onnz, hdr);
  } else {
    if (plan->form == kF64)
      hipLaunchKernelGGL((k_reuse_gather<int, double>), dim3(g), dim3(256), 0, s, static_cast<const int*>(X.subs),
                         X.stride_e, sjm, static_cast<const double*>(X.vals), perm, plan->nnz,
                         reinterpret_cast<double*>(d + plan->off_sv), reinterpret_cast<int*>(d + plan->off_sidx),
                         onnz, hdr);
    else
      hipLaunchKernelGGL((k_reuse_gather<int, float>), dim3(g), dim3(256), 0, s, static_cast<const int*>(X.subs),
                         X.stride_e, sjm, static_cast<const float*>(X.vals), perm, plan->nnz,
                         reinterpret_cast<float*>(d + plan->off_sv), reinterpret_cast<int*>(d + plan->off_sidx),
                         onnz, hdr);
  }
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
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  char* d = static_cast<char*>(plan->data);
  ReuseArgs A;
  A.sv = d + plan->off_sv;
  A.sidx = d + plan->off_sidx;
  A.rowid = reinterpret_cast<const int32_t*>(d + plan->off_rowid);
  A.carry = reinterpret_cast<Carry*>(d + plan->off_carry);
  A.v = v;
  A.out = out_vals;
  A.nnz = plan->nnz;
  A.nchunks = plan->nchunks;
  A.out_f64 = plan->out_f64;
  const int ga = (int)std::min<long long>(plan->nchunks, 1LL << 20);
  const int gc = (int)std::min<long long>(std::max<long long>(1, (2 * plan->nchunks + 255) / 256), 1024);
  prof_begin(TTV_PROF_REUSE, s);
  if (plan->form == kF64) {
    if (plan->idx64)
      hipLaunchKernelGGL((k_reuse_apply<long long, kF64>), dim3(ga), dim3(kReuseThreads), 0, s, A);
    else
      hipLaunchKernelGGL((k_reuse_apply<int, kF64>), dim3(ga), dim3(kReuseThreads), 0, s, A);
  } else {
    if (plan->idx64)
      hipLaunchKernelGGL((k_reuse_apply<long long, kC32>), dim3(ga), dim3(kReuseThreads), 0, s, A);
    else
      hipLaunchKernelGGL((k_reuse_apply<int, kC32>), dim3(ga), dim3(kReuseThreads), 0, s, A);
  }
  prof_end(TTV_PROF_REUSE, s);
  if (plan->form == kF64)
    hipLaunchKernelGGL(k_reuse_combine<kF64>, dim3(gc), dim3(256), 0, s, A);
  else
    hipLaunchKernelGGL(k_reuse_combine<kC32>, dim3(gc), dim3(256), 0, s, A);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_last_hip_error((int)e);
    return TTV_E_HIP;
  }
  return TTV_OK;
}

void ttv_reuse_plan_destroy(ttv_reuse_plan* plan) { delete plan; }

}  // extern "C"
