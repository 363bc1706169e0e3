// Product with a vector in every mode (n_v = d in Sec. 3.3): the scalar
//     y = sum over the nonzeros e of vals[e] * prod_j vecs[j][subs(e, j)]
// (factors in ascending mode order).  For d = 1 it is the dot product of a
// sparse and a dense vector (Sec. 3.1).
//
// One streaming pass: a fixed set of kFullWaves waves takes tiles of 64 x
// kFullIPT nonzeros in a fixed order (wave w: tiles w, w + kFullWaves, ...);
// the vectors that fit are staged in each block's LDS;
// every lane sums its products in order (FP64; the compensated form keeps
// exact FP32 product pairs and Dot2 sums), the wave adds its lanes with a
// fixed butterfly in FP64, and one block adds the kFullWaves wave sums with a
// fixed tree.  The order of every addition depends only on nnz: the result is
// bitwise repeatable, on any device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>

#include "ttv.h"
#include "ttv_device.hpp"
#include "ttv_host.h"

namespace ttv {
namespace {

constexpr int kFullWaves = 8192;               // wave sums: fixed, whatever the block shape
// threads per block: 16 waves for narrow rows (room for staged vectors), 4
// for wide ones (their registers)
template <int MO>
constexpr int full_threads() { return MO <= 3 ? 1024 : 256; }
constexpr size_t kFullLdsBudget = 128 * 1024;                // LDS per block: row stage + staged vectors
constexpr int kFullIPT = 4;                                  // nonzeros per lane per tile
constexpr int kFullCombine = 1024;                           // threads of the final sum
constexpr size_t kFullHdr = 256;                             // error word at Ctrl's offset

struct FullArgs {
  const void* subs;
  const void* vals;
  long long se, sj;  // subs element (e, j) at subs[e*se + j*sj]
  long long dims[kMaxOrder];
  const void* vec[kMaxOrder];
  long long nnz;
  int order;
  int validate;
  int32_t* err;
  double* partials;  // kFullWaves wave sums
  long long lds_off[kMaxOrder];  // byte offset of a vector staged in LDS, -1 if read from global memory
};

template <typename IdxT, int F, int MO>
__global__ __launch_bounds__(full_threads<MO>()) void k_full(FullArgs A) {
  constexpr int kFullThreads = full_threads<MO>();
  using FO = FormOps<F>;
  using Acc = typename FO::Acc;
  using In = typename FO::In;
  constexpr int IPT = kFullIPT;
  constexpr long long T = 64LL * IPT;
  __shared__ IdxT stage[kFullThreads / 64][64 * MO];
  extern __shared__ __attribute__((aligned(16))) unsigned char vsm[];  // staged vectors
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const unsigned ln = lane_id();
  // the vectors that fit in LDS, copied once per block (16 loads per thread
  // issued together, then their stores): a gather from LDS instead of a
  // cache line from L2 per lane
  for (int m = 0; m < (MO <= 3 ? MO : 0); ++m) {
    if (m >= A.order || A.lds_off[m] < 0) continue;
    In* vs = reinterpret_cast<In*>(vsm + A.lds_off[m]);
    const gptr<const In> gv = to_global(static_cast<const In*>(A.vec[m]));
    const long long len = A.dims[m];
    for (long long b = 0; b < len; b += 16LL * kFullThreads) {
      In t[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const long long i = b + (long long)q * kFullThreads + threadIdx.x;
        t[q] = i < len ? gv[i] : (In)0;
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const long long i = b + (long long)q * kFullThreads + threadIdx.x;
        if (i < len) vs[i] = t[q];
      }
    }
  }
  __syncthreads();
  const long long gw = (long long)blockIdx.x * (kFullThreads / 64) + w;
  const gptr<const In> vals = to_global(static_cast<const In*>(A.vals));
  const bool rowmajor = rows_coalesced(A.order, A.se, A.sj);
  const long long ntiles = (A.nnz + T - 1) / T;
  Acc acc = FO::zero();
  for (long long t = gw; t < ntiles; t += kFullWaves) {
    const long long e0 = t * T;
    const long long n = std::min<long long>(T, A.nnz - e0);
    In a[IPT];
#pragma unroll
    for (int j = 0; j < IPT; ++j) a[j] = (long long)j * 64 + ln < n ? vals[e0 + j * 64 + ln] : (In)0;
    // vector entries gathered as the indices arrive (no index kept)
    In g[MO][IPT];
#pragma unroll
    for (int m = 0; m < MO; ++m)
#pragma unroll
      for (int j = 0; j < IPT; ++j) g[m][j] = (In)1;
    for_rows<IdxT, IPT, MO>(static_cast<const IdxT*>(A.subs), A.se, A.sj, A.order, rowmajor, e0, n, stage[w],
                            [&](int m, int j, long long x) {
                              if ((long long)j * 64 + ln >= n) return;
                              if (A.validate && (x < 0 || x >= A.dims[m])) {
                                atomicCAS(A.err, 0, TTV_E_INDEX);
                                x = 0;
                              }
                              if (MO <= 3 && A.lds_off[m] >= 0)
                                g[m][j] = reinterpret_cast<const In*>(vsm + A.lds_off[m])[x];
                              else
                                g[m][j] = to_global(static_cast<const In*>(A.vec[m]))[x];
                            });
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      uint64_t p = FO::start_prod(a[j]);
#pragma unroll
      for (int m = 0; m < MO; ++m)
        if (m < A.order) p = FO::mul_prod(p, g[m][j]);
      if ((long long)j * 64 + ln < n) acc = FO::add(acc, FO::from_pay(p));
    }
  }
  double s = FO::to_f64(acc);
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
  if (ln == 0) to_global(A.partials)[gw] = s;
}

// y = the sum of the wave sums: every thread adds kFullWaves / kFullCombine
// consecutive ones, then a tree in LDS.
__global__ __launch_bounds__(kFullCombine) void k_full_combine(const double* partials, void* y, int out_f64) {
  constexpr int K = kFullWaves / kFullCombine;
  __shared__ double s[kFullCombine];
  const int t = threadIdx.x;
  const gptr<const double> p = to_global(partials);
  double v = 0.0;
#pragma unroll
  for (int i = 0; i < K; ++i) v += p[t * K + i];
  s[t] = v;
  __syncthreads();
  for (int h = kFullCombine / 2; h >= 1; h >>= 1) {
    if (t < h) s[t] += s[t + h];
    __syncthreads();
  }
  if (t == 0) {
    if (out_f64)
      *to_global(static_cast<double*>(y)) = s[0];
    else
      *to_global(static_cast<float*>(y)) = (float)s[0];
  }
}

static_assert(kFullWaves % kFullCombine == 0, "wave sums split evenly over the final block");

int check_full(const ttv_coo_desc* X, int& form, int& idx64) {
  if (!X) return TTV_E_NULL;
  const int d = X->order;
  if (d < 1 || d > TTV_MAX_ORDER) return TTV_E_ORDER;
  if (X->index_dtype != TTV_I32 && X->index_dtype != TTV_I64) return TTV_E_DTYPE;
  if (X->value_dtype != TTV_F32 && X->value_dtype != TTV_F64) return TTV_E_DTYPE;
  if (X->nnz < 0) return TTV_E_ARG;
  for (int j = 0; j < d; ++j)
    if (X->shape[j] < 1) return TTV_E_SHAPE;
  if (X->nnz > 0 && (!X->subs || !X->vals)) return TTV_E_NULL;
  form = X->value_dtype == TTV_F64 ? kF64 : kC32;
  idx64 = X->index_dtype == TTV_I64 ? 1 : 0;
  return TTV_OK;
}

// Stages in LDS, in mode order, every vector that still fits in the budget
// left by the kernel's row stage; returns the dynamic LDS bytes.
size_t plan_staging(FullArgs& A, int order, size_t vsz, size_t stage_bytes) {
  size_t used = 0;
  for (int m = 0; m < kMaxOrder; ++m) {
    A.lds_off[m] = -1;
    if (m >= order) continue;
    const size_t b = ((size_t)A.dims[m] * vsz + 15) & ~(size_t)15;
    if (stage_bytes + used + b <= kFullLdsBudget) {
      A.lds_off[m] = (long long)used;
      used += b;
    }
  }
  return used;
}

template <typename IdxT, int F, int MO>
void launch_full_k(FullArgs A, int order, hipStream_t s) {
  using In = typename FormOps<F>::In;
  constexpr int NT = full_threads<MO>();
  size_t lds = 0;
  if (MO <= 3) {
    lds = plan_staging(A, order, sizeof(In), sizeof(IdxT) * (NT / 64) * 64 * MO);
  } else {
    for (int m = 0; m < kMaxOrder; ++m) A.lds_off[m] = -1;
  }
  if (lds > 0)
    hipFuncSetAttribute((const void*)k_full<IdxT, F, MO>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((k_full<IdxT, F, MO>), dim3(kFullWaves * 64 / NT), dim3(NT), lds, s, A);
}

template <typename IdxT, int F>
void launch_full_mo(const FullArgs& A, int mo, int order, hipStream_t s) {
  if (mo <= 3)
    launch_full_k<IdxT, F, 3>(A, order, s);
  else if (mo <= 5)
    launch_full_k<IdxT, F, 5>(A, order, s);
  else
    launch_full_k<IdxT, F, kMaxOrder>(A, order, s);
}

}  // namespace
}  // namespace ttv

using namespace ttv;

extern "C" {

int ttv_coo_full_workspace(const ttv_coo_desc* X, int32_t flags, size_t* bytes) {
  if (flags & TTV_DROP_ZEROS) return TTV_E_ARG;  // sparse products only
  if (!bytes) return TTV_E_NULL;
  int form, idx64;
  if (int rc = check_full(X, form, idx64)) return rc;
  *bytes = kFullHdr + sizeof(double) * (size_t)kFullWaves;
  return TTV_OK;
}

int ttv_coo_full(const ttv_coo_desc* X, const void* const* vecs, const int64_t* vec_lens, void* y, void* ws,
                 size_t ws_bytes, int32_t flags, ttv_stream_t stream) {
  if (flags & TTV_DROP_ZEROS) return TTV_E_ARG;  // sparse products only
  int form, idx64;
  if (int rc = check_full(X, form, idx64)) return rc;
  if (!vecs || !vec_lens || !y) return TTV_E_NULL;
  for (int j = 0; j < X->order; ++j) {
    if (vec_lens[j] != X->shape[j]) return TTV_E_SHAPE;
    if (!vecs[j] && X->nnz > 0) return TTV_E_NULL;
  }
  if (!ws || ws_bytes < kFullHdr + sizeof(double) * (size_t)kFullWaves) return TTV_E_WORKSPACE;
  if (int f = fault_launch()) return f;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  (void)hipGetLastError();  // errors left by earlier, unrelated runtime calls are not ours
  char* w = static_cast<char*>(ws);
  if (int rc = launch_zero(w, kFullHdr, s)) return rc;
  FullArgs A;
  A.subs = X->subs;
  A.vals = X->vals;
  A.se = X->stride_e;
  A.sj = X->stride_j;
  for (int j = 0; j < kMaxOrder; ++j) {
    A.dims[j] = j < X->order ? X->shape[j] : 1;
    A.vec[j] = j < X->order ? vecs[j] : nullptr;
  }
  A.nnz = X->nnz;
  A.order = X->order;
  A.validate = (flags & TTV_VALIDATE) ? 1 : 0;
  A.err = reinterpret_cast<int32_t*>(w + offsetof(Ctrl, error));
  A.partials = reinterpret_cast<double*>(w + kFullHdr);
  const int mo = row_width_class(X->order, X->stride_e, X->stride_j);
  const int out_f64 = (form == kF64 || (flags & TTV_OUT_F64)) ? 1 : 0;
  prof_begin(TTV_PROF_FULL, s);
  if (idx64) {
    if (form == kF64)
      launch_full_mo<long long, kF64>(A, mo, X->order, s);
    else
      launch_full_mo<long long, kC32>(A, mo, X->order, s);
  } else {
    if (form == kF64)
      launch_full_mo<int, kF64>(A, mo, X->order, s);
    else
      launch_full_mo<int, kC32>(A, mo, X->order, s);
  }
  prof_end(TTV_PROF_FULL, s);
  hipLaunchKernelGGL(k_full_combine, dim3(1), dim3(kFullCombine), 0, s, A.partials, y, out_f64);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_last_hip_error((int)e);
    return TTV_E_HIP;
  }
  return TTV_OK;
}

}  // extern "C"
