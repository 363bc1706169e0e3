// Options of the pyttb procedure that Sec. 3.3 lists besides the product
// itself: removing output entries whose sum is exactly zero (its `nonzero`
// step), and converting a result to a dense array when more than half of its
// cells are stored.  Both run after the product, on its sparse result, with
// every decision taken on the device (no host synchronisation).
//
// Drop: a fixed number of blocks each take a contiguous range of rows; the
// first kernel counts each range's kept rows, the second gives every block
// its output offset (the sum of the counts before it) and writes its kept
// rows in order.  Dense: one kernel writes the flag and the zeros, the next
// places every row's value at the row-major cell of its tuple (rows are
// distinct, so every cell has at most one writer).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ttv.h"
#include "ttv_device.hpp"
#include "ttv_host.h"

namespace ttv {
namespace {

constexpr int kOptThreads = 1024;

struct DropArgs {
  const void* in_subs;
  const void* in_vals;
  const long long* in_nnz;
  void* out_subs;
  void* out_vals;
  long long* out_nnz;
  long long* counts;  // one per block
  int nrem;
};

__device__ __forceinline__ void block_range(long long n, long long& lo, long long& hi) {
  lo = n * (long long)blockIdx.x / gridDim.x;
  hi = n * (long long)(blockIdx.x + 1) / gridDim.x;
}

template <typename V>
__device__ __forceinline__ bool kept(V x) {
  return x != (V)0;  // +0 and -0 are dropped
}

template <typename V>
__global__ __launch_bounds__(kOptThreads) void k_drop_count(DropArgs A) {
  __shared__ unsigned wsum[kOptThreads / 64];
  long long lo, hi;
  block_range(*A.in_nnz, lo, hi);
  const gptr<const V> vals = to_global(static_cast<const V*>(A.in_vals));
  unsigned c = 0;
  for (long long r = lo + threadIdx.x; r < hi; r += kOptThreads) c += kept(vals[r]) ? 1u : 0u;
  const unsigned tot = block_sum<kOptThreads>(c, wsum);
  if (threadIdx.x == 0) A.counts[blockIdx.x] = tot;
}

template <typename IdxT, typename V>
__global__ __launch_bounds__(kOptThreads) void k_drop_write(DropArgs A) {
  __shared__ unsigned wsum[kOptThreads / 64];
  __shared__ long long sbase[kOptThreads / 64];
  long long lo, hi;
  block_range(*A.in_nnz, lo, hi);
  // output offset of this block: the kept rows of the blocks before it
  long long b = 0;
  for (int q = threadIdx.x; q < (int)blockIdx.x; q += kOptThreads) b += A.counts[q];
  for (int d = 32; d >= 1; d >>= 1) b += __shfl_xor(b, d, 64);
  if (lane_id() == 0) sbase[threadIdx.x >> 6] = b;
  __syncthreads();
  long long base = 0;
  for (int i = 0; i < kOptThreads / 64; ++i) base += sbase[i];
  const gptr<const V> vals = to_global(static_cast<const V*>(A.in_vals));
  const gptr<const IdxT> subs = to_global(static_cast<const IdxT*>(A.in_subs));
  const gptr<V> ovals = to_global(static_cast<V*>(A.out_vals));
  const gptr<IdxT> osubs = to_global(static_cast<IdxT*>(A.out_subs));
  const int nr = A.nrem;
  for (long long r0 = lo; r0 < hi; r0 += kOptThreads) {
    const long long r = r0 + threadIdx.x;
    const V x = r < hi ? vals[r] : (V)0;
    const bool k = r < hi && kept(x);
    unsigned tot;
    const unsigned pos = block_excl_scan<kOptThreads>(k ? 1u : 0u, wsum, tot);
    if (k) {
      const long long o = base + pos;
      ovals[o] = x;
      for (int j = 0; j < nr; ++j) osubs[o * nr + j] = subs[r * nr + j];
    }
    base += tot;
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *A.out_nnz = base;
}

// Dense conversion.
struct DenseOut {
  const void* subs;
  const void* vals;
  const long long* nnz;
  void* dense;
  int32_t* is_dense;
  long long cells;  // product of the dimensions (clamped)
  long long cap;
  long long stride[kMaxOrder];  // row-major cell strides
  int order;
};

__device__ __forceinline__ bool dense_wanted(const DenseOut& D) {
  const long long n = *D.nnz;
  return D.cells <= D.cap && 2 * n > D.cells;
}

template <typename V>
__global__ __launch_bounds__(256) void k_dense_fill(DenseOut D) {
  const bool want = dense_wanted(D);
  if (blockIdx.x == 0 && threadIdx.x == 0) *D.is_dense = want ? 1 : 0;
  if (!want) return;
  const gptr<V> out = to_global(static_cast<V*>(D.dense));
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < D.cells;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = (V)0;
}

template <typename IdxT, typename V>
__global__ __launch_bounds__(256) void k_dense_place(DenseOut D) {
  if (!dense_wanted(D)) return;
  const long long n = *D.nnz;
  const gptr<const IdxT> subs = to_global(static_cast<const IdxT*>(D.subs));
  const gptr<const V> vals = to_global(static_cast<const V*>(D.vals));
  const gptr<V> out = to_global(static_cast<V*>(D.dense));
  for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (long long)gridDim.x * blockDim.x) {
    long long lin = 0;
    for (int j = 0; j < D.order; ++j) lin += (long long)subs[r * D.order + j] * D.stride[j];
    if (lin >= 0 && lin < D.cells) out[lin] = vals[r];
  }
}

}  // namespace

size_t drop_zeros_ws(long long nnz, int nrem, int idx64, int out_f64) {
  const size_t isz = idx64 ? 8 : 4, vsz = out_f64 ? 8 : 4;
  size_t o = 256;  // result count
  o += (size_t)kDropBlocks * 8;
  o = (o + 255) & ~(size_t)255;
  o += ((size_t)nnz * nrem * isz + 255) & ~(size_t)255;
  o += ((size_t)nnz * vsz + 255) & ~(size_t)255;
  return o;
}

void drop_zeros_layout(void* tmp, long long nnz, int nrem, int idx64, long long*& cnt, long long*& counts,
                       void*& subs, void*& vals) {
  const size_t isz = idx64 ? 8 : 4;
  char* t = static_cast<char*>(tmp);
  cnt = reinterpret_cast<long long*>(t);
  counts = reinterpret_cast<long long*>(t + 256);
  size_t o = (256 + (size_t)kDropBlocks * 8 + 255) & ~(size_t)255;
  subs = t + o;
  o += ((size_t)nnz * nrem * isz + 255) & ~(size_t)255;
  vals = t + o;
}

int launch_drop_zeros(const void* in_subs, const void* in_vals, const long long* in_nnz, long long* counts,
                      void* out_subs, void* out_vals, long long* out_nnz, int nrem, int idx64, int out_f64,
                      hipStream_t s) {
  DropArgs A{in_subs, in_vals, in_nnz, out_subs, out_vals, out_nnz, counts, nrem};
  const dim3 g(kDropBlocks), b(kOptThreads);
  if (out_f64)
    hipLaunchKernelGGL(k_drop_count<double>, g, b, 0, s, A);
  else
    hipLaunchKernelGGL(k_drop_count<float>, g, b, 0, s, A);
  if (idx64) {
    if (out_f64)
      hipLaunchKernelGGL((k_drop_write<long long, double>), g, b, 0, s, A);
    else
      hipLaunchKernelGGL((k_drop_write<long long, float>), g, b, 0, s, A);
  } else {
    if (out_f64)
      hipLaunchKernelGGL((k_drop_write<int, double>), g, b, 0, s, A);
    else
      hipLaunchKernelGGL((k_drop_write<int, float>), g, b, 0, s, A);
  }
  return TTV_OK;
}

}  // namespace ttv

using namespace ttv;

extern "C" {

int ttv_result_densify(int32_t order, const int64_t* shape, int32_t index_dtype, int32_t value_dtype,
                       const void* subs, const void* vals, const int64_t* nnz, void* dense, int64_t dense_cap,
                       int32_t* is_dense, ttv_stream_t stream) {
  if (order < 1 || order > TTV_MAX_ORDER) return TTV_E_ORDER;
  if (!shape || !nnz || !is_dense) return TTV_E_NULL;
  if (index_dtype != TTV_I32 && index_dtype != TTV_I64) return TTV_E_DTYPE;
  if (value_dtype != TTV_F32 && value_dtype != TTV_F64) return TTV_E_DTYPE;
  if (dense_cap < 0) return TTV_E_ARG;
  if (dense_cap > 0 && !dense) return TTV_E_NULL;
  DenseOut D;
  D.subs = subs;
  D.vals = vals;
  D.nnz = reinterpret_cast<const long long*>(nnz);
  D.dense = dense;
  D.is_dense = is_dense;
  D.cap = dense_cap;
  D.order = order;
  unsigned __int128 cells = 1;
  for (int j = order - 1; j >= 0; --j) {
    if (shape[j] < 1) return TTV_E_SHAPE;
    D.stride[j] = (long long)std::min<unsigned __int128>(cells, (unsigned __int128)1 << 62);
    cells *= (unsigned __int128)shape[j];
    if (cells > ((unsigned __int128)1 << 62)) cells = (unsigned __int128)1 << 62;  // never dense
  }
  D.cells = (long long)cells;
  if (int f = fault_launch()) return f;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  (void)hipGetLastError();  // errors left by earlier, unrelated runtime calls are not ours
  const int cus = device_cus();
  const long long want_cells = std::min<long long>(D.cells, std::max<long long>(dense_cap, 1));
  const int gf = (int)std::min<long long>(std::max<long long>(1, (want_cells + 255) / 256), 8LL * cus);
  const int gp = 4 * cus;
  const bool f64 = value_dtype == TTV_F64;
  if (f64)
    hipLaunchKernelGGL(k_dense_fill<double>, dim3(gf), dim3(256), 0, s, D);
  else
    hipLaunchKernelGGL(k_dense_fill<float>, dim3(gf), dim3(256), 0, s, D);
  if (index_dtype == TTV_I64) {
    if (f64)
      hipLaunchKernelGGL((k_dense_place<long long, double>), dim3(gp), dim3(256), 0, s, D);
    else
      hipLaunchKernelGGL((k_dense_place<long long, float>), dim3(gp), dim3(256), 0, s, D);
  } else {
    if (f64)
      hipLaunchKernelGGL((k_dense_place<int, double>), dim3(gp), dim3(256), 0, s, D);
    else
      hipLaunchKernelGGL((k_dense_place<int, float>), dim3(gp), dim3(256), 0, s, D);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_last_hip_error((int)e);
    return TTV_E_HIP;
  }
  return TTV_OK;
}

}  // extern "C"
