// Products whose remaining modes span few keys, without a sort.  Small ones
// in one launch.  When a product's nonzeros are few and
// the remaining dimensions span few keys (the 1e4-nnz 100x80x60 workload:
// 8000 keys), the sorting pipeline's thirteen launches dominate its time.
// Here one block computes the whole product: every nonzero's packed key (the
// mixed-radix key of the remaining modes, ordered like the index tuples) and
// its product with the vectors (Eq. 3's summand) are added to a dense LDS
// array of sums indexed by the key, with a presence bit per key; then the
// present keys are written in key order -- which is the lexicographic order
// of the output tuples -- with their sums.  Every key's sum adds its products
// in input order (tiles in order, the block's waves taking turns, a wave's
// items in order, and the lanes of one LDS atomic that hit the same sum
// applied in lane order), so results are bitwise repeatable.  The sums are
// FP64; FP32 inputs add their exact product pair widened to FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <type_traits>

#include "ttv_device.hpp"
#include "ttv_host.h"

namespace ttv {
namespace {

constexpr int kTinyThreads = 1024;
// keys held in LDS: 16384 FP64 sums (128 KB) beside the row stage of rows of
// up to 3 indices, 8192 beside the wider ones; a product uses the smallest
// capacity that holds its keys (less to clear and scan)
template <int MO>
constexpr int key_cap() { return MO <= 3 ? 2 * kTinyKeys : kTinyKeys; }

template <typename IdxT, int F, int MO, int KC>
__global__ __launch_bounds__(kTinyThreads) void k_tiny(TDesc D, long long range, int32_t* err) {
  using FO = FormOps<F>;
  using In = typename FO::In;
  constexpr int NW = kTinyThreads / 64;
  constexpr int IPT = MO <= 5 ? 4 : 2;  // nonzeros per lane per tile
  static_assert(KC <= key_cap<MO>() && KC % kTinyThreads == 0, "LDS sums by key");
  constexpr int KPT = KC / kTinyThreads;  // keys per thread when writing
  __shared__ double acc[KC];
  __shared__ unsigned pres[KC / 32];
  __shared__ IdxT stage[NW][64 * MO];
  __shared__ unsigned wsum[NW];
  const int tid = threadIdx.x, w = tid >> 6;
  const unsigned ln = lane_id();
  if (tid == 0) *to_global(err) = 0;
  for (int i = tid; i < KC; i += kTinyThreads) acc[i] = 0.0;
  for (int i = tid; i < KC / 32; i += kTinyThreads) pres[i] = 0u;
  __syncthreads();
  const gptr<const In> vals = to_global(static_cast<const In*>(D.vals));
  const bool rowmajor = rows_coalesced(D.order, D.stride_e, D.stride_j);
  constexpr long long TA = (long long)kTinyThreads * IPT;
  for (long long e0 = 0; e0 < D.nnz; e0 += TA) {
    const long long s0 = e0 + (long long)w * 64 * IPT;  // this wave's slice
    const long long n = D.nnz - s0;
    unsigned long long key[IPT];
    uint64_t p[IPT];  // product payload (FP64, or the FP32 pair)
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      key[j] = 0;
      p[j] = FO::start_prod((long long)j * 64 + ln < n ? vals[s0 + j * 64 + ln] : (In)0);
    }
    for_rows<IdxT, IPT, MO>(static_cast<const IdxT*>(D.subs), D.stride_e, D.stride_j, D.order, rowmajor, s0, n,
                            stage[w], [&](int m, int j, long long x) {
                              if ((long long)j * 64 + ln >= n) return;
                              if (D.validate && (x < 0 || x >= D.dims[m])) {
                                atomicCAS(err, 0, TTV_E_INDEX);
                                x = 0;
                              }
                              if (D.mrem[m])
                                key[j] += (unsigned long long)x * D.mstride[m];
                              else if (D.vec[m])
                                p[j] = FO::mul_prod(p[j], to_global(static_cast<const In*>(D.vec[m]))[x]);
                            });
    // the waves take turns adding to the sums (input order per key)
    for (int turn = 0; turn < NW; ++turn) {
      if (w == turn) {
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
          if ((long long)j * 64 + ln < n) {
            const unsigned k = (unsigned)key[j];
            atomicAdd(&acc[k], FO::to_f64(FO::from_pay(p[j])));
            atomicOr(&pres[k >> 5], 1u << (k & 31));
          }
        }
      }
      __syncthreads();
    }
  }
  // present keys in key order: every thread takes KPT consecutive keys
  const int k0 = tid * KPT;
  unsigned c = 0;
#pragma unroll
  for (int q = 0; q < KPT; ++q) {
    const int k = k0 + q;
    c += (k < range && ((pres[k >> 5] >> (k & 31)) & 1u)) ? 1u : 0u;
  }
  unsigned total;
  unsigned pos = block_excl_scan<kTinyThreads>(c, wsum, total);
  const gptr<IdxT> osubs = to_global(static_cast<IdxT*>(D.out_subs));
  const bool of64 = F == kF64 || D.out_f64;
  for (int q = 0; q < KPT; ++q) {
    const int k = k0 + q;
    if (k < range && ((pres[k >> 5] >> (k & 31)) & 1u)) {
      if (of64)
        to_global(static_cast<double*>(D.out_vals))[pos] = acc[k];
      else
        to_global(static_cast<float*>(D.out_vals))[pos] = (float)acc[k];
      for (int i = 0; i < D.nrem; ++i)
        osubs[(long long)pos * D.nrem + i] =
            (IdxT)(((unsigned long long)k / D.kstride[i]) % (unsigned long long)D.dims[D.rem[i]]);
      ++pos;
    }
  }
  if (tid == 0) *to_global(D.out_nnz) = (long long)total;
}

// ---------------------------------------------------------------------------
// Larger products whose remaining modes span at most key_cap keys (a large
// contracted mode: many nonzeros per output row).  The same dense sums by
// key, per block: a fixed number of blocks take tiles in a fixed order, each
// adds its products into its own LDS sums (in order, as above) and ORs its
// presence bits into a global bitmap; the blocks' sums are added per key in
// block order (FP64), and the present keys written in key order.
// ---------------------------------------------------------------------------
constexpr int kKeyedBlocks = 512;  // most blocks: the sum order depends on nnz only

template <typename IdxT, int F, int MO, int KC>
__global__ __launch_bounds__(kTinyThreads) void k_keyed(TDesc D, long long range, int32_t* err, double* partials,
                                                         unsigned* present) {
  using FO = FormOps<F>;
  using In = typename FO::In;
  constexpr int NW = kTinyThreads / 64;
  constexpr int IPT = MO <= 5 ? 4 : 2;
  constexpr long long TA = (long long)kTinyThreads * IPT;
  static_assert(KC <= key_cap<MO>() && KC % kTinyThreads == 0, "LDS sums by key");
  __shared__ double acc[KC];
  __shared__ unsigned pres[KC / 32];
  __shared__ IdxT stage[NW][64 * MO];
  const int tid = threadIdx.x, w = tid >> 6;
  const unsigned ln = lane_id();
  for (int i = tid; i < KC; i += kTinyThreads) acc[i] = 0.0;
  for (int i = tid; i < KC / 32; i += kTinyThreads) pres[i] = 0u;
  __syncthreads();
  const gptr<const In> vals = to_global(static_cast<const In*>(D.vals));
  const bool rowmajor = rows_coalesced(D.order, D.stride_e, D.stride_j);
  const long long ntiles = (D.nnz + TA - 1) / TA;
  for (long long t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const long long s0 = t * TA + (long long)w * 64 * IPT;  // this wave's slice
    const long long n = D.nnz - s0;
    unsigned long long key[IPT];
    uint64_t p[IPT];
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      key[j] = 0;
      p[j] = FO::start_prod((long long)j * 64 + ln < n ? vals[s0 + j * 64 + ln] : (In)0);
    }
    for_rows<IdxT, IPT, MO>(static_cast<const IdxT*>(D.subs), D.stride_e, D.stride_j, D.order, rowmajor, s0, n,
                            stage[w], [&](int m, int j, long long x) {
                              if ((long long)j * 64 + ln >= n) return;
                              if (D.validate && (x < 0 || x >= D.dims[m])) {
                                atomicCAS(err, 0, TTV_E_INDEX);
                                x = 0;
                              }
                              if (D.mrem[m])
                                key[j] += (unsigned long long)x * D.mstride[m];
                              else if (D.vec[m])
                                p[j] = FO::mul_prod(p[j], to_global(static_cast<const In*>(D.vec[m]))[x]);
                            });
    for (int turn = 0; turn < NW; ++turn) {
      if (w == turn) {
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
          if ((long long)j * 64 + ln < n) {
            const unsigned k = (unsigned)key[j];
            atomicAdd(&acc[k], FO::to_f64(FO::from_pay(p[j])));
            atomicOr(&pres[k >> 5], 1u << (k & 31));
          }
        }
      }
      __syncthreads();
    }
  }
  __syncthreads();
  const gptr<double> part = to_global(partials) + (size_t)blockIdx.x * range;
  for (long long i = tid; i < range; i += kTinyThreads) part[i] = acc[i];
  for (long long i = tid; i < (range + 31) / 32; i += kTinyThreads)
    if (pres[i]) atomicOr(&present[i], pres[i]);
}

// Per key: the blocks' sums in block order; then the present keys in key
// order (one block).
__global__ __launch_bounds__(256) void k_keyed_sum(const double* partials, int nparts, long long range, double* y) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= range) return;
  const gptr<const double> part = to_global(partials);
  double s = 0.0;
#pragma unroll 8
  for (int b = 0; b < nparts; ++b) s += part[(size_t)b * range + k];
  to_global(y)[k] = s;
}

template <typename IdxT, int KC>
__global__ __launch_bounds__(kTinyThreads) void k_keyed_write(TDesc D, long long range, const double* y,
                                                              const unsigned* present) {
  constexpr int KPT = KC / kTinyThreads;
  __shared__ unsigned wsum[kTinyThreads / 64];
  const int k0 = (int)threadIdx.x * KPT;
  const gptr<const unsigned> pr = to_global(present);
  unsigned c = 0;
#pragma unroll
  for (int q = 0; q < KPT; ++q) {
    const int k = k0 + q;
    c += (k < range && ((pr[k >> 5] >> (k & 31)) & 1u)) ? 1u : 0u;
  }
  unsigned total;
  unsigned pos = block_excl_scan<kTinyThreads>(c, wsum, total);
  const gptr<IdxT> osubs = to_global(static_cast<IdxT*>(D.out_subs));
  const bool of64 = D.out_f64 != 0;  // FP64 values (FP64 inputs or TTV_OUT_F64), set by the launcher
  for (int q = 0; q < KPT; ++q) {
    const int k = k0 + q;
    if (k < range && ((pr[k >> 5] >> (k & 31)) & 1u)) {
      const double v = to_global(y)[k];
      if (of64)
        to_global(static_cast<double*>(D.out_vals))[pos] = v;
      else
        to_global(static_cast<float*>(D.out_vals))[pos] = (float)v;
      for (int i = 0; i < D.nrem; ++i)
        osubs[(long long)pos * D.nrem + i] =
            (IdxT)(((unsigned long long)k / D.kstride[i]) % (unsigned long long)D.dims[D.rem[i]]);
      ++pos;
    }
  }
  if (threadIdx.x == 0) *to_global(D.out_nnz) = (long long)total;
}

}  // namespace

// The product's key count if it fits the LDS sums of its row class, else -1.
long long keyed_range(const PipePlan& P) {
  unsigned __int128 range = 1;
  for (int i = 0; i < P.d0.nrem; ++i) range *= (unsigned __int128)P.d0.dims[P.d0.rem[i]];
  const int mo = row_width_class(P.d0.order, P.d0.stride_e, P.d0.stride_j);
  const int cap = mo <= 3 ? key_cap<3>() : key_cap<kMaxOrder>();
  return range <= (unsigned __int128)cap ? (long long)range : -1;
}

bool keyed_fits(const PipePlan& P, int flags) {
  return !(flags & TTV_DROP_ZEROS) && P.d0.nnz > kTinyNnz && keyed_range(P) > 0;
}

static long long keyed_parts(long long nnz) {
  const long long tiles = (nnz + 4096 - 1) / 4096;
  return std::max<long long>(1, std::min<long long>(kKeyedBlocks, tiles));
}

size_t keyed_ws(const PipePlan& P) {
  const long long range = keyed_range(P);
  if (range <= 0) return 0;
  // header (error word) | bitmap | y | partials
  return 256 + 256 * 8 + (size_t)range * 8 + (size_t)keyed_parts(P.d0.nnz) * range * 8 + 256;
}

int launch_keyed(const PipePlan& P, void* ws, hipStream_t s) {
  (void)hipGetLastError();  // errors left by earlier, unrelated runtime calls are not ours
  const long long range = keyed_range(P);
  char* w = static_cast<char*>(ws);
  int32_t* err = reinterpret_cast<int32_t*>(w + offsetof(Ctrl, error));
  unsigned* present = reinterpret_cast<unsigned*>(w + 256);
  double* y = reinterpret_cast<double*>(w + 256 + 256 * 8);
  double* partials = reinterpret_cast<double*>(w + 256 + 256 * 8 + ((range * 8 + 255) & ~255LL));
  if (int rc = launch_zero(w, 256 + 256 * 8, s)) return rc;  // error word and bitmap
  const int G = (int)keyed_parts(P.d0.nnz);
  TDesc D = P.d0;
  D.out_f64 = (P.form == kF64 || D.out_f64) ? 1 : 0;
  const int mo = row_width_class(D.order, D.stride_e, D.stride_j);
  auto go = [&](auto idx_tag, auto form_tag) {
    using IdxT = decltype(idx_tag);
    constexpr int F = decltype(form_tag)::value;
    const bool wide = range > kTinyKeys;  // only rows of up to 3 indices get here with more keys
    if (mo <= 3 && wide)
      hipLaunchKernelGGL((k_keyed<IdxT, F, 3, key_cap<3>()>), dim3(G), dim3(kTinyThreads), 0, s, D, range, err,
                         partials, present);
    else if (mo <= 3)
      hipLaunchKernelGGL((k_keyed<IdxT, F, 3, kTinyKeys>), dim3(G), dim3(kTinyThreads), 0, s, D, range, err, partials,
                         present);
    else if (mo <= 5)
      hipLaunchKernelGGL((k_keyed<IdxT, F, 5, kTinyKeys>), dim3(G), dim3(kTinyThreads), 0, s, D, range, err, partials,
                         present);
    else
      hipLaunchKernelGGL((k_keyed<IdxT, F, kMaxOrder, kTinyKeys>), dim3(G), dim3(kTinyThreads), 0, s, D, range, err,
                         partials, present);
    hipLaunchKernelGGL(k_keyed_sum, dim3((unsigned)((range + 255) / 256)), dim3(256), 0, s, partials, G, range, y);
    if (wide)
      hipLaunchKernelGGL((k_keyed_write<IdxT, key_cap<3>()>), dim3(1), dim3(kTinyThreads), 0, s, D, range, y, present);
    else
      hipLaunchKernelGGL((k_keyed_write<IdxT, kTinyKeys>), dim3(1), dim3(kTinyThreads), 0, s, D, range, y, present);
  };
  auto by_form = [&](auto idx_tag) {
    if (P.form == kF64)
      go(idx_tag, std::integral_constant<int, kF64>());
    else
      go(idx_tag, std::integral_constant<int, kC32>());
  };
  if (P.idx64)
    by_form((long long)0);
  else
    by_form((int)0);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_last_hip_error((int)e);
    return TTV_E_HIP;
  }
  return TTV_OK;
}

bool tiny_fits(const PipePlan& P, int flags) {
  return !(flags & TTV_DROP_ZEROS) && P.d0.nnz <= kTinyNnz && keyed_range(P) >= 0;
}

int launch_tiny(const PipePlan& P, void* ws, hipStream_t s) {
  (void)hipGetLastError();  // errors left by earlier, unrelated runtime calls are not ours
  long long range = 1;
  for (int i = 0; i < P.d0.nrem; ++i) range *= P.d0.dims[P.d0.rem[i]];
  int32_t* err = reinterpret_cast<int32_t*>(static_cast<char*>(ws) + offsetof(Ctrl, error));
  const int mo = row_width_class(P.d0.order, P.d0.stride_e, P.d0.stride_j);
  auto go = [&](auto idx_tag, auto form_tag) {
    using IdxT = decltype(idx_tag);
    constexpr int F = decltype(form_tag)::value;
    if (mo <= 3 && range > kTinyKeys)  // only rows of up to 3 indices get here with more keys
      hipLaunchKernelGGL((k_tiny<IdxT, F, 3, key_cap<3>()>), dim3(1), dim3(kTinyThreads), 0, s, P.d0, range, err);
    else if (mo <= 3)
      hipLaunchKernelGGL((k_tiny<IdxT, F, 3, kTinyKeys>), dim3(1), dim3(kTinyThreads), 0, s, P.d0, range, err);
    else if (mo <= 5)
      hipLaunchKernelGGL((k_tiny<IdxT, F, 5, kTinyKeys>), dim3(1), dim3(kTinyThreads), 0, s, P.d0, range, err);
    else
      hipLaunchKernelGGL((k_tiny<IdxT, F, kMaxOrder, kTinyKeys>), dim3(1), dim3(kTinyThreads), 0, s, P.d0, range,
                         err);
  };
  auto by_form = [&](auto idx_tag) {
    if (P.form == kF64)
      go(idx_tag, std::integral_constant<int, kF64>());
    else
      go(idx_tag, std::integral_constant<int, kC32>());
  };
  if (P.idx64)
    by_form((long long)0);
  else
    by_form((int)0);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_last_hip_error((int)e);
    return TTV_E_HIP;
  }
  return TTV_OK;
}

}  // namespace ttv
