// Dense accumulation kernels: the all-but-one product (n_v = d - 1 vectors,
// Sec. 3.3) and the adjoints of both products.
//
// Each accumulator `a` sums, over the nonzeros e of X,
//     vals[e] * prod_{j in factor modes, j != key_a} f_j[subs(e, j)]  (* gseg[seg[e]])
// into a dense vector indexed by subs(e, key_a).  The forward all-but-one
// product is one accumulator (key = kept mode, factors = the other vectors);
// the adjoint of the all-but-one product has one accumulator per vector
// (factors = the vectors with the cotangent in the kept mode); the adjoint of
// the sparse product keys by the contracted mode with the cotangent gathered
// through the segment map.  The optional per-nonzero output is the product of
// all factors (the gradient with respect to vals).
//
// Accumulation is free of global atomics and deterministic: a block takes
// tiles of nonzeros in a fixed order and adds every product into its private
// dense LDS partial in FP64 (for FP32 inputs, the exact FP32 product pair
// widened to FP64), in nonzero order; the blocks' partials are summed in a
// fixed block order in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ttv_dense.h"
#include "ttv_device.hpp"
#include "ttv_host.h"

namespace ttv {

namespace {

constexpr int NT = kDenseThreads;
constexpr int NW = NT / 64;

template <typename IdxT, int F, int MO, int NACC>
__global__ __launch_bounds__(kDenseThreads) void k_dense(DenseArgs A) {
  using FO = FormOps<F>;
  using In = typename FO::In;
  constexpr int IPT = dense_ipt(F, sizeof(IdxT) == 8);
  constexpr int TA = NT * IPT;  // nonzeros per tile
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  // layout: FP64 accumulators | row stage IdxT[NW][64*MO] | staged factor vectors
  double* accs = reinterpret_cast<double*>(smem);
  IdxT* stage = reinterpret_cast<IdxT*>(smem + A.acc_bytes);
  In* vst = reinterpret_cast<In*>(smem + A.vst_at);
  const int tid = threadIdx.x, w = tid >> 6;
  const unsigned ln = lane_id();
  for (int i = tid; i < A.acc_total; i += NT) accs[i] = 0.0;
  // factor vectors that fit beside the accumulators are copied in once: their
  // random per-nonzero gathers then read LDS instead of L2
#pragma unroll
  for (int m = 0; m < MO; ++m) {
    if (m < A.order && A.vst_off[m] >= 0) {
      const gptr<const In> src = to_global(static_cast<const In*>(A.fac[m]));
      for (long long i = tid; i < A.dims[m]; i += NT) vst[A.vst_off[m] + i] = src[i];
    }
  }
  __syncthreads();
  const gptr<const In> vals = to_global(static_cast<const In*>(A.vals));
  // Row-major indices and the values of the block's next tile are loaded
  // during the current tile's turns: after the current tile's gathers (the
  // memory counter retires in issue order, so loads issued before them would
  // hold them up) and before the adds, which wait only for LDS.  Only with
  // one accumulator: the adjoints' several accumulators leave no registers
  // for it (measured slower).
  const bool rowmajor = rows_coalesced(A.order, A.se, A.sj[1]);
  const bool pre = NACC == 1 && rowmajor;
  const int s0 = w * 64 * IPT;  // this wave's slice of a tile
  IdxT rawn[IPT][MO];
  In an[IPT];
  auto issue = [&](long long t) {
    const long long e0 = t * TA;
    const int n = (int)((A.nnz - e0 < (long long)TA) ? A.nnz - e0 : (long long)TA);
    rows_issue<IdxT, IPT, MO>(static_cast<const IdxT*>(A.subs), A.se, A.order, e0 + s0, (long long)n - s0, rawn);
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      const int i = s0 + j * 64 + (int)ln;
      an[j] = i < n ? vals[e0 + i] : (In)0;
    }
  };
  if (pre && blockIdx.x < A.ntiles) issue(blockIdx.x);
  for (long long t = blockIdx.x; t < A.ntiles; t += gridDim.x) {
    const long long e0 = t * TA;
    const int n = (int)((A.nnz - e0 < (long long)TA) ? A.nnz - e0 : (long long)TA);
    // ---- per nonzero: indices of the key modes, products ----
    unsigned key[NACC][IPT];
    uint64_t pay[NACC][IPT];
    {
      uint64_t full[IPT];  // product of all factors (gradient w.r.t. vals)
      uint64_t pa[NACC][IPT];
      In a[IPT];
#pragma unroll
      for (int j = 0; j < IPT; ++j) {
        const int i = s0 + j * 64 + (int)ln;
        a[j] = pre ? an[j] : (i < n ? vals[e0 + i] : (In)0);
        full[j] = FO::start_prod((In)1);
#pragma unroll
        for (int q = 0; q < NACC; ++q) {
          pa[q][j] = FO::start_prod(a[j]);
          key[q][j] = 0;
        }
      }
      long long x[MO][IPT];
#pragma unroll
      for (int m = 0; m < MO; ++m)
#pragma unroll
        for (int j = 0; j < IPT; ++j) x[m][j] = 0;
      if (pre)
        rows_deliver<IdxT, IPT, MO>(rawn, A.se, A.order, stage + (size_t)w * 64 * MO,
                                    [&](int m, int j, long long v) { x[m][j] = v; });
      else
        for_rows<IdxT, IPT, MO>(static_cast<const IdxT*>(A.subs), A.se, A.sj[1], A.order, rowmajor, e0 + s0,
                                (long long)n - s0, stage + (size_t)w * 64 * MO,
                                [&](int m, int j, long long v) { x[m][j] = v; });
      if (A.validate) {
#pragma unroll
        for (int m = 0; m < MO; ++m)
#pragma unroll
          for (int j = 0; j < IPT; ++j)
            if (m < A.order && s0 + j * 64 + (int)ln < n && (x[m][j] < 0 || x[m][j] >= A.dims[m])) {
              atomicCAS(A.err, 0, TTV_E_INDEX);
              x[m][j] = 0;
            }
      }
      // vector entries of every factor mode, gathered together
      In g[MO][IPT];
#pragma unroll
      for (int m = 0; m < MO; ++m) {
        const In* fac = m < A.order ? static_cast<const In*>(A.fac[m]) : nullptr;
        const gptr<const In> f = to_global(fac);
        const long long so = m < A.order ? A.vst_off[m] : -1;  // uniform over the launch
        if (fac && so >= 0) {
#pragma unroll
          for (int j = 0; j < IPT; ++j) g[m][j] = s0 + j * 64 + (int)ln < n ? vst[so + x[m][j]] : (In)1;
        } else {
#pragma unroll
          for (int j = 0; j < IPT; ++j) g[m][j] = (fac && s0 + j * 64 + (int)ln < n) ? f[x[m][j]] : (In)1;
        }
      }
#pragma unroll
      for (int m = 0; m < MO; ++m) {
        if (m >= A.order) break;
#pragma unroll
        for (int q = 0; q < NACC; ++q)
          if (q < A.nacc && A.key_mode[q] == m) {
#pragma unroll
            for (int j = 0; j < IPT; ++j) key[q][j] = (unsigned)x[m][j];
          }
        if (A.fac[m]) {
#pragma unroll
          for (int j = 0; j < IPT; ++j) {
            full[j] = FO::mul_prod(full[j], g[m][j]);
#pragma unroll
            for (int q = 0; q < NACC; ++q)
              if (q < A.nacc && A.key_mode[q] != m) pa[q][j] = FO::mul_prod(pa[q][j], g[m][j]);
          }
        }
      }
      if (A.gseg) {
        const gptr<const In> gs = to_global(static_cast<const In*>(A.gseg));
        const gptr<const int32_t> sg = to_global(A.seg);
        In h[IPT];
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
          const int i = s0 + j * 64 + (int)ln;
          h[j] = i < n ? gs[sg[e0 + i]] : (In)0;
        }
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
          full[j] = FO::mul_prod(full[j], h[j]);
#pragma unroll
          for (int q = 0; q < NACC; ++q) pa[q][j] = FO::mul_prod(pa[q][j], h[j]);
        }
      }
      if (A.grad_vals) {
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
          const int i = s0 + j * 64 + (int)ln;
          if (i < n) {
            const double v = FO::to_f64(FO::from_pay(full[j]));
            if (F == kF64)
              to_global(static_cast<double*>(A.grad_vals))[e0 + i] = v;
            else
              to_global(static_cast<float*>(A.grad_vals))[e0 + i] = (float)v;
          }
        }
      }
#pragma unroll
      for (int q = 0; q < NACC; ++q)
#pragma unroll
        for (int j = 0; j < IPT; ++j) pay[q][j] = pa[q][j];
    }
    if (pre && t + gridDim.x < A.ntiles) issue(t + gridDim.x);
    // ---- LDS atomic adds in FP64, in nonzero order.  Waves take turns; in
    // a wave, items in order, and the lanes of one ds_add_f64 that hit the
    // same entry are applied in ascending lane order (as for the integer
    // adds the stable ranks rely on).  The block's partial is therefore the
    // in-order sum of its tiles, bitwise repeatable.  FP32 inputs add their
    // exact product pair widened to FP64 (no rounding before the sum). ----
#pragma unroll
    for (int q = 0; q < NACC; ++q) {
      if (q >= A.nacc) break;
      double* acc = accs + A.acc_off[q];
      for (int turn = 0; turn < NW; ++turn) {
        if (w == turn) {
#pragma unroll
          for (int j = 0; j < IPT; ++j)
            if (w * 64 * IPT + j * 64 + (int)ln < n) atomicAdd(&acc[key[q][j]], FO::to_f64(FO::from_pay(pay[q][j])));
        }
        __syncthreads();
      }
    }
  }
  __syncthreads();
  // block partials, FP64
  for (int i = tid; i < A.acc_total; i += NT)
    to_global(A.partials)[(size_t)blockIdx.x * A.acc_total + i] = accs[i];
}

// Sum the block partials of every output entry in block order (FP64).
// Block = 64 entries x 16 groups of blocks; group sums are added in order.
__global__ __launch_bounds__(1024) void k_dense_combine(DenseArgs A, int nparts) {
  __shared__ double part[16][64];
  const int dd = threadIdx.x & 63, g = threadIdx.x >> 6;
  const long long c0 = (long long)blockIdx.x * 64;
  const long long c = c0 + dd;
  const int per = (nparts + 15) / 16;
  const int b0 = g * per, b1 = std::min(nparts, b0 + per);
  double s = 0.0;
  if (c < A.acc_total) {
    const gptr<const double> P = to_global((const double*)A.partials);
    for (int b = b0; b < b1; ++b) s += P[(size_t)b * A.acc_total + c];
  }
  part[g][dd] = s;
  __syncthreads();
  if (g == 0 && c < A.acc_total) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) t += part[q][dd];
    // which accumulator / entry
    int q = 0;
    while (q + 1 < A.nacc && c >= A.acc_off[q + 1]) ++q;
    const long long i = c - A.acc_off[q];
    if (A.out_f64)
      to_global(static_cast<double*>(A.out[q]))[i] = t;
    else
      to_global(static_cast<float*>(A.out[q]))[i] = (float)t;
  }
}

// Dense output from a sparse one: zero-fill, then scatter the values.
__global__ __launch_bounds__(256) void k_fill_zero(void* out, long long n_out, int f64) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n_out;
       i += (long long)gridDim.x * blockDim.x) {
    if (f64)
      static_cast<double*>(out)[i] = 0.0;
    else
      static_cast<float*>(out)[i] = 0.f;
  }
}

// vals: FP64 values of the sparse result, idx: its single index column
template <typename IdxT>
__global__ __launch_bounds__(256) void k_scatter_dense(const IdxT* idx, const double* vals, const long long* cnt,
                                                       void* out, long long n_out, int f64) {
  const long long m = *cnt;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (long long)gridDim.x * blockDim.x) {
    const long long k = (long long)idx[i];
    if (k < 0 || k >= n_out) continue;
    if (f64)
      static_cast<double*>(out)[k] = vals[i];
    else
      static_cast<float*>(out)[k] = (float)vals[i];
  }
}

template <typename IdxT, int F, int MO, int NACC>
void launch_dense_k(const DenseArgs& A, int grid, size_t lds, hipStream_t s) {
  hipFuncSetAttribute((const void*)k_dense<IdxT, F, MO, NACC>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  prof_begin(TTV_PROF_DENSE, s);
  hipLaunchKernelGGL((k_dense<IdxT, F, MO, NACC>), dim3(grid), dim3(kDenseThreads), lds, s, A);
  prof_end(TTV_PROF_DENSE, s);
}

// one accumulator (the forward all-but-one product) or up to kDenseMaxAcc
template <typename IdxT, int F, int MO>
int launch_dense_impl(const DenseArgs& A, int grid, size_t lds, hipStream_t s) {
  if (A.nacc <= 1)
    launch_dense_k<IdxT, F, MO, 1>(A, grid, lds, s);
  else
    launch_dense_k<IdxT, F, MO, kDenseMaxAcc>(A, grid, lds, s);
  const int cb = (int)((A.acc_total + 63) / 64);
  hipLaunchKernelGGL(k_dense_combine, dim3(std::max(cb, 1)), dim3(1024), 0, s, A, grid);
  return 0;
}

}  // namespace

size_t dense_tile_lds(int form, int idx64, int mo) {
  (void)form;
  return (size_t)NW * 64 * mo * (idx64 ? 8 : 4);
}

template <typename IdxT, int F>
int launch_dense_mo(const DenseArgs& A, int mo, int grid, size_t lds, hipStream_t s) {
  switch (mo) {
    case 3: return launch_dense_impl<IdxT, F, 3>(A, grid, lds, s);
    case 5: return launch_dense_impl<IdxT, F, 5>(A, grid, lds, s);
    default: return launch_dense_impl<IdxT, F, kMaxOrder>(A, grid, lds, s);
  }
}

int launch_dense(const DenseArgs& A, int idx64, int form, int grid, size_t lds, hipStream_t s) {
  const int mo = row_width_class(A.order, A.se, A.sj[1]);
  if (form == kF64) {
    if (idx64) return launch_dense_mo<long long, kF64>(A, mo, grid, lds, s);
    return launch_dense_mo<int, kF64>(A, mo, grid, lds, s);
  }
  if (idx64) return launch_dense_mo<long long, kC32>(A, mo, grid, lds, s);
  return launch_dense_mo<int, kC32>(A, mo, grid, lds, s);
}

int launch_zero(void* p, size_t bytes, hipStream_t s) {
  const long long n = (long long)(bytes / 4);
  const int g = (int)std::min<long long>(std::max<long long>(1, (n + 255) / 256), 1024);
  hipLaunchKernelGGL(k_fill_zero, dim3(g), dim3(256), 0, s, p, n, 0);
  return 0;
}

int launch_densify(const void* idx, int idx64, const void* vals, const long long* cnt, void* out, long long n_out,
                   int f64, int cus, hipStream_t s) {
  const int g = (int)std::min<long long>(std::max<long long>(1, (n_out + 255) / 256), 4LL * cus);
  hipLaunchKernelGGL(k_fill_zero, dim3(g), dim3(256), 0, s, out, n_out, f64);
  if (idx64)
    hipLaunchKernelGGL(k_scatter_dense<long long>, dim3(g), dim3(256), 0, s, (const long long*)idx,
                       (const double*)vals, cnt, out, n_out, f64);
  else
    hipLaunchKernelGGL(k_scatter_dense<int>, dim3(g), dim3(256), 0, s, (const int*)idx, (const double*)vals, cnt,
                       out, n_out, f64);
  return 0;
}

}  // namespace ttv
