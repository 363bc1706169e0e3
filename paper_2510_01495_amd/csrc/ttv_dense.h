// Arguments of the dense-accumulation kernels (all-but-one product and the
// adjoints).  Passed by value to the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "ttv_internal.h"

namespace ttv {

constexpr int kDenseThreads = 1024;
// Nonzeros per lane and tile: 4 for FP32 values with 32-bit indices (fewer
// ordered-add turns per nonzero; their registers allow it), 2 otherwise
// (wider index rows and FP64 values would spill).
__host__ __device__ constexpr int dense_ipt(int form, bool idx64) { return (form == kC32 && !idx64) ? 4 : 2; }
constexpr int kDenseMaxAcc = 4;

struct DenseArgs {
  const void* subs;
  const void* vals;
  long long se;                  // subs element stride
  long long sj[kMaxOrder];       // subs mode stride times mode
  long long dims[kMaxOrder];
  const void* fac[kMaxOrder];    // factor vector per mode (null: no factor)
  const void* gseg;              // optional factor gathered through `seg`
  const int32_t* seg;            // output row of every nonzero (with gseg)
  void* grad_vals;               // optional per-nonzero product of all factors
  double* partials;              // [grid][acc_total] FP64
  void* out[kDenseMaxAcc];       // dense results (FP64, or FP32 unless out_f64)
  int32_t* err;                  // device error word
  long long nnz;
  long long ntiles;
  int order;
  int validate;
  int nacc;
  int key_mode[kDenseMaxAcc];
  int key_bits[kDenseMaxAcc];
  long long acc_off[kDenseMaxAcc];  // entry offsets of the accumulators
  long long acc_total;              // sum of the accumulator lengths
  size_t acc_bytes;                 // LDS bytes of the accumulators (16-byte aligned)
  size_t vst_at;                    // LDS byte offset of the staged factor vectors
  long long vst_off[kMaxOrder];     // per mode: element offset of its staged vector, or -1 (gathered from HBM)
  int out_f64;
};

size_t dense_tile_lds(int form, int idx64, int mo);  // LDS of one block besides its accumulators
int launch_dense(const DenseArgs& A, int idx64, int form, int grid, size_t lds, hipStream_t s);
int launch_densify(const void* idx, int idx64, const void* vals, const long long* cnt, void* out, long long n_out,
                   int f64, int cus, hipStream_t s);

}  // namespace ttv
