// Host-side planning structures shared by the C ABI and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "ttv_internal.h"

namespace ttv {

// A fully planned run of the keyed-reduction pipeline over `count` tensors.
struct PipePlan {
  int count = 0;
  int levels = 1;
  int form = kF64;
  int idx64 = 1;
  int pipe_mode = kPipeTTV;
  int T1 = 16384;       // records per level-1 tile
  int T2 = 16384;       // records per tile at deeper levels
  int cus = 256;
  int spin_limit = 1 << 22;
  long long total = 0;
  long long tiles1 = 0;
  TDesc d0{};                       // single tensor: passed by value to the init kernel
  const TDesc* descs_dev = nullptr; // batched: device-readable descriptor array
  std::vector<TDesc> descs;         // host copies
  Layout L{};
};

void set_last_hip_error(int e);
int device_cus();
// Environment switches, read on every call.
//   TTV_LOG=1          the planners print each plan to stderr (what runs, its
//                      sizes and workspace).
//   TTV_FAULT=launch   every entry point that would launch kernels returns
//                      TTV_E_HIP (hipErrorLaunchFailure) after validating its
//                      arguments, without touching the device.
//   TTV_FAULT=spin     the bounded waits of the sorting pipeline give up at
//                      once (TTV_E_DEVICE from the device error word); every
//                      kernel still ends and writes only inside its buffers.
// TTV_FAULT takes a comma-separated list of these names.
bool log_on();
bool fault_on(const char* what);
int fault_launch();  // TTV_E_HIP if TTV_FAULT names "launch", else TTV_OK
int launch_pipeline(const PipePlan& P, void* ws, hipStream_t s);
int plan_tensor(const ttv_coo_desc* X, int ncon, const int32_t* modes, int flags, TDesc& D, int& form, int& idx64);
int plan_single(const ttv_coo_desc* X, int ncon, const int32_t* modes, int flags, int pipe_mode, PipePlan& P);
// dense: buckets of at most kDenseBits relative key bits may become dense
// leaves (every pipeline mode except kPipePerm, whose leaves must be sorted)
// aux: the nonzero-index arrays beside the record buffers (kPipeTTVSeg)
Layout make_layout(long long total, int count, int levels, int T1, int T2, long long tiles1, bool dense,
                   bool aux = false);
inline int dense_bits_of(int pipe_mode) { return pipe_mode == kPipePerm ? 0 : kDenseBits; }
int finish_plan(PipePlan& P);  // levels, tiles and layout of a planned single tensor
int launch_zero(void* p, size_t bytes, hipStream_t s);
void set_divmagic(unsigned long long d, unsigned long long& m, int& sh1, int& sh2);
int choose_r1(long long nnz, unsigned __int128 range, int bits);

// measurement hook (see ttv_profile_events)
void prof_begin(int kernel, hipStream_t s);
void prof_end(int kernel, hipStream_t s);

// Removal of exact-zero sums from a sparse result (TTV_DROP_ZEROS): the
// product writes into a temporary area laid out by drop_zeros_layout, then
// launch_drop_zeros compacts the kept rows into the caller's output.
constexpr int kDropBlocks = 512;
size_t drop_zeros_ws(long long nnz, int nrem, int idx64, int out_f64);
void drop_zeros_layout(void* tmp, long long nnz, int nrem, int idx64, long long*& cnt, long long*& counts,
                       void*& subs, void*& vals);
int launch_drop_zeros(const void* in_subs, const void* in_vals, const long long* in_nnz, long long* counts,
                      void* out_subs, void* out_vals, long long* out_nnz, int nrem, int idx64, int out_f64,
                      hipStream_t s);

// Small products in one block and one launch (at most kTinyNnz nonzeros and
// kTinyKeys keys of the remaining modes -- twice that for rows of at most
// three indices), FP64 sums.
constexpr long long kTinyNnz = 1 << 15;
constexpr int kTinyKeys = 8192;
bool tiny_fits(const PipePlan& P, int flags);
int launch_tiny(const PipePlan& P, void* ws, hipStream_t s);
// Larger products with at most kTinyKeys keys: per-block dense sums by key,
// added in block order.
bool keyed_fits(const PipePlan& P, int flags);
size_t keyed_ws(const PipePlan& P);
int launch_keyed(const PipePlan& P, void* ws, hipStream_t s);

constexpr int kAssumedCUs = 256;  // MI355X; tiling never depends on the device queried at call time

}  // namespace ttv
