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

// Dense (all-but-one / adjoint) accumulation plan.
struct DensePlan {
  TDesc D{};
  int keep = 0;
  int form = kF64;
  int idx64 = 1;
  int nkeep = 0;
  int tile = 4096;
  int blocks = 256;
  int cus = 256;
  size_t ws_bytes = 0;
};

void set_last_hip_error(int e);
int device_cus();
int launch_pipeline(const PipePlan& P, void* ws, hipStream_t s);

}  // namespace ttv
