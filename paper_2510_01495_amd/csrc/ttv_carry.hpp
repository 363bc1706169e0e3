// Carries of a streaming segmented sum over a sorted order (plan reuse and
// MTTKRP): the sorted positions are cut into chunks of CHUNK; every chunk
// sums its rows, writes the rows that start and end inside it, and leaves two
// partial sums: entry 2c for chunk c's first run (its row may continue from
// the previous chunk) and entry 2c+1 for its last run (unused when the chunk
// holds a single run).  A row's entries are consecutive among the used ones:
// the entry that opens it, then entry 2c of every following chunk whose
// first row is the same.  Which entries belong together depends only on the
// sorted order, so it is computed once, when the order is.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

#include "ttv_device.hpp"

namespace ttv {

struct CarryGroup {
  long long row;  // output row (rank) of the entry that opens it; -1: the entry opens none
  long long cnt;  // following entries of the same row (entries 2c of the next cnt chunks)
};

// groups[e] for every carry entry, from the output row of every sorted
// position (rowid) and of every chunk's first position (row0, nondecreasing).
template <int CHUNK>
__global__ __launch_bounds__(256) void k_carry_groups(const int32_t* rowid, const long long* row0, long long nnz,
                                                      long long nchunks, CarryGroup* groups) {
  const gptr<const int32_t> gr = to_global(rowid);
  const long long E = 2 * nchunks;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < E;
       e += (long long)gridDim.x * blockDim.x) {
    const long long c = e >> 1, k0 = c * CHUNK;
    const long long n = std::min<long long>(CHUNK, nnz - k0);
    const long long first = gr[k0], last = gr[k0 + n - 1];
    const long long r = (e & 1) ? (last != first ? last : -1) : first;
    // the previous used entry's row: entry 2c's for entry 2c+1, else the
    // previous chunk's last row
    const long long prev = (e & 1) ? first : (c > 0 ? (long long)gr[k0 - 1] : -1);
    CarryGroup g{-1, 0};
    if (r >= 0 && r != prev) {
      long long lo = c + 1, hi = nchunks;  // first chunk after c whose first row exceeds r
      while (lo < hi) {
        const long long mid = (lo + hi) >> 1;
        if (row0[mid] > r)
          hi = mid;
        else
          lo = mid + 1;
      }
      g = CarryGroup{r, lo - (c + 1)};
    }
    groups[e] = g;
  }
}

// A wave-uniform 64-bit value moved to scalar registers.
__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}

}  // namespace ttv
