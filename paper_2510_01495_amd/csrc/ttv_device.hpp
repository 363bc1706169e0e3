// Device primitives for gfx950 (CDNA4, wave64): lane masks, ballot
// multisplit, DPP prefix scans, error-free FP32 transforms and the two
// value forms (FP64, compensated FP32).
#pragma once

#include <hip/hip_runtime.h>

#include "ttv_internal.h"

namespace ttv {

// ---------------------------------------------------------------------------
// Lanes and masks
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
// Number of set bits of m in the lanes below this one.
__device__ __forceinline__ unsigned count_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Orders LDS accesses of one wave across lanes (a wave's LDS instructions
// execute in issue order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lanes of `valid` whose r-bit digit equals this lane's (ballot multisplit:
// one ballot per digit bit, keep the lanes that agree on every bit).
__device__ __forceinline__ uint64_t match_digit(unsigned d, int r, uint64_t valid) {
  uint64_t m = valid;
  for (int b = 0; b < r; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t bb = __ballot(bit);
    m &= bit ? bb : ~bb;
  }
  return m;
}

// ---------------------------------------------------------------------------
// DPP wave prefix sums (u32).  Rows of 16 lanes scan with row_shr 1/2/4/8,
// then row_bcast:15 and row_bcast:31 carry the row totals across rows.
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned wave_incl_scan(unsigned v) {
  v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return v;
}
__device__ __forceinline__ unsigned wave_total(unsigned incl) {
  return (unsigned)__builtin_amdgcn_readlane((int)incl, 63);
}

// Block-wide exclusive scan of one u32 per thread.  `wsum` holds NT/64
// entries of LDS.  Returns the exclusive prefix; `total` gets the block sum.
template <int NT>
__device__ __forceinline__ unsigned block_excl_scan(unsigned v, unsigned* wsum, unsigned& total) {
  const unsigned inc = wave_incl_scan(v);
  const int w = threadIdx.x >> 6;
  if (lane_id() == 63) wsum[w] = inc;
  __syncthreads();
  unsigned off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) {
    const unsigned s = wsum[i];
    off += (i < w) ? s : 0u;
    tot += s;
  }
  __syncthreads();
  total = tot;
  return off + inc - v;
}

template <int NT>
__device__ __forceinline__ unsigned block_sum(unsigned v, unsigned* wsum) {
  unsigned t;
  block_excl_scan<NT>(v, wsum, t);
  return t;
}

// ---------------------------------------------------------------------------
// Error-free transformations (Knuth's TwoSum; TwoProduct through fmaf) and
// the Dot2 accumulator of Ogita, Rump and Oishi ("Accurate Sum and Dot
// Product", SISC 2005): the running sum s plus an FP32 accumulator c of the
// exact rounding errors.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}
__device__ __forceinline__ void two_prod(float a, float b, float& p, float& e) {
  p = a * b;
  e = __builtin_fmaf(a, b, -p);
}

struct C2 {
  float s, c;
};

// ---------------------------------------------------------------------------
// Value forms.  A record payload is 64 bits: an FP64 product, or the FP32
// pair (hi, lo) with hi + lo the exact product of FP32 inputs.
// ---------------------------------------------------------------------------
template <int F>
struct FormOps;

template <>
struct FormOps<kF64> {
  using In = double;
  using Acc = double;
  static __device__ __forceinline__ Acc zero() { return 0.0; }
  static __device__ __forceinline__ Acc from_pay(uint64_t p) { return __longlong_as_double((long long)p); }
  static __device__ __forceinline__ Acc add(Acc a, Acc b) { return a + b; }
  static __device__ __forceinline__ double to_f64(Acc a) { return a; }
  // product of the value with the vector entries of the contracted modes
  static __device__ __forceinline__ uint64_t start_prod(In a) { return (uint64_t)__double_as_longlong(a); }
  static __device__ __forceinline__ uint64_t mul_prod(uint64_t p, In x) {
    return (uint64_t)__double_as_longlong(__longlong_as_double((long long)p) * x);
  }
  static __device__ __forceinline__ Acc shfl_up(Acc a, int d) { return __shfl_up(a, d, 64); }
  static __device__ __forceinline__ Acc shfl_last(Acc a) { return __shfl(a, 63, 64); }
};

template <>
struct FormOps<kC32> {
  using In = float;
  using Acc = C2;
  static __device__ __forceinline__ Acc zero() { return C2{0.f, 0.f}; }
  static __device__ __forceinline__ Acc from_pay(uint64_t p) {
    return C2{__uint_as_float((unsigned)p), __uint_as_float((unsigned)(p >> 32))};
  }
  static __device__ __forceinline__ uint64_t make_pay(float hi, float lo) {
    return (uint64_t)__float_as_uint(hi) | ((uint64_t)__float_as_uint(lo) << 32);
  }
  // Dot2 combination of two partial sums: TwoSum of the leading parts, the
  // error terms added in FP32.
  static __device__ __forceinline__ Acc add(Acc a, Acc b) {
    float s, q;
    two_sum(a.s, b.s, s, q);
    return C2{s, (a.c + b.c) + q};
  }
  static __device__ __forceinline__ double to_f64(Acc a) { return (double)a.s + (double)a.c; }
  // Compensated product: TwoProduct of the leading part, the error term
  // carried and scaled by every further factor.
  static __device__ __forceinline__ uint64_t start_prod(In a) { return make_pay(a, 0.f); }
  static __device__ __forceinline__ uint64_t mul_prod(uint64_t p, In x) {
    const C2 v = from_pay(p);
    float hi, e;
    two_prod(v.s, x, hi, e);
    return make_pay(hi, __builtin_fmaf(v.c, x, e));
  }
  static __device__ __forceinline__ Acc shfl_up(Acc a, int d) {
    return C2{__shfl_up(a.s, d, 64), __shfl_up(a.c, d, 64)};
  }
  static __device__ __forceinline__ Acc shfl_last(Acc a) { return C2{__shfl(a.s, 63, 64), __shfl(a.c, 63, 64)}; }
};

// Segmented-scan element: `f` marks that a segment head lies inside.
template <int F>
struct Seg {
  typename FormOps<F>::Acc v;
  int f;
};
template <int F>
__device__ __forceinline__ Seg<F> seg_combine(const Seg<F>& a, const Seg<F>& b) {
  Seg<F> r;
  r.f = a.f | b.f;
  r.v = b.f ? b.v : FormOps<F>::add(a.v, b.v);
  return r;
}

// Pointers in the global address space: loads and stores through them are
// global_* instructions rather than flat ones.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> to_global(T* p) {
  return (gptr<T>)p;
}
template <typename T>
__device__ __forceinline__ gptr<const T> to_global(const T* p) {
  return (gptr<const T>)p;
}

// A record as one 16-byte vector (key, payload) for single load/store
// instructions in any address space.
typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));

// DPP move of a 32-bit value; lanes whose source is outside the pattern (or
// whose row is masked off) receive 0.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ int dpp32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWMASK, 0xf, false);
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp32<CTRL, ROWMASK>((int)(unsigned)b);
  const int hi = dpp32<CTRL, ROWMASK>((int)(unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dppf(float v) {
  return __int_as_float(dpp32<CTRL, ROWMASK>(__float_as_int(v)));
}

template <int F, int CTRL, int ROWMASK>
__device__ __forceinline__ Seg<F> seg_dpp_step(const Seg<F>& e) {
  Seg<F> y;
  y.f = dpp32<CTRL, ROWMASK>(e.f);
  if constexpr (F == kF64) {
    y.v = dpp64<CTRL, ROWMASK>(e.v);
  } else {
    y.v.s = dppf<CTRL, ROWMASK>(e.v.s);
    y.v.c = dppf<CTRL, ROWMASK>(e.v.c);
  }
  return seg_combine<F>(y, e);  // y is the identity where the source lane is invalid
}

// Inclusive segmented scan across the 64 lanes of a wave: row_shr 1/2/4/8
// within rows of 16, then row_bcast:15 and row_bcast:31 across rows.
template <int F>
__device__ __forceinline__ Seg<F> wave_seg_scan(Seg<F> e) {
  e = seg_dpp_step<F, 0x111, 0xf>(e);
  e = seg_dpp_step<F, 0x112, 0xf>(e);
  e = seg_dpp_step<F, 0x114, 0xf>(e);
  e = seg_dpp_step<F, 0x118, 0xf>(e);
  e = seg_dpp_step<F, 0x142, 0xa>(e);
  e = seg_dpp_step<F, 0x143, 0xc>(e);
  return e;
}

// Index loads from either index type.
template <typename IdxT>
__device__ __forceinline__ long long ld_idx(const TDesc& D, long long e, int j) {
  return (long long)static_cast<const IdxT*>(D.subs)[e * D.stride_e + (long long)j * D.stride_j];
}

__device__ __forceinline__ void set_error(Ctrl* C, int code) { atomicCAS(&C->error, 0, code); }

// n / d for an invariant divisor d, from its magic multiplier (see the
// planner): t = mulhi(m, n), q = (t + ((n - t) >> sh1)) >> sh2.
__device__ __forceinline__ unsigned long long udiv_magic(unsigned long long n, unsigned long long m, int sh1,
                                                         int sh2) {
  const unsigned long long t = __umul64hi(m, n);
  return (t + ((n - t) >> sh1)) >> sh2;
}

__device__ __forceinline__ int bitlen64(unsigned long long x) { return x ? 64 - __clzll((long long)x) : 0; }


// ---------------------------------------------------------------------------
// Index columns of one round of nonzeros: item j of this lane is nonzero
// r0 + j*64 + lane, valid while j*64 + lane < nrec (r0 is the first nonzero of
// the wave's slice); f(m, j, index) is called for every mode m < order.
//   Row-major rows (se <= MO consecutive indices per nonzero): the wave reads
//   its slice as consecutive words (every lane one word per load, so a load
//   covers whole cache lines) and transposes 64 rows at a time through its
//   LDS stage of 64*MO words.  A lane reading its own row directly touches
//   64 rows' worth of lines per load for one index each, which caps the read
//   rate well below HBM bandwidth.
//   Other strides (structure of arrays): one load per mode, lane-consecutive.
// ---------------------------------------------------------------------------
// The row-major read, in two steps so that a caller can issue the next
// round's loads before it consumes the current one: rows_issue loads the
// words, rows_deliver transposes them and calls f.
template <typename IdxT, int IPT, int MO>
__device__ __forceinline__ void rows_issue(const IdxT* subs_p, long long se, int order, long long r0, long long nrec,
                                           IdxT (&raw)[IPT][MO]) {
  const unsigned ln = lane_id();
  const long long nr = nrec <= 0 ? 0 : (nrec < 64 * IPT ? nrec : 64 * IPT);
  const long long wend = nr ? (nr - 1) * se + order : 0;  // the last row's padding is not read
  const gptr<const IdxT> p = to_global(subs_p) + r0 * se;
#pragma unroll
  for (int j = 0; j < IPT; ++j)
#pragma unroll
    for (int c = 0; c < MO; ++c) {
      const long long wi = (long long)j * 64 * se + c * 64 + ln;
      raw[j][c] = (c < se && wi < wend) ? p[wi] : (IdxT)0;
    }
}

template <typename IdxT, int IPT, int MO, typename Fn>
__device__ __forceinline__ void rows_deliver(const IdxT (&raw)[IPT][MO], long long se, int order, IdxT* stage,
                                             Fn&& f) {
  const unsigned ln = lane_id();
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    wave_lds_sync();
#pragma unroll
    for (int c = 0; c < MO; ++c)
      if (c < se) stage[c * 64 + ln] = raw[j][c];
    wave_lds_sync();
#pragma unroll
    for (int m = 0; m < MO; ++m)
      if (m < order) f(m, j, (long long)stage[ln * se + m]);
  }
  wave_lds_sync();
}

template <typename IdxT, int IPT, int MO, typename Fn>
__device__ __forceinline__ void for_rows(const IdxT* subs_p, long long se, long long sj, int order, bool rowmajor,
                                         long long r0, long long nrec, IdxT* stage, Fn&& f) {
  const gptr<const IdxT> subs = to_global(subs_p);
  const unsigned ln = lane_id();
  if (rowmajor) {
    IdxT raw[IPT][MO];
    rows_issue<IdxT, IPT, MO>(subs_p, se, order, r0, nrec, raw);
    rows_deliver<IdxT, IPT, MO>(raw, se, order, stage, f);
  } else {
#pragma unroll
    for (int m = 0; m < MO; ++m) {
      if (m >= order) break;
      long long x[IPT];
#pragma unroll
      for (int j = 0; j < IPT; ++j) {
        const long long i = (long long)j * 64 + ln;
        x[j] = i < nrec ? (long long)subs[(r0 + i) * se + (long long)m * sj] : 0;
      }
#pragma unroll
      for (int j = 0; j < IPT; ++j) f(m, j, x[j]);
    }
  }
}

}  // namespace ttv
