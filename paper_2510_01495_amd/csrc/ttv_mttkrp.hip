// Sparse MTTKRP, the matricized tensor times Khatri-Rao product that the
// paper names as its next target (TTV's per-nonzero product with one factor
// row per mode instead of one vector entry):
//     M[i, r] = sum over nonzeros e with subs(e, mode) = i of
//               vals[e] * prod_{j != mode} U_j[subs(e, j), r],   r < R.
//
// The tensor is fixed across calls (CP-ALS and tensor regression call MTTKRP
// on the same tensor with new factors every iteration), so the keyed sort by
// the mode's index runs once, in setup (the sorting pipeline in its
// permutation mode, every mode but `mode` contracted), and every apply is
// one streaming pass over the nonzeros in output-row order:
//   setup: the nonzero at every sorted position and its output row (rank of
//          its mode index among the distinct ones); a gather stores, in
//          sorted order, the values, the other modes' indices (uint32, one
//          array per mode), one bit per position marking where a row starts,
//          the first row of every unit of kMUnit positions, the mode index of
//          every row, and the carry groups (which unit partials make one row).
//   apply: a group of GS lanes (one per column r, GS = the power of two >= R,
//          at most 64; NC columns per lane beyond 64) walks one unit's
//          positions in order: per position the product of the value with
//          every factor row (coalesced row reads), added to the open row's
//          sums; a finished row is written (with the zero rows before the
//          next stored row), the unit's first and last rows go to carries,
//          which a second kernel adds per row in a fixed order (FP64).
// Every sum has one fixed order: bitwise repeatable.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>

#include "ttv.h"
#include "ttv_carry.hpp"
#include "ttv_device.hpp"
#include "ttv_host.h"

struct ttv_mttkrp_plan {
  ttv::PipePlan P;  // permutation-mode pipeline keyed by the mode's index
  ttv_coo_desc X;   // descriptor (its arrays are read by setup only)
  int mode = 0;
  int R = 0;
  int nf = 0;  // other modes
  int others[TTV_MAX_ORDER] = {0};
  int idx64 = 1;
  int form = ttv::kF64;
  int out_f64 = 1;
  long long nnz = 0;
  long long nunits = 0;
  long long dcap = 0;  // rows the distinct-index list can hold: min(nnz, shape[mode])
  size_t off_sv = 0, off_sidx = 0, off_heads = 0, off_rank0 = 0, off_dist = 0, off_groups = 0, off_carry = 0;
  size_t off_hier = 0;
  int hlevels = 0;                         // unit-carry hierarchy levels above 0
  int long_rows = 0;                       // some row spans more than kSerial units (setup)
  long long hoff[8] = {0}, hcnt[8] = {0};  // entry offset and count of every level
  size_t data_bytes = 0;
  size_t off_perm = 0, off_rowid = 0, off_osubs = 0, setup_bytes = 0;
  void* data = nullptr;  // bound by setup
};

namespace ttv {
namespace {

constexpr int kMUnit = 128;       // sorted positions per unit (one lane group, in order)
constexpr int kMThreads = 256;    // 4 waves
constexpr int kMMaxR = 256;
constexpr size_t kMHdr = 256;     // int64 nnz_out at offset 0

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Setup gather.  sv[k] = vals[perm[k]]; sidx[f][k] = subs(perm[k], others[f]);
// heads bit k set when position k starts a row; rank0[u] = row of position
// u * kMUnit; dist[r] = the mode index of row r.  One wave per 64 positions.
struct GatherArgs {
  const void* subs;
  const void* vals;
  long long se, sj;
  const int32_t* perm;
  const int32_t* rowid;
  const void* osubs;  // distinct mode indices from the pipeline (input index type)
  const long long* out_nnz;
  long long nnz, dcap;
  int others[kMaxOrder];
  int nf;
  void* sv;
  uint32_t* sidx;
  unsigned long long* heads;
  long long* rank0;
  long long* dist;
};

template <typename IdxT, typename In>
__global__ __launch_bounds__(256) void k_mttkrp_gather(GatherArgs A) {
  const gptr<const IdxT> gs = to_global(static_cast<const IdxT*>(A.subs));
  const gptr<const In> gv = to_global(static_cast<const In*>(A.vals));
  const gptr<const int32_t> gp = to_global(A.perm);
  const gptr<const int32_t> gr = to_global(A.rowid);
  const long long nout = *A.out_nnz;
  const gptr<const IdxT> os = to_global(static_cast<const IdxT*>(A.osubs));
  for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < nout && r < A.dcap;
       r += (long long)gridDim.x * blockDim.x)
    A.dist[r] = (long long)os[r];
  const unsigned ln = lane_id();
  const long long nw = (A.nnz + 63) / 64;
  const long long tw = (long long)gridDim.x * (blockDim.x / 64);
  In* sv = static_cast<In*>(A.sv);
  for (long long q = (long long)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); q < nw; q += tw) {
    const long long k = q * 64 + ln;
    bool h = false;
    if (k < A.nnz) {
      const long long e = gp[k];
      sv[k] = gv[e];
      for (int f = 0; f < A.nf; ++f) A.sidx[(size_t)f * A.nnz + k] = (uint32_t)gs[e * A.se + A.others[f] * A.sj];
      const int32_t r = gr[k];
      h = k == 0 || r != gr[k - 1];
      if (k % kMUnit == 0) A.rank0[k / kMUnit] = r;
    }
    const uint64_t m = ballot(h);
    if (ln == 0) A.heads[q] = m;
  }
}

constexpr long long kSerial = 32;  // rows spanning at most this many more units: carries added one by one
constexpr int kMaxHier = 6;        // hierarchy levels: 32^5 units exceed any supported nnz

struct MArgs {
  const void* sv;
  const uint32_t* sidx;
  const unsigned long long* heads;
  const long long* rank0;
  const long long* dist;
  const long long* hdr;
  const CarryGroup* groups;
  double* carry;  // [2 * nunits][R]
  double* hier;   // levels 1.. of the unit-carry hierarchy, [hoff[h] + i][R]
  const long long* longest;  // largest row span in units (setup), 0 if none above kSerial
  long long hoff[kMaxHier + 1];
  long long hcnt[kMaxHier + 1];  // entries per level (hcnt[0] = nunits)
  int hlevels;                   // levels above 0
  const void* fac[kMaxOrder];  // factor of the f-th other mode, (shape, R) row-major
  void* M;
  long long nnz, nunits, nrows;
  int R, GS, nf, out_f64;
};

template <int NC>
__device__ __forceinline__ void store_m(const MArgs& A, long long i, int rl, const double (&v)[NC]) {
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const int r = rl + 64 * k;
    if (r < A.R) {
      if (A.out_f64)
        to_global(static_cast<double*>(A.M))[i * A.R + r] = v[k];
      else
        to_global(static_cast<float*>(A.M))[i * A.R + r] = (float)v[k];
    }
  }
}

// Row `rank` of the result (its mode index from dist), then the rows that no
// nonzero reaches up to the next stored row (and, for the first row, the
// ones before it), written as zeros by the lanes of the group.
template <int NC>
__device__ __forceinline__ void write_row(const MArgs& A, long long rank, int rl, const double (&v)[NC]) {
  const long long nout = A.hdr[0];
  const long long i = A.dist[rank];
  store_m<NC>(A, i, rl, v);
  const long long next = rank + 1 < nout ? A.dist[rank + 1] : A.nrows;
  double z[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) z[k] = 0.0;
  for (long long q = i + 1; q < next; ++q) store_m<NC>(A, q, rl, z);
  if (rank == 0)
    for (long long q = 0; q < i; ++q) store_m<NC>(A, q, rl, z);
}

// One unit per lane group: positions in order, B at a time (their loads
// issued together), the open row's sums per column.
template <int F, int NC, int MO>
__global__ __launch_bounds__(kMThreads) void k_mttkrp_apply(MArgs A) {
  using FO = FormOps<F>;
  using Acc = typename FO::Acc;
  using In = typename FO::In;
  constexpr int B = MO <= 2 ? 8 : (MO <= 4 ? 4 : 2);
  const unsigned ln = lane_id();
  const int GS = A.GS;
  const int grp = (int)ln / GS, rl = (int)ln % GS;
  const long long wv = (long long)blockIdx.x * (kMThreads / 64) + (threadIdx.x >> 6);
  const long long u = wv * (64 / GS) + grp;
  const bool active = u < A.nunits;
  const long long k0 = u * kMUnit;
  const int n = active ? (int)std::min<long long>(kMUnit, A.nnz - k0) : 0;
  const gptr<const In> sv = to_global(static_cast<const In*>(A.sv));
  const gptr<const uint32_t> sidx = to_global(A.sidx);
  long long rank = active ? A.rank0[u] : 0;
  bool firstrun = true;
  Acc acc[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) acc[k] = FO::zero();
  for (int p0 = 0; p0 < kMUnit; p0 += B) {
    In a[B];
    uint32_t ix[MO][B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const bool ok = p0 + b < n;
      a[b] = ok ? sv[k0 + p0 + b] : (In)0;
#pragma unroll
      for (int f = 0; f < MO; ++f) ix[f][b] = (ok && f < A.nf) ? sidx[(size_t)f * A.nnz + k0 + p0 + b] : 0u;
    }
    const uint64_t word = p0 < n ? A.heads[(k0 + p0) >> 6] : 0ull;
    const int sh = (int)((k0 + p0) & 63);
    In x[MO][B][NC];
#pragma unroll
    for (int f = 0; f < MO; ++f) {
      const gptr<const In> U = to_global(f < A.nf ? static_cast<const In*>(A.fac[f]) : nullptr);
#pragma unroll
      for (int b = 0; b < B; ++b)
#pragma unroll
        for (int k = 0; k < NC; ++k) {
          const int r = rl + 64 * k;
          x[f][b][k] = (f < A.nf && p0 + b < n && r < A.R) ? U[(long long)ix[f][b] * A.R + r] : (In)1;
        }
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
      if (p0 + b >= n) break;
      if (p0 + b > 0 && ((word >> (sh + b)) & 1ull)) {  // a new row starts: the open one is complete
        double v[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) v[k] = FO::to_f64(acc[k]);
        if (firstrun) {
#pragma unroll
          for (int k = 0; k < NC; ++k) {
            const int r = rl + 64 * k;
            if (r < A.R) A.carry[(2 * u) * A.R + r] = v[k];
          }
        } else {
          write_row<NC>(A, rank, rl, v);
        }
        firstrun = false;
        ++rank;
#pragma unroll
        for (int k = 0; k < NC; ++k) acc[k] = FO::zero();
      }
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        uint64_t p = FO::start_prod(a[b]);
#pragma unroll
        for (int f = 0; f < MO; ++f)
          if (f < A.nf) p = FO::mul_prod(p, x[f][b][k]);
        acc[k] = FO::add(acc[k], FO::from_pay(p));
      }
    }
  }
  if (active) {  // the unit's last run
    const long long e = firstrun ? 2 * u : 2 * u + 1;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const int r = rl + 64 * k;
      if (r < A.R) A.carry[e * A.R + r] = FO::to_f64(acc[k]);
    }
  }
}

// Entry i of hierarchy level h (R columns): level 0 is the first-run carry
// of unit i (entry 2i), level h >= 1 the sum of 32 consecutive entries of
// level h - 1.
__device__ __forceinline__ const double* level_entry(const MArgs& A, int h, long long i) {
  return h == 0 ? A.carry + (2 * i) * A.R : A.hier + (A.hoff[h] + i) * A.R;
}

// Level h of the hierarchy, one lane group per entry: its 32 level h - 1
// entries added in order (FP64).  Skipped when no row spans more than kSerial
// units (the largest span is computed at setup).
template <int NC>
__global__ __launch_bounds__(kMThreads) void k_mttkrp_level(MArgs A, int h) {
  if (*A.longest <= kSerial) return;
  const unsigned ln = lane_id();
  const int GS = A.GS;
  const int grp = (int)ln / GS, rl = (int)ln % GS;
  const long long wv = (long long)blockIdx.x * (kMThreads / 64) + (threadIdx.x >> 6);
  const long long b = wv * (64 / GS) + grp;
  if (b >= A.hcnt[h]) return;
  const long long n = A.hcnt[h - 1];
  double s[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) s[k] = 0.0;
  for (long long i = 32 * b; i < 32 * b + 32 && i < n; ++i) {
    const gptr<const double> src = to_global(level_entry(A, h - 1, i));
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const int r = rl + 64 * k;
      if (r < A.R) s[k] += src[r];
    }
  }
  double* dst = A.hier + (A.hoff[h] + b) * A.R;
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const int r = rl + 64 * k;
    if (r < A.R) to_global(dst)[r] = s[k];
  }
}

// Adds entries [lo, hi) of level h to s, in order.
template <int NC>
__device__ __forceinline__ void add_range(const MArgs& A, int h, long long lo, long long hi, int rl, double (&s)[NC]) {
#pragma unroll 4
  for (long long i = lo; i < hi; ++i) {
    const gptr<const double> src = to_global(level_entry(A, h, i));
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const int r = rl + 64 * k;
      if (r < A.R) s[k] += src[r];
    }
  }
}

// Rows that touch a unit boundary: the entry that opens a row adds the
// first-run carries of the next cnt units, in a fixed order (FP64), one lane
// group per entry.  Up to kSerial of them one by one; longer spans as the
// level-0 entries up to a multiple of 32, then the same on the next level
// for the whole blocks, ..., and the partial blocks at the end, highest
// level first.
template <int NC>
__global__ __launch_bounds__(kMThreads) void k_mttkrp_combine(MArgs A) {
  const unsigned ln = lane_id();
  const int GS = A.GS;
  const int grp = (int)ln / GS, rl = (int)ln % GS;
  const long long wv = (long long)blockIdx.x * (kMThreads / 64) + (threadIdx.x >> 6);
  const long long e = wv * (64 / GS) + grp;
  if (e >= 2 * A.nunits) return;
  const long long row = to_global(A.groups)[e].row, cnt = to_global(A.groups)[e].cnt;
  if (row < 0) return;
  const gptr<const double> cv = to_global(static_cast<const double*>(A.carry));
  double s[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const int r = rl + 64 * k;
    s[k] = r < A.R ? cv[e * A.R + r] : 0.0;
  }
  long long lo = (e >> 1) + 1, hi = lo + cnt;  // level-0 entries of the following units
  if (cnt <= kSerial) {
    add_range<NC>(A, 0, lo, hi, rl, s);
  } else {
    double tail[kMaxHier][NC];
    int top = 0;  // the level whose remaining range is added whole
    bool open = true;
#pragma unroll
    for (int h = 0; h < kMaxHier; ++h) {
#pragma unroll
      for (int k = 0; k < NC; ++k) tail[h][k] = 0.0;
      if (open && h < A.hlevels) {
        const long long lo2 = (lo + 31) / 32, hi2 = hi / 32;
        if (lo2 >= hi2) {  // no whole block on the next level
          open = false;
        } else {
          add_range<NC>(A, h, lo, lo2 * 32, rl, s);
          add_range<NC>(A, h, hi2 * 32, hi, rl, tail[h]);
          lo = lo2;
          hi = hi2;
          top = h + 1;
        }
      } else {
        open = false;
      }
    }
    add_range<NC>(A, top, lo, hi, rl, s);
#pragma unroll
    for (int h = kMaxHier - 1; h >= 0; --h)
      if (h < top)
#pragma unroll
        for (int k = 0; k < NC; ++k) s[k] += tail[h][k];
  }
  write_row<NC>(A, row, rl, s);
}

// The longest span (units after the opening entry) of any row, for skipping
// the hierarchy when every row is short.
__global__ __launch_bounds__(256) void k_mttkrp_longest(const CarryGroup* groups, long long E, long long* longest) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += (long long)gridDim.x * blockDim.x) {
    const long long c = to_global(groups)[e].cnt;
    if (to_global(groups)[e].row >= 0 && c > kSerial) atomicMax(reinterpret_cast<unsigned long long*>(longest),
                                                                (unsigned long long)c);
  }
}

__global__ __launch_bounds__(256) void k_mttkrp_zero(void* M, long long n, int f64) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    if (f64)
      to_global(static_cast<double*>(M))[i] = 0.0;
    else
      to_global(static_cast<float*>(M))[i] = 0.f;
  }
}

int check_plan(const ttv_mttkrp_plan* p) { return p ? TTV_OK : TTV_E_NULL; }

template <int F, int NC>
void launch_apply_mo(const MArgs& A, int mo, dim3 g, hipStream_t s) {
  if (mo <= 2)
    hipLaunchKernelGGL((k_mttkrp_apply<F, NC, 2>), g, dim3(kMThreads), 0, s, A);
  else if (mo <= 4)
    hipLaunchKernelGGL((k_mttkrp_apply<F, NC, 4>), g, dim3(kMThreads), 0, s, A);
  else
    hipLaunchKernelGGL((k_mttkrp_apply<F, NC, kMaxOrder - 1>), g, dim3(kMThreads), 0, s, A);
}

template <int F>
void launch_apply(const MArgs& A, int nc, int mo, dim3 g, hipStream_t s) {
  if (nc == 1)
    launch_apply_mo<F, 1>(A, mo, g, s);
  else if (nc == 2)
    launch_apply_mo<F, 2>(A, mo, g, s);
  else
    launch_apply_mo<F, 4>(A, mo, g, s);
}

}  // namespace
}  // namespace ttv

using namespace ttv;

extern "C" {

int ttv_mttkrp_plan_create(const ttv_coo_desc* X, int32_t mode, int32_t R, int32_t flags, ttv_mttkrp_plan** plan) {
  if (flags & TTV_DROP_ZEROS) return TTV_E_ARG;  // the result is dense
  if (!plan) return TTV_E_NULL;
  *plan = nullptr;
  if (R < 1 || R > kMMaxR) return TTV_E_ARG;
  if (!X) return TTV_E_NULL;
  if (X->order < 2 || X->order > TTV_MAX_ORDER) return TTV_E_ORDER;
  if (mode < 0 || mode >= X->order) return TTV_E_MODE;
  int others[TTV_MAX_ORDER], nf = 0;
  for (int j = 0; j < X->order; ++j)
    if (j != mode) others[nf++] = j;
  for (int f = 0; f < nf; ++f)
    if (X->shape[others[f]] > (1LL << 32)) return TTV_E_SIZE;  // indices are kept as uint32
  ttv_mttkrp_plan* p = new (std::nothrow) ttv_mttkrp_plan();
  if (!p) return TTV_E_ARG;
  int rc = plan_single(X, nf, others, flags, kPipePerm, p->P);
  if (rc) {
    delete p;
    return rc;
  }
  p->X = *X;
  p->mode = mode;
  p->R = R;
  p->nf = nf;
  for (int f = 0; f < nf; ++f) p->others[f] = others[f];
  p->idx64 = X->index_dtype == TTV_I64 ? 1 : 0;
  p->form = X->value_dtype == TTV_F64 ? kF64 : kC32;
  p->out_f64 = (p->form == kF64 || (flags & TTV_OUT_F64)) ? 1 : 0;
  p->nnz = X->nnz;
  p->nunits = (X->nnz + kMUnit - 1) / kMUnit;
  p->dcap = std::max<long long>(1, std::min<long long>(X->nnz, X->shape[mode]));
  const size_t vsz = p->form == kF64 ? 8 : 4, isz = p->idx64 ? 8 : 4;
  size_t o = kMHdr;
  p->off_sv = o;
  o = align256(o + (size_t)p->nnz * vsz);
  p->off_sidx = o;
  o = align256(o + (size_t)p->nnz * 4 * nf);
  p->off_heads = o;
  o = align256(o + (size_t)((p->nnz + 63) / 64) * 8);
  p->off_rank0 = o;
  o = align256(o + (size_t)p->nunits * 8);
  p->off_dist = o;
  o = align256(o + (size_t)p->dcap * 8);
  p->off_groups = o;
  o = align256(o + (size_t)(2 * p->nunits) * sizeof(CarryGroup));
  p->off_carry = o;
  o = align256(o + (size_t)(2 * p->nunits) * R * sizeof(double));
  // hierarchy of first-run carries: level h + 1 sums 32 entries of level h
  p->hcnt[0] = p->nunits;
  long long hs = 0;
  while (p->hlevels + 1 < kMaxHier && p->hcnt[p->hlevels] > 32) {
    const int h = ++p->hlevels;
    p->hcnt[h] = (p->hcnt[h - 1] + 31) / 32;
    p->hoff[h] = hs;
    hs += p->hcnt[h];
  }
  p->off_hier = o;
  o = align256(o + (size_t)std::max<long long>(hs, 1) * R * sizeof(double));
  p->data_bytes = o;
  p->off_perm = align256(p->P.L.end);
  p->off_rowid = p->off_perm + align256((size_t)p->nnz * 4);
  p->off_osubs = p->off_rowid + align256((size_t)p->nnz * 4);
  p->setup_bytes = p->off_osubs + align256((size_t)p->dcap * isz);
  *plan = p;
  return TTV_OK;
}

int ttv_mttkrp_sizes(const ttv_mttkrp_plan* plan, size_t* data_bytes, size_t* setup_ws_bytes) {
  if (int rc = check_plan(plan)) return rc;
  if (!data_bytes || !setup_ws_bytes) return TTV_E_NULL;
  *data_bytes = plan->data_bytes;
  *setup_ws_bytes = plan->setup_bytes;
  return TTV_OK;
}

int ttv_mttkrp_setup(ttv_mttkrp_plan* plan, void* data, size_t data_bytes, void* ws, size_t ws_bytes,
                     ttv_stream_t stream) {
  if (int rc = check_plan(plan)) return rc;
  if (!data || data_bytes < plan->data_bytes || !ws || ws_bytes < plan->setup_bytes) return TTV_E_WORKSPACE;
  if (int f = fault_launch()) return f;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  (void)hipGetLastError();  // errors left by earlier, unrelated runtime calls are not ours
  char* d = static_cast<char*>(data);
  char* w = static_cast<char*>(ws);
  if (plan->nnz == 0) {
    // no sort: only the device error word that ttv_check_device_error reads
    if (int rc = launch_zero(w, 256, s)) return rc;
  } else {
    if (int rc = launch_zero(d, kMHdr, s)) return rc;  // the count and the longest span
    PipePlan P = plan->P;
    P.d0.out_subs = w + plan->off_osubs;
    P.d0.out_nnz = reinterpret_cast<long long*>(d);  // the header's count
    P.d0.seg_out = reinterpret_cast<int32_t*>(w + plan->off_rowid);
    P.d0.perm_out = reinterpret_cast<int32_t*>(w + plan->off_perm);
    P.cus = device_cus();
    int rc = launch_pipeline(P, ws, s);
    if (rc) return rc;
    GatherArgs G;
    const ttv_coo_desc& X = plan->X;
    G.subs = X.subs;
    G.vals = X.vals;
    G.se = X.stride_e;
    G.sj = X.stride_j;
    G.perm = P.d0.perm_out;
    G.rowid = P.d0.seg_out;
    G.osubs = P.d0.out_subs;
    G.out_nnz = P.d0.out_nnz;
    G.nnz = plan->nnz;
    G.dcap = plan->dcap;
    for (int f = 0; f < kMaxOrder; ++f) G.others[f] = f < plan->nf ? plan->others[f] : 0;
    G.nf = plan->nf;
    G.sv = d + plan->off_sv;
    G.sidx = reinterpret_cast<uint32_t*>(d + plan->off_sidx);
    G.heads = reinterpret_cast<unsigned long long*>(d + plan->off_heads);
    G.rank0 = reinterpret_cast<long long*>(d + plan->off_rank0);
    G.dist = reinterpret_cast<long long*>(d + plan->off_dist);
    const int g = (int)std::min<long long>(std::max<long long>(1, (plan->nnz + 255) / 256), 8LL * P.cus);
    if (plan->idx64) {
      if (plan->form == kF64)
        hipLaunchKernelGGL((k_mttkrp_gather<long long, double>), dim3(g), dim3(256), 0, s, G);
      else
        hipLaunchKernelGGL((k_mttkrp_gather<long long, float>), dim3(g), dim3(256), 0, s, G);
    } else {
      if (plan->form == kF64)
        hipLaunchKernelGGL((k_mttkrp_gather<int, double>), dim3(g), dim3(256), 0, s, G);
      else
        hipLaunchKernelGGL((k_mttkrp_gather<int, float>), dim3(g), dim3(256), 0, s, G);
    }
    const long long ge = std::min<long long>((2 * plan->nunits + 255) / 256, 4LL * P.cus);
    hipLaunchKernelGGL(k_carry_groups<kMUnit>, dim3((unsigned)ge), dim3(256), 0, s, G.rowid,
                       static_cast<const long long*>(G.rank0), plan->nnz, plan->nunits,
                       reinterpret_cast<CarryGroup*>(d + plan->off_groups));
    hipLaunchKernelGGL(k_mttkrp_longest, dim3((unsigned)ge), dim3(256), 0, s,
                       reinterpret_cast<const CarryGroup*>(d + plan->off_groups), 2 * plan->nunits,
                       reinterpret_cast<long long*>(d + 8));
    // whether any row spans more than kSerial units: the applies launch the
    // hierarchy kernels only then
    long long longest = 0;
    hipError_t e = hipMemcpyAsync(&longest, d + 8, sizeof(longest), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      set_last_hip_error((int)e);
      return TTV_E_HIP;
    }
    plan->long_rows = longest > kSerial ? 1 : 0;
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_last_hip_error((int)e);
    return TTV_E_HIP;
  }
  plan->data = data;
  return TTV_OK;
}

int ttv_mttkrp_apply(const ttv_mttkrp_plan* plan, const void* const* factors, void* M, ttv_stream_t stream) {
  if (int rc = check_plan(plan)) return rc;
  if (!plan->data) return TTV_E_ARG;  // setup has not run
  if (!factors || !M) return TTV_E_NULL;
  for (int f = 0; f < plan->nf; ++f)
    if (!factors[plan->others[f]] && plan->nnz > 0) return TTV_E_NULL;
  if (int f = fault_launch()) return f;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  const int cus = device_cus();
  if (plan->nnz == 0) {
    const long long n = plan->X.shape[plan->mode] * (long long)plan->R;
    const int g = (int)std::min<long long>(std::max<long long>(1, (n + 255) / 256), 4LL * cus);
    hipLaunchKernelGGL(k_mttkrp_zero, dim3(g), dim3(256), 0, s, M, n, plan->out_f64);
  } else {
    char* d = static_cast<char*>(plan->data);
    MArgs A;
    A.sv = d + plan->off_sv;
    A.sidx = reinterpret_cast<const uint32_t*>(d + plan->off_sidx);
    A.heads = reinterpret_cast<const unsigned long long*>(d + plan->off_heads);
    A.rank0 = reinterpret_cast<const long long*>(d + plan->off_rank0);
    A.dist = reinterpret_cast<const long long*>(d + plan->off_dist);
    A.hdr = reinterpret_cast<const long long*>(d);
    A.groups = reinterpret_cast<const CarryGroup*>(d + plan->off_groups);
    A.carry = reinterpret_cast<double*>(d + plan->off_carry);
    A.hier = reinterpret_cast<double*>(d + plan->off_hier);
    A.longest = reinterpret_cast<const long long*>(d + 8);
    A.hlevels = plan->hlevels;
    for (int h = 0; h <= kMaxHier; ++h) {
      A.hoff[h] = h < 8 ? plan->hoff[h] : 0;
      A.hcnt[h] = h < 8 ? plan->hcnt[h] : 0;
    }
    for (int f = 0; f < kMaxOrder; ++f) A.fac[f] = f < plan->nf ? factors[plan->others[f]] : nullptr;
    A.M = M;
    A.nnz = plan->nnz;
    A.nunits = plan->nunits;
    A.nrows = plan->X.shape[plan->mode];
    A.R = plan->R;
    int gs = 1;
    while (gs < plan->R && gs < 64) gs <<= 1;
    A.GS = gs;
    A.nf = plan->nf;
    A.out_f64 = plan->out_f64;
    const int nc = (plan->R + 63) / 64 <= 1 ? 1 : ((plan->R + 63) / 64 <= 2 ? 2 : 4);
    const long long per_wave = 64 / gs;
    const long long ga = (plan->nunits + per_wave * (kMThreads / 64) - 1) / (per_wave * (kMThreads / 64));
    const long long gc = (2 * plan->nunits + per_wave * (kMThreads / 64) - 1) / (per_wave * (kMThreads / 64));
    prof_begin(TTV_PROF_MTTKRP, s);
    if (plan->form == kF64)
      launch_apply<kF64>(A, nc, plan->nf, dim3((unsigned)ga), s);
    else
      launch_apply<kC32>(A, nc, plan->nf, dim3((unsigned)ga), s);
    prof_end(TTV_PROF_MTTKRP, s);
    for (int h = 1; plan->long_rows && h <= plan->hlevels; ++h) {
      const long long gh = (plan->hcnt[h] + per_wave * (kMThreads / 64) - 1) / (per_wave * (kMThreads / 64));
      if (nc == 1)
        hipLaunchKernelGGL(k_mttkrp_level<1>, dim3((unsigned)gh), dim3(kMThreads), 0, s, A, h);
      else if (nc == 2)
        hipLaunchKernelGGL(k_mttkrp_level<2>, dim3((unsigned)gh), dim3(kMThreads), 0, s, A, h);
      else
        hipLaunchKernelGGL(k_mttkrp_level<4>, dim3((unsigned)gh), dim3(kMThreads), 0, s, A, h);
    }
    if (nc == 1)
      hipLaunchKernelGGL(k_mttkrp_combine<1>, dim3((unsigned)gc), dim3(kMThreads), 0, s, A);
    else if (nc == 2)
      hipLaunchKernelGGL(k_mttkrp_combine<2>, dim3((unsigned)gc), dim3(kMThreads), 0, s, A);
    else
      hipLaunchKernelGGL(k_mttkrp_combine<4>, dim3((unsigned)gc), dim3(kMThreads), 0, s, A);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_last_hip_error((int)e);
    return TTV_E_HIP;
  }
  return TTV_OK;
}

void ttv_mttkrp_plan_destroy(ttv_mttkrp_plan* plan) { delete plan; }

}  // extern "C"
