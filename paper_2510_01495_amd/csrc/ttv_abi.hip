// C ABI: argument validation, key-layout planning, workspace layout and
// dispatch of the sparse TTV pipeline (Eq. 3, Sec. 3.3).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#include <algorithm>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <vector>

#include "ttv.h"
#include "ttv_host.h"

namespace ttv {

static thread_local int g_last_hip_error = 0;
void set_last_hip_error(int e) { g_last_hip_error = e; }

struct ProfHook {
  int kernel = 0;
  int count = 0;
  std::vector<void*> starts, stops;
};
static ProfHook g_prof;

void prof_begin(int kernel, hipStream_t s) {
  if (g_prof.kernel != kernel || g_prof.count >= (int)g_prof.starts.size()) return;
  hipEventRecord(static_cast<hipEvent_t>(g_prof.starts[g_prof.count]), s);
}
void prof_end(int kernel, hipStream_t s) {
  if (g_prof.kernel != kernel || g_prof.count >= (int)g_prof.stops.size()) return;
  hipEventRecord(static_cast<hipEvent_t>(g_prof.stops[g_prof.count]), s);
  ++g_prof.count;
}

bool log_on() {
  const char* e = std::getenv("TTV_LOG");
  return e && e[0] && std::strcmp(e, "0") != 0;
}

bool fault_on(const char* what) {
  const char* e = std::getenv("TTV_FAULT");
  if (!e) return false;
  const size_t n = std::strlen(what);
  for (const char* p = e; *p;) {
    const char* q = std::strchr(p, ',');
    const size_t len = q ? (size_t)(q - p) : std::strlen(p);
    if (len == n && std::strncmp(p, what, n) == 0) return true;
    if (!q) break;
    p = q + 1;
  }
  return false;
}

int fault_launch() {
  if (!fault_on("launch")) return TTV_OK;
  set_last_hip_error((int)hipErrorLaunchFailure);
  return TTV_E_HIP;
}

int device_cus() {
  static std::mutex mu;
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  std::lock_guard<std::mutex> g(mu);
  if (cache[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
    cache[dev] = v;
  }
  return cache[dev];
}

static int bitlen(unsigned long long x) {
  int b = 0;
  while (x) {
    ++b;
    x >>= 1;
  }
  return b;
}

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Division of 64-bit keys by an invariant divisor d >= 1 (Granlund and
// Montgomery, "Division by invariant integers using multiplication", 1994):
// with l = ceil(log2 d) and m = floor(2^64 (2^l - d) / d) + 1,
// n / d = (t + ((n - t) >> min(l, 1))) >> max(l - 1, 0), t = mulhi(m, n).
void set_divmagic(unsigned long long d, unsigned long long& m, int& sh1, int& sh2) {
  int l = 0;
  while (l < 64 && ((unsigned __int128)1 << l) < (unsigned __int128)d) ++l;
  const unsigned __int128 two_l = (unsigned __int128)1 << l;
  m = (unsigned long long)(((two_l - d) << 64) / d + 1);
  sh1 = l < 1 ? l : 1;
  sh2 = l > 1 ? l - 1 : 0;
}

// First-level digit: the smallest width (<= kRMax) whose used digits leave
// about 0.6 * kSmall nonzeros per bucket on uniform keys.
int choose_r1(long long nnz, unsigned __int128 range, int bits) {
  const double target = 0.6 * kSmall;
  int r1 = 0;
  while (r1 < kRMax && r1 < bits) {
    const int shift = bits - r1;
    const double used = (double)((range + (((unsigned __int128)1 << shift) - 1)) >> shift);
    if ((double)nnz / used <= target) break;
    ++r1;
  }
  return r1;
}

// Validates a descriptor and fills the tensor part of a TDesc: remaining
// modes (all modes minus the contracted ones, ascending -- the set
// difference of Sec. 3.3), their key fields (first remaining mode most
// significant, so numeric key order is lexicographic tuple order) and the
// first-level digit.
int plan_tensor(const ttv_coo_desc* X, int ncon, const int32_t* modes, int flags, TDesc& D, int& form,
                int& idx64) {
  if (!X || !modes) return TTV_E_NULL;
  const int d = X->order;
  if (d < 2 || d > TTV_MAX_ORDER) return TTV_E_ORDER;
  if (X->index_dtype != TTV_I32 && X->index_dtype != TTV_I64) return TTV_E_DTYPE;
  if (X->value_dtype != TTV_F32 && X->value_dtype != TTV_F64) return TTV_E_DTYPE;
  if (X->nnz < 0) return TTV_E_ARG;
  if (X->nnz > 0x7fffffffLL) return TTV_E_SIZE;
  for (int j = 0; j < d; ++j)
    if (X->shape[j] < 1) return TTV_E_SHAPE;
  if (X->index_dtype == TTV_I32)
    for (int j = 0; j < d; ++j)
      if (X->shape[j] > 0x7fffffffLL) return TTV_E_SIZE;
  if (X->nnz > 0 && (!X->subs || !X->vals)) return TTV_E_NULL;
  if (ncon < 1 || ncon > d - 1) return TTV_E_MODE;
  bool con[TTV_MAX_ORDER] = {false};
  for (int c = 0; c < ncon; ++c) {
    if (modes[c] < 0 || modes[c] >= d || con[modes[c]]) return TTV_E_MODE;
    con[modes[c]] = true;
  }
  std::memset(&D, 0, sizeof(D));
  D.subs = X->subs;
  D.vals = X->vals;
  D.nnz = X->nnz;
  D.stride_e = X->stride_e;
  D.stride_j = X->stride_j;
  D.order = d;
  for (int j = 0; j < d; ++j) D.dims[j] = X->shape[j];
  int nr = 0, nc = 0;
  for (int j = 0; j < d; ++j) {
    if (con[j])
      D.con[nc++] = j;
    else
      D.rem[nr++] = j;
  }
  D.nrem = nr;
  D.ncon = nc;
  // mixed-radix key over the remaining modes (first remaining mode most
  // significant): numeric order = lexicographic order of the index tuples
  unsigned __int128 range = 1;
  for (int i = nr - 1; i >= 0; --i) {
    D.kstride[i] = (unsigned long long)range;
    range *= (unsigned __int128)X->shape[D.rem[i]];
    if (range > ((unsigned __int128)1 << 64)) return TTV_E_KEYBITS;
  }
  for (int i = 0; i < nr; ++i) set_divmagic(D.kstride[i], D.kmagic[i], D.ksh1[i], D.ksh2[i]);
  for (int j = 0; j < TTV_MAX_ORDER; ++j) {
    D.mstride[j] = 0;
    D.mrem[j] = 0;
  }
  for (int i = 0; i < nr; ++i) {
    D.mstride[D.rem[i]] = D.kstride[i];
    D.mrem[D.rem[i]] = 1;
  }
  const int bits = bitlen((unsigned long long)(range - 1));
  D.keybits = bits;
  D.r1 = choose_r1(X->nnz, range, bits);
  D.validate = (flags & TTV_VALIDATE) ? 1 : 0;
  D.out_f64 = (flags & TTV_OUT_F64) ? 1 : 0;
  form = X->value_dtype == TTV_F64 ? kF64 : kC32;
  idx64 = X->index_dtype == TTV_I64 ? 1 : 0;
  return TTV_OK;
}

// Bucket levels of a tensor: the first digit, then 12-bit digits for the
// rest of the key; one more when the first level's buckets are expected to
// be nearly full on average and the second level would be the last one
// (it would then have to take all the remaining bits): most buckets split at
// the second level, which takes only the few bits they need, and the level
// after it the rest.
static int levels_of(const TDesc& D, int dense_bits) {
  const int rest = std::max(0, D.keybits - D.r1);
  // buckets left with at most dense_bits key bits need no further level
  int levels = 1 + (std::max(0, rest - dense_bits) + kRMax - 1) / kRMax;
  if (dense_bits == 0 && rest > 0 && D.nnz > 0) {
    unsigned __int128 range = 1;
    for (int i = 0; i < D.nrem; ++i) range *= (unsigned __int128)D.dims[D.rem[i]];
    const double used = (double)((range + (((unsigned __int128)1 << rest) - 1)) >> rest);
    const bool full = (double)D.nnz / used > 0.9 * kCap;
    if (full && levels == 2 && rest > 2) ++levels;
  }
  return std::min(kMaxLevels, levels);
}

Layout make_layout(long long total, int count, int levels, int T1, int T2, long long tiles1, bool dense,
                   bool aux) {
  Layout L{};
  L.count = count;
  L.levels = levels;
  L.jcap = std::max<long long>(count, total / kCap + 2);
  L.tcap = std::max<long long>(tiles1, total / T2 + L.jcap + 1);
  L.lcap = (long long)levels * (3 * ((total + kSmall - 1) / kSmall) + L.jcap) + count + 64;
  // a dense leaf of s > kCap records holds ceil(s / kDenseTile) <= s / kDenseTile + 1 partial tiles, each
  // a slot of at most dense_slot_words(kDenseBits) words
  const long long dtiles = dense ? total / kDenseTile + total / kCap + count + 1 : 0;
  L.pcap = total / kPureTile + total / kCap + dtiles + count + 2;
  L.dpcap = dtiles * dense_slot_words(kDenseBits);
  L.words = (total + 31) / 32 + 1;
  L.wblocks = (L.words + kBitmapWordsPerBlock - 1) / kBitmapWordsPerBlock;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  L.ctrl = take(sizeof(Ctrl));
  L.desc = take((size_t)std::max(count, 1) * sizeof(TDesc));
  L.jobs = take((size_t)levels * L.jcap * sizeof(Job));
  L.tiles = take((size_t)levels * L.tcap * sizeof(int));
  L.table = take((size_t)L.tcap * kNDig * sizeof(unsigned));
  L.starts = take((size_t)L.jcap * kNDig * sizeof(unsigned));
  L.leaves = take((size_t)L.lcap * sizeof(Leaf));
  L.ordered = take((size_t)L.lcap * sizeof(Leaf));
  L.status = take((size_t)L.lcap * sizeof(unsigned long long));
  L.bitmap = take((size_t)L.words * sizeof(unsigned));
  L.wordpre = take((size_t)L.words * sizeof(unsigned));
  L.blockpre = take((size_t)L.wblocks * sizeof(unsigned));
  L.partials = take((size_t)L.pcap * sizeof(double));
  L.ptile_leaf = take((size_t)L.pcap * sizeof(int));
  L.dpool = take((size_t)L.dpcap * sizeof(unsigned long long));
  L.recA = take((size_t)total * sizeof(Rec));
  L.recB = take(levels > 1 ? (size_t)total * sizeof(Rec) : 0);
  L.auxA = take(aux ? (size_t)total * sizeof(int32_t) : 0);
  L.auxB = take(aux && levels > 1 ? (size_t)total * sizeof(int32_t) : 0);
  L.end = o;
  return L;
}

static int choose_T1(long long total) {
  long long t = (total + 2 * 256 - 1) / (2 * 256);
  t = (t + 1023) / 1024 * 1024;
  return (int)std::min<long long>(65536, std::max<long long>(4096, t));
}

int finish_plan(PipePlan& P) {
  P.count = 1;
  P.total = P.d0.nnz;
  P.d0.base = 0;
  P.levels = levels_of(P.d0, dense_bits_of(P.pipe_mode));
  P.T1 = choose_T1(P.total);
  P.T2 = 16384;
  P.tiles1 = (P.total + P.T1 - 1) / P.T1;
  P.L = make_layout(P.total, 1, P.levels, P.T1, P.T2, P.tiles1, dense_bits_of(P.pipe_mode) > 0,
                    P.pipe_mode == kPipeTTVSeg);
  if (log_on())
    std::fprintf(stderr,
                 "ttv: plan mode=%d form=%s index=%s nnz=%lld order=%d kept=%d key_bits=%d digit1=%d levels=%d "
                 "tile1=%d tile=%d workspace=%zu\n",
                 P.pipe_mode, P.form == kF64 ? "f64" : "c32", P.idx64 ? "i64" : "i32", (long long)P.total,
                 (int)P.d0.order, (int)P.d0.nrem, (int)P.d0.keybits, (int)P.d0.r1, P.levels, P.T1, P.T2, P.L.end);
  return TTV_OK;
}

// Plans a single-tensor pipeline run (ncon contracted modes).
int plan_single(const ttv_coo_desc* X, int ncon, const int32_t* modes, int flags, int pipe_mode,
                PipePlan& P) {
  int rc = plan_tensor(X, ncon, modes, flags, P.d0, P.form, P.idx64);
  if (rc) return rc;
  P.pipe_mode = pipe_mode;
  return finish_plan(P);
}

}  // namespace ttv

using namespace ttv;

extern "C" {

const char* ttv_strerror(int s) {
  switch (s) {
    case TTV_OK: return "success";
    case TTV_E_NULL: return "a required pointer is null";
    case TTV_E_ORDER: return "tensor order must be in [2, TTV_MAX_ORDER]";
    case TTV_E_MODE: return "mode out of range or repeated";
    case TTV_E_SHAPE: return "invalid dimension or vector length";
    case TTV_E_DTYPE: return "unsupported or mixed index/value type";
    case TTV_E_KEYBITS: return "the product of the remaining dimensions exceeds 2^64";
    case TTV_E_WORKSPACE: return "workspace missing or too small";
    case TTV_E_INDEX: return "an index is out of range";
    case TTV_E_HIP: return "a HIP runtime call failed";
    case TTV_E_SIZE: return "size beyond what this build supports";
    case TTV_E_DEVICE: return "a device-side bounded wait or capacity check failed";
    case TTV_E_ARG: return "invalid argument";
    default: return "unknown status";
  }
}

int ttv_version(void) { return 100; }

int ttv_last_hip_error(void) { return g_last_hip_error; }

int ttv_plan_query(const ttv_coo_desc* X, int32_t ncon, const int32_t* modes, int32_t flags,
                   ttv_plan_info* out) {
  if (!out) return TTV_E_NULL;
  PipePlan P;
  const int rc = plan_single(X, ncon, modes, flags, kPipeTTV, P);
  if (rc) return rc;
  std::memset(out, 0, sizeof(*out));
  out->order = P.d0.order;
  out->nrem = P.d0.nrem;
  out->key_bits = P.d0.keybits;
  out->levels = P.levels;
  for (int i = 0; i < P.d0.nrem; ++i) {
    out->rem_modes[i] = P.d0.rem[i];
    out->bits[i] = bitlen((unsigned long long)(X->shape[P.d0.rem[i]] - 1));
    out->stride[i] = (int64_t)P.d0.kstride[i];
  }
  out->digit1_bits = P.d0.r1;
  out->workspace_bytes = (int64_t)P.L.end;
  return TTV_OK;
}

// Whether the product writes FP64 values (FP64 inputs, or TTV_OUT_F64).
static int out_is_f64(const PipePlan& P, int flags) {
  return (P.form == kF64 || (flags & TTV_OUT_F64)) ? 1 : 0;
}

int ttv_coo_multi_workspace(const ttv_coo_desc* X, int32_t ncon, const int32_t* modes, int32_t flags,
                            size_t* bytes) {
  if (!bytes) return TTV_E_NULL;
  PipePlan P;
  const int rc = plan_single(X, ncon, modes, flags, kPipeTTV, P);
  if (rc) return rc;
  *bytes = P.L.end;
  if (keyed_fits(P, flags)) *bytes = std::max(*bytes, keyed_ws(P));
  if (flags & TTV_DROP_ZEROS)
    *bytes = ((P.L.end + 255) & ~(size_t)255) + drop_zeros_ws(X->nnz, P.d0.nrem, P.idx64, out_is_f64(P, flags));
  return TTV_OK;
}

int ttv_coo_workspace(const ttv_coo_desc* X, int32_t mode, int32_t flags, size_t* bytes) {
  return ttv_coo_multi_workspace(X, 1, &mode, flags, bytes);
}

int ttv_coo_multi(const ttv_coo_desc* X, int32_t ncon, const int32_t* modes, const void* const* vecs,
                  const int64_t* vec_lens, void* out_subs, void* out_vals, int64_t* out_nnz, void* ws,
                  size_t ws_bytes, int32_t flags, ttv_stream_t stream) {
  PipePlan P;
  int rc = plan_single(X, ncon, modes, flags, kPipeTTV, P);
  if (rc) return rc;
  if (!vecs || !vec_lens || !out_nnz) return TTV_E_NULL;
  for (int c = 0; c < ncon; ++c) {
    if (vec_lens[c] != X->shape[modes[c]]) return TTV_E_SHAPE;
    if (!vecs[c] && X->nnz > 0) return TTV_E_NULL;
    P.d0.vec[modes[c]] = vecs[c];
  }
  if (X->nnz > 0 && (!out_subs || !out_vals)) return TTV_E_NULL;
  const bool drop = (flags & TTV_DROP_ZEROS) != 0;
  const size_t tmp_off = (P.L.end + 255) & ~(size_t)255;
  const int of64 = out_is_f64(P, flags);
  size_t need = drop ? tmp_off + drop_zeros_ws(X->nnz, P.d0.nrem, P.idx64, of64) : P.L.end;
  if (keyed_fits(P, flags)) need = std::max(need, keyed_ws(P));
  if (!ws || ws_bytes < need) return TTV_E_WORKSPACE;
  if (int f = fault_launch()) return f;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  P.cus = device_cus();
  if (!drop) {
    P.d0.out_subs = out_subs;
    P.d0.out_vals = out_vals;
    P.d0.out_nnz = reinterpret_cast<long long*>(out_nnz);
    if (tiny_fits(P, flags)) return launch_tiny(P, ws, s);
    if (keyed_fits(P, flags)) return launch_keyed(P, ws, s);
    return launch_pipeline(P, ws, s);
  }
  // the product into the temporary area, then its rows with nonzero sums
  long long *cnt, *counts;
  void *tsubs, *tvals;
  drop_zeros_layout(static_cast<char*>(ws) + tmp_off, X->nnz, P.d0.nrem, P.idx64, cnt, counts, tsubs, tvals);
  P.d0.out_subs = tsubs;
  P.d0.out_vals = tvals;
  P.d0.out_nnz = cnt;
  if (int rc2 = launch_pipeline(P, ws, s)) return rc2;
  launch_drop_zeros(tsubs, tvals, cnt, counts, out_subs, out_vals, reinterpret_cast<long long*>(out_nnz),
                    P.d0.nrem, P.idx64, of64, s);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_last_hip_error((int)e);
    return TTV_E_HIP;
  }
  return TTV_OK;
}

int ttv_coo(const ttv_coo_desc* X, int32_t mode, const void* v, int64_t v_len, void* out_subs,
            void* out_vals, int64_t* out_nnz, void* ws, size_t ws_bytes, int32_t flags,
            ttv_stream_t stream) {
  const void* vecs[1] = {v};
  const int64_t lens[1] = {v_len};
  return ttv_coo_multi(X, 1, &mode, vecs, lens, out_subs, out_vals, out_nnz, ws, ws_bytes, flags, stream);
}

int ttv_coo_save_workspace(const ttv_coo_desc* X, int32_t mode, int32_t flags, size_t* bytes) {
  if (!bytes) return TTV_E_NULL;
  if (flags & TTV_DROP_ZEROS) return TTV_E_ARG;  // the saved rows are the rows before any removal
  PipePlan P;
  const int rc = plan_single(X, 1, &mode, flags, kPipeTTVSeg, P);
  if (rc) return rc;  // (nnz above 2^31 - 1 is refused there: rows and indices fit int32)
  *bytes = P.L.end;
  return TTV_OK;
}

int ttv_coo_save(const ttv_coo_desc* X, int32_t mode, const void* v, int64_t v_len, void* out_subs, void* out_vals,
                 int64_t* out_nnz, int32_t* seg, void* ws, size_t ws_bytes, int32_t flags, ttv_stream_t stream) {
  if (flags & TTV_DROP_ZEROS) return TTV_E_ARG;
  PipePlan P;
  int rc = plan_single(X, 1, &mode, flags, kPipeTTVSeg, P);
  if (rc) return rc;
  if (!out_nnz) return TTV_E_NULL;
  if (v_len != X->shape[mode]) return TTV_E_SHAPE;
  if (X->nnz > 0 && (!v || !out_subs || !out_vals || !seg)) return TTV_E_NULL;
  if (!ws || ws_bytes < P.L.end) return TTV_E_WORKSPACE;
  if (int f = fault_launch()) return f;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  P.d0.vec[mode] = v;
  P.d0.out_subs = out_subs;
  P.d0.out_vals = out_vals;
  P.d0.out_nnz = reinterpret_cast<long long*>(out_nnz);
  P.d0.seg_out = seg;
  P.cus = device_cus();
  if (X->nnz == 0) {  // no leaf would write the count: a zero count and a clear error word
    (void)hipGetLastError();
    launch_zero(out_nnz, sizeof(int64_t), s);
    launch_zero(ws, sizeof(Ctrl), s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      set_last_hip_error((int)e);
      return TTV_E_HIP;
    }
    return TTV_OK;
  }
  return launch_pipeline(P, ws, s);
}

int ttv_profile_events(int32_t kernel, void* const* starts, void* const* stops, int32_t capacity) {
  if (kernel != TTV_PROF_NONE && (!starts || !stops || capacity < 0)) return TTV_E_NULL;
  g_prof.kernel = kernel;
  g_prof.starts.assign(starts, starts + (kernel ? capacity : 0));
  g_prof.stops.assign(stops, stops + (kernel ? capacity : 0));
  g_prof.count = 0;
  return TTV_OK;
}

int ttv_profile_count(void) { return g_prof.count; }

int ttv_check_device_error(const void* ws, ttv_stream_t stream) {
  if (!ws) return TTV_E_NULL;
  hipError_t e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    set_last_hip_error((int)e);
    return TTV_E_HIP;
  }
  int32_t err = 0;
  e = hipMemcpy(&err, static_cast<const char*>(ws) + offsetof(Ctrl, error), sizeof(err), hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    set_last_hip_error((int)e);
    return TTV_E_HIP;
  }
  return err;
}

}  // extern "C"
