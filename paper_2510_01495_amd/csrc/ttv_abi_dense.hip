// C ABI of the all-but-one product (n_v = d - 1 vectors, Sec. 3.3) and of
// the adjoints of both products.
//
// When every dense accumulator of a pass fits in LDS the work runs in the
// dense-accumulation kernels (one streaming pass over the nonzeros).
// Otherwise an accumulator falls back to the keyed-reduction pipeline with a
// single remaining mode, whose sparse result is scattered into the dense
// output.
#include <hip/hip_runtime.h>

#include <cstdio>

#include <algorithm>
#include <cstddef>
#include <cstring>
#include <mutex>

#include "ttv.h"
#include "ttv_dense.h"
#include "ttv_host.h"

namespace ttv {

namespace {

constexpr size_t kHdr = 256;                  // error word lives here (same offset as Ctrl::error)
constexpr size_t kLdsBudget = 150 * 1024;     // dynamic LDS of one dense block
constexpr size_t kLdsPerCU = 160 * 1024;
constexpr size_t kMaxWavesPerCU = 32;         // gfx950: 8 waves per SIMD, 4 SIMDs
// nonzeros per tile of the dense kernel for this tensor's value and index types
int tile_of(const ttv_coo_desc* X) {
  return kDenseThreads * dense_ipt(X->value_dtype == TTV_F64 ? kF64 : kC32, X->index_dtype == TTV_I64);
}

size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t acc_lds(long long nk) { return align16((size_t)nk * 8); }

struct Pass {
  int nacc = 0;
  int mode[kDenseMaxAcc] = {0, 0, 0, 0};
  long long nk[kDenseMaxAcc] = {0, 0, 0, 0};
  bool grad_vals = false;
  size_t lds = 0;
  int grid = 1;
  long long acc_total = 0;
  size_t tile = 0;  // LDS of a block besides its accumulators
};

// Tile LDS of the dense kernel for this tensor: the row stage, plus the sort
// buffers of the compensated-FP32 form.
size_t tile_lds_of(const ttv_coo_desc* X) {
  return dense_tile_lds(X->value_dtype == TTV_F64 ? kF64 : kC32, X->index_dtype == TTV_I64 ? 1 : 0,
                        row_width_class(X->order, X->stride_e, X->stride_j));
}

void finish_pass(Pass& p, long long nnz, int tile_nnz) {
  size_t acc = 0;
  p.acc_total = 0;
  for (int q = 0; q < p.nacc; ++q) {
    acc += acc_lds(p.nk[q]);
    p.acc_total += p.nk[q];
  }
  p.lds = acc + p.tile;
  // blocks per CU: LDS-limited, and at most kMaxWavesPerCU / 16 waves of a block
  const int bpc = (int)std::max<size_t>(
      1, std::min<size_t>(kMaxWavesPerCU / (kDenseThreads / 64), kLdsPerCU / std::max<size_t>(p.lds, 1)));
  const long long ntiles = std::max<long long>(1, (nnz + tile_nnz - 1) / tile_nnz);
  p.grid = (int)std::max<long long>(1, std::min<long long>((long long)kAssumedCUs * bpc, ntiles));
}

size_t pass_ws(const Pass& p) { return (size_t)p.grid * (size_t)p.acc_total * 8; }

// Splits the requested accumulators (key modes) into dense passes; modes whose
// accumulator alone exceeds the LDS budget go to `fallback`.
void plan_passes(const ttv_coo_desc* X, const int* modes, int nm, bool grad_vals, Pass* passes, int& npass,
                 int* fallback, int& nfb) {
  npass = 0;
  nfb = 0;
  const size_t tile = tile_lds_of(X);
  Pass cur;
  cur.tile = tile;
  size_t used = tile;
  for (int i = 0; i < nm; ++i) {
    const long long nk = X->shape[modes[i]];
    const size_t need = acc_lds(nk);
    if (need + tile > kLdsBudget) {
      fallback[nfb++] = modes[i];
      continue;
    }
    if (cur.nacc == kDenseMaxAcc || used + need > kLdsBudget) {
      passes[npass++] = cur;
      cur = Pass();
      cur.tile = tile;
      used = tile;
    }
    cur.mode[cur.nacc] = modes[i];
    cur.nk[cur.nacc] = nk;
    ++cur.nacc;
    used += need;
  }
  if (cur.nacc > 0) passes[npass++] = cur;
  if (grad_vals) {
    if (npass == 0) {  // a pass for the per-nonzero gradient only
      passes[npass] = Pass();
      passes[npass++].tile = tile;
    }
    passes[0].grad_vals = true;
  }
  for (int p = 0; p < npass; ++p) finish_pass(passes[p], X->nnz, tile_of(X));
}

// Pipeline plan whose key is the single mode `m` (all other modes contracted).
int plan_keyed(const ttv_coo_desc* X, int m, int flags, PipePlan& P) {
  int modes[TTV_MAX_ORDER], nc = 0;
  for (int j = 0; j < X->order; ++j)
    if (j != m) modes[nc++] = j;
  const int rc = plan_tensor(X, nc, modes, flags, P.d0, P.form, P.idx64);
  if (rc) return rc;
  P.d0.out_f64 = 1;  // the temporary sparse result is FP64
  P.pipe_mode = kPipeTTV;
  return finish_plan(P);
}

size_t tmp_bytes(const ttv_coo_desc* X) {
  const size_t isz = X->index_dtype == TTV_I64 ? 8 : 4;
  return align256((size_t)X->nnz * isz) + align256((size_t)X->nnz * 8) + 256;
}

void dense_base(const ttv_coo_desc* X, int flags, DenseArgs& A) {
  std::memset(&A, 0, sizeof(A));
  A.subs = X->subs;
  A.vals = X->vals;
  A.se = X->stride_e;
  for (int j = 0; j < X->order; ++j) {
    A.sj[j] = (long long)j * X->stride_j;
    A.dims[j] = X->shape[j];
  }
  A.nnz = X->nnz;
  A.ntiles = (X->nnz + tile_of(X) - 1) / tile_of(X);
  A.order = X->order;
  A.validate = (flags & TTV_VALIDATE) ? 1 : 0;
}

int bitlen(long long x) {
  int b = 0;
  while (x > 0) {
    ++b;
    x >>= 1;
  }
  return b;
}

int run_pass(const Pass& p, DenseArgs A, char* ws, size_t part_off, void* const* outs, void* grad_vals, int idx64,
             int form, int out_f64, hipStream_t s) {
  A.nacc = p.nacc;
  size_t lo = 0;
  long long off = 0;
  for (int q = 0; q < p.nacc; ++q) {
    A.key_mode[q] = p.mode[q];
    A.key_bits[q] = bitlen(p.nk[q] - 1);
    A.acc_off[q] = off;
    off += p.nk[q];
    lo += acc_lds(p.nk[q]);
    A.out[q] = outs[q];
  }
  // accumulators are laid out back to back as Acc (8 bytes each)
  A.acc_total = off;
  A.acc_bytes = align16((size_t)off * 8);
  (void)lo;
  A.grad_vals = p.grad_vals ? grad_vals : nullptr;
  A.partials = reinterpret_cast<double*>(ws + part_off);
  A.err = reinterpret_cast<int32_t*>(ws + offsetof(Ctrl, error));
  A.out_f64 = out_f64;
  // factor vectors staged in LDS (mode order) while the block's LDS stays
  // within the budget; the grid follows the blocks per CU that fit (never
  // more than the pass was sized for)
  size_t lds = A.acc_bytes + p.tile;
  A.vst_at = lds;
  const size_t esz = form == kF64 ? 8 : 4;
  long long vo = 0;
  for (int m = 0; m < kMaxOrder; ++m) {
    A.vst_off[m] = -1;
    if (m >= A.order || !A.fac[m]) continue;
    const size_t bytes = align16((size_t)A.dims[m] * esz);
    if (lds + bytes > kLdsBudget) continue;
    A.vst_off[m] = vo;
    vo += (long long)(bytes / esz);
    lds += bytes;
  }
  int grid = p.grid;
  if (lds > A.acc_bytes + p.tile) {
    const int bpc = (int)std::max<size_t>(
        1, std::min<size_t>(kMaxWavesPerCU / (kDenseThreads / 64), kLdsPerCU / std::max<size_t>(lds, 1)));
    grid = std::min(grid, kAssumedCUs * bpc);
  }
  if (log_on())
    std::fprintf(stderr,
                 "ttv: dense pass accumulators=%d entries=%lld grad_vals=%d grid=%d lds=%zu staged=%lld nnz=%lld\n",
                 p.nacc, (long long)off, A.grad_vals ? 1 : 0, grid, lds, vo, (long long)A.nnz);
  return launch_dense(A, idx64, form, grid, lds, s);
}

int run_fallback(const ttv_coo_desc* X, int m, int flags, const void* const* fac, const void* segfac,
                 const int32_t* segidx, void* out, int out_f64, char* ws, size_t pipe_off, size_t tmp_off,
                 hipStream_t s) {
  PipePlan P;
  int rc = plan_keyed(X, m, flags, P);
  if (rc) return rc;
  for (int j = 0; j < X->order; ++j) P.d0.vec[j] = (j == m) ? nullptr : fac[j];
  P.d0.segfac = segfac;
  P.d0.segidx = segidx;
  const size_t isz = X->index_dtype == TTV_I64 ? 8 : 4;
  char* tmp = ws + tmp_off;
  P.d0.out_subs = tmp;
  P.d0.out_vals = tmp + align256((size_t)X->nnz * isz);
  P.d0.out_nnz = reinterpret_cast<long long*>(tmp + align256((size_t)X->nnz * isz) + align256((size_t)X->nnz * 8));
  P.cus = device_cus();
  rc = launch_pipeline(P, ws + pipe_off, s);
  if (rc) return rc;
  return launch_densify(P.d0.out_subs, P.idx64, P.d0.out_vals, P.d0.out_nnz, out, X->shape[m], out_f64, P.cus, s);
}

size_t fallback_pipe_ws(const ttv_coo_desc* X, int m, int flags) {
  PipePlan P;
  if (plan_keyed(X, m, flags, P)) return 0;
  return P.L.end;
}

int check_common(const ttv_coo_desc* X, int keep_or_mode, int& form, int& idx64) {
  if (!X) return TTV_E_NULL;
  int modes[TTV_MAX_ORDER], nc = 0;
  if (X->order < 2 || X->order > TTV_MAX_ORDER) return TTV_E_ORDER;
  if (keep_or_mode < 0 || keep_or_mode >= X->order) return TTV_E_MODE;
  for (int j = 0; j < X->order; ++j)
    if (j != keep_or_mode) modes[nc++] = j;
  TDesc D;
  return plan_tensor(X, nc, modes, 0, D, form, idx64);
}

// Largest partials region of the adjoint of the all-but-one product over
// every subset of requested vector gradients (null grad_vecs entries are
// skipped): a pass with fewer accumulators uses less LDS, so it can run more
// blocks per CU and write more partials than the pass of all modes.
size_t allbut_bwd_partials(const ttv_coo_desc* X, int keep) {
  int all[TTV_MAX_ORDER], na = 0;
  for (int j = 0; j < X->order; ++j)
    if (j != keep) all[na++] = j;
  size_t part = 0;
  for (unsigned sub = 0; sub < (1u << na); ++sub) {
    int modes[TTV_MAX_ORDER], nm = 0;
    for (int i = 0; i < na; ++i)
      if (sub & (1u << i)) modes[nm++] = all[i];
    Pass passes[TTV_MAX_ORDER];
    int npass, fb[TTV_MAX_ORDER], nfb;
    plan_passes(X, modes, nm, true, passes, npass, fb, nfb);
    for (int p = 0; p < npass; ++p) part = std::max(part, pass_ws(passes[p]));
  }
  return part;
}

// Workspace of the all-but-one product / its adjoint.
struct DenseWs {
  size_t total = kHdr;
  size_t pipe_off = 0, seg_off = 0, tmp_off = 0, part_off = 0;
};

DenseWs layout_dense(const ttv_coo_desc* X, int flags, const Pass* passes, int npass, const int* fb, int nfb,
                     size_t segmap_ws, bool need_seg, size_t min_part = 0) {
  DenseWs W;
  size_t pipe = segmap_ws;
  for (int i = 0; i < nfb; ++i) pipe = std::max(pipe, fallback_pipe_ws(X, fb[i], flags));
  size_t o = align256(std::max(kHdr, pipe));
  W.pipe_off = 0;
  if (need_seg) {
    W.seg_off = o;
    o = align256(o + (size_t)X->nnz * 4);
  }
  if (nfb > 0) {
    W.tmp_off = o;
    o = align256(o + tmp_bytes(X));
  }
  size_t part = min_part;
  for (int p = 0; p < npass; ++p) part = std::max(part, pass_ws(passes[p]));
  W.part_off = o;
  o = align256(o + part);
  W.total = o;
  return W;
}

// Scratch of ttv_coo_allbut_noalloc: one copy per GPU, held until the process
// ends.  Host code never passes `scratch` itself (on the host it names a
// stand-in, not device memory): it passes the address hipGetSymbolAddress
// returned for the current device.
constexpr size_t kNoAllocScratch = (size_t)48 << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratch];

std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {nullptr};

// Device address of `scratch` on the current device (looked up once per
// device, with that device current).
int scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    set_last_hip_error((int)e);
    return TTV_E_HIP;
  }
  if (dev < 0 || dev >= 64) return TTV_E_ARG;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_last_hip_error((int)e);
      return TTV_E_HIP;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return TTV_OK;
}

// The sparse form's adjoint from the output row of every nonzero (seg):
// grad_v of the contracted mode keyed by its index (dense passes, or the
// sorting pipeline for a mode too long for LDS) and grad_vals per nonzero.
int sparse_adjoint(const ttv_coo_desc* X, int mode, const void* const* vecs, const int32_t* seg,
                   const void* grad_out, void* const* grad_vecs, void* grad_vals, const Pass* passes, int npass,
                   const int* fb, int nfb, const DenseWs& W, char* w, int flags, int idx64, int form, int out_f64,
                   hipStream_t s) {
  int rc;
  for (int i = 0; i < nfb; ++i) {
    const void* nofac[TTV_MAX_ORDER] = {nullptr};
    rc = run_fallback(X, fb[i], flags, nofac, grad_out, seg, grad_vecs[fb[i]], out_f64, w, W.pipe_off, W.tmp_off,
                      s);
    if (rc) return rc;
  }
  DenseArgs A;
  dense_base(X, flags, A);
  A.fac[mode] = vecs[mode];
  A.gseg = grad_out;
  A.seg = seg;
  for (int p = 0; p < npass; ++p) {
    void* outs[kDenseMaxAcc] = {nullptr, nullptr, nullptr, nullptr};
    for (int q = 0; q < passes[p].nacc; ++q) outs[q] = grad_vecs[passes[p].mode[q]];
    rc = run_pass(passes[p], A, w, W.part_off, outs, grad_vals, idx64, form, out_f64, s);
    if (rc) return rc;
  }
  return TTV_OK;
}

}  // namespace

}  // namespace ttv

using namespace ttv;

extern "C" {

int ttv_coo_allbut_workspace(const ttv_coo_desc* X, int32_t keep, int32_t flags, size_t* bytes) {
  if (flags & TTV_DROP_ZEROS) return TTV_E_ARG;  // sparse products only
  if (!bytes) return TTV_E_NULL;
  int form, idx64;
  int rc = check_common(X, keep, form, idx64);
  if (rc) return rc;
  Pass passes[TTV_MAX_ORDER];
  int npass, fb[TTV_MAX_ORDER], nfb;
  plan_passes(X, &keep, 1, false, passes, npass, fb, nfb);
  *bytes = layout_dense(X, flags, passes, npass, fb, nfb, 0, false).total;
  return TTV_OK;
}

int ttv_coo_allbut(const ttv_coo_desc* X, int32_t keep, const void* const* vecs, const int64_t* vec_lens, void* y,
                   void* ws, size_t ws_bytes, int32_t flags, ttv_stream_t stream) {
  if (flags & TTV_DROP_ZEROS) return TTV_E_ARG;  // sparse products only
  int form, idx64;
  int rc = check_common(X, keep, form, idx64);
  if (rc) return rc;
  if (!vecs || !vec_lens || !y) return TTV_E_NULL;
  for (int j = 0; j < X->order; ++j) {
    if (j == keep) continue;
    if (vec_lens[j] != X->shape[j]) return TTV_E_SHAPE;
    if (!vecs[j] && X->nnz > 0) return TTV_E_NULL;
  }
  Pass passes[TTV_MAX_ORDER];
  int npass, fb[TTV_MAX_ORDER], nfb;
  plan_passes(X, &keep, 1, false, passes, npass, fb, nfb);
  const DenseWs W = layout_dense(X, flags, passes, npass, fb, nfb, 0, false);
  if (!ws || ws_bytes < W.total) return TTV_E_WORKSPACE;
  if (int f = fault_launch()) return f;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  (void)hipGetLastError();  // errors left by earlier, unrelated runtime calls are not ours
  const int out_f64 = (form == kF64 || (flags & TTV_OUT_F64)) ? 1 : 0;
  const void* fac[TTV_MAX_ORDER] = {nullptr};
  for (int j = 0; j < X->order; ++j) fac[j] = (j == keep) ? nullptr : vecs[j];
  if (nfb) {
    rc = run_fallback(X, keep, flags, fac, nullptr, nullptr, y, out_f64, w, W.pipe_off, W.tmp_off, s);
  } else {
    launch_zero(w, kHdr, s);
    DenseArgs A;
    dense_base(X, flags, A);
    for (int j = 0; j < X->order; ++j) A.fac[j] = fac[j];
    void* outs[kDenseMaxAcc] = {y, nullptr, nullptr, nullptr};
    rc = run_pass(passes[0], A, w, W.part_off, outs, nullptr, idx64, form, out_f64, s);
  }
  if (rc) return rc;
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_last_hip_error((int)e);
    return TTV_E_HIP;
  }
  return TTV_OK;
}

int ttv_coo_allbut_noalloc(const ttv_coo_desc* X, int32_t keep, const void* const* vecs, const int64_t* vec_lens,
                           void* y, int32_t flags, ttv_stream_t stream) {
  if (flags & (TTV_DROP_ZEROS | TTV_VALIDATE)) return TTV_E_ARG;  // no workspace to read a device error from
  int form, idx64;
  int rc = check_common(X, keep, form, idx64);
  if (rc) return rc;
  if (!vecs || !vec_lens || !y) return TTV_E_NULL;
  for (int j = 0; j < X->order; ++j) {
    if (j == keep) continue;
    if (vec_lens[j] != X->shape[j]) return TTV_E_SHAPE;
    if (!vecs[j] && X->nnz > 0) return TTV_E_NULL;
  }
  Pass passes[TTV_MAX_ORDER];
  int npass, fb[TTV_MAX_ORDER], nfb;
  plan_passes(X, &keep, 1, false, passes, npass, fb, nfb);
  if (nfb) return TTV_E_SIZE;  // the kept mode's accumulator does not fit in LDS: needs the sorting pipeline
  const DenseWs W = layout_dense(X, flags, passes, npass, fb, nfb, 0, false);
  if (W.total > kNoAllocScratch) return TTV_E_SIZE;
  if (int f = fault_launch()) return f;
  void* ws = nullptr;
  rc = scratch_address(&ws);
  if (rc) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  (void)hipGetLastError();  // errors left by earlier, unrelated runtime calls are not ours
  const int out_f64 = (form == kF64 || (flags & TTV_OUT_F64)) ? 1 : 0;
  launch_zero(w, kHdr, s);
  DenseArgs A;
  dense_base(X, flags, A);
  for (int j = 0; j < X->order; ++j) A.fac[j] = (j == keep) ? nullptr : vecs[j];
  void* outs[kDenseMaxAcc] = {y, nullptr, nullptr, nullptr};
  rc = run_pass(passes[0], A, w, W.part_off, outs, nullptr, idx64, form, out_f64, s);
  if (rc) return rc;
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_last_hip_error((int)e);
    return TTV_E_HIP;
  }
  return TTV_OK;
}

int ttv_coo_backward_workspace(const ttv_coo_desc* X, int32_t kind, int32_t mode_or_keep, int32_t flags,
                               size_t* bytes) {
  if (flags & TTV_DROP_ZEROS) return TTV_E_ARG;  // sparse products only
  if (!bytes) return TTV_E_NULL;
  int form, idx64;
  int rc = check_common(X, mode_or_keep, form, idx64);
  if (rc) return rc;
  Pass passes[TTV_MAX_ORDER];
  int npass, fb[TTV_MAX_ORDER], nfb;
  if (kind == TTV_BWD_ALLBUT) {
    int modes[TTV_MAX_ORDER], nm = 0;
    for (int j = 0; j < X->order; ++j)
      if (j != mode_or_keep) modes[nm++] = j;
    plan_passes(X, modes, nm, true, passes, npass, fb, nfb);
    *bytes = layout_dense(X, flags, passes, npass, fb, nfb, 0, false, allbut_bwd_partials(X, mode_or_keep)).total;
    return TTV_OK;
  }
  if (kind != TTV_BWD_SPARSE) return TTV_E_ARG;
  PipePlan P;
  rc = plan_single(X, 1, &mode_or_keep, flags, kPipeSegMap, P);
  if (rc) return rc;
  plan_passes(X, &mode_or_keep, 1, true, passes, npass, fb, nfb);
  *bytes = layout_dense(X, flags, passes, npass, fb, nfb, P.L.end, true).total;
  return TTV_OK;
}

int ttv_coo_backward(const ttv_coo_desc* X, int32_t kind, int32_t mode_or_keep, const void* const* vecs,
                     const int64_t* vec_lens, const void* grad_out, void* const* grad_vecs, void* grad_vals,
                     void* ws, size_t ws_bytes, int32_t flags, ttv_stream_t stream) {
  if (flags & TTV_DROP_ZEROS) return TTV_E_ARG;  // sparse products only
  int form, idx64;
  int rc = check_common(X, mode_or_keep, form, idx64);
  if (rc) return rc;
  if (!vecs || !vec_lens || !grad_vecs) return TTV_E_NULL;
  if (!grad_out && X->nnz > 0) return TTV_E_NULL;
  if (int f = fault_launch()) return f;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  (void)hipGetLastError();  // errors left by earlier, unrelated runtime calls are not ours
  const int out_f64 = form == kF64 ? 1 : 0;  // gradients have the value type of X
  Pass passes[TTV_MAX_ORDER];
  int npass, fb[TTV_MAX_ORDER], nfb;
  if (kind == TTV_BWD_ALLBUT) {
    const int keep = mode_or_keep;
    int modes[TTV_MAX_ORDER], nm = 0;
    for (int j = 0; j < X->order; ++j) {
      if (j == keep) continue;
      if (vec_lens[j] != X->shape[j]) return TTV_E_SHAPE;
      if (!vecs[j] && X->nnz > 0) return TTV_E_NULL;
      if (grad_vecs[j]) modes[nm++] = j;
    }
    Pass wpasses[TTV_MAX_ORDER];
    int wnp, wfb[TTV_MAX_ORDER], wnfb;
    int all[TTV_MAX_ORDER], na = 0;
    for (int j = 0; j < X->order; ++j)
      if (j != keep) all[na++] = j;
    plan_passes(X, all, na, true, wpasses, wnp, wfb, wnfb);  // what the workspace query sized
    const DenseWs W = layout_dense(X, flags, wpasses, wnp, wfb, wnfb, 0, false, allbut_bwd_partials(X, keep));
    if (!ws || ws_bytes < W.total) return TTV_E_WORKSPACE;
    plan_passes(X, modes, nm, grad_vals != nullptr, passes, npass, fb, nfb);
    for (int p = 0; p < npass; ++p)  // every pass's partials fit the region sized above
      if (W.part_off + pass_ws(passes[p]) > W.total) return TTV_E_WORKSPACE;
    const void* fac[TTV_MAX_ORDER] = {nullptr};
    for (int j = 0; j < X->order; ++j) fac[j] = (j == keep) ? grad_out : vecs[j];
    for (int i = 0; i < nfb; ++i) {
      rc = run_fallback(X, fb[i], flags, fac, nullptr, nullptr, grad_vecs[fb[i]], out_f64, w, W.pipe_off, W.tmp_off,
                        s);
      if (rc) return rc;
    }
    if (nfb == 0) launch_zero(w, kHdr, s);
    DenseArgs A;
    dense_base(X, flags, A);
    for (int j = 0; j < X->order; ++j) A.fac[j] = fac[j];
    for (int p = 0; p < npass; ++p) {
      void* outs[kDenseMaxAcc] = {nullptr, nullptr, nullptr, nullptr};
      for (int q = 0; q < passes[p].nacc; ++q) outs[q] = grad_vecs[passes[p].mode[q]];
      rc = run_pass(passes[p], A, w, W.part_off, outs, grad_vals, idx64, form, out_f64, s);
      if (rc) return rc;
    }
  } else if (kind == TTV_BWD_SPARSE) {
    const int mode = mode_or_keep;
    if (vec_lens[mode] != X->shape[mode]) return TTV_E_SHAPE;
    if (!vecs[mode] && X->nnz > 0) return TTV_E_NULL;
    PipePlan P;
    rc = plan_single(X, 1, &mode, flags, kPipeSegMap, P);
    if (rc) return rc;
    Pass wpasses[TTV_MAX_ORDER];
    int wnp, wfb[TTV_MAX_ORDER], wnfb;
    plan_passes(X, &mode, 1, true, wpasses, wnp, wfb, wnfb);
    const DenseWs W = layout_dense(X, flags, wpasses, wnp, wfb, wnfb, P.L.end, true);
    if (!ws || ws_bytes < W.total) return TTV_E_WORKSPACE;
    int modes[1] = {mode};
    const int nm = grad_vecs[mode] ? 1 : 0;
    plan_passes(X, modes, nm, grad_vals != nullptr, passes, npass, fb, nfb);
    for (int p = 0; p < npass; ++p)
      if (W.part_off + pass_ws(passes[p]) > W.total) return TTV_E_WORKSPACE;
    // 1. the output row of every nonzero (the forward's grouping)
    int32_t* seg = reinterpret_cast<int32_t*>(w + W.seg_off);
    P.d0.seg_out = seg;
    P.d0.out_nnz = nullptr;
    P.cus = device_cus();
    rc = launch_pipeline(P, w + W.pipe_off, s);
    if (rc) return rc;
    // 2. grad_v keyed by the contracted mode, grad_vals per nonzero
    rc = sparse_adjoint(X, mode, vecs, seg, grad_out, grad_vecs, grad_vals, passes, npass, fb, nfb, W, w, flags,
                        idx64, form, out_f64, s);
    if (rc) return rc;
  } else {
    return TTV_E_ARG;
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_last_hip_error((int)e);
    return TTV_E_HIP;
  }
  return TTV_OK;
}

int ttv_coo_backward_saved_workspace(const ttv_coo_desc* X, int32_t mode, int32_t flags, size_t* bytes) {
  if (flags & TTV_DROP_ZEROS) return TTV_E_ARG;
  if (!bytes) return TTV_E_NULL;
  int form, idx64;
  int rc = check_common(X, mode, form, idx64);
  if (rc) return rc;
  Pass passes[TTV_MAX_ORDER];
  int npass, fb[TTV_MAX_ORDER], nfb;
  plan_passes(X, &mode, 1, true, passes, npass, fb, nfb);
  *bytes = layout_dense(X, flags, passes, npass, fb, nfb, 0, false).total;
  return TTV_OK;
}

int ttv_coo_backward_saved(const ttv_coo_desc* X, int32_t mode, const void* const* vecs, const int64_t* vec_lens,
                           const int32_t* seg, const void* grad_out, void* const* grad_vecs, void* grad_vals,
                           void* ws, size_t ws_bytes, int32_t flags, ttv_stream_t stream) {
  if (flags & TTV_DROP_ZEROS) return TTV_E_ARG;
  int form, idx64;
  int rc = check_common(X, mode, form, idx64);
  if (rc) return rc;
  if (!vecs || !vec_lens || !grad_vecs) return TTV_E_NULL;
  if (vec_lens[mode] != X->shape[mode]) return TTV_E_SHAPE;
  if (X->nnz > 0 && (!grad_out || !seg || !vecs[mode])) return TTV_E_NULL;
  Pass wpasses[TTV_MAX_ORDER];
  int wnp, wfb[TTV_MAX_ORDER], wnfb;
  plan_passes(X, &mode, 1, true, wpasses, wnp, wfb, wnfb);  // what the workspace query sized
  const DenseWs W = layout_dense(X, flags, wpasses, wnp, wfb, wnfb, 0, false);
  if (!ws || ws_bytes < W.total) return TTV_E_WORKSPACE;
  Pass passes[TTV_MAX_ORDER];
  int npass, fb[TTV_MAX_ORDER], nfb;
  int modes[1] = {mode};
  plan_passes(X, modes, grad_vecs[mode] ? 1 : 0, grad_vals != nullptr, passes, npass, fb, nfb);
  for (int p = 0; p < npass; ++p)
    if (W.part_off + pass_ws(passes[p]) > W.total) return TTV_E_WORKSPACE;
  if (int f = fault_launch()) return f;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  (void)hipGetLastError();  // errors left by earlier, unrelated runtime calls are not ours
  const int out_f64 = form == kF64 ? 1 : 0;
  if (nfb == 0) launch_zero(ws, kHdr, s);  // the error word (a fallback's pipeline clears its own)
  rc = sparse_adjoint(X, mode, vecs, seg, grad_out, grad_vecs, grad_vals, passes, npass, fb, nfb, W,
                      static_cast<char*>(ws), flags, idx64, form, out_f64, s);
  if (rc) return rc;
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_last_hip_error((int)e);
    return TTV_E_HIP;
  }
  return TTV_OK;
}

}  // extern "C"
