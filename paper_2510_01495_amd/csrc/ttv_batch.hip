// Batched sparse TTV: many independent tensors, each with its own mode and
// vector, run by one fixed sequence of persistent kernels (the same
// keyed-reduction pipeline, whose work lists span every tensor).  A plan
// binds all pointers, so a call is a fixed set of kernel launches on one
// stream -- no host synchronisation, allocation or read-back -- and can be
// captured into a hipGraph and replayed.
//
// The autotuner times candidate level-1 tile sizes and first-digit widths on
// the bound batch and keeps the fastest; results are cached in a small JSON
// file keyed by architecture, library version and batch shape.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ttv.h"
#include "ttv_host.h"

namespace ttv {
namespace {

struct Tuning {
  int T1;
  int r1_bias;
};

const Tuning kCandidates[] = {{8192, 0},  {16384, 0}, {32768, 0}, {65536, 0},
                              {16384, -1}, {32768, -1}, {16384, 1}, {32768, 1}};
constexpr int kNumCandidates = sizeof(kCandidates) / sizeof(kCandidates[0]);

std::mutex g_cache_mu;

}  // namespace
}  // namespace ttv

struct ttv_batch_plan {
  ttv::PipePlan P;
  std::vector<int> base_r1;   // r1 of every tensor before the bias
  ttv::TDesc* descs_dev = nullptr;
  ttv::Tuning tuning{16384, 0};
  size_t ws_max = 0;          // workspace for every candidate
  std::string cache_path;
  std::string cache_key;
};

namespace ttv {
namespace {

void apply_tuning(ttv_batch_plan* p, const Tuning& t) {
  PipePlan& P = p->P;
  P.T1 = t.T1;
  P.T2 = 16384;
  int levels = 1;
  long long tiles1 = 0;
  for (int i = 0; i < P.count; ++i) {
    TDesc& D = P.descs[i];
    int r1 = std::min(std::max(p->base_r1[i] + t.r1_bias, 0), std::min(kRMax, D.keybits));
    if (p->base_r1[i] == 0) r1 = 0;  // tiny tensors stay a single bucket
    D.r1 = r1;
    const int rest = std::max(0, D.keybits - r1);
    levels = std::max(levels, std::min(kMaxLevels, 1 + (std::max(0, rest - kDenseBits) + kRMax - 1) / kRMax));
    tiles1 += (D.nnz + P.T1 - 1) / P.T1;
  }
  P.levels = levels;
  P.tiles1 = tiles1;
  P.L = make_layout(P.total, P.count, P.levels, P.T1, P.T2, tiles1, true);
  if (log_on())
    std::fprintf(stderr, "ttv: batch plan tensors=%d records=%lld levels=%d tile1=%d digit1_bias=%d workspace=%zu\n",
                 P.count, (long long)P.total, P.levels, P.T1, t.r1_bias, P.L.end);
  p->tuning = t;
  if (p->descs_dev)  // the device copy follows the tuning (never while a call may run)
    hipMemcpy(p->descs_dev, P.descs.data(), sizeof(TDesc) * (size_t)P.count, hipMemcpyHostToDevice);
}

std::string make_key(const ttv_batch_plan* p) {
  const PipePlan& P = p->P;
  int maxbits = 0;
  for (const TDesc& D : P.descs) maxbits = std::max(maxbits, D.keybits);
  int dev = 0;
  hipGetDevice(&dev);
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%s|lib%d|f%d|i%d|n%d|nnz2^%d|bits%d", arch.c_str(), ttv_version(), P.form, P.idx64,
                P.count, (int)std::lround(std::log2((double)std::max<long long>(P.total, 1))), maxbits);
  return buf;
}

std::string read_file(const std::string& path) {
  std::string s;
  FILE* f = std::fopen(path.c_str(), "rb");
  if (!f) return s;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) s.append(buf, n);
  std::fclose(f);
  return s;
}

// Cache format: {"<key>": {"T1": n, "r1_bias": m, "us": t}, ...}.  Anything
// that does not parse is ignored (and rewritten by the next autotune).
bool cache_lookup(const std::string& path, const std::string& key, Tuning& t) {
  if (path.empty()) return false;
  std::lock_guard<std::mutex> g(g_cache_mu);
  const std::string s = read_file(path);
  const std::string k = "\"" + key + "\"";
  const size_t at = s.find(k);
  if (at == std::string::npos) return false;
  int T1 = 0, bias = 0;
  const size_t a = s.find("\"T1\":", at);
  const size_t b = s.find("\"r1_bias\":", at);
  const size_t end = s.find('}', at);
  if (a == std::string::npos || b == std::string::npos || end == std::string::npos || a > end || b > end) return false;
  if (std::sscanf(s.c_str() + a + 5, "%d", &T1) != 1) return false;
  if (std::sscanf(s.c_str() + b + 10, "%d", &bias) != 1) return false;
  for (const Tuning& c : kCandidates)
    if (c.T1 == T1 && c.r1_bias == bias) {
      t = c;
      return true;
    }
  return false;
}

void cache_store(const std::string& path, const std::string& key, const Tuning& t, double us) {
  if (path.empty()) return;
  std::lock_guard<std::mutex> g(g_cache_mu);
  std::string s = read_file(path);
  // keep the other well-formed entries: drop this key's entry and any garbage
  std::vector<std::string> entries;
  size_t pos = 0;
  while (true) {
    const size_t q0 = s.find('"', pos);
    if (q0 == std::string::npos) break;
    const size_t q1 = s.find('"', q0 + 1);
    if (q1 == std::string::npos) break;
    const size_t o = s.find('{', q1);
    const size_t c = s.find('}', q1);
    if (o == std::string::npos || c == std::string::npos || o > c) break;
    const std::string k = s.substr(q0 + 1, q1 - q0 - 1);
    const std::string body = s.substr(o, c - o + 1);
    if (k != key && k.find('|') != std::string::npos && body.find("\"T1\":") != std::string::npos)
      entries.push_back("\"" + k + "\": " + body);
    pos = c + 1;
  }
  char buf[256];
  std::snprintf(buf, sizeof(buf), "\"%s\": {\"T1\": %d, \"r1_bias\": %d, \"us\": %.1f}", key.c_str(), t.T1,
                t.r1_bias, us);
  entries.push_back(buf);
  std::string out = "{\n";
  for (size_t i = 0; i < entries.size(); ++i) out += "  " + entries[i] + (i + 1 < entries.size() ? ",\n" : "\n");
  out += "}\n";
  const std::string tmp = path + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) return;
  std::fwrite(out.data(), 1, out.size(), f);
  std::fclose(f);
  std::rename(tmp.c_str(), path.c_str());
}

}  // namespace
}  // namespace ttv

using namespace ttv;

extern "C" {

int ttv_batch_plan_create(int32_t count, const ttv_coo_desc* Xs, const int32_t* modes, const void* const* vs,
                          void* const* out_subs, void* const* out_vals, int64_t* out_nnz, int32_t flags,
                          const char* tune_cache, ttv_batch_plan** plan) {
  if (flags & TTV_DROP_ZEROS) return TTV_E_ARG;  // not offered for batches
  if (!plan) return TTV_E_NULL;
  *plan = nullptr;
  if (count < 1) return TTV_E_ARG;
  if (!Xs || !modes || !vs || !out_subs || !out_vals || !out_nnz) return TTV_E_NULL;
  ttv_batch_plan* p = new (std::nothrow) ttv_batch_plan();
  if (!p) return TTV_E_ARG;
  PipePlan& P = p->P;
  P.count = count;
  P.pipe_mode = kPipeTTV;
  P.descs.resize(count);
  p->base_r1.resize(count);
  long long base = 0;
  for (int i = 0; i < count; ++i) {
    int form = 0, idx64 = 0;
    const int rc = plan_tensor(&Xs[i], 1, &modes[i], flags, P.descs[i], form, idx64);
    if (rc) {
      delete p;
      return rc;
    }
    if (i == 0) {
      P.form = form;
      P.idx64 = idx64;
    } else if (form != P.form || idx64 != P.idx64) {
      delete p;
      return TTV_E_DTYPE;
    }
    if (Xs[i].nnz > 0 && (!vs[i] || !out_subs[i] || !out_vals[i])) {
      delete p;
      return TTV_E_NULL;
    }
    TDesc& D = P.descs[i];
    D.vec[modes[i]] = vs[i];
    D.out_subs = out_subs[i];
    D.out_vals = out_vals[i];
    D.out_nnz = reinterpret_cast<long long*>(out_nnz + i);
    D.base = base;
    base += Xs[i].nnz;
    p->base_r1[i] = D.r1;
  }
  P.total = base;
  P.cus = device_cus();
  // workspace big enough for every tuning candidate
  for (const Tuning& t : kCandidates) {
    apply_tuning(p, t);
    p->ws_max = std::max(p->ws_max, P.L.end);
  }
  p->cache_path = tune_cache ? tune_cache : "";
  p->cache_key = make_key(p);
  Tuning t{16384, 0};
  cache_lookup(p->cache_path, p->cache_key, t);
  apply_tuning(p, t);
  hipError_t e = hipMalloc(&p->descs_dev, sizeof(TDesc) * (size_t)count);
  if (e == hipSuccess)
    e = hipMemcpy(p->descs_dev, P.descs.data(), sizeof(TDesc) * (size_t)count, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    set_last_hip_error((int)e);
    if (p->descs_dev) hipFree(p->descs_dev);
    delete p;
    return TTV_E_HIP;
  }
  P.descs_dev = p->descs_dev;
  *plan = p;
  return TTV_OK;
}

int ttv_batch_workspace(const ttv_batch_plan* plan, size_t* bytes) {
  if (!plan || !bytes) return TTV_E_NULL;
  *bytes = plan->ws_max;
  return TTV_OK;
}

int ttv_coo_batched(const ttv_batch_plan* plan, void* ws, size_t ws_bytes, ttv_stream_t stream) {
  if (!plan) return TTV_E_NULL;
  if (!ws || ws_bytes < plan->P.L.end) return TTV_E_WORKSPACE;
  if (int f = fault_launch()) return f;
  return launch_pipeline(plan->P, ws, reinterpret_cast<hipStream_t>(stream));
}

int ttv_batch_autotune(ttv_batch_plan* plan, void* ws, size_t ws_bytes, ttv_stream_t stream) {
  if (!plan) return TTV_E_NULL;
  if (!ws || ws_bytes < plan->ws_max) return TTV_E_WORKSPACE;
  if (int f = fault_launch()) return f;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return TTV_E_HIP;
  double best_us = 1e30;
  Tuning best = plan->tuning;
  for (const Tuning& t : kCandidates) {
    apply_tuning(plan, t);
    int rc = launch_pipeline(plan->P, ws, s);  // warm-up
    if (rc) {
      hipEventDestroy(e0);
      hipEventDestroy(e1);
      return rc;
    }
    constexpr int reps = 3;
    hipEventRecord(e0, s);
    for (int r = 0; r < reps; ++r) launch_pipeline(plan->P, ws, s);
    hipEventRecord(e1, s);
    hipEventSynchronize(e1);
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    const double us = 1000.0 * ms / reps;
    if (us < best_us) {
      best_us = us;
      best = t;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  apply_tuning(plan, best);
  cache_store(plan->cache_path, plan->cache_key, best, best_us);
  const hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    set_last_hip_error((int)e);
    return TTV_E_HIP;
  }
  return TTV_OK;
}

void ttv_batch_plan_destroy(ttv_batch_plan* plan) {
  if (!plan) return;
  if (plan->descs_dev) hipFree(plan->descs_dev);
  delete plan;
}

}  // extern "C"
