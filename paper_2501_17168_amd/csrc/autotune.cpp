// Autotuner for the evaluation schedule.
//
// The paper switches between its hybrid and data-parallel fitness modes by
// comparing the number of data points with the GPU's core count (§III-C,
// "Choose Parallelism Adaptively"; the crossover is measured in §V-B). Here
// the choice is measured instead: every candidate (schedule x points per
// lane x waves per workgroup x trees per unit) is timed on the caller's own
// population and data, and the fastest is cached under the shape key
// (device architecture and compute-unit count, P, Lmax, V, D, n_out,
// gradient flag). The gradient call has one schedule (point-major); its
// candidates are the points per lane (2 to 4), the workgroup shape and the
// trees per unit.
//
// The cache lives for the process. With TGP_AUTOTUNE_CACHE naming a file it
// also persists: the file is read on the first lookup or tuning run, and each
// new result is appended to it as one JSON line. A line that does not parse
// exactly, or whose values are out of range, is skipped (that shape is then
// tuned again or runs the default configuration).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "tgp_autotune.h"
#include "tgp_isa.h"

namespace tgp {

namespace {

// (architecture, compute units, P, Lmax, V, D, n_out, gradient)
using Key = std::tuple<std::string, int32_t, int64_t, int32_t, int32_t, int64_t, int32_t, int32_t>;
std::mutex g_mu;
std::map<Key, tgp_cfg> g_cache;
bool g_env_loaded = false;

constexpr int kArchChars = 31;

// The current device's architecture name (up to its first ':') and compute-unit count,
// looked up once per device.
bool device_id(std::string* arch, int* cus) {
  constexpr int kMaxDevices = 64;
  static std::mutex m;
  static std::string names[kMaxDevices];
  static int counts[kMaxDevices];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return false;
  std::lock_guard<std::mutex> g(m);
  if (counts[dev] == 0) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return false;
    const size_t len = strcspn(p.gcnArchName, ":");
    if (len == 0 || len > (size_t)kArchChars || p.multiProcessorCount < 1) return false;
    names[dev].assign(p.gcnArchName, len);
    counts[dev] = p.multiProcessorCount;
  }
  *arch = names[dev];
  *cus = counts[dev];
  return true;
}

bool key_of(const tgp_pop* pop, const tgp_data* d, int n_out, bool grad, Key* k) {
  std::string arch;
  int cus = 0;
  if (!device_id(&arch, &cus)) return false;
  *k = Key(arch, cus, pop->P, pop->Lmax, d->V, d->D, n_out, grad ? 1 : 0);
  return true;
}

bool valid_entry(const Key& k, const tgp_cfg& c) {
  const int32_t cus = std::get<1>(k), Lmax = std::get<3>(k), V = std::get<4>(k), n_out = std::get<6>(k);
  const int64_t P = std::get<2>(k), D = std::get<5>(k);
  const int32_t grad = std::get<7>(k);
  for (char ch : std::get<0>(k))
    if (!((ch >= 'a' && ch <= 'z') || (ch >= '0' && ch <= '9'))) return false;
  if (cus < 1 || P < 1 || Lmax < 1 || Lmax > kMaxLmax || V < 1 || V > kMaxV || D < 1) return false;
  if (grad != 0 && grad != 1) return false;
  if (n_out < 1 || n_out > (grad ? kMaxOutGrad : kMaxOut)) return false;
  if (c.block_waves != 1 && c.block_waves != 2 && c.block_waves != 4) return false;
  if (c.trees_per_unit < 1 || c.trees_per_unit > 4096) return false;
  if (grad) {
    if (c.mode != TGP_MODE_POINT_MAJOR || c.points_per_lane < 2 || c.points_per_lane > 4) return false;
    if (c.flags & ~TGP_FLAG_ADJ_RECOMPUTE) return false;
  } else {
    if (c.mode < TGP_MODE_TREE_MAJOR || c.mode > TGP_MODE_PERSISTENT) return false;
    if (c.points_per_lane != 4 && c.points_per_lane != 8 && c.points_per_lane != 16) return false;
    if (c.flags & ~(TGP_FLAG_NO_TAIL_CHECK | TGP_FLAG_STATIC_ORDER)) return false;
  }
  return true;
}

const char kLineFmt[] =
    "{\"arch\":\"%s\",\"cus\":%d,\"P\":%lld,\"Lmax\":%d,\"V\":%d,\"D\":%lld,\"n_out\":%d,"
    "\"grad\":%d,\"mode\":%d,\"block_waves\":%d,\"points_per_lane\":%d,\"trees_per_unit\":%d,"
    "\"flags\":%d}\n";

void write_line(FILE* f, const Key& k, const tgp_cfg& c) {
  fprintf(f, kLineFmt, std::get<0>(k).c_str(), std::get<1>(k), (long long)std::get<2>(k), std::get<3>(k),
          std::get<4>(k), (long long)std::get<5>(k), std::get<6>(k), std::get<7>(k), c.mode, c.block_waves,
          c.points_per_lane, c.trees_per_unit, c.flags);
}

// One cache line, exactly as write_line prints it (trailing blanks allowed).
bool parse_line(const char* line, Key* k, tgp_cfg* c) {
  char arch[kArchChars + 1];
  int cus, Lmax, V, n_out, grad, n = -1;
  long long P, D;
  tgp_cfg x{};
  const int got = sscanf(line,
                         "{\"arch\":\"%31[a-z0-9]\",\"cus\":%d,\"P\":%lld,\"Lmax\":%d,\"V\":%d,\"D\":%lld,"
                         "\"n_out\":%d,\"grad\":%d,\"mode\":%d,\"block_waves\":%d,\"points_per_lane\":%d,"
                         "\"trees_per_unit\":%d,\"flags\":%d}%n",
                         arch, &cus, &P, &Lmax, &V, &D, &n_out, &grad, &x.mode, &x.block_waves, &x.points_per_lane,
                         &x.trees_per_unit, &x.flags, &n);
  if (got != 13 || n < 0) return false;
  for (const char* r = line + n; *r; ++r)
    if (*r != ' ' && *r != '\t' && *r != '\r' && *r != '\n') return false;
  *k = Key(std::string(arch), cus, P, Lmax, V, D, n_out, grad);
  *c = x;
  return valid_entry(*k, *c);
}

// Read a cache file into g_cache (caller holds g_mu). Lines longer than the buffer are rejected.
bool load_file(const char* path, int* loaded, int* rejected) {
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char buf[512];
  int ok = 0, bad = 0;
  while (fgets(buf, sizeof buf, f)) {
    const size_t len = strlen(buf);
    if (len + 1 == sizeof buf && buf[len - 1] != '\n') {  // overlong: skip to its end
      ++bad;
      int ch;
      while ((ch = fgetc(f)) != EOF && ch != '\n') {
      }
      continue;
    }
    if (len == 0 || (len == 1 && buf[0] == '\n')) continue;
    Key k;
    tgp_cfg c;
    if (parse_line(buf, &k, &c)) {
      g_cache[k] = c;
      ++ok;
    } else {
      ++bad;
    }
  }
  fclose(f);
  if (loaded) *loaded = ok;
  if (rejected) *rejected = bad;
  return true;
}

const char* env_path() {
  const char* p = getenv("TGP_AUTOTUNE_CACHE");
  return (p && *p) ? p : nullptr;
}

// First use in the process: read the file TGP_AUTOTUNE_CACHE names, if any (caller holds g_mu).
void load_env_once() {
  if (g_env_loaded) return;
  g_env_loaded = true;
  if (const char* p = env_path()) load_file(p, nullptr, nullptr);
}

}  // namespace

bool autotune_lookup(const tgp_pop* pop, const tgp_data* d, int n_out, bool grad, tgp_cfg* out) {
  Key k;
  if (!key_of(pop, d, n_out, grad, &k)) return false;
  std::lock_guard<std::mutex> g(g_mu);
  load_env_once();
  auto it = g_cache.find(k);
  if (it == g_cache.end()) return false;
  *out = it->second;
  return true;
}

tgp_status autotune_run(const tgp_pop* pop, const tgp_data* d, int n_out, bool grad, tgp_cfg* out, void* ws,
                        size_t ws_bytes, hipStream_t s) {
  if (pop->P == 0) {
    *out = grad ? tgp_cfg{TGP_MODE_POINT_MAJOR, 1, 4, 1, 0} : tgp_cfg{TGP_MODE_TREE_MAJOR, 1, 8, 1, 0};
    return TGP_OK;
  }
  float* mse = nullptr;
  float* gv = nullptr;
  float* gx = nullptr;
  if (hipMalloc(&mse, sizeof(float) * (size_t)pop->P) != hipSuccess) return TGP_E_HIP;
  if (grad && (hipMalloc(&gv, sizeof(float) * (size_t)pop->P * pop->row_stride) != hipSuccess ||
               hipMalloc(&gx, sizeof(float) * (size_t)d->V * d->ldx) != hipSuccess)) {
    (void)hipFree(mse);
    if (gv) (void)hipFree(gv);
    return TGP_E_HIP;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    (void)hipFree(mse);
    if (gv) (void)hipFree(gv);
    if (gx) (void)hipFree(gx);
    return TGP_E_HIP;
  }
  auto run = [&](const tgp_cfg& c) {
    return grad ? tgp_eval_mse_grad(pop, d, &c, nullptr, mse, gv, gx, nullptr, ws, ws_bytes, s)
                : tgp_internal_forward(pop, d, &c, n_out, mse, ws, ws_bytes, s);
  };
  std::vector<tgp_cfg> cands;
  if (grad) {
    for (int k : {4, 3, 2})
      for (int bw : {1, 2})
        for (int tpu : {1, 4, 16, 64}) cands.push_back(tgp_cfg{TGP_MODE_POINT_MAJOR, bw, k, tpu, 0});
  } else {
    for (int k : {16, 8, 4}) {
      if (k == 16 && d->V > 2) continue;
      if (k == 8 && d->V > 8) continue;
      if (k > 4 && n_out > kMaxOutNarrow) continue;  // many outputs: 4 points per lane only
      for (int bw : {1, 2, 4}) cands.push_back(tgp_cfg{TGP_MODE_TREE_MAJOR, bw, k, 1, 0});
      for (int tpu : {1, 4, 16, 64})
        cands.push_back(tgp_cfg{TGP_MODE_POINT_MAJOR, 4, k, tpu, 0});
      for (int bw : {1, 4})
        for (int tpu : {1, 2, 4}) cands.push_back(tgp_cfg{TGP_MODE_PERSISTENT, bw, k, tpu, 0});
      cands.push_back(tgp_cfg{TGP_MODE_PERSISTENT, 4, k, 1, TGP_FLAG_STATIC_ORDER});
    }
  }
  tgp_cfg best{};
  float best_ms = 1e30f;
  tgp_status st = TGP_OK;
  for (const tgp_cfg& c : cands) {
    // warm-up, then the median of three timed runs
    st = run(c);
    if (st != TGP_OK) break;
    float t[3];
    for (int r = 0; r < 3; ++r) {
      hipEventRecord(e0, s);
      run(c);
      hipEventRecord(e1, s);
      if (hipEventSynchronize(e1) != hipSuccess) { st = TGP_E_HIP; break; }
      hipEventElapsedTime(&t[r], e0, e1);
    }
    if (st != TGP_OK) break;
    std::sort(t, t + 3);
    if (t[1] < best_ms) {
      best_ms = t[1];
      best = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(mse);
  if (gv) (void)hipFree(gv);
  if (gx) (void)hipFree(gx);
  if (st != TGP_OK) return st;
  Key k;
  if (key_of(pop, d, n_out, grad, &k)) {
    std::lock_guard<std::mutex> g(g_mu);
    load_env_once();
    g_cache[k] = best;
    if (const char* p = env_path()) {
      if (FILE* f = fopen(p, "a")) {
        write_line(f, k, best);
        fclose(f);
      }
    }
  }
  *out = best;
  return TGP_OK;
}

}  // namespace tgp

extern "C" __attribute__((visibility("default"))) tgp_status tgp_autotune_cache_load(const char* path,
                                                                                   int32_t* n_loaded,
                                                                                   int32_t* n_rejected) {
  if (!path) return TGP_E_ARG;
  int ok = 0, bad = 0;
  {
    std::lock_guard<std::mutex> g(tgp::g_mu);
    if (!tgp::load_file(path, &ok, &bad)) return TGP_E_IO;
  }
  if (n_loaded) *n_loaded = ok;
  if (n_rejected) *n_rejected = bad;
  return TGP_OK;
}

extern "C" __attribute__((visibility("default"))) tgp_status tgp_autotune_cache_save(const char* path) {
  if (!path) return TGP_E_ARG;
  const std::string tmp = std::string(path) + ".tmp";
  std::lock_guard<std::mutex> g(tgp::g_mu);
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return TGP_E_IO;
  for (const auto& e : tgp::g_cache) tgp::write_line(f, e.first, e.second);
  const bool ok = fflush(f) == 0;
  if (fclose(f) != 0 || !ok || rename(tmp.c_str(), path) != 0) {
    remove(tmp.c_str());
    return TGP_E_IO;
  }
  return TGP_OK;
}
