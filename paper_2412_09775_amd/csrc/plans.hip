// FFT schedule table and its tuner.
//
// Each tunable FFT pass (rows, strided columns, the fused Z pass) has a key
// (pass kind, length, columns, batch) and a schedule (workgroup tile, threads,
// radix plan).  wo_fft_tune runs one library call while recording every
// tunable launch, then times every candidate schedule of each recorded pass
// on the call's own buffers and keeps the fastest.  The table is process-wide
// and can be exported and imported as text.
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>

#include "../../include/waveorder.h"
#include "internal.hpp"

namespace wo {

namespace {
std::mutex g_plan_mu;
std::map<FftKey, FftChoice> g_plans;
unsigned long long g_plan_version = 0;
thread_local std::vector<std::pair<FftKey, std::function<hipError_t()>>>* g_rec = nullptr;

const char* kind_name(int k) {
  switch (k) {
    case kFftRowsR2C: return "rows_r2c";
    case kFftRowsC2R: return "rows_c2r";
    case kFftCols: return "cols";
    case kFftZop: return "zop";
    case kFftTfRows: return "tf_rows";
    case kFftTfFields: return "tf_fields";
    default: return "?";
  }
}

int kind_of(const char* s) {
  for (int k = 0; k < kFftKinds; ++k)
    if (strcmp(s, kind_name(k)) == 0) return k;
  return -1;
}

std::string line_of(const FftKey& k, const FftChoice& c) {
  char b[160];
  snprintf(b, sizeof(b), "%s %d %ld %ld %d %d %d %d\n", kind_name(k.kind), k.n, k.m, k.batch, k.extra,
           c.w, c.threads, c.plan);
  return b;
}

int copy_out(const std::string& t, char* buf, size_t len, size_t* needed) {
  if (needed) *needed = t.size() + 1;
  if (buf && len) {
    const size_t n = t.size() < len - 1 ? t.size() : len - 1;
    memcpy(buf, t.data(), n);
    buf[n] = 0;
  }
  return WO_OK;
}
}  // namespace

bool make_plan_variant(int n, int variant, FftPlan* p) {
  if (!make_plan(n, p)) return false;
  if (variant == 2) {
    unsigned long long r = 0;
    for (int q = 0; q < p->npass; ++q)
      r |= (unsigned long long)plan_radix(*p, p->npass - 1 - q) << (4 * q);
    p->radices = r;
  } else if (variant == 3) {
    int m = n, np = 0;
    unsigned long long r = 0;
    for (int f : {5, 3, 8, 4, 2})
      while (m % f == 0 && np < kMaxPasses) {
        r |= (unsigned long long)f << (4 * np++);
        m /= f;
      }
    p->radices = r;
    p->npass = np;
  }
  return true;
}

bool fft_lookup(const FftKey& k, FftChoice* c) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  auto it = g_plans.find(k);
  if (it == g_plans.end()) return false;
  *c = it->second;
  return true;
}

void fft_store(const FftKey& k, const FftChoice& c) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  g_plans[k] = c;
  ++g_plan_version;
}

unsigned long long fft_table_version() {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  return g_plan_version;
}

bool fft_recording() { return g_rec != nullptr; }

void fft_record(const FftKey& k, std::function<hipError_t()> relaunch) {
  for (auto& e : *g_rec)
    if (!(e.first < k) && !(k < e.first)) return;   // first launch of a key is enough
  g_rec->push_back({k, std::move(relaunch)});
}

}  // namespace wo

using namespace wo;

extern "C" {

int wo_fft_tune(int32_t op, const wo_optics* o, int32_t n, const void* tf, const float* in, float* out,
                double eta, int32_t reps, void* ws, size_t ws_bytes, void* stream) {
  if (!o || n < 1 || reps < 1 || !ws) return WO_EINVAL;
  hipStream_t hs = (hipStream_t)stream;
  const bool band = (op & WO_FFT_TUNE_BAND) != 0;
  const int op0 = op & ~WO_FFT_TUNE_BAND;
  auto run_op = [&]() -> int {
    if (band)
      return op0 == WO_OP_TRANSFER_FUNCTION
                 ? wo_transfer_function_band(o, n, out, ws, ws_bytes, stream)
                 : wo_linear_band(op0, o, n, tf, in, nullptr, eta, out, ws, ws_bytes, stream);
    switch (op0) {
      case WO_OP_TRANSFER_FUNCTION: return wo_transfer_function(o, n, out, ws, ws_bytes, stream);
      case WO_OP_FORWARD: return wo_forward(o, n, tf, in, nullptr, out, ws, ws_bytes, stream);
      case WO_OP_RECONSTRUCT: return wo_reconstruct(o, n, tf, in, nullptr, eta, out, ws, ws_bytes, stream);
      case WO_OP_ADJOINT: return wo_adjoint(o, n, tf, in, out, ws, ws_bytes, stream);
      default: return WO_EINVAL;
    }
  };
  // one recorded call names the passes to tune
  std::vector<std::pair<FftKey, std::function<hipError_t()>>> rec;
  g_rec = &rec;
  int st = run_op();
  g_rec = nullptr;
  if (st) return st;
  const bool was_timing = timing_enabled();
  if (was_timing) wo_timing_enable(0);
  hipEvent_t a = nullptr, b = nullptr;
  int status = WO_OK;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) status = WO_EHIP;
  // Each pass in turn, the others keeping their current schedules: every
  // candidate is timed over the whole call, so the pass sees the caches and
  // the neighbouring passes it meets in use (timing one kernel alone on a
  // buffer it keeps in the Infinity Cache favoured other schedules).
  for (size_t r = 0; r < rec.size() && status == WO_OK; ++r) {
    const FftKey& key = rec[r].first;
    const std::vector<FftChoice> cand = fft_candidates(key);
    float best_ms = 0.f;
    int best = -1;
    for (size_t i = 0; i < cand.size() && status == WO_OK; ++i) {
      fft_store(key, cand[i]);
      if (run_op() != WO_OK) continue;   // warm-up; a failing schedule is skipped
      // the fastest of `reps` timed calls (the least disturbed)
      float ms = -1.f;
      for (int k = 0; k < reps && status == WO_OK; ++k) {
        if (hipEventRecord(a, hs) != hipSuccess) { status = WO_EHIP; break; }
        const bool ok = run_op() == WO_OK;
        if (hipEventRecord(b, hs) != hipSuccess || hipEventSynchronize(b) != hipSuccess) {
          status = WO_EHIP;
          break;
        }
        float t = 0.f;
        if (!ok || hipEventElapsedTime(&t, a, b) != hipSuccess) { ms = -1.f; break; }
        if (ms < 0.f || t < ms) ms = t;
      }
      if (ms < 0.f) continue;
      if (best < 0 || ms < best_ms) {
        best = (int)i;
        best_ms = ms;
      }
    }
    fft_store(key, best >= 0 ? cand[best] : cand[0]);
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (was_timing) wo_timing_enable(1);
  if (status == WO_OK && hipStreamSynchronize(hs) != hipSuccess) status = WO_EHIP;
  return status;
}

int wo_fft_plans_export(char* buf, size_t len, size_t* needed) {
  std::string t;
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    for (auto& kv : g_plans) t += line_of(kv.first, kv.second);
  }
  return copy_out(t, buf, len, needed);
}

int wo_fft_plans_import(const char* text) {
  if (!text) return WO_EINVAL;
  std::vector<std::pair<FftKey, FftChoice>> parsed;
  const char* p = text;
  while (*p) {
    const char* e = strchr(p, '\n');
    std::string ln = e ? std::string(p, e - p) : std::string(p);
    p = e ? e + 1 : p + ln.size();
    if (ln.find_first_not_of(" \t\r") == std::string::npos) continue;
    char kind[32];
    FftKey k;
    FftChoice c;
    if (sscanf(ln.c_str(), "%31s %d %ld %ld %d %d %d %d", kind, &k.n, &k.m, &k.batch, &k.extra, &c.w,
               &c.threads, &c.plan) != 8)
      return WO_EINVAL;
    k.kind = kind_of(kind);
    if (k.kind < 0 || k.n < 1 || k.m < 0 || k.batch < 0) return WO_EINVAL;
    bool accepted = false;
    for (auto& x : fft_candidates(k))
      accepted |= x.w == c.w && x.threads == c.threads && x.plan == c.plan;
    if (!accepted) return WO_EINVAL;
    parsed.push_back({k, c});
  }
  for (auto& kc : parsed) fft_store(kc.first, kc.second);
  return WO_OK;
}

int wo_fft_plans_clear(void) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  g_plans.clear();
  ++g_plan_version;
  return WO_OK;
}

int wo_fft_candidates(const char* key_line, char* buf, size_t len, size_t* needed) {
  if (!key_line) return WO_EINVAL;
  char kind[32];
  FftKey k;
  if (sscanf(key_line, "%31s %d %ld %ld %d", kind, &k.n, &k.m, &k.batch, &k.extra) != 5) return WO_EINVAL;
  k.kind = kind_of(kind);
  if (k.kind < 0 || k.n < 1 || k.m < 0 || k.batch < 0) return WO_EINVAL;
  std::string t;
  for (auto& c : fft_candidates(k)) t += line_of(k, c);
  return copy_out(t, buf, len, needed);
}

}  // extern "C"
