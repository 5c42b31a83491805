// Per-stage device timers (the paper profiles its GPU solve with per-stage
// device timers, Sec. 5.4 "GPU Kernel Profiling", Table profile).
//
// When tracing is on, every launch site brackets its kernel with a pair of
// HIP events on the launch stream and records the algorithmic flops and
// bytes of that launch.  hp_trace_read() waits for the events and returns,
// per stage, the number of launches, the summed kernel time and the summed
// algorithmic work.  Off (the default) it costs one branch per launch.
#include "common.h"

#include <mutex>
#include <vector>

namespace hp {

namespace {
struct Rec {
  int cat;
  hipEvent_t a, b;
  double flops, bytes;
};
std::mutex g_mu;
bool g_on = false;
unsigned g_mask = 0;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t get_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

const char *const kTraceNames[TR_COUNT] = {"assemble", "panel",    "laswp",   "trsm",    "gemm_c128",  "gemm_c64",
                                           "residual", "refine",   "rmatrix", "smatrix", "gemm_f16x3"};

bool trace_on() { return g_on; }

TraceScope::TraceScope(int cat, hipStream_t st, double flops, double bytes)
    : cat_(cat), st_(st), flops_(flops), bytes_(bytes), a_(nullptr) {
  if (!g_on || !((g_mask >> cat) & 1u)) return;
  // launches recorded into a graph are not timed (their events would be
  // replayed many times under one record)
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return;
  std::lock_guard<std::mutex> lk(g_mu);
  a_ = get_event();
  if (a_) hipEventRecord((hipEvent_t)a_, st_);
}

TraceScope::~TraceScope() {
  if (!a_) return;
  std::lock_guard<std::mutex> lk(g_mu);
  hipEvent_t b = get_event();
  if (!b) return;
  hipEventRecord(b, st_);
  g_recs.push_back(Rec{cat_, (hipEvent_t)a_, b, flops_, bytes_});
}

}  // namespace hp

using namespace hp;

extern "C" int hp_trace_enable(int mask) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (Rec &r : g_recs) {
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  g_on = (mask != 0);
  g_mask = mask < 0 ? ((1u << TR_COUNT) - 1u) : (unsigned)mask;
  return HP_OK;
}

extern "C" int hp_trace_read(hp_trace_stat *out, int max_stats) {
  if (!out || max_stats < TR_COUNT) return HP_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_mu);
  for (int c = 0; c < TR_COUNT; ++c) {
    out[c].name = kTraceNames[c];
    out[c].launches = 0;
    out[c].ms = 0.0;
    out[c].flops = 0.0;
    out[c].bytes = 0.0;
  }
  for (Rec &r : g_recs) {
    if (hipEventSynchronize(r.b) != hipSuccess) return HP_ERR_HIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return HP_ERR_HIP;
    hp_trace_stat &s = out[r.cat];
    s.launches += 1;
    s.ms += ms;
    s.flops += r.flops;
    s.bytes += r.bytes;
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  return TR_COUNT;
}
