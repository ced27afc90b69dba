// Event profiler: when enabled, each timed launch gets two HIP events, so
// benchmarks can read per-launch device durations of kernels that run inside
// library calls.  Single kernels carry the events in their dispatch
// (hipExtLaunchKernel: no extra packets between launches); a scope spanning
// several launches records them on its stream around the launches.
#include <mutex>

#include "common.h"

namespace gift {
namespace {

struct Rec {
  hipEvent_t a, b;
  int cls;
  double bytes;
};

struct Profiler {
  std::mutex m;
  bool on = false;
  bool paused = false;
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;

  hipEvent_t take() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};

Profiler &prof() {
  static Profiler *p = new Profiler();  // never destroyed: events may outlive exit order
  return *p;
}

}  // namespace

ProfScope::ProfScope(hipStream_t s, int cls, double bytes) : idx_(-1), stream_(s) {
  Profiler &p = prof();
  std::lock_guard<std::mutex> lk(p.m);
  if (!p.on || p.paused) return;
  hipEvent_t a = p.take(), b = p.take();
  if (!a || !b || hipEventRecord(a, s) != hipSuccess) {
    if (a) p.pool.push_back(a);
    if (b) p.pool.push_back(b);
    return;
  }
  idx_ = static_cast<int>(p.recs.size());
  p.recs.push_back(Rec{a, b, cls, bytes});
}

ProfScope::~ProfScope() {
  if (idx_ < 0) return;
  Profiler &p = prof();
  std::lock_guard<std::mutex> lk(p.m);
  if (idx_ < static_cast<int>(p.recs.size())) (void)hipEventRecord(p.recs[idx_].b, stream_);
}

bool prof_launch_events(int cls, double bytes, hipEvent_t *start, hipEvent_t *stop) {
  *start = *stop = nullptr;
  Profiler &p = prof();
  std::lock_guard<std::mutex> lk(p.m);
  if (!p.on || p.paused) return false;
  hipEvent_t a = p.take(), b = p.take();
  if (!a || !b) {
    if (a) p.pool.push_back(a);
    if (b) p.pool.push_back(b);
    return false;
  }
  p.recs.push_back(Rec{a, b, cls, bytes});
  *start = a;
  *stop = b;
  return true;
}

}  // namespace gift

using namespace gift;

extern "C" gift_status gift_profile_enable(int32_t on) {
  clear_error();
  Profiler &p = prof();
  std::lock_guard<std::mutex> lk(p.m);
  for (Rec &r : p.recs) {
    (void)hipEventSynchronize(r.b);
    p.pool.push_back(r.a);
    p.pool.push_back(r.b);
  }
  p.recs.clear();
  p.on = on != 0;
  p.paused = false;
  return GIFT_OK;
}

extern "C" gift_status gift_profile_pause(int32_t paused) {
  clear_error();
  Profiler &p = prof();
  std::lock_guard<std::mutex> lk(p.m);
  p.paused = paused != 0;
  return GIFT_OK;
}

extern "C" gift_status gift_profile_collect(int32_t cls, int64_t *launches, double *total_ms,
                                            double *max_ms, double *bytes) {
  clear_error();
  if (cls < 0 || cls >= GIFT_PROF_NUM_CLASSES)
    return set_error(GIFT_EINVAL, "unknown profiler class %d", cls);
  Profiler &p = prof();
  std::lock_guard<std::mutex> lk(p.m);
  int64_t n = 0;
  double tot = 0.0, mx = 0.0, by = 0.0;
  std::vector<Rec> keep;
  for (Rec &r : p.recs) {
    if (r.cls != cls) {
      keep.push_back(r);
      continue;
    }
    GIFT_HIP(hipEventSynchronize(r.b));
    float ms = 0.0f;
    GIFT_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    ++n;
    tot += ms;
    mx = ms > mx ? ms : mx;
    by += r.bytes;
    p.pool.push_back(r.a);
    p.pool.push_back(r.b);
  }
  p.recs.swap(keep);
  if (launches) *launches = n;
  if (total_ms) *total_ms = tot;
  if (max_ms) *max_ms = mx;
  if (bytes) *bytes = by;
  return GIFT_OK;
}
