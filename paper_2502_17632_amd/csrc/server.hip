// Request-serving engine: filter requests for many designs, graphs kept
// resident on the device, admission by a device-memory budget, continuous
// batching of ready requests, latency statistics.
//
// Threads (all on the server's device):
//   - the dispatcher admits pending requests, hands builds to the builders,
//     groups ready requests of similar size into one launch sequence on one
//     of the filter streams, and retires launches whose completion event has
//     fired;
//   - each builder turns a netlist into a resident graph on its own stream.
// A request is admitted as soon as an execution slot is free and its memory
// fits the budget (resident graphs that no admitted request uses are evicted,
// least recently used first); requests that arrive while others run join the
// next launch, so work of different requests overlaps on the device.
//
// Every launch filters each of its graphs with the arithmetic of filtering it
// alone (tile class 0, widest column chunks), so a result does not depend on
// what else was in the mix.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.h"
#include "filter.h"

namespace gift {
namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

enum class Phase { kPending, kBuilding, kWaitGraph, kReady, kRunning, kDone };

struct Request {
  uint64_t ticket = 0;
  gift_request req{};
  Phase phase = Phase::kPending;
  gift_status status = GIFT_OK;
  std::string error;
  int32_t built = 0;
  int64_t reserved = 0;  // bytes reserved for this request's filter work
  int64_t est_graph = 0, est_peak = 0;  // bounds for a build of its netlist
  Clock::time_point t_submit, t_admit, t_done;
};

struct Resident {
  gift_graph *g = nullptr;
  int64_t bytes = 0;        // actual device bytes (estimate while building)
  bool ready = false;       // built
  bool failed = false;
  int refs = 0;             // admitted requests that use it
  uint64_t last_use = 0;
  std::vector<uint64_t> waiting;  // requests waiting for the build
};

struct Launch {
  hipEvent_t done = nullptr;
  int stream = 0;
  std::vector<uint64_t> tickets;
};

// Device bytes of a graph built from this netlist, and the build's peak
// scratch (upper bounds from the pin counts).
void estimate_graph(const gift_request &r, const gift_server_config &c, int64_t *graph,
                    int64_t *peak) {
  int64_t z = 0, v = 0;
  const int64_t T = c.star_threshold;
  for (int64_t e = 0; e < r.num_nets; ++e) {
    const int64_t m = r.net_ptr[e + 1] - r.net_ptr[e];
    if (m < 2) continue;
    if (T > 0 && m > T) {
      // a star, or a clique of at most T distinct cells if pins repeat
      z += std::max(2 * m, T * (T - 1));
      ++v;
    } else {
      z += m * (m - 1);
    }
  }
  const int64_t R = r.num_cells + v;
  const int64_t bv = static_cast<int64_t>(dtype_size(c.storage));
  const int64_t ba = static_cast<int64_t>(accum_size(c.storage));
  int64_t sig = 0;
  for (int32_t t = 0; t < c.num_terms; ++t) {
    bool dup = false;
    for (int32_t u = 0; u < t; ++u) dup |= c.terms[u].sigma == c.terms[t].sigma;
    if (!dup) sig += bv * z + ba * R;
  }
  const int64_t tiles = 2 * (z / 256 + R / 64 + 2) * 16;
  *graph = 4 * (R + 1) + 12 * z + 8 * R + sig + tiles + (1 << 20);
  const int64_t P = r.net_ptr[r.num_nets];
  *peak = *graph + 40 * z + 24 * P + 48 * r.num_nets + 16 * R + (8 << 20);
}

}  // namespace
}  // namespace gift

using namespace gift;

struct gift_server {
  gift_server_config cfg{};
  std::vector<gift_term> terms;
  int device = 0;

  std::mutex m;
  std::condition_variable cv_dispatch;  // new work for the dispatcher
  std::condition_variable cv_done;      // a request finished
  std::condition_variable cv_build;     // new work for the builders
  bool stopping = false;        // drain, then the dispatcher exits
  bool builders_stop = false;   // set after the dispatcher has exited

  uint64_t next_ticket = 1;
  std::unordered_map<uint64_t, Request> reqs;
  std::deque<uint64_t> pending;  // submitted, not admitted (FIFO)
  std::deque<uint64_t> ready;    // graph resident, not launched
  std::deque<uint64_t> build_queue;
  std::unordered_map<uint64_t, Resident> graphs;  // by design id
  uint64_t use_clock = 0;
  int64_t reserved = 0;  // graphs + admitted requests' work
  int64_t peak_reserved = 0;
  int32_t admitted = 0;  // admitted and not finished
  std::vector<Launch> inflight;

  std::vector<hipStream_t> streams;
  std::vector<PinnedRing *> rings;
  std::vector<int> stream_load;  // launches in flight per stream
  std::vector<hipStream_t> build_streams;

  std::vector<double> latencies;  // completed requests since the last reset
  gift_server_stats st{};
  Clock::time_point t_first, t_last;
  bool any = false;

  std::thread dispatcher;
  std::vector<std::thread> builders;
};

namespace gift {
namespace {

int64_t bucket_of(int64_t rows) {
  int64_t b = 0;
  while (rows > 1) {
    rows >>= 1;
    ++b;
  }
  return b;
}

void finish_locked(gift_server *s, Request &r, gift_status status, const std::string &err) {
  r.phase = Phase::kDone;
  r.status = status;
  r.error = err;
  r.t_done = Clock::now();
  s->reserved -= r.reserved;
  r.reserved = 0;
  --s->admitted;
  auto it = s->graphs.find(r.req.design_id);
  if (it != s->graphs.end() && it->second.refs > 0) --it->second.refs;
  if (status == GIFT_OK) {
    s->latencies.push_back(ms_between(r.t_submit, r.t_done));
    ++s->st.completed;
  } else {
    ++s->st.failed;
  }
  s->t_last = r.t_done;
  s->cv_done.notify_all();
}

// Evicts unused resident graphs (least recently used first) until `need`
// more bytes fit; returns whether they do.
bool make_room_locked(gift_server *s, int64_t need) {
  while (s->reserved + need > s->cfg.hbm_budget_bytes) {
    uint64_t victim = 0;
    uint64_t oldest = UINT64_MAX;
    for (auto &kv : s->graphs) {
      const Resident &g = kv.second;
      if (g.ready && g.refs == 0 && g.last_use < oldest) {
        oldest = g.last_use;
        victim = kv.first;
      }
    }
    if (oldest == UINT64_MAX) return false;
    Resident &g = s->graphs[victim];
    // refs == 0: every launch that used it has completed
    (void)gift_destroy_graph(g.g, s->build_streams[0]);
    s->reserved -= g.bytes;
    ++s->st.evictions;
    s->graphs.erase(victim);
  }
  return true;
}

int64_t work_bytes(const gift_server *s, int64_t rows_est) {
  const int64_t rb = static_cast<int64_t>(dtype_size(s->cfg.storage)) *
                     chunk_width(s->cfg.num_cols) * rows_est;
  return (3 + s->cfg.num_terms) * (rb + 256) + rows_est / 8 + (1 << 20);
}

// Admits pending requests in arrival order while slots and memory allow; a
// request that does not fit stays pending and does not block smaller ones.
void admit_locked(gift_server *s) {
  for (auto it = s->pending.begin(); it != s->pending.end();) {
    if (s->admitted >= s->cfg.max_inflight) return;
    Request &r = s->reqs[*it];
    auto gi = s->graphs.find(r.req.design_id);
    const bool have = gi != s->graphs.end() && !gi->second.failed;
    int64_t peak = 0;
    int64_t rows = r.req.num_cells;
    if (have && gi->second.ready) {
      rows = gi->second.g->num_rows;
    } else if (!have) {
      // evicted since it was submitted: bound the build now
      if (r.est_peak == 0) estimate_graph(r.req, s->cfg, &r.est_graph, &r.est_peak);
      peak = r.est_peak;
      rows = r.req.num_cells + r.req.num_nets;
    }
    const int64_t wb = work_bytes(s, rows);
    const int64_t need = wb + (have ? 0 : peak);
    if (need > s->cfg.hbm_budget_bytes) {
      ++s->admitted;
      r.t_admit = Clock::now();
      finish_locked(s, r, GIFT_ENOMEM, "request needs more device memory than the budget");
      it = s->pending.erase(it);
      continue;
    }
    if (have) ++gi->second.refs;  // protect it from eviction while making room
    const bool fits = make_room_locked(s, need);
    if (have) --gi->second.refs;
    if (!fits) {
      ++it;
      continue;
    }
    ++s->admitted;
    r.t_admit = Clock::now();
    r.reserved = wb;
    s->reserved += wb;
    if (have) {
      Resident &g = s->graphs[r.req.design_id];
      ++g.refs;
      g.last_use = ++s->use_clock;
      if (g.ready) {
        r.phase = Phase::kReady;
        s->ready.push_back(r.ticket);
      } else {
        r.phase = Phase::kWaitGraph;
        g.waiting.push_back(r.ticket);
      }
    } else {
      Resident &g = s->graphs[r.req.design_id];
      g.bytes = peak;  // the build's peak until it is done
      g.refs = 1;
      g.last_use = ++s->use_clock;
      s->reserved += peak;
      r.phase = Phase::kBuilding;
      s->build_queue.push_back(r.ticket);
      s->cv_build.notify_one();
    }
    s->peak_reserved = std::max(s->peak_reserved, s->reserved);
    it = s->pending.erase(it);
  }
}

// Retires launches whose event has fired.
void retire_locked(gift_server *s) {
  for (size_t i = 0; i < s->inflight.size();) {
    Launch &l = s->inflight[i];
    hipError_t e = hipEventQuery(l.done);
    if (e == hipErrorNotReady) {
      ++i;
      continue;
    }
    const gift_status st = e == hipSuccess ? GIFT_OK : GIFT_EDEVICE;
    const std::string err = e == hipSuccess ? "" : hipGetErrorString(e);
    for (uint64_t t : l.tickets) finish_locked(s, s->reqs[t], st, err);
    (void)hipEventDestroy(l.done);
    --s->stream_load[l.stream];
    s->inflight.erase(s->inflight.begin() + i);
  }
}

// Groups ready requests by size bucket and launches them; the lock is held
// only while choosing the group.
bool launch_one(gift_server *s, std::unique_lock<std::mutex> &lk) {
  if (s->ready.empty()) return false;
  int stream = -1;
  for (size_t i = 0; i < s->streams.size(); ++i)
    if (s->stream_load[i] < 2 && (stream < 0 || s->stream_load[i] < s->stream_load[stream]))
      stream = static_cast<int>(i);
  if (stream < 0) return false;
  // the oldest ready request fixes the bucket
  const uint64_t head = s->ready.front();
  const int64_t b0 = bucket_of(s->graphs[s->reqs[head].req.design_id].g->num_rows);
  std::vector<uint64_t> group;
  int64_t rows = 0;
  for (auto it = s->ready.begin(); it != s->ready.end();) {
    Request &r = s->reqs[*it];
    const gift_graph *g = s->graphs[r.req.design_id].g;
    const bool same = bucket_of(g->num_rows) == b0;
    const bool room = group.empty() || (static_cast<int32_t>(group.size()) < s->cfg.max_batch &&
                                        rows + g->num_rows <= s->cfg.max_batch_rows);
    if (same && room) {
      group.push_back(*it);
      rows += g->num_rows;
      it = s->ready.erase(it);
    } else {
      ++it;
    }
  }
  std::vector<const gift_graph *> gs;
  std::vector<GraphIO> ios;
  for (uint64_t t : group) {
    Request &r = s->reqs[t];
    r.phase = Phase::kRunning;
    gs.push_back(s->graphs[r.req.design_id].g);
    ios.push_back(GraphIO{r.req.x_in, r.req.ld_in, r.req.y_out, r.req.ld_out, r.req.fixed_mask, 0});
  }
  ++s->stream_load[stream];
  lk.unlock();
  hipStream_t st = s->streams[stream];
  gift_status status =
      enqueue_dynamic_batch(gs.data(), ios.data(), static_cast<int32_t>(gs.size()),
                            s->terms.data(), s->cfg.num_terms, s->cfg.num_cols,
                            s->cfg.in_dtype, s->cfg.out_dtype, st, *s->rings[stream]);
  std::string err = status == GIFT_OK ? "" : gift_last_error();
  hipEvent_t ev = nullptr;
  if (status == GIFT_OK && (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
                            hipEventRecord(ev, st) != hipSuccess)) {
    status = GIFT_EDEVICE;
    err = "hipEventRecord failed";
    if (ev) (void)hipEventDestroy(ev);
    ev = nullptr;
  }
  lk.lock();
  if (status != GIFT_OK) {
    --s->stream_load[stream];
    for (uint64_t t : group) finish_locked(s, s->reqs[t], status, err);
    return true;
  }
  ++s->st.batches;
  s->st.batched_requests += static_cast<int64_t>(group.size());
  s->inflight.push_back(Launch{ev, stream, std::move(group)});
  return true;
}

void dispatcher_main(gift_server *s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->m);
  for (;;) {
    retire_locked(s);
    admit_locked(s);
    bool launched = false;
    while (launch_one(s, lk)) launched = true;
    if (s->stopping && s->pending.empty() && s->ready.empty() && s->inflight.empty() &&
        s->build_queue.empty() && s->admitted == 0)
      return;
    if (launched) continue;
    // poll in-flight launches often, sleep longer when idle
    const auto wait = s->inflight.empty() ? std::chrono::milliseconds(5)
                                          : std::chrono::milliseconds(0);
    if (s->inflight.empty())
      s->cv_dispatch.wait_for(lk, wait);
    else {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    }
  }
}

void builder_main(gift_server *s, int idx) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->m);
  for (;;) {
    s->cv_build.wait(lk, [&] { return s->builders_stop || !s->build_queue.empty(); });
    if (s->build_queue.empty()) {
      if (s->builders_stop) return;
      continue;
    }
    const uint64_t t = s->build_queue.front();
    s->build_queue.pop_front();
    Request &r = s->reqs[t];
    const gift_request req = r.req;
    lk.unlock();
    std::vector<double> sig;
    for (const gift_term &tm : s->terms)
      if (std::find(sig.begin(), sig.end(), tm.sigma) == sig.end()) sig.push_back(tm.sigma);
    gift_graph_desc d{req.num_cells, req.num_nets, req.net_ptr, req.pin_cell, GIFT_MEM_HOST,
                      s->cfg.weight_model, s->cfg.star_threshold, s->cfg.storage,
                      static_cast<int32_t>(sig.size()), sig.data(), -1};
    gift_graph *g = nullptr;
    gift_status status = gift_build_graph(&d, s->build_streams[idx], &g);
    // the build's last kernels may still run on the builder's stream; the
    // graph is used on the filter streams, so wait for them
    if (status == GIFT_OK && hipStreamSynchronize(s->build_streams[idx]) != hipSuccess) {
      (void)gift_destroy_graph(g, s->build_streams[idx]);
      g = nullptr;
      status = set_error(GIFT_EDEVICE, "build stream failed");
    }
    std::string err = status == GIFT_OK ? "" : gift_last_error();
    lk.lock();
    Resident &res = s->graphs[req.design_id];
    s->reserved -= res.bytes;  // the build's peak
    Request &rr = s->reqs[t];
    ++s->st.builds;
    if (status != GIFT_OK) {
      res.failed = true;
      std::vector<uint64_t> w = std::move(res.waiting);
      s->graphs.erase(req.design_id);
      finish_locked(s, rr, status, err);
      for (uint64_t u : w) finish_locked(s, s->reqs[u], status, err);
    } else {
      res.g = g;
      res.bytes = g->bytes;
      res.ready = true;
      s->reserved += res.bytes;
      rr.built = 1;
      rr.phase = Phase::kReady;
      s->ready.push_back(t);
      for (uint64_t u : res.waiting) {
        s->reqs[u].phase = Phase::kReady;
        s->ready.push_back(u);
      }
      res.waiting.clear();
    }
    s->cv_dispatch.notify_one();
  }
}

void stop_threads(gift_server *s) {
  {
    std::lock_guard<std::mutex> lk(s->m);
    s->stopping = true;
  }
  s->cv_dispatch.notify_all();
  s->cv_build.notify_all();
  if (s->dispatcher.joinable()) s->dispatcher.join();
  {
    std::lock_guard<std::mutex> lk(s->m);
    s->builders_stop = true;
  }
  s->cv_build.notify_all();
  for (auto &b : s->builders)
    if (b.joinable()) b.join();
}

void free_server(gift_server *s) {
  stop_threads(s);
  for (auto &kv : s->graphs)
    if (kv.second.g) (void)gift_destroy_graph(kv.second.g, s->build_streams.empty() ? nullptr : s->build_streams[0]);
  for (PinnedRing *r : s->rings) delete r;
  for (hipStream_t st : s->streams) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  for (hipStream_t st : s->build_streams) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  delete s;
}

double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double pos = q * static_cast<double>(v.size() - 1);
  const size_t i = static_cast<size_t>(pos);
  const double f = pos - static_cast<double>(i);
  return i + 1 < v.size() ? v[i] * (1.0 - f) + v[i + 1] * f : v[i];
}

}  // namespace
}  // namespace gift

extern "C" gift_status gift_server_create(const gift_server_config *cfg, gift_server **out) {
  clear_error();
  if (!out) return set_error(GIFT_EINVAL, "gift_server_create: out is NULL");
  *out = nullptr;
  if (!cfg) return set_error(GIFT_EINVAL, "gift_server_create: cfg is NULL");
  const gift_server_config &c = *cfg;
  if (c.hbm_budget_bytes < (int64_t(1) << 20))
    return set_error(GIFT_EINVAL, "hbm_budget_bytes %lld < 1 MiB",
                     static_cast<long long>(c.hbm_budget_bytes));
  if (c.max_inflight < 1 || c.num_streams < 1 || c.num_builders < 1 || c.max_batch < 1 ||
      c.max_batch_rows < 1)
    return set_error(GIFT_EINVAL, "max_inflight, num_streams, num_builders, max_batch and "
                                  "max_batch_rows must be >= 1");
  if (c.num_streams > 16 || c.num_builders > 16)
    return set_error(GIFT_EINVAL, "at most 16 filter streams and 16 builders");
  if (!dtype_valid(c.storage)) return set_error(GIFT_EINVAL, "storage %d", c.storage);
  if (c.weight_model != GIFT_W_INV_M1 && c.weight_model != GIFT_W_TWO_OVER_M)
    return set_error(GIFT_EINVAL, "weight_model %d", c.weight_model);
  if (c.star_threshold < 0) return set_error(GIFT_EINVAL, "star_threshold < 0");
  if (c.num_cols < 1) return set_error(GIFT_EINVAL, "num_cols %d < 1", c.num_cols);
  if ((c.in_dtype != GIFT_F32 && c.in_dtype != GIFT_F64) ||
      (c.out_dtype != GIFT_F32 && c.out_dtype != GIFT_F64))
    return set_error(GIFT_EUNSUPPORTED, "in_dtype and out_dtype must be F32 or F64");
  if (!c.terms || c.num_terms < 1 || c.num_terms > kMaxTerms)
    return set_error(GIFT_EINVAL, "terms: need 1..64");
  for (int32_t t = 0; t < c.num_terms; ++t) {
    const gift_term &tm = c.terms[t];
    if (!(tm.sigma >= 0.0) || !std::isfinite(tm.sigma) || tm.order < 1 ||
        !std::isfinite(tm.alpha) || tm.reserved != 0)
      return set_error(GIFT_EINVAL, "term %d is invalid", t);
  }
  gift_server *s = new (std::nothrow) gift_server();
  if (!s) return set_error(GIFT_ENOMEM, "gift_server_create: host allocation");
  s->cfg = c;
  s->terms.assign(c.terms, c.terms + c.num_terms);
  s->cfg.terms = s->terms.data();
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return set_error(GIFT_EDEVICE, "hipGetDevice failed");
  }
  auto fail = [&](const char *what) {
    std::string msg = what;
    free_server(s);
    return set_error(GIFT_EDEVICE, "%s", msg.c_str());
  };
  for (int i = 0; i < c.num_streams; ++i) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
      return fail("hipStreamCreateWithFlags failed");
    s->streams.push_back(st);
    s->rings.push_back(new PinnedRing());
    s->stream_load.push_back(0);
  }
  for (int i = 0; i < c.num_builders; ++i) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
      return fail("hipStreamCreateWithFlags failed");
    s->build_streams.push_back(st);
  }
  try {
    s->dispatcher = std::thread(dispatcher_main, s);
    for (int i = 0; i < c.num_builders; ++i) s->builders.emplace_back(builder_main, s, i);
  } catch (...) {
    return fail("could not start the server threads");
  }
  *out = s;
  return GIFT_OK;
}

extern "C" gift_status gift_server_submit(gift_server *s, const gift_request *req,
                                          uint64_t *ticket) {
  clear_error();
  if (!s || !req || !ticket) return set_error(GIFT_EINVAL, "gift_server_submit: NULL argument");
  const gift_request &r = *req;
  if (r.num_cells < 0 || r.num_nets < 0) return set_error(GIFT_EINVAL, "negative sizes");
  if (!r.net_ptr || (!r.pin_cell && r.num_nets > 0 && r.net_ptr[r.num_nets] > 0))
    return set_error(GIFT_EINVAL, "net_ptr / pin_cell is NULL");
  if (r.num_cells > 0 && (!r.x_in || !r.y_out))
    return set_error(GIFT_EINVAL, "x_in / y_out is NULL");
  if (r.ld_in < s->cfg.num_cols || r.ld_out < s->cfg.num_cols)
    return set_error(GIFT_EINVAL, "leading dimension smaller than num_cols");
  Request q;
  q.req = r;
  q.t_submit = Clock::now();
  bool resident = false;
  {
    std::lock_guard<std::mutex> lk(s->m);
    auto it = s->graphs.find(r.design_id);
    resident = it != s->graphs.end() && !it->second.failed;
  }
  // the build bound walks the netlist (O(nets)): only for a design that is
  // not resident, and outside the lock
  if (!resident) estimate_graph(r, s->cfg, &q.est_graph, &q.est_peak);
  std::lock_guard<std::mutex> lk(s->m);
  if (s->stopping) return set_error(GIFT_EBUSY, "server is stopping");
  q.ticket = s->next_ticket++;
  if (!s->any) {
    s->t_first = q.t_submit;
    s->any = true;
  }
  ++s->st.submitted;
  s->reqs.emplace(q.ticket, q);
  s->pending.push_back(q.ticket);
  *ticket = q.ticket;
  s->cv_dispatch.notify_one();
  return GIFT_OK;
}

extern "C" gift_status gift_server_wait(gift_server *s, uint64_t ticket, double timeout_s,
                                        gift_request_result *res) {
  clear_error();
  if (!s) return set_error(GIFT_EINVAL, "gift_server_wait: NULL server");
  std::unique_lock<std::mutex> lk(s->m);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return set_error(GIFT_EINVAL, "unknown ticket %llu",
                                            static_cast<unsigned long long>(ticket));
  auto done = [&] { return s->reqs[ticket].phase == Phase::kDone; };
  if (timeout_s < 0) {
    s->cv_done.wait(lk, done);
  } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done)) {
    return set_error(GIFT_EBUSY, "request %llu not finished",
                     static_cast<unsigned long long>(ticket));
  }
  Request r = s->reqs[ticket];
  s->reqs.erase(ticket);
  if (res) {
    res->status = r.status;
    res->built = r.built;
    res->latency_ms = ms_between(r.t_submit, r.t_done);
    res->queue_ms = ms_between(r.t_submit, r.t_admit);
    res->service_ms = ms_between(r.t_admit, r.t_done);
  }
  if (r.status != GIFT_OK) return set_error(r.status, "request %llu: %s",
                                            static_cast<unsigned long long>(ticket),
                                            r.error.c_str());
  return GIFT_OK;
}

extern "C" gift_status gift_server_get_stats(gift_server *s, int32_t reset,
                                             gift_server_stats *out) {
  clear_error();
  if (!s || !out) return set_error(GIFT_EINVAL, "gift_server_get_stats: NULL argument");
  std::lock_guard<std::mutex> lk(s->m);
  gift_server_stats st = s->st;
  st.p50_ms = percentile(s->latencies, 0.50);
  st.p99_ms = percentile(s->latencies, 0.99);
  double sum = 0, mx = 0;
  for (double v : s->latencies) {
    sum += v;
    mx = std::max(mx, v);
  }
  st.mean_ms = s->latencies.empty() ? 0.0 : sum / static_cast<double>(s->latencies.size());
  st.max_ms = mx;
  st.elapsed_s = s->any ? ms_between(s->t_first, s->t_last) * 1e-3 : 0.0;
  int64_t rb = 0, rg = 0;
  for (auto &kv : s->graphs)
    if (kv.second.ready) {
      rb += kv.second.bytes;
      ++rg;
    }
  st.resident_graphs = rg;
  st.resident_bytes = rb;
  st.reserved_bytes = s->reserved;
  st.peak_reserved_bytes = s->peak_reserved;
  *out = st;
  if (reset) {
    s->latencies.clear();
    s->st = gift_server_stats{};
    s->any = false;
    s->peak_reserved = s->reserved;
  }
  return GIFT_OK;
}

extern "C" gift_status gift_server_destroy(gift_server *s) {
  clear_error();
  if (!s) return GIFT_OK;
  free_server(s);
  return GIFT_OK;
}
