// C ABI plumbing: errors, stream-ordered allocation, graph info/export/destroy.
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "common.h"

namespace gift {

namespace {
thread_local std::string t_last_error;
}

gift_status set_error(gift_status s, const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  t_last_error = buf;
  return s;
}

void clear_error() { t_last_error.clear(); }

gift_status check_launch(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return set_error(GIFT_EDEVICE, "launch of %s failed: %s", what, hipGetErrorString(e));
  return GIFT_OK;
}

namespace {

// Stream-ordered caching allocator, or the caller's allocator when one is set
// (gift_set_allocator).  Device memory comes from hipMalloc in
// blocks that are never returned to the runtime while cached: a freed block
// goes back to the free list of the stream it was freed on and is handed out
// again only for work on that same stream, so stream order alone makes the
// reuse safe (the previous user's kernels precede the new user's).  A free
// block is reused for a request when it is at most 25% larger.  This keeps
// the runtime's allocation calls (tens of microseconds each, more for large
// frees) off the build and filter paths.
struct Block {
  void *ptr;
  size_t size;
};

// A block in use: its size, device, and whether the caller's allocator
// (rather than the cache) provided it, with that allocator's callbacks.
struct Live {
  size_t size;
  int device;
  bool hooked;
  gift_allocator hook;
};

struct Pool {
  std::mutex m;
  // per (device, stream): free blocks by size
  std::map<std::pair<int, hipStream_t>, std::multimap<size_t, void *>> free_lists;
  std::unordered_map<void *, Live> live;
  int64_t bytes_held = 0;    // cached blocks and blocks in use from the cache
  int64_t bytes_in_use = 0;  // every block in use, cache or caller's allocator
  bool hook_set = false;
  gift_allocator hook{};
};

Pool &pool() {
  static Pool *p = new Pool();  // outlives static destructors of callers
  return *p;
}

size_t round_size(size_t n) {
  if (n < 256) return 256;
  if (n < (size_t(2) << 20)) return (n + 255) & ~size_t(255);
  return (n + (size_t(2) << 20) - 1) & ~((size_t(2) << 20) - 1);
}

}  // namespace

gift_status dev_alloc(void **p, size_t bytes, hipStream_t s, const char *what) {
  *p = nullptr;
  const size_t need = round_size(bytes == 0 ? 16 : bytes);
  int dev = 0;
  (void)hipGetDevice(&dev);
  Pool &pl = pool();
  gift_allocator hook{};
  bool hooked = false;
  {
    std::lock_guard<std::mutex> lk(pl.m);
    hooked = pl.hook_set;
    hook = pl.hook;
    if (!hooked) {
      auto &fl = pl.free_lists[{dev, s}];
      auto it = fl.lower_bound(need);
      if (it != fl.end() && it->first <= need + need / 4) {
        *p = it->second;
        pl.live[it->second] = Live{it->first, dev, false, {}};
        pl.bytes_in_use += static_cast<int64_t>(it->first);
        fl.erase(it);
        return GIFT_OK;
      }
    }
  }
  if (hooked) {
    // the caller's allocator, called outside the lock
    void *q = hook.alloc(need, dev, s, hook.ctx);
    if (!q)
      return set_error(GIFT_ENOMEM, "the caller's allocator returned NULL for %zu bytes (%s)",
                       need, what);
    std::lock_guard<std::mutex> lk(pl.m);
    pl.live[q] = Live{need, dev, true, hook};
    pl.bytes_in_use += static_cast<int64_t>(need);
    *p = q;
    return GIFT_OK;
  }
  hipError_t e = hipMalloc(p, need);
  if (e != hipSuccess) {
    // drop this device's cached blocks and retry once
    (void)hipGetLastError();
    gift_status st = release_cached(dev);
    if (st != GIFT_OK) return st;
    e = hipMalloc(p, need);
  }
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return set_error(e == hipErrorOutOfMemory ? GIFT_ENOMEM : GIFT_EDEVICE,
                     "device allocation of %zu bytes for %s failed: %s", bytes, what,
                     hipGetErrorString(e));
  }
  std::lock_guard<std::mutex> lk(pl.m);
  pl.live[*p] = Live{need, dev, false, {}};
  pl.bytes_held += static_cast<int64_t>(need);
  pl.bytes_in_use += static_cast<int64_t>(need);
  return GIFT_OK;
}

void dev_free(void *p, hipStream_t s) {
  if (!p) return;
  Pool &pl = pool();
  Live lv{};
  {
    std::lock_guard<std::mutex> lk(pl.m);
    auto it = pl.live.find(p);
    if (it == pl.live.end()) return;
    lv = it->second;
    pl.live.erase(it);
    pl.bytes_in_use -= static_cast<int64_t>(lv.size);
    if (!lv.hooked) {
      pl.free_lists[{lv.device, s}].emplace(lv.size, p);
      return;
    }
  }
  // back to the allocator that provided it, outside the lock
  lv.hook.free(p, lv.size, lv.device, s, lv.hook.ctx);
}

gift_status set_allocator(const gift_allocator *a) {
  Pool &pl = pool();
  std::lock_guard<std::mutex> lk(pl.m);
  if (a) {
    pl.hook = *a;
    pl.hook_set = true;
  } else {
    pl.hook = gift_allocator{};
    pl.hook_set = false;
  }
  return GIFT_OK;
}

gift_status release_cached(int dev) {
  Pool &pl = pool();
  std::vector<void *> drop;
  {
    std::lock_guard<std::mutex> lk(pl.m);
    for (auto it = pl.free_lists.begin(); it != pl.free_lists.end();) {
      if (dev >= 0 && it->first.first != dev) {
        ++it;
        continue;
      }
      for (auto &kv : it->second) {
        drop.push_back(kv.second);
        pl.bytes_held -= static_cast<int64_t>(kv.first);
      }
      it = pl.free_lists.erase(it);
    }
  }
  if (drop.empty()) return GIFT_OK;
  // blocks may still be referenced by queued work on their streams
  GIFT_HIP(hipDeviceSynchronize());
  for (void *q : drop) GIFT_HIP(hipFree(q));
  return GIFT_OK;
}

void pool_stats(int64_t *held, int64_t *in_use) {
  Pool &pl = pool();
  std::lock_guard<std::mutex> lk(pl.m);
  if (held) *held = pl.bytes_held;
  if (in_use) *in_use = pl.bytes_in_use;
}

namespace {
struct ReadbackPool {
  std::mutex m;
  std::map<int, std::vector<Readback>> free;  // per device
};
ReadbackPool &readback_pool() {
  static ReadbackPool *p = new ReadbackPool();
  return *p;
}
}  // namespace

gift_status readback_acquire(Readback *r) {
  int dev = 0;
  GIFT_HIP(hipGetDevice(&dev));
  ReadbackPool &pl = readback_pool();
  {
    std::lock_guard<std::mutex> lk(pl.m);
    auto &fl = pl.free[dev];
    if (!fl.empty()) {
      *r = fl.back();
      fl.pop_back();
      return GIFT_OK;
    }
  }
  Readback n{nullptr, nullptr, nullptr, dev, 0};
  GIFT_HIP(hipHostMalloc(reinterpret_cast<void **>(&n.host), kReadbackSlots * sizeof(int64_t),
                         hipHostMallocCoherent | hipHostMallocPortable));
  n.host[kReadbackFlag] = 0;
  hipError_t e = hipHostGetDevicePointer(reinterpret_cast<void **>(&n.dev), n.host, 0);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&n.done, hipEventDisableTiming);
  if (e != hipSuccess) {
    (void)hipHostFree(n.host);
    (void)hipGetLastError();
    return set_error(GIFT_EDEVICE, "readback event: %s", hipGetErrorString(e));
  }
  *r = n;
  return GIFT_OK;
}

void readback_release(const Readback &r) {
  if (!r.host) return;
  ReadbackPool &pl = readback_pool();
  std::lock_guard<std::mutex> lk(pl.m);
  pl.free[r.device].push_back(r);
}

gift_status readback_wait(const Readback &r, hipStream_t st) {
  GIFT_HIP(hipEventRecord(r.done, st));
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    const hipError_t q = hipEventQuery(r.done);
    if (q == hipSuccess) return GIFT_OK;
    if (q != hipErrorNotReady) {
      (void)hipGetLastError();
      return set_error(GIFT_EDEVICE, "readback: %s", hipGetErrorString(q));
    }
    if (std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(300)) break;
  }
  GIFT_HIP(hipEventSynchronize(r.done));
  return GIFT_OK;
}

namespace {
struct SidePool {
  std::mutex m;
  std::map<int, std::vector<SideStream>> free;  // per device
};
SidePool &side_pool() {
  static SidePool *p = new SidePool();
  return *p;
}
}  // namespace

gift_status side_stream_acquire(SideStream *r) {
  int dev = 0;
  GIFT_HIP(hipGetDevice(&dev));
  SidePool &pl = side_pool();
  {
    std::lock_guard<std::mutex> lk(pl.m);
    auto &fl = pl.free[dev];
    if (!fl.empty()) {
      *r = fl.back();
      fl.pop_back();
      return GIFT_OK;
    }
  }
  SideStream n{nullptr, nullptr, nullptr, dev};
  hipError_t e = hipStreamCreateWithFlags(&n.stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&n.ready, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&n.done, hipEventDisableTiming);
  if (e != hipSuccess) {
    if (n.done) (void)hipEventDestroy(n.done);
    if (n.ready) (void)hipEventDestroy(n.ready);
    if (n.stream) (void)hipStreamDestroy(n.stream);
    (void)hipGetLastError();
    return set_error(GIFT_EDEVICE, "side stream: %s", hipGetErrorString(e));
  }
  *r = n;
  return GIFT_OK;
}

void side_stream_release(const SideStream &r) {
  if (!r.stream) return;
  SidePool &pl = side_pool();
  std::lock_guard<std::mutex> lk(pl.m);
  pl.free[r.device].push_back(r);
}

const SigmaBlock *find_sigma(const gift_graph *g, double sigma) {
  for (const SigmaBlock &b : g->sig)
    if (b.sigma == sigma) return &b;
  return nullptr;
}

}  // namespace gift

using namespace gift;

extern "C" {

const char *gift_status_string(gift_status s) {
  switch (s) {
    case GIFT_OK: return "GIFT_OK";
    case GIFT_EINVAL: return "GIFT_EINVAL: invalid argument";
    case GIFT_ENOMEM: return "GIFT_ENOMEM: out of memory";
    case GIFT_EDEVICE: return "GIFT_EDEVICE: HIP runtime error";
    case GIFT_EUNSUPPORTED: return "GIFT_EUNSUPPORTED: unsupported combination or size";
    case GIFT_EBUSY: return "GIFT_EBUSY: object in use";
  }
  return "unknown gift_status";
}

const char *gift_last_error(void) { return t_last_error.c_str(); }

int32_t gift_abi_version(void) { return GIFT_ABI_VERSION; }

gift_status gift_memory_stats(int64_t *bytes_held, int64_t *bytes_in_use) {
  clear_error();
  pool_stats(bytes_held, bytes_in_use);
  return GIFT_OK;
}

gift_status gift_set_allocator(const gift_allocator *allocator) {
  clear_error();
  if (allocator && (!allocator->alloc || !allocator->free))
    return set_error(GIFT_EINVAL, "gift_set_allocator: alloc and free must both be set");
  return set_allocator(allocator);
}

gift_status gift_release_cached_memory(void) {
  clear_error();
  return release_cached(-1);
}

gift_status gift_graph_get_info(const gift_graph *g, gift_graph_info *info) {
  clear_error();
  if (!g || !info) return set_error(GIFT_EINVAL, "gift_graph_get_info: NULL argument");
  info->num_cells = g->num_cells;
  info->num_virtual = g->num_virtual;
  info->num_rows = g->num_rows;
  info->nnz = g->nnz;
  info->bytes_resident = g->bytes;
  info->storage = g->storage;
  info->num_sigmas = static_cast<int32_t>(g->sig.size());
  return GIFT_OK;
}

gift_status gift_graph_set_tile_class(gift_graph *g, int32_t tile_class) {
  clear_error();
  if (!g) return set_error(GIFT_EINVAL, "gift_graph_set_tile_class: NULL graph");
  if (tile_class < 0 || tile_class >= kTileClasses)
    return set_error(GIFT_EINVAL, "tile_class %d not in [0, %d)", tile_class, kTileClasses);
  g->tile_class = tile_class;
  return GIFT_OK;
}

gift_status gift_graph_export(const gift_graph *g, int64_t *row_ptr, int32_t *col, double *w,
                              double *deg, void *stream) {
  clear_error();
  if (!g) return set_error(GIFT_EINVAL, "gift_graph_export: NULL graph");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (row_ptr) {
    std::vector<int32_t> tmp(static_cast<size_t>(g->num_rows + 1));
    GIFT_HIP(hipMemcpyAsync(tmp.data(), g->row_ptr, tmp.size() * 4, hipMemcpyDeviceToHost, s));
    GIFT_HIP(hipStreamSynchronize(s));
    for (size_t i = 0; i < tmp.size(); ++i) row_ptr[i] = tmp[i];
  }
  if (col && g->nnz)
    GIFT_HIP(hipMemcpyAsync(col, g->col, g->nnz * 4, hipMemcpyDeviceToHost, s));
  if (w && g->nnz) GIFT_HIP(hipMemcpyAsync(w, g->w, g->nnz * 8, hipMemcpyDeviceToHost, s));
  if (deg && g->num_rows)
    GIFT_HIP(hipMemcpyAsync(deg, g->deg, g->num_rows * 8, hipMemcpyDeviceToHost, s));
  GIFT_HIP(hipStreamSynchronize(s));
  return GIFT_OK;
}

gift_status gift_destroy_graph(gift_graph *g, void *stream) {
  clear_error();
  if (!g) return GIFT_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  dev_free(g->row_ptr, s);
  dev_free(g->col, s);
  dev_free(g->w, s);
  dev_free(g->deg, s);
  for (int c = 0; c < kTileClasses; ++c) dev_free(g->tiles[c], s);
  for (SigmaBlock &b : g->sig) {
    dev_free(b.val, s);
    dev_free(b.diag, s);
  }
  delete g;
  return GIFT_OK;
}

}  // extern "C"
