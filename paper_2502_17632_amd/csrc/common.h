// Internal declarations shared by the library's HIP sources.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <type_traits>
#include <vector>

#include "gift.h"

namespace gift {

// ---------------------------------------------------------------------------
// Errors: every entry point returns a status and records a message per host
// thread.
// ---------------------------------------------------------------------------
gift_status set_error(gift_status s, const char *fmt, ...);
void clear_error();

#define GIFT_HIP(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      return ::gift::set_error(e_ == hipErrorOutOfMemory ? GIFT_ENOMEM : GIFT_EDEVICE, \
                               "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                               __FILE__, __LINE__);                                \
  } while (0)

#define GIFT_TRY(expr)                  \
  do {                                  \
    gift_status s_ = (expr);            \
    if (s_ != GIFT_OK) return s_;       \
  } while (0)

// Checks the launch that was just enqueued.
gift_status check_launch(const char *what);

// Brackets the launches made while it is alive with profiler events (when
// the profiler is enabled); `bytes` is their algorithmic traffic.
class ProfScope {
 public:
  ProfScope(hipStream_t s, int cls, double bytes);
  ~ProfScope();
  ProfScope(const ProfScope &) = delete;
  ProfScope &operator=(const ProfScope &) = delete;

 private:
  int idx_;
  hipStream_t stream_;
};

// When the profiler is on, takes a pair of events for one launch of class
// `cls` (to be recorded by the launch itself) and returns true.
bool prof_launch_events(int cls, double bytes, hipEvent_t *start, hipEvent_t *stop);

// Launches kern<<<grid, 256>>>(args...) on `st`; when `timed` and the
// profiler is on, the dispatch itself records the launch's start and end.
template <typename... Args>
gift_status launch_timed(void (*kern)(Args...), unsigned grid, hipStream_t st, bool timed,
                         int cls, double bytes, const char *what, Args... args) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (timed && prof_launch_events(cls, bytes, &e0, &e1))
    hipExtLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, st, e0, e1, 0, args...);
  else
    kern<<<grid, 256, 0, st>>>(args...);
  return check_launch(what);
}

// ---------------------------------------------------------------------------
// Device memory: a stream-ordered caching allocator (see api.hip).  A block
// freed on stream s is reused only by later allocations for stream s.
// ---------------------------------------------------------------------------
gift_status dev_alloc(void **p, size_t bytes, hipStream_t s, const char *what);
void dev_free(void *p, hipStream_t s);
// Returns the cached (free) blocks of device `dev` (all devices if < 0) to
// the runtime; synchronises the device first.
gift_status release_cached(int dev);
// Routes later allocations to the caller's allocator (NULL: the cache).
gift_status set_allocator(const gift_allocator *a);
void pool_stats(int64_t *held, int64_t *in_use);

// Host readback of a few device scalars without a copy: a slot of
// kReadbackSlots int64 values in pinned, host-coherent memory that a kernel
// writes directly, and an event recorded after that kernel.  Slots come from
// a per-device pool (allocated once, kept for the life of the process) and
// are returned with readback_release.  A kernel may also announce its values
// by writing the slot's next ticket into value kReadbackFlag after them.
constexpr int kReadbackSlots = 16;
constexpr int kReadbackFlag = kReadbackSlots - 1;
struct Readback {
  int64_t *host;  // kReadbackSlots values, read by the host
  int64_t *dev;   // the same memory as device code addresses it
  hipEvent_t done;
  int device;
  int64_t ticket;  // the last ticket used with this slot (0: none)
};
gift_status readback_acquire(Readback *r);
void readback_release(const Readback &r);
// Records the event on `st` and waits for it: polls for a short while (the
// usual case: the readback ends a short chain of kernels), then blocks.
gift_status readback_wait(const Readback &r, hipStream_t st);

// Reads `n` (<= kReadScalarsMax) device int64 scalars with one launch and
// one wait on `st`: a kernel writes them straight into a pinned host slot.
constexpr int kReadScalarsMax = 8;
gift_status read_scalars(hipStream_t st, const int64_t *const *ptrs, int n, int64_t *out);

// A second stream (default priority) with two events, for work a call runs
// beside its caller's stream: `ready` is recorded on the caller's stream and
// waited on by `stream`; `done` is free for the caller.  From a per-device
// pool kept for the life of the process.
struct SideStream {
  hipStream_t stream;
  hipEvent_t ready;
  hipEvent_t done;
  int device;
};
gift_status side_stream_acquire(SideStream *s);
void side_stream_release(const SideStream &s);

// RAII holder for build/filter scratch, released in stream order.
struct Scratch {
  hipStream_t stream;
  std::vector<void *> ptrs;
  explicit Scratch(hipStream_t s) : stream(s) {}
  ~Scratch() {
    for (void *p : ptrs) dev_free(p, stream);
  }
  template <typename T>
  gift_status get(T **p, size_t count, const char *what) {
    void *v = nullptr;
    gift_status st = dev_alloc(&v, count * sizeof(T) + 16, stream, what);
    if (st != GIFT_OK) return st;
    ptrs.push_back(v);
    *p = static_cast<T *>(v);
    return GIFT_OK;
  }
};

// ---------------------------------------------------------------------------
// Resident graph.
// ---------------------------------------------------------------------------
// A row tile: rows [r0, r1), stored entries [p0, p1).
struct TileDesc {
  int32_t r0, r1, p0, p1;
};
constexpr int kTileClasses = 2;

struct SigmaBlock {
  double sigma;
  void *val;  // storage type [nnz]: a_ij = (w_ij s_i) s_j
  void *diag; // accumulation type [R]: (sigma s_i) s_i
};

}  // namespace gift

struct gift_graph {
  int64_t num_cells = 0;    // N
  int64_t num_virtual = 0;  // V
  int64_t num_rows = 0;     // R
  int64_t nnz = 0;
  int64_t nnz_cells = 0;     // entries in rows [0, N)
  int32_t storage = GIFT_F32;
  int32_t weight_model = GIFT_W_INV_M1;
  int64_t star_threshold = 0;
  int32_t *row_ptr = nullptr;  // int32[R+1]
  int32_t *col = nullptr;      // int32[nnz]
  double *w = nullptr;         // float64[nnz]
  double *deg = nullptr;       // float64[R]
  std::vector<gift::SigmaBlock> sig;
  int64_t bytes = 0;
  int device = 0;
  // Row tiles of the SpMM for every tile class (see tiles.hip): tiles[c][t]
  // covers rows [r0, r1) and entries [p0, p1); the first num_tiles_cells[c]
  // tiles cover the cell rows [0, N).
  gift::TileDesc *tiles[gift::kTileClasses] = {};
  int64_t num_tiles[gift::kTileClasses] = {};
  int64_t num_tiles_cells[gift::kTileClasses] = {};
  int32_t tile_class = 0;  // class used by gift_filter_placement
};

namespace gift {

inline size_t dtype_size(int32_t d) {
  switch (d) {
    case GIFT_F32: return 4;
    case GIFT_F64: return 8;
    case GIFT_BF16: return 2;
    case GIFT_F16: return 2;
  }
  return 0;
}
inline bool dtype_valid(int32_t d) { return d >= GIFT_F32 && d <= GIFT_F16; }
// Accumulation type of a storage type: float64 for F64, float32 otherwise.
inline size_t accum_size(int32_t storage) { return storage == GIFT_F64 ? 8 : 4; }

const SigmaBlock *find_sigma(const gift_graph *g, double sigma);
gift_status prepare_sigma(gift_graph *g, double sigma, hipStream_t s);

// Exclusive prefix sum: out[0..n] with out[n] = total (int64 output); with
// out32, also a 32-bit copy of out[0..n] (values past 2^31 are not kept).
gift_status scan_i32_to_i64(const int32_t *in, int64_t *out, int64_t n, hipStream_t s,
                            int32_t *out32 = nullptr);
gift_status scan_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t s);

// Row tiles (see tiles.hip): a tile is a single row longer than long_row or
// rows starting in one window of `entries` entries, at most `rows` rows.
struct TileShape {
  int32_t entries, rows, long_row;
};
// The SpMM's tile classes: class 0 stages up to 2303 entries of at most 512
// rows per block, class 1 up to 1151 entries of at most 256 rows.
template <int TC>
struct TileClass;
template <>
struct TileClass<0> {
  static constexpr int kEntries = 2048, kRows = 512, kLong = 256;
  static constexpr int kCap = kEntries + kLong - 1;
};
template <>
struct TileClass<1> {
  static constexpr int kEntries = 1024, kRows = 256, kLong = 128;
  static constexpr int kCap = kEntries + kLong - 1;
};
constexpr TileShape kSpmmTiles[kTileClasses] = {
    {TileClass<0>::kEntries, TileClass<0>::kRows, TileClass<0>::kLong},
    {TileClass<1>::kEntries, TileClass<1>::kRows, TileClass<1>::kLong}};
// Tile descriptors from tile starts (tile_row[0..T]) and 64-bit row offsets.
gift_status tile_descs(const int32_t *tile_row, const int64_t *rp64, int64_t T, hipStream_t st,
                       TileDesc *out);
// tile_row must hold R + 1 entries; counts_dev[0] = number of tiles T,
// counts_dev[1] = tiles that start before row `split`.  With `narrow`, the
// same pass copies off[0..R] to 32 bits (read it only once off[R] < 2^31
// is known).
gift_status build_tiles64(const int64_t *off, int64_t R, int64_t split, TileShape sh,
                          hipStream_t st, int32_t *tile_row, int64_t *counts_dev,
                          int32_t *narrow = nullptr);
// The tiles of two shapes over the same offsets in one pass (one flag
// kernel, one scan, one scatter); the results equal two build_tiles64 calls.
gift_status build_tiles64_pair(const int64_t *off, int64_t R, int64_t split, TileShape s0,
                               TileShape s1, hipStream_t st, int32_t *tile_row0,
                               int32_t *tile_row1, int64_t *counts0, int64_t *counts1);

// ---------------------------------------------------------------------------
// Storage types.  bf16 and f16 are stored as raw 16-bit patterns; values are
// rounded to nearest-even when stored.
// ---------------------------------------------------------------------------
struct bf16 {
  uint16_t bits;
};
struct f16 {
  uint16_t bits;
};

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  return __uint_as_float(static_cast<uint32_t>(h) << 16);
}
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<uint16_t>((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float f16_to_f32(uint16_t h) {
  _Float16 v;
  __builtin_memcpy(&v, &h, 2);
  return static_cast<float>(v);
}
__device__ __forceinline__ uint16_t f32_to_f16(float f) {
  _Float16 v = static_cast<_Float16>(f);
  uint16_t h;
  __builtin_memcpy(&h, &v, 2);
  return h;
}
// float64 -> float32 rounded to odd: exact results stay exact, inexact ones
// get their last bit set.  A second rounding to a format with at least two
// fewer significand bits (bf16, f16) is then correctly rounded.
__device__ __forceinline__ float f64_to_f32_odd(double d) {
  float t = __double2float_rz(d);
  if (static_cast<double>(t) != d) t = __uint_as_float(__float_as_uint(t) | 1u);
  return t;
}

template <int D>
struct Store;
template <>
struct Store<GIFT_F32> {
  using T = float;
  using A = float;
  static __device__ __forceinline__ A load(T v) { return v; }
  static __device__ __forceinline__ T from_acc(A a) { return a; }
  static __device__ __forceinline__ T from_f64(double d) { return static_cast<float>(d); }
};
template <>
struct Store<GIFT_F64> {
  using T = double;
  using A = double;
  static __device__ __forceinline__ A load(T v) { return v; }
  static __device__ __forceinline__ T from_acc(A a) { return a; }
  static __device__ __forceinline__ T from_f64(double d) { return d; }
};
template <>
struct Store<GIFT_BF16> {
  using T = uint16_t;
  using A = float;
  static __device__ __forceinline__ A load(T v) { return bf16_to_f32(v); }
  static __device__ __forceinline__ T from_acc(A a) { return f32_to_bf16(a); }
  static __device__ __forceinline__ T from_f64(double d) { return f32_to_bf16(f64_to_f32_odd(d)); }
};
template <>
struct Store<GIFT_F16> {
  using T = uint16_t;
  using A = float;
  static __device__ __forceinline__ A load(T v) { return f16_to_f32(v); }
  static __device__ __forceinline__ T from_acc(A a) { return f32_to_f16(a); }
  static __device__ __forceinline__ T from_f64(double d) { return f32_to_f16(f64_to_f32_odd(d)); }
};

// Pointers into global memory.  Accesses through a pointer that was loaded
// from a table compile to FLAT instructions unless its address space is
// spelled out; to_global does that.
template <typename T>
using gptr = __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ gptr<T> to_global(T *p) {
  return (gptr<T>)p;
}

// Loads/stores p[i] of a trivially copyable struct through global
// instructions, in the widest words its alignment allows (C++ cannot copy a
// class object out of a qualified address space directly).
template <typename T>
struct GWord {
  typedef uint32_t v4 __attribute__((ext_vector_type(4)));
  typedef uint32_t v2 __attribute__((ext_vector_type(2)));
  using type = std::conditional_t<
      alignof(T) >= 16 && sizeof(T) % 16 == 0, v4,
      std::conditional_t<alignof(T) >= 8 && sizeof(T) % 8 == 0, v2,
                         std::conditional_t<alignof(T) >= 4 && sizeof(T) % 4 == 0, uint32_t,
                                            uint16_t>>>;
  static constexpr int kWords = sizeof(T) / sizeof(type);
  static_assert(sizeof(T) % sizeof(type) == 0, "struct size must be a multiple of 2 bytes");
};
template <typename T>
__device__ __forceinline__ T gload(const T *p, int64_t i) {
  using W = typename GWord<T>::type;
  const gptr<const W> q = to_global(reinterpret_cast<const W *>(p + i));
  W w[GWord<T>::kWords];
#pragma unroll
  for (int k = 0; k < GWord<T>::kWords; ++k) w[k] = q[k];
  T t;
  __builtin_memcpy(&t, w, sizeof(T));
  return t;
}
template <typename T>
__device__ __forceinline__ void gstore(T *p, int64_t i, const T &t) {
  using W = typename GWord<T>::type;
  const gptr<W> q = to_global(reinterpret_cast<W *>(p + i));
  W w[GWord<T>::kWords];
  __builtin_memcpy(w, &t, sizeof(T));
#pragma unroll
  for (int k = 0; k < GWord<T>::kWords; ++k) q[k] = w[k];
}

// Blocks are dispatched round-robin over the 8 XCDs.  Remap logical tiles so
// that every XCD works on chunks of kXcdChunk consecutive tiles (and so of
// rows), the chunks dealt round-robin to the XCDs: the signal rows a tile
// gathers from its neighbourhood are then mostly in its own XCD's L2, while
// a heavy region of the tile list (the star rows at its end) is still spread
// over all XCDs.  Tiles past the last whole round of chunks keep their index.
// A bijection on [0, n) for any n.
constexpr uint32_t kXcds = 8;
constexpr uint32_t kXcdChunk = 64;
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t n) {
  const uint32_t full = n / (kXcds * kXcdChunk) * (kXcds * kXcdChunk);
  if (b >= full) return b;
  const uint32_t x = b % kXcds, i = b / kXcds;
  return ((i / kXcdChunk) * kXcds + x) * kXcdChunk + (i % kXcdChunk);
}

inline unsigned grid_for(int64_t threads, int block = 256) {
  int64_t b = (threads + block - 1) / block;
  if (b < 1) b = 1;
  return static_cast<unsigned>(b);
}

}  // namespace gift
