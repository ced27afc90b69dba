// Netlist -> resident normalised cell graph.
//
// Clique net model (Section 3.2, the paragraph after Algorithm 1): a net of M
// distinct cells adds w(M) to every ordered pair of its cells, w(M) = 1/(M-1)
// or 2/M (Section 2.2, eq. wire_eq).  Nets with more than T cells may instead
// become a star around a virtual node with weight M w(M).  Parallel edges are
// summed (A is a weight sum, Section 2.1), degrees d_i = sum_j w_ij, and for
// every self-loop weight sigma the entries of
// A~_sigma = (D + sigma I)^-1/2 (A + sigma I) (D + sigma I)^-1/2
// (eq. A_formulation) are rounded once to the storage type.
//
// Pipeline (device work on the caller's stream and on a pooled side stream
// that it forks to and joins with events):
//   0. check net_ptr; tile the nets (consecutive nets, about a thousand pins
//      per tile, long nets alone)
//   1. per net tile, in LDS: distinct cells of every net, ascending (rank of
//      each pin among the net's first occurrences); long nets by a block-wide
//      bitonic sort in LDS or a merge sort through global memory.  The same
//      kernel counts the directed entries of every cell row: one atomic add
//      per distinct (net, cell), whose old value is the slice of that cell's
//      entries from this net within the row (arbitrary order of the slices;
//      the atomics overlap the LDS work of the net tiles)
//   2. per net: clique or star, weight; the star nets' virtual rows in
//      ascending order of their median cell (then net id), by bucketing on
//      the median and sorting each bucket in one block
//   3. exclusive scan of the row counts -> row slices and row tiles (side
//      stream, beside step 2); emit each pin's (col, net) keys into its slice
//   4. per row tile, in LDS: sort each row's keys by (col, net) (rank among
//      the row's keys, which are distinct), count distinct columns.  The
//      sorted order fixes every summation order below, so the result does
//      not depend on the emission order
//   5. scan of distinct counts -> row_ptr; the SpMM row tiles of both
//      classes in one pass (side stream, beside step 6)
//   6. per row tile, in LDS: merge runs of equal col (weights summed in
//      ascending net id, float64), write col / w, degree summed in ascending
//      col; star rows copy the net's sorted cells with weight M w(M) (side
//      stream)
//   7. per sigma: s_i = 1/sqrt(d_i + sigma), a_ij = (w_ij s_i) s_j,
//      diag_i = (sigma s_i) s_i
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>

#include "common.h"
#include "devutil.h"

namespace gift {
namespace {

enum : uint32_t { kFlagBadNetPtr = 1u, kFlagBadPin = 2u };

// Tiles of the build kernels: smaller than the SpMM's so that the LDS each
// block stages (keys, offsets, segment ids, merged weights) stays small and
// many blocks share a CU.
constexpr int kBTileEntries = 1024;
constexpr int kBTileRows = 256;
constexpr int kBLongRow = 128;
constexpr int kBTileCap = kBTileEntries + kBLongRow - 1;
constexpr TileShape kBuildTiles{kBTileEntries, kBTileRows, kBLongRow};
constexpr int kNetSortCap = 2048;  // longest net sorted in LDS (32-bit keys, 8 KB)
constexpr int kRowSortCap = 2048;  // longest row sorted in LDS (64-bit keys, 16 KB)
constexpr int kChunk32 = 2048;     // LDS chunk of the global merge sort (u32)
constexpr int kChunk64 = 2048;     // LDS chunk of the global merge sort (u64)
// Items per thread when a block stages a tile's offsets (up to kBTileRows + 1),
// its entries (up to kBTileCap) or a long row (up to 2048) into LDS.  Each
// thread issues all its loads before its first store, so a block waits for
// one memory latency instead of one per item.
constexpr int kOffItems = (kBTileRows + 1 + kBlock - 1) / kBlock;
constexpr int kTileItems = (kBTileCap + kBlock - 1) / kBlock;
constexpr int kLongItems = 2048 / kBlock;
static_assert(kNetSortCap <= kLongItems * kBlock && kRowSortCap <= kLongItems * kBlock,
              "long rows staged in one pass");

__device__ __forceinline__ double clique_weight(int64_t m, int model) {
  return model == GIFT_W_TWO_OVER_M ? 2.0 / static_cast<double>(m)
                                    : 1.0 / static_cast<double>(m - 1);
}
__device__ __forceinline__ double star_weight(int64_t m, int model) {
  return model == GIFT_W_TWO_OVER_M ? 2.0
                                    : static_cast<double>(m) / static_cast<double>(m - 1);
}

// An emitted entry is one 64-bit key: its column in the high bits, the net
// in the middle and, when the three fit, the net's distinct cell count M in
// the low bits (the merge then derives the weight from M instead of reading
// it per net).  Sorting keys sorts by (column, net): a row never holds two
// keys of one (column, net).
struct KeyLayout {
  int32_t col_shift;  // column = key >> col_shift
  int32_t net_shift;  // net = (key >> net_shift) & net_mask
  uint64_t net_mask;
  uint64_t m_mask;    // M = key & m_mask; 0 when M is not in the key
};
__device__ __forceinline__ uint32_t key_col(uint64_t k, const KeyLayout &L) {
  return static_cast<uint32_t>(k >> L.col_shift);
}
__device__ __forceinline__ uint32_t key_net(uint64_t k, const KeyLayout &L) {
  return static_cast<uint32_t>((k >> L.net_shift) & L.net_mask);
}

int bits_for(int64_t v) {  // bits to hold 0..v
  int b = 1;
  while (b < 63 && (int64_t(1) << b) <= v) ++b;
  return b;
}

// The widest layout that fits: M packed when bits(max column) + bits(max
// net) + bits(max M) <= 64, else column and net in 32 bits each.
KeyLayout key_layout(int64_t max_col, int64_t max_net, int64_t max_m) {
  const int cb = bits_for(max_col), nb = bits_for(max_net), mb = bits_for(max_m);
  if (cb + nb + mb <= 64)
    return KeyLayout{nb + mb, mb, (uint64_t(1) << nb) - 1, (uint64_t(1) << mb) - 1};
  return KeyLayout{32, 0, 0xffffffffull, 0};
}

// ---------------------------------------------------------------------------
// 0. netlist checks
// ---------------------------------------------------------------------------
// net_ptr must start at 0 and not decrease (so it ends at the pin count,
// which is read back with this flag).
__global__ void k_check_netptr(const int64_t *net_ptr, int64_t E, uint32_t *flag) {
  int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e > E) return;
  const int64_t v = net_ptr[e];
  bool bad = v < 0 || (e == 0 && v != 0) || (e < E && net_ptr[e + 1] < v);
  if (bad) atomicOr(flag, kFlagBadNetPtr);
}

// ---------------------------------------------------------------------------
// 1. distinct cells of each net
// ---------------------------------------------------------------------------
struct NetArgs {
  const int64_t *net_ptr;
  const int32_t *pin;
  int64_t E, P, N;
  int32_t *M;        // distinct cells per net
  int32_t *ucell;    // sorted distinct cells at the net's pin offset
  int32_t *pin_net;  // net of every pin slot
  uint32_t *flag;
  uint32_t *tmp32;   // scratch of the global merge sort [P]
  const TileDesc *tiles;  // nets [r0, r1), pins [p0, p1) of every tile
  int64_t T;         // star threshold (0: no stars)
  int32_t *cnt;      // entries per cell row (zeroed before the launch)
  int32_t *slot;     // per distinct-cell slot: its slice start within the row
};

// Entries a net of m distinct cells adds to each of its cells' rows: m - 1
// for a clique, 1 (the virtual node) for a star, none for m < 2.
__device__ __forceinline__ int32_t row_entries(int64_t m, int64_t T) {
  if (m < 2) return 0;
  return (T > 0 && m > T) ? 1 : static_cast<int32_t>(m - 1);
}

// Reserves the slice of cell c's entries from a net of m distinct cells in
// row c; q is the cell's slot in ucell.  Cells outside [0, N) were flagged
// and get no slice (the build fails on the flag).
__device__ __forceinline__ void reserve_slice(const NetArgs &a, int64_t q, int32_t c, int64_t m) {
  const int32_t k = row_entries(m, a.T);
  if (k > 0 && c >= 0 && c < a.N) a.slot[q] = atomicAdd(&a.cnt[c], k);
}

// Writes the distinct values of the sorted keys src[0..n) to out[0..) and
// returns their count.  Force-inlined at call sites whose `src` is known to be
// LDS or global memory: a single pointer that may be either would make the
// compiler address LDS through FLAT instructions.
__device__ __forceinline__ int64_t write_distinct(const uint32_t *src, int64_t n, int32_t *out,
                                                  int32_t *tmp) {
  int64_t base = 0;
  for (int64_t c0 = 0; c0 < n; c0 += kBlock) {
    const int64_t i = c0 + threadIdx.x;
    int f = 0;
    if (i < n) f = (i == 0 || src[i] != src[i - 1]) ? 1 : 0;
    int32_t total;
    const int32_t pos = block_excl_scan<int32_t>(f, &total, tmp);
    if (f) out[base + pos] = static_cast<int32_t>(src[i]);
    base += total;
  }
  return base;
}

// A net longer than kBLongRow pins, alone in its tile.
__device__ __forceinline__ void net_long(const NetArgs &a, int64_t e, int64_t lo, int64_t n,
                                         unsigned char *smem) {
  uint32_t *keys = reinterpret_cast<uint32_t *>(smem);
  __shared__ int bad_s;
  __shared__ int32_t tmp[kBlock / kWave];
  if (threadIdx.x == 0) bad_s = 0;
  __syncthreads();
  int64_t m;
  if (n <= kNetSortCap) {
    const int np = next_pow2_i(static_cast<int>(n));
    int32_t c[kLongItems];
#pragma unroll
    for (int k = 0; k < kLongItems; ++k) {
      const int i = threadIdx.x + k * kBlock;
      c[k] = i < n ? a.pin[lo + i] : 0;
    }
#pragma unroll
    for (int k = 0; k < kLongItems; ++k) {
      const int i = threadIdx.x + k * kBlock;
      if (i < n) {
        a.pin_net[lo + i] = static_cast<int32_t>(e);
        if (c[k] < 0 || c[k] >= a.N) bad_s = 1;
      }
      if (i < np) keys[i] = i < n ? static_cast<uint32_t>(c[k]) : 0xffffffffu;
    }
    __syncthreads();
    lds_bitonic_sort<uint32_t>(keys, np);
    m = write_distinct(keys, n, a.ucell + lo, tmp);
  } else {
    uint32_t *ka = reinterpret_cast<uint32_t *>(a.ucell) + lo, *kb = a.tmp32 + lo;
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
      const int32_t c = a.pin[lo + i];
      a.pin_net[lo + i] = static_cast<int32_t>(e);
      if (c < 0 || c >= a.N) bad_s = 1;
      ka[i] = static_cast<uint32_t>(c);
    }
    __syncthreads();
    if (!block_merge_sort_global<uint32_t, kChunk32>(ka, kb, n, keys, 0xffffffffu)) {
      for (int64_t i = threadIdx.x; i < n; i += kBlock) kb[i] = ka[i];
      __syncthreads();
    }
    m = write_distinct(kb, n, a.ucell + lo, tmp);
  }
  if (threadIdx.x == 0) {
    a.M[e] = static_cast<int32_t>(m);
    if (bad_s) atomicOr(a.flag, kFlagBadPin);
  }
  // the distinct cells this block just wrote (visible to it after the
  // barrier)
  __syncthreads();
  for (int64_t i = threadIdx.x; i < m; i += kBlock) reserve_slice(a, lo + i, a.ucell[lo + i], m);
}

constexpr int kNetSmem = 10 * 1024;
static_assert((kBTileCap + 1) * 4 + (kBTileRows + 2) * 4 + (kBTileCap + 1) * 2 + kBTileCap <= kNetSmem,
              "net tile LDS");
static_assert(kNetSortCap * 4 <= kNetSmem && kChunk32 * 4 <= kNetSmem, "long net LDS");

__global__ __launch_bounds__(kBlock) void k_net_tiles(NetArgs a) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[kNetSmem];
  __shared__ int32_t mloc[kBTileRows];
  __shared__ int bad_s;
  const TileDesc td = a.tiles[blockIdx.x];
  const int64_t e0 = td.r0, e1 = td.r1, q0 = td.p0, q1 = td.p1;
  const int ns = static_cast<int>(e1 - e0);
  const int64_t n64 = q1 - q0;
  if (ns == 1 && n64 > kBLongRow) {
    net_long(a, e0, q0, n64, smem);
    return;
  }
  const int n = static_cast<int>(n64);  // <= kBTileCap
  uint32_t *key = reinterpret_cast<uint32_t *>(smem);
  int32_t *loff = reinterpret_cast<int32_t *>(key + kBTileCap + 1);
  uint16_t *seg = reinterpret_cast<uint16_t *>(loff + kBTileRows + 2);
  uint8_t *first = reinterpret_cast<uint8_t *>(seg + kBTileCap + 1);
  if (threadIdx.x == 0) bad_s = 0;
  __syncthreads();
  {
    int64_t o[kOffItems];
    int32_t c[kTileItems];
#pragma unroll
    for (int k = 0; k < kOffItems; ++k) {
      const int i = threadIdx.x + k * kBlock;
      o[k] = i <= ns ? a.net_ptr[e0 + i] : q0;
    }
#pragma unroll
    for (int k = 0; k < kTileItems; ++k) {
      const int i = threadIdx.x + k * kBlock;
      c[k] = i < n ? a.pin[q0 + i] : 0;
    }
#pragma unroll
    for (int k = 0; k < kOffItems; ++k) {
      const int i = threadIdx.x + k * kBlock;
      if (i <= ns) loff[i] = static_cast<int32_t>(o[k] - q0);
    }
#pragma unroll
    for (int k = 0; k < kTileItems; ++k) {
      const int i = threadIdx.x + k * kBlock;
      if (i < n) {
        if (c[k] < 0 || c[k] >= a.N) bad_s = 1;
        key[i] = static_cast<uint32_t>(c[k]);
      }
    }
  }
  __syncthreads();
  fill_segment_ids(loff, ns, seg);
  __syncthreads();
  // (both loops take four pins per step, so four LDS reads are in flight
  // per wait)
  for (int i = threadIdx.x; i < n; i += kBlock) {
    const int k = seg[i];
    a.pin_net[q0 + i] = static_cast<int32_t>(e0 + k);
    const uint32_t me = key[i];
    bool f = true;
    int j = loff[k];
    for (; j + 4 <= i; j += 4)
      f = f & (key[j] != me) & (key[j + 1] != me) & (key[j + 2] != me) & (key[j + 3] != me);
    for (; j < i; ++j) f = f & (key[j] != me);
    first[i] = f ? 1 : 0;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < ns; k += kBlock) {
    int m = 0;
    for (int i = loff[k]; i < loff[k + 1]; ++i) m += first[i];
    a.M[e0 + k] = m;
    mloc[k] = m;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += kBlock) {
    if (!first[i]) continue;
    const int k = seg[i];
    const uint32_t me = key[i];
    int ur = 0;
    int j = loff[k];
    const int end = loff[k + 1];
    for (; j + 4 <= end; j += 4)
      ur += ((first[j] != 0) & (key[j] < me)) + ((first[j + 1] != 0) & (key[j + 1] < me)) +
            ((first[j + 2] != 0) & (key[j + 2] < me)) + ((first[j + 3] != 0) & (key[j + 3] < me));
    for (; j < end; ++j) ur += (first[j] && key[j] < me) ? 1 : 0;
    const int64_t q = q0 + loff[k] + ur;
    a.ucell[q] = static_cast<int32_t>(me);
    reserve_slice(a, q, static_cast<int32_t>(me), mloc[k]);
  }
  if (threadIdx.x == 0 && bad_s) atomicOr(a.flag, kFlagBadPin);
}

// ---------------------------------------------------------------------------
// 2. classify nets
// ---------------------------------------------------------------------------
// Labels of the virtual rows: row N + v for the v-th star net in ascending
// order of (median cell, net id), the median being the distinct cell at
// index M/2 of the net's ascending list.  Neighbouring virtual rows then
// gather from neighbouring cells, and a filter pass's tiles of virtual rows
// read a few lines of the signal instead of lines from all over it.  The
// classification writes each star net's key and counts it in its median
// bucket (2^kStarShift cells per bucket); the keys are then placed in their
// buckets and every bucket is sorted by one block (step 2b).
constexpr int kStarShift = 12;

struct StarKeys {
  const int64_t *net_ptr;
  const int32_t *ucell;
  uint64_t *key;  // per net: (median << 32 | e), star nets only
  int32_t *bcnt;  // star nets per median bucket (zeroed before)
};

__device__ __forceinline__ void star_key(const StarKeys &sk, int64_t e, int64_t m) {
  const int32_t med = sk.ucell[sk.net_ptr[e] + m / 2];
  sk.key[e] = (static_cast<uint64_t>(med) << 32) | static_cast<uint32_t>(e);
  atomicAdd(sk.bcnt + (med >> kStarShift), 1);
}

// Per net: star or clique and weight, the star net's label key (above); per
// block the largest net size into bmax[blockIdx.x] and the star nets' cells
// (the star rows' entries) into bstar[blockIdx.x] (one atomic per block on a
// single word would serialise thousands of blocks at the memory side).
__global__ __launch_bounds__(kBlock) void k_classify(const int32_t *M, int64_t E, int64_t T,
                                                     int model, int32_t *is_star, double *wnet,
                                                     int32_t *bmax, int64_t *bstar,
                                                     StarKeys sk) {
  __shared__ int32_t red[kBlock];
  __shared__ int64_t tmp[kBlock / kWave];
  int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  int32_t mine = 0;
  int64_t star_m = 0;
  if (e < E) {
    int64_t m = M[e];
    bool star = m >= 2 && T > 0 && m > T;
    is_star[e] = star ? 1 : 0;
    wnet[e] = m < 2 ? 0.0 : (star ? star_weight(m, model) : clique_weight(m, model));
    mine = static_cast<int32_t>(m);
    if (star) {
      star_key(sk, e, m);
      star_m = m;
    }
  }
  const int64_t stars = block_sum<int64_t>(star_m, tmp);
  red[threadIdx.x] = mine;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off && red[threadIdx.x + off] > red[threadIdx.x])
      red[threadIdx.x] = red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    bmax[blockIdx.x] = red[0];
    bstar[blockIdx.x] = stars;
  }
}

// out[0] = max of v[0..n), out[1] = sum of w[0..n), one block (integers, so
// the order does not matter).  Each thread has kU loads of each array in
// flight per step instead of waiting for every load in turn.
__global__ __launch_bounds__(kBlock) void k_max_reduce(const int32_t *v, const int64_t *w,
                                                       int64_t n, int64_t *out) {
  constexpr int kU = 8;
  __shared__ int32_t red[kBlock];
  __shared__ int64_t tmp[kBlock / kWave];
  int32_t m = 0;
  int64_t sum = 0;
  int64_t i = threadIdx.x;
  for (; i + (kU - 1) * kBlock < n; i += kU * kBlock) {
    int32_t vv[kU];
    int64_t ww[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      vv[u] = v[i + u * kBlock];
      ww[u] = w[i + u * kBlock];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      m = vv[u] > m ? vv[u] : m;
      sum += ww[u];
    }
  }
  for (; i < n; i += kBlock) {
    m = v[i] > m ? v[i] : m;
    sum += w[i];
  }
  const int64_t total = block_sum<int64_t>(sum, tmp);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off && red[threadIdx.x + off] > red[threadIdx.x])
      red[threadIdx.x] = red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = red[0];
    out[1] = total;
  }
}

// ---------------------------------------------------------------------------
// 2b. labels of the virtual rows (see step 2)
// ---------------------------------------------------------------------------
// The star nets' keys into their buckets' ranges (in any order within a
// bucket).
__global__ void k_star_scatter(const int32_t *is_star, const uint64_t *skey, int64_t E,
                               const int64_t *boff, int32_t *bfill, uint64_t *bkey) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= E || !is_star[e]) return;
  const uint64_t k = skey[e];
  const int64_t b = static_cast<int64_t>(k >> (32 + kStarShift));
  bkey[boff[b] + atomicAdd(bfill + b, 1)] = k;
}

// Block b sorts bucket b (keys are distinct, so the order is unique) and
// labels its nets: virt_net[v] = e and vrow[e] = v; the star row N + v has
// one entry per distinct cell of net e, so its distinct count is M[e].
__global__ __launch_bounds__(kBlock) void k_star_sort(uint64_t *bkey, uint64_t *btmp,
                                                      const int64_t *boff, int32_t *virt_net,
                                                      int32_t *vrow, const int32_t *M,
                                                      int64_t N, int32_t *ucnt) {
  __shared__ uint64_t lds[kChunk64];
  const int64_t lo = boff[blockIdx.x], n = boff[blockIdx.x + 1] - lo;
  if (n == 0) return;
  const bool in_tmp =
      block_merge_sort_global<uint64_t, kChunk64>(bkey + lo, btmp + lo, n, lds, ~0ull);
  const uint64_t *sorted = (in_tmp ? btmp : bkey) + lo;
  for (int64_t i = threadIdx.x; i < n; i += kBlock) {
    const int32_t e = static_cast<int32_t>(sorted[i] & 0xffffffffu);
    virt_net[lo + i] = e;
    vrow[e] = static_cast<int32_t>(lo + i);
    ucnt[N + lo + i] = M[e];
  }
}

// ---------------------------------------------------------------------------
// 3. count and emit the directed entries of cell rows
// ---------------------------------------------------------------------------
struct EmitArgs {
  const int64_t *net_ptr;
  const int32_t *ucell, *pin_net, *M, *is_star;
  const int32_t *vrow;  // virtual row label of each star net
  int64_t E, P, N;
  KeyLayout L;
};

// Writes each pin's (col, net) keys into the slice k_net_tiles reserved.  The
// block's 256 pins first publish their slices in LDS (start, length, net,
// position in the net); then the block's threads take the keys one each,
// in slice order, so consecutive threads write consecutive addresses of a
// slice instead of every thread looping over its own slice.
__global__ __launch_bounds__(kBlock) void k_emit(EmitArgs a, const int32_t *zoff,
                                                 const int32_t *slot, uint64_t *zkey) {
  __shared__ int32_t first[kBlock + 1];  // exclusive prefix of the keys per pin
  __shared__ int64_t dst[kBlock];        // first key of the pin's slice in zkey
  __shared__ int64_t lo_of[kBlock];      // first pin of the pin's net
  __shared__ int64_t net_of[kBlock];
  __shared__ int32_t self_of[kBlock];    // the pin's index in its net; -1: star
  __shared__ int32_t m_of[kBlock];
  __shared__ int32_t tmp[kBlock / kWave];
  const int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  int32_t n = 0;
  if (p < a.P) {
    const int64_t e = a.pin_net[p];
    const int64_t lo = a.net_ptr[e];
    const int64_t i = p - lo;
    const int64_t m = a.M[e];
    if (m >= 2 && i < m) {
      const bool star = a.is_star[e] != 0;
      n = star ? 1 : static_cast<int32_t>(m - 1);
      dst[threadIdx.x] = static_cast<int64_t>(zoff[a.ucell[p]]) + slot[p];
      lo_of[threadIdx.x] = star ? a.N + a.vrow[e] : lo;
      net_of[threadIdx.x] = e;
      self_of[threadIdx.x] = star ? -1 : static_cast<int32_t>(i);
      m_of[threadIdx.x] = static_cast<int32_t>(m);
    }
  }
  int32_t total = 0;
  first[threadIdx.x] = block_excl_scan<int32_t>(n, &total, tmp);
  if (threadIdx.x == 0) first[kBlock] = total;
  __syncthreads();
  for (int32_t q = threadIdx.x; q < total; q += kBlock) {
    int lo = 0, hi = kBlock;  // last pin t with first[t] <= q
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (first[mid] <= q) lo = mid;
      else hi = mid;
    }
    const int t = lo;
    const int32_t idx = q - first[t];
    const uint64_t tail = (static_cast<uint64_t>(net_of[t]) << a.L.net_shift) |
                          (a.L.m_mask ? static_cast<uint64_t>(m_of[t]) : 0);
    uint64_t col;
    if (self_of[t] < 0) {
      col = static_cast<uint64_t>(lo_of[t]);  // the star's virtual node
    } else {
      const int32_t j = idx + (idx >= self_of[t] ? 1 : 0);
      col = static_cast<uint32_t>(a.ucell[lo_of[t] + j]);
    }
    zkey[dst[t] + idx] = (col << a.L.col_shift) | tail;
  }
}

// ---------------------------------------------------------------------------
// 4. sort each cell row's keys by (col, net); count distinct columns
// ---------------------------------------------------------------------------
struct RowArgs {
  const int64_t *zoff;
  uint64_t *zkey;   // emitted keys (also scratch of the global merge sort)
  uint64_t *zsort;  // sorted keys
  int32_t *ucnt;    // distinct columns per row
  const TileDesc *tiles;  // rows [r0, r1), emitted keys [p0, p1) of every tile
  KeyLayout L;
};

__device__ int32_t count_heads_block(const uint64_t *k, int64_t n, int32_t *tmp,
                                     const KeyLayout &L) {
  int32_t heads = 0;
  for (int64_t i = threadIdx.x; i < n; i += kBlock)
    if (i == 0 || key_col(k[i], L) != key_col(k[i - 1], L)) ++heads;
  return block_sum<int32_t>(heads, tmp);
}

constexpr int kSortSmem = 16 * 1024;
static_assert((kBTileCap + 1) * 8 + (kBTileRows + 2) * 4 + (kBTileCap + 1) * 2 + kBTileCap <=
                  kSortSmem,
              "row sort LDS");
static_assert(kRowSortCap * 8 <= kSortSmem && kChunk64 * 8 <= kSortSmem, "long row LDS");

__global__ __launch_bounds__(kBlock) void k_row_sort_tiles(RowArgs a) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[kSortSmem];
  __shared__ int32_t tmp[kBlock / kWave];
  const TileDesc td = a.tiles[blockIdx.x];
  const int64_t r0 = td.r0, r1 = td.r1, z0 = td.p0, z1 = td.p1;
  const int ns = static_cast<int>(r1 - r0);
  const int64_t n64 = z1 - z0;
  if (ns == 1 && n64 > kBLongRow) {
    uint64_t *keys = reinterpret_cast<uint64_t *>(smem);
    int32_t total;
    if (n64 <= kRowSortCap) {
      const int np = next_pow2_i(static_cast<int>(n64));
      uint64_t v[kLongItems];
#pragma unroll
      for (int k = 0; k < kLongItems; ++k) {
        const int i = threadIdx.x + k * kBlock;
        v[k] = i < n64 ? a.zkey[z0 + i] : ~0ull;
      }
#pragma unroll
      for (int k = 0; k < kLongItems; ++k) {
        const int i = threadIdx.x + k * kBlock;
        if (i < np) keys[i] = v[k];
      }
      __syncthreads();
      lds_bitonic_sort<uint64_t>(keys, np);
      for (int i = threadIdx.x; i < n64; i += kBlock) a.zsort[z0 + i] = keys[i];
      total = count_heads_block(keys, n64, tmp, a.L);
    } else {
      uint64_t *ka = a.zkey + z0, *kb = a.zsort + z0;
      if (!block_merge_sort_global<uint64_t, kChunk64>(ka, kb, n64, keys, ~0ull)) {
        for (int64_t i = threadIdx.x; i < n64; i += kBlock) kb[i] = ka[i];
        __syncthreads();
      }
      total = count_heads_block(kb, n64, tmp, a.L);
    }
    if (threadIdx.x == 0) a.ucnt[r0] = total;
    return;
  }
  const int n = static_cast<int>(n64);
  uint64_t *key = reinterpret_cast<uint64_t *>(smem);
  int32_t *loff = reinterpret_cast<int32_t *>(key + kBTileCap + 1);
  uint16_t *seg = reinterpret_cast<uint16_t *>(loff + kBTileRows + 2);
  uint8_t *head = reinterpret_cast<uint8_t *>(seg + kBTileCap + 1);
  {
    int64_t o[kOffItems];
    uint64_t v[kTileItems];
#pragma unroll
    for (int k = 0; k < kOffItems; ++k) {
      const int i = threadIdx.x + k * kBlock;
      o[k] = i <= ns ? a.zoff[r0 + i] : z0;
    }
#pragma unroll
    for (int k = 0; k < kTileItems; ++k) {
      const int i = threadIdx.x + k * kBlock;
      v[k] = i < n ? a.zkey[z0 + i] : 0;
    }
#pragma unroll
    for (int k = 0; k < kOffItems; ++k) {
      const int i = threadIdx.x + k * kBlock;
      if (i <= ns) loff[i] = static_cast<int32_t>(o[k] - z0);
    }
#pragma unroll
    for (int k = 0; k < kTileItems; ++k) {
      const int i = threadIdx.x + k * kBlock;
      if (i < n) key[i] = v[k];
    }
  }
  __syncthreads();
  fill_segment_ids(loff, ns, seg);
  __syncthreads();
  // rank of each key in its row (keys of a row are distinct).  The keys of
  // the same column that sort before me lie in [first_of_col, me), so the
  // key heads its column exactly when as many keys sort below first_of_col
  // as below me (four keys per step, so four LDS reads are in flight per
  // wait)
  for (int i = threadIdx.x; i < n; i += kBlock) {
    const int k = seg[i];
    const uint64_t me = key[i];
    const uint64_t col_lo = (me >> a.L.col_shift) << a.L.col_shift;
    int rank = 0, below = 0;
    int j = loff[k];
    const int end = loff[k + 1];
    for (; j + 4 <= end; j += 4) {
      const uint64_t o0 = key[j], o1 = key[j + 1], o2 = key[j + 2], o3 = key[j + 3];
      rank += (o0 < me ? 1 : 0) + (o1 < me ? 1 : 0) + (o2 < me ? 1 : 0) + (o3 < me ? 1 : 0);
      below += (o0 < col_lo ? 1 : 0) + (o1 < col_lo ? 1 : 0) + (o2 < col_lo ? 1 : 0) +
               (o3 < col_lo ? 1 : 0);
    }
    for (; j < end; ++j) {
      const uint64_t o = key[j];
      rank += o < me ? 1 : 0;
      below += o < col_lo ? 1 : 0;
    }
    a.zsort[z0 + loff[k] + rank] = me;
    head[i] = rank == below ? 1 : 0;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < ns; k += kBlock) {
    int h = 0;
    for (int i = loff[k]; i < loff[k + 1]; ++i) h += head[i];
    a.ucnt[r0 + k] = h;
  }
}




// ---------------------------------------------------------------------------
// 6. merge into the CSR of A, degrees
// ---------------------------------------------------------------------------
struct MergeArgs {
  const int64_t *zoff;
  const uint64_t *zsort;
  const double *wnet;
  const int32_t *row_ptr;
  const TileDesc *tiles;  // as in the row sort
  int32_t *col;
  double *w;
  double *deg;
  KeyLayout L;
  int64_t N;
  int32_t model;
};

// Weight one key adds: from the M packed in the key (a column >= N is a star
// node: weight M w(M)), else the net's weight.
__device__ __forceinline__ double key_weight(uint64_t k, const MergeArgs &a) {
  if (a.L.m_mask) {
    const int64_t m = static_cast<int64_t>(k & a.L.m_mask);
    return static_cast<int64_t>(key_col(k, a.L)) >= a.N ? star_weight(m, a.model)
                                                        : clique_weight(m, a.model);
  }
  return a.wnet[key_net(k, a.L)];
}

// Weight of the run of equal columns starting at sorted entry i (ascending
// net id), reading the keys from `k` (length n).
__device__ __forceinline__ double run_weight(const uint64_t *k, int64_t i, int64_t n,
                                             const MergeArgs &a) {
  const uint32_t c = key_col(k[i], a.L);
  double s = key_weight(k[i], a);
  for (int64_t j = i + 1; j < n && key_col(k[j], a.L) == c; ++j) s = s + key_weight(k[j], a);
  return s;
}

constexpr int kMergeSmem = 14 * 1024;
static_assert((kBTileCap + 1) * 8 + 2 * (kBTileRows + 2) * 4 + (kBTileCap + 1) * 2 <= kMergeSmem,
              "row merge LDS");

__global__ __launch_bounds__(kBlock) void k_row_merge_tiles(MergeArgs a) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[kMergeSmem];
  // merged columns of a short-row tile, written out coalesced with the
  // weights
  __shared__ int32_t mcol[kBTileCap + 1];
  __shared__ int32_t tmp[kBlock / kWave];
  const TileDesc td = a.tiles[blockIdx.x];
  const int64_t r0 = td.r0, r1 = td.r1, z0 = td.p0, z1 = td.p1;
  const int ns = static_cast<int>(r1 - r0);
  const int64_t n64 = z1 - z0;
  const int64_t o0 = a.row_ptr[r0];
  if (ns == 1 && n64 > kBLongRow) {
    // one long row: chunks of kBlock keys straight from global memory
    const uint64_t *k = a.zsort + z0;
    double *mw = reinterpret_cast<double *>(smem);
    int64_t base = 0;
    for (int64_t c0 = 0; c0 < n64; c0 += kBlock) {
      const int64_t i = c0 + threadIdx.x;
      const int f =
          (i < n64 && (i == 0 || key_col(k[i], a.L) != key_col(k[i - 1], a.L))) ? 1 : 0;
      int32_t total;
      const int32_t pos = block_excl_scan<int32_t>(f, &total, tmp);
      if (f) {
        a.col[o0 + base + pos] = static_cast<int32_t>(key_col(k[i], a.L));
        a.w[o0 + base + pos] = run_weight(k, i, n64, a);
      }
      base += total;
    }
    __syncthreads();
    // degree: ascending column, staged through LDS in chunks
    double d = 0.0;
    constexpr int kChunk = kMergeSmem / 8;
    for (int64_t c0 = 0; c0 < base; c0 += kChunk) {
      const int len = static_cast<int>(base - c0 < kChunk ? base - c0 : kChunk);
      for (int i = threadIdx.x; i < len; i += kBlock) mw[i] = a.w[o0 + c0 + i];
      __syncthreads();
      if (threadIdx.x == 0)
        for (int i = 0; i < len; ++i) d = d + mw[i];
      __syncthreads();
    }
    if (threadIdx.x == 0) a.deg[r0] = d;
    return;
  }
  const int n = static_cast<int>(n64);
  uint64_t *key = reinterpret_cast<uint64_t *>(smem);
  // the merged weights replace the keys once every thread has read them
  double *mw = reinterpret_cast<double *>(key);
  int32_t *loff = reinterpret_cast<int32_t *>(key + kBTileCap + 1);
  int32_t *moff = loff + kBTileRows + 2;
  uint16_t *seg = reinterpret_cast<uint16_t *>(moff + kBTileRows + 2);
  {
    int64_t o[kOffItems];
    int32_t m[kOffItems];
    uint64_t v[kTileItems];
#pragma unroll
    for (int k = 0; k < kOffItems; ++k) {
      const int i = threadIdx.x + k * kBlock;
      o[k] = i <= ns ? a.zoff[r0 + i] : z0;
      m[k] = i <= ns ? a.row_ptr[r0 + i] : static_cast<int32_t>(o0);
    }
#pragma unroll
    for (int k = 0; k < kTileItems; ++k) {
      const int i = threadIdx.x + k * kBlock;
      v[k] = i < n ? a.zsort[z0 + i] : 0;
    }
#pragma unroll
    for (int k = 0; k < kOffItems; ++k) {
      const int i = threadIdx.x + k * kBlock;
      if (i <= ns) {
        loff[i] = static_cast<int32_t>(o[k] - z0);
        moff[i] = static_cast<int32_t>(m[k] - o0);
      }
    }
#pragma unroll
    for (int k = 0; k < kTileItems; ++k) {
      const int i = threadIdx.x + k * kBlock;
      if (i < n) key[i] = v[k];
    }
  }
  __syncthreads();
  fill_segment_ids(loff, ns, seg);
  __syncthreads();
  // each thread owns a contiguous chunk of entries; heads are numbered by a
  // block scan, which also numbers the merged entries of the tile in order
  constexpr int kPer = (kBTileCap + kBlock - 1) / kBlock;
  const int b = threadIdx.x * kPer;
  int mine = 0;
  for (int i = b; i < b + kPer && i < n; ++i)
    mine += (i == loff[seg[i]] || key_col(key[i], a.L) != key_col(key[i - 1], a.L)) ? 1 : 0;
  int32_t total;
  int32_t pos = block_excl_scan<int32_t>(mine, &total, tmp);
  // each head's merged weight waits in a register until every thread is
  // done reading keys
  double hw[kPer];
  int32_t hp[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int i = b + u;
    hp[u] = -1;
    if (i < n) {
      const int k = seg[i];
      const int end = loff[k + 1];
      if (i == loff[k] || key_col(key[i], a.L) != key_col(key[i - 1], a.L)) {
        const uint32_t c = key_col(key[i], a.L);
        double s = key_weight(key[i], a);
        for (int j = i + 1; j < end && key_col(key[j], a.L) == c; ++j)
          s = s + key_weight(key[j], a);
        mcol[pos] = static_cast<int32_t>(c);
        hw[u] = s;
        hp[u] = pos;
        ++pos;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kPer; ++u)
    if (hp[u] >= 0) mw[hp[u]] = hw[u];
  __syncthreads();
  // columns and weights leave LDS coalesced
  for (int i = threadIdx.x; i < total; i += kBlock) {
    a.col[o0 + i] = mcol[i];
    a.w[o0 + i] = mw[i];
  }
  for (int k = threadIdx.x; k < ns; k += kBlock) {
    double d = 0.0;
    for (int i = moff[k]; i < moff[k + 1]; ++i) d = d + mw[i];
    a.deg[r0 + k] = d;
  }
}

// One wave per star row: the net's sorted cells, weight M w(M).
__global__ __launch_bounds__(kBlock) void k_star_rows(const int32_t *virt_net,
                                                      const int64_t *net_ptr, const int32_t *M,
                                                      const int32_t *ucell, const double *wnet,
                                                      const int32_t *row_ptr, int64_t N,
                                                      int64_t V, int32_t *col, double *w,
                                                      double *deg) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t waves = static_cast<int64_t>(gridDim.x) * (kBlock / kWave);
  for (int64_t v = static_cast<int64_t>(blockIdx.x) * (kBlock / kWave) + threadIdx.x / kWave;
       v < V; v += waves) {
    const int64_t e = virt_net[v];
    const int64_t lo = net_ptr[e];
    const int32_t m = M[e];
    const double g = wnet[e];
    const int64_t out = row_ptr[N + v];
    int32_t i = lane;
    for (; i + 3 * kWave < m; i += 4 * kWave) {  // four loads in flight per lane
      const int32_t c0 = ucell[lo + i], c1 = ucell[lo + i + kWave];
      const int32_t c2 = ucell[lo + i + 2 * kWave], c3 = ucell[lo + i + 3 * kWave];
      col[out + i] = c0;
      col[out + i + kWave] = c1;
      col[out + i + 2 * kWave] = c2;
      col[out + i + 3 * kWave] = c3;
      w[out + i] = g;
      w[out + i + kWave] = g;
      w[out + i + 2 * kWave] = g;
      w[out + i + 3 * kWave] = g;
    }
    for (; i < m; i += kWave) {
      col[out + i] = ucell[lo + i];
      w[out + i] = g;
    }
    if (lane == 0) {
      double d = 0.0;
      for (int32_t i = 0; i < m; ++i) d = d + g;
      deg[N + v] = d;
    }
  }
}

// ---------------------------------------------------------------------------
// 7. normalisation for one sigma
// ---------------------------------------------------------------------------
template <int D>
__global__ void k_sigma_scale(const double *deg, int64_t R, double sigma, double *s,
                              typename Store<D>::A *diag) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= R) return;
  double t = deg[i] + sigma;
  double si = (t == 0.0) ? 0.0 : 1.0 / sqrt(t);
  s[i] = si;
  diag[i] = static_cast<typename Store<D>::A>((sigma * si) * si);
}

// One block per SpMM row tile (class 0): a_ij = (w_ij s_i) s_j for the tile's
// entries.
template <int D>
__global__ __launch_bounds__(kBlock) void k_sigma_values(const int32_t *row_ptr,
                                                         const TileDesc *tiles,
                                                         const int32_t *col, const double *w,
                                                         const double *s,
                                                         typename Store<D>::T *val) {
  using TCL = TileClass<0>;
  __shared__ int32_t loff[TCL::kRows + 2];
  __shared__ uint16_t seg[TCL::kCap + 1];
  __shared__ double ls[TCL::kRows + 1];
  // each XCD takes chunks of consecutive tiles (xcd_remap), so the s_j of
  // neighbouring rows that its tiles share stay in its L2
  const TileDesc td = tiles[xcd_remap(blockIdx.x, gridDim.x)];
  const int64_t r0 = td.r0, r1 = td.r1, p0 = td.p0, p1 = td.p1;
  const int ns = static_cast<int>(r1 - r0);
  if (ns == 1 && p1 - p0 > TCL::kLong) {
    const double si = s[r0];
    for (int64_t p = p0 + threadIdx.x; p < p1; p += kBlock)
      val[p] = Store<D>::from_f64((w[p] * si) * s[col[p]]);
    return;
  }
  const int n = static_cast<int>(p1 - p0);
  for (int k = threadIdx.x; k <= ns; k += kBlock) loff[k] = static_cast<int32_t>(row_ptr[r0 + k] - p0);
  for (int k = threadIdx.x; k < ns; k += kBlock) ls[k] = s[r0 + k];
  __syncthreads();
  fill_segment_ids(loff, ns, seg);
  __syncthreads();
  // every load of the thread is issued before the first use: the entries'
  // weights and columns, then the column scales.  Inactive slots read entry
  // 0 (the arrays always hold at least one element) and use column 0 (the
  // graph has rows, since it has this tile).
  constexpr int kStage = (TCL::kCap + kBlock - 1) / kBlock;
  double wv[kStage], sj[kStage];
  int32_t cj[kStage];
#pragma unroll
  for (int k = 0; k < kStage; ++k) {
    const int i = threadIdx.x + k * kBlock;
    const int64_t p = i < n ? p0 + i : 0;
    wv[k] = w[p];
    const int32_t c = col[p];
    cj[k] = i < n ? c : 0;
  }
#pragma unroll
  for (int k = 0; k < kStage; ++k) sj[k] = s[cj[k]];
#pragma unroll
  for (int k = 0; k < kStage; ++k) {
    const int i = threadIdx.x + k * kBlock;
    if (i < n) val[p0 + i] = Store<D>::from_f64((wv[k] * ls[seg[i]]) * sj[k]);
  }
}

template <int D>
gift_status sigma_kernels(gift_graph *g, double sigma, SigmaBlock &b, hipStream_t st) {
  using A = typename Store<D>::A;
  using T = typename Store<D>::T;
  Scratch sc(st);
  double *s = nullptr;
  GIFT_TRY(sc.get(&s, g->num_rows, "normalisation scale"));
  k_sigma_scale<D><<<grid_for(g->num_rows), kBlock, 0, st>>>(g->deg, g->num_rows, sigma, s,
                                                               static_cast<A *>(b.diag));
  GIFT_TRY(check_launch("k_sigma_scale"));
  if (g->num_tiles[0] > 0) {
    k_sigma_values<D><<<static_cast<unsigned>(g->num_tiles[0]), kBlock, 0, st>>>(
        g->row_ptr, g->tiles[0], g->col, g->w, s, static_cast<T *>(b.val));
    GIFT_TRY(check_launch("k_sigma_values"));
  }
  return GIFT_OK;
}

}  // namespace

gift_status prepare_sigma(gift_graph *g, double sigma, hipStream_t st) {
  if (!(sigma >= 0.0) || !std::isfinite(sigma))
    return set_error(GIFT_EINVAL, "sigma must be finite and >= 0 (got %g)", sigma);
  if (find_sigma(g, sigma)) return GIFT_OK;
  SigmaBlock b{sigma, nullptr, nullptr};
  size_t vb = dtype_size(g->storage) * static_cast<size_t>(g->nnz);
  size_t db = accum_size(g->storage) * static_cast<size_t>(g->num_rows);
  GIFT_TRY(dev_alloc(&b.val, vb, st, "normalised values"));
  gift_status s = dev_alloc(&b.diag, db, st, "normalised diagonal");
  if (s != GIFT_OK) {
    dev_free(b.val, st);
    return s;
  }
  switch (g->storage) {
    case GIFT_F32: s = sigma_kernels<GIFT_F32>(g, sigma, b, st); break;
    case GIFT_F64: s = sigma_kernels<GIFT_F64>(g, sigma, b, st); break;
    case GIFT_BF16: s = sigma_kernels<GIFT_BF16>(g, sigma, b, st); break;
    case GIFT_F16: s = sigma_kernels<GIFT_F16>(g, sigma, b, st); break;
  }
  if (s != GIFT_OK) {
    dev_free(b.val, st);
    dev_free(b.diag, st);
    return s;
  }
  g->sig.push_back(b);
  g->bytes += static_cast<int64_t>(vb + db);
  return GIFT_OK;
}

namespace {

constexpr int kMaxReadback = kReadScalarsMax;
static_assert(kMaxReadback <= kReadbackFlag, "readback slots");

// Copies int64 scalars from device memory into the host slot, then writes the
// ticket that tells the host they are there: every thread's value is made
// visible to the host (system-scope fence) before the block's barrier, and
// the ticket is stored after it.
struct ReadbackPtrs {
  const int64_t *p[kMaxReadback];
};
__global__ void k_gather_i64(ReadbackPtrs src, int n, int64_t *dst, int64_t ticket) {
  if (threadIdx.x < n) dst[threadIdx.x] = *src.p[threadIdx.x];
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0)
    __hip_atomic_store(dst + kReadbackFlag, ticket, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

}  // namespace

// Reads `n` device int64 scalars with one launch and one wait: the kernel
// writes them straight into a pinned host slot, then the slot's next ticket.
// The host spins on the ticket for a short while (no event to record or
// query), then falls back to an event wait, which also reports a failed
// kernel.  A slot whose wait failed is not returned to the pool (its kernel
// may still write it).
gift_status read_scalars(hipStream_t st, const int64_t *const *ptrs, int n, int64_t *out) {
  Readback rb{};
  GIFT_TRY(readback_acquire(&rb));
  ReadbackPtrs rp{};
  for (int i = 0; i < n; ++i) rp.p[i] = ptrs[i];
  const int64_t ticket = ++rb.ticket;
  k_gather_i64<<<1, 64, 0, st>>>(rp, n, rb.dev, ticket);
  gift_status s = check_launch("k_gather_i64");
  if (s != GIFT_OK) {
    readback_release(rb);
    return s;
  }
  const volatile int64_t *h = rb.host;
  bool seen = false;
  const auto t0 = std::chrono::steady_clock::now();
  while (!(seen = h[kReadbackFlag] == ticket) &&
         std::chrono::steady_clock::now() - t0 < std::chrono::microseconds(300)) {
  }
  if (!seen) GIFT_TRY(readback_wait(rb, st));
  for (int i = 0; i < n; ++i) out[i] = h[i];
  readback_release(rb);
  return GIFT_OK;
}

namespace {

// A pooled side stream held for the rest of a build.  On an early return its
// queued work may still use the build's scratch, so the stream is drained
// before it goes back to the pool (and before the scratch, declared earlier,
// is released).
struct SideGuard {
  SideStream s{};
  bool idle = false;  // set once the build knows the stream has no work left
  ~SideGuard() {
    if (!s.stream) return;
    if (!idle) (void)hipStreamSynchronize(s.stream);
    side_stream_release(s);
  }
};

// Makes `side` wait for everything enqueued on `st` so far.
gift_status fork_to(hipStream_t st, const SideStream &side) {
  if (hipEventRecord(side.ready, st) != hipSuccess ||
      hipStreamWaitEvent(side.stream, side.ready, 0) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(GIFT_EDEVICE, "side stream ordering failed");
  }
  return GIFT_OK;
}

gift_status build_impl(const gift_graph_desc *d, hipStream_t st, gift_graph *g) {
  const int64_t N = d->num_cells, E = d->num_nets;
  Scratch sc(st);
  // --- netlist on the device
  int64_t P = 0;
  const int64_t *net_ptr = d->net_ptr;
  const int32_t *pin = d->pin_cell;
  if (d->mem_space == GIFT_MEM_HOST) {
    P = d->net_ptr[E];
    if (P < 0) return set_error(GIFT_EINVAL, "net_ptr[num_nets] is negative");
    int64_t *dn = nullptr;
    int32_t *dp = nullptr;
    GIFT_TRY(sc.get(&dn, E + 1, "net_ptr copy"));
    GIFT_TRY(sc.get(&dp, P, "pin_cell copy"));
    GIFT_HIP(hipMemcpyAsync(dn, d->net_ptr, (E + 1) * 8, hipMemcpyHostToDevice, st));
    if (P) GIFT_HIP(hipMemcpyAsync(dp, d->pin_cell, P * 4, hipMemcpyHostToDevice, st));
    net_ptr = dn;
    pin = dp;
  }
  if (N + E >= (int64_t(1) << 31))
    return set_error(GIFT_EUNSUPPORTED, "netlist too large (cells+nets %lld)",
                     (long long)(N + E));

  // one zeroed block: the error flags (the low word of a 64-bit word, read
  // back as int64), the row counts (N + 1 int32) and the star buckets'
  // counts and fill levels (NB int32 each)
  const int64_t NB = (N >> kStarShift) + 1;
  int64_t *zero_blk = nullptr;
  const int64_t zero_words = 1 + (N + 2) / 2 + NB;
  GIFT_TRY(sc.get(&zero_blk, zero_words, "flags, row counts, star buckets"));
  GIFT_HIP(hipMemsetAsync(zero_blk, 0, zero_words * 8, st));
  int64_t *flag64 = zero_blk;
  uint32_t *flag = reinterpret_cast<uint32_t *>(flag64);
  int32_t *cnt = reinterpret_cast<int32_t *>(zero_blk + 1);
  int32_t *bcnt = reinterpret_cast<int32_t *>(zero_blk + 1 + (N + 2) / 2);
  int32_t *bfill = bcnt + NB;

  // 0. check net_ptr and tile the nets, then read the flag, the pin count
  //    and the tile count back together; nothing reads pins before the check
  //    passed (tiling reads net_ptr only and stays in bounds for any values)
  k_check_netptr<<<grid_for(E + 1), kBlock, 0, st>>>(net_ptr, E, flag);
  GIFT_TRY(check_launch("k_check_netptr"));
  int32_t *net_tiles = nullptr;
  int64_t *net_tile_counts = nullptr;
  GIFT_TRY(sc.get(&net_tiles, E + 2, "net tiles"));
  GIFT_TRY(sc.get(&net_tile_counts, 2, "net tile counts"));
  GIFT_TRY(build_tiles64(net_ptr, E, E, kBuildTiles, st, net_tiles, net_tile_counts));
  int64_t h0[3] = {0, 0, 0};
  {
    const int64_t *ptrs[3] = {flag64, net_ptr + E, net_tile_counts};
    GIFT_TRY(read_scalars(st, ptrs, 3, h0));
  }
  if (h0[0] & kFlagBadNetPtr)
    return set_error(GIFT_EINVAL, "net_ptr must start at 0, end at the pin count and not decrease");
  if (d->mem_space != GIFT_MEM_HOST) {
    P = h0[1];
    if (d->num_pins >= 0 && P != d->num_pins)
      return set_error(GIFT_EINVAL, "pin_cell has %lld entries but net_ptr[num_nets] = %lld",
                       (long long)d->num_pins, (long long)P);
  }
  const int64_t num_net_tiles = h0[2];
  if (P >= (int64_t(1) << 31))
    return set_error(GIFT_EUNSUPPORTED, "netlist too large (pins %lld)", (long long)P);

  int32_t *M = nullptr, *ucell = nullptr, *pin_net = nullptr;
  uint32_t *tmp32 = nullptr;
  GIFT_TRY(sc.get(&M, E, "net sizes"));
  GIFT_TRY(sc.get(&ucell, P, "distinct cells"));
  GIFT_TRY(sc.get(&pin_net, P, "pin nets"));
  GIFT_TRY(sc.get(&tmp32, P, "net sort scratch"));

  // 1. distinct cells per net and the row counts (tile descriptors first:
  //    one load per block instead of two dependent ones; pin offsets fit
  //    int32 by the check above)
  int32_t *slot = nullptr;
  GIFT_TRY(sc.get(&slot, P, "pin slices"));
  TileDesc *net_descs = nullptr;
  GIFT_TRY(sc.get(&net_descs, num_net_tiles + 1, "net tile descriptors"));
  GIFT_TRY(tile_descs(net_tiles, net_ptr, num_net_tiles, st, net_descs));
  if (num_net_tiles > 0) {
    NetArgs na{net_ptr, pin,   E,         P,   N,   M,   ucell, pin_net,
               flag,    tmp32, net_descs, d->star_threshold, cnt, slot};
    k_net_tiles<<<static_cast<unsigned>(num_net_tiles), kBlock, 0, st>>>(na);
    GIFT_TRY(check_launch("k_net_tiles"));
  }

  // 2-3. two independent chains: the net classes here, the row offsets and
  //      row tiles on a side stream.  The sizes are read back once the
  //      classes and the row offsets are done; the emit starts then, and the
  //      row tile count is read back while it runs
  SideGuard side;
  GIFT_TRY(side_stream_acquire(&side.s));
  int32_t *row_tiles = nullptr;
  int64_t *zoff = nullptr, *row_tile_counts = nullptr;
  int32_t *zoff32 = nullptr;
  GIFT_TRY(sc.get(&zoff, N + 1, "row offsets"));
  GIFT_TRY(sc.get(&zoff32, N + 1, "row offsets (32-bit)"));
  GIFT_TRY(sc.get(&row_tiles, N + 2, "row tiles"));
  GIFT_TRY(sc.get(&row_tile_counts, 2, "row tile counts"));
  // (these blocks and cnt were allocated on this stream before the fork, so
  // the event orders the side stream after their earlier users)
  GIFT_TRY(fork_to(st, side.s));
  // with a 32-bit copy of the row offsets: the emit's random lookups of them
  // then touch an 8 MB table instead of 16 MB, more of it in L2
  GIFT_TRY(scan_i32_to_i64(cnt, zoff, N, side.s.stream, zoff32));
  // (the main stream waits for this record before it reads the offsets)
  if (hipEventRecord(side.s.done, side.s.stream) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(GIFT_EDEVICE, "side stream ordering failed");
  }
  GIFT_TRY(build_tiles64(zoff, N, N, kBuildTiles, side.s.stream, row_tiles, row_tile_counts));

  // 2. classify
  int32_t *is_star = nullptr, *virt_net = nullptr;
  double *wnet = nullptr;
  GIFT_TRY(sc.get(&is_star, E, "star flags"));
  GIFT_TRY(sc.get(&wnet, E, "net weights"));
  GIFT_TRY(sc.get(&virt_net, E, "virtual nets"));
  int32_t *bmax = nullptr;
  int64_t *bstar = nullptr, *totals = nullptr;
  uint64_t *skey = nullptr;
  GIFT_TRY(sc.get(&bmax, grid_for(E), "largest net per block"));
  GIFT_TRY(sc.get(&bstar, grid_for(E), "star entries per block"));
  GIFT_TRY(sc.get(&totals, 2, "largest net, star entries"));
  GIFT_TRY(sc.get(&skey, E, "star keys by net"));
  k_classify<<<grid_for(E), kBlock, 0, st>>>(M, E, d->star_threshold, d->weight_model, is_star,
                                             wnet, bmax, bstar,
                                             StarKeys{net_ptr, ucell, skey, bcnt});
  GIFT_TRY(check_launch("k_classify"));
  k_max_reduce<<<1, kBlock, 0, st>>>(bmax, bstar, grid_for(E), totals);
  GIFT_TRY(check_launch("k_max_reduce"));

  // 2b. virtual row labels
  int32_t *vrow = nullptr;
  int64_t *boff = nullptr;
  uint64_t *bkey = nullptr, *btmp = nullptr;
  GIFT_TRY(sc.get(&vrow, E, "virtual row of each star net"));
  GIFT_TRY(sc.get(&boff, NB + 1, "star bucket offsets"));
  GIFT_TRY(sc.get(&bkey, E, "star keys by bucket"));
  GIFT_TRY(sc.get(&btmp, E, "star key sort scratch"));
  // distinct columns per row: the star rows' counts come from the star sort,
  // the cell rows' from the row sort (N + E bounds the rows: V <= E)
  int32_t *ucnt = nullptr;
  GIFT_TRY(sc.get(&ucnt, N + E, "distinct counts"));
  GIFT_TRY(scan_i32_to_i64(bcnt, boff, NB, st));
  k_star_scatter<<<grid_for(E), kBlock, 0, st>>>(is_star, skey, E, boff, bfill, bkey);
  GIFT_TRY(check_launch("k_star_scatter"));
  k_star_sort<<<static_cast<unsigned>(NB), kBlock, 0, st>>>(bkey, btmp, boff, virt_net, vrow,
                                                            M, N, ucnt);
  GIFT_TRY(check_launch("k_star_sort"));

  // this stream waits for the row offsets (the record after their scan)
  if (hipStreamWaitEvent(st, side.s.done, 0) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(GIFT_EDEVICE, "side stream ordering failed");
  }
  EmitArgs ea{net_ptr, ucell, pin_net, M, is_star, vrow, E, P, N, KeyLayout{}};

  // sizes back to the host: flag, V (the star nets counted in the median
  // buckets), Z, largest net, star entries
  int64_t h1[5] = {0, 0, 0, 0, 0};
  {
    const int64_t *ptrs[5] = {flag64, boff + NB, zoff + N, totals, totals + 1};
    GIFT_TRY(read_scalars(st, ptrs, 5, h1));
  }
  if (h1[0] & kFlagBadPin) return set_error(GIFT_EINVAL, "a pin names a cell outside [0, num_cells)");
  const int64_t V = h1[1], star_entries = h1[4];
  const int64_t Z = h1[2], R = N + V;
  const KeyLayout L = key_layout(R > 0 ? R - 1 : 0, E > 0 ? E - 1 : 0, h1[3]);
  ea.L = L;
  if (R >= (int64_t(1) << 31))
    return set_error(GIFT_EUNSUPPORTED, "too many rows (%lld)", (long long)R);
  // merging only removes entries: Z + star_entries bounds the stored count,
  // so the CSR is allocated now and its exact size read back at the end
  const int64_t cap = Z + star_entries;
  if (cap >= (int64_t(1) << 31))
    return set_error(GIFT_EUNSUPPORTED, "too many stored entries (up to %lld)", (long long)cap);
  // 3b. emit (launched before the host's other allocations, so that the
  // device starts on it as soon as the sizes are known)
  uint64_t *zkey = nullptr, *zsort = nullptr;
  GIFT_TRY(sc.get(&zkey, Z, "emitted keys"));
  // (zoff32 is exact: Z < 2^31 was checked above)
  k_emit<<<grid_for(P), kBlock, 0, st>>>(ea, zoff32, slot, zkey);
  GIFT_TRY(check_launch("k_emit"));
  GIFT_TRY(sc.get(&zsort, Z, "sorted keys"));
  g->num_cells = N;
  g->num_virtual = V;
  g->num_rows = R;
  GIFT_TRY(dev_alloc(reinterpret_cast<void **>(&g->row_ptr), (R + 1) * 4, st, "row_ptr"));
  GIFT_TRY(dev_alloc(reinterpret_cast<void **>(&g->col), cap * 4, st, "col"));
  GIFT_TRY(dev_alloc(reinterpret_cast<void **>(&g->w), cap * 8, st, "weights"));
  GIFT_TRY(dev_alloc(reinterpret_cast<void **>(&g->deg), R * 8, st, "degrees"));
  g->bytes = (R + 1) * 4 + cap * 12 + R * 8;

  // the row tile count, read back from the side stream while the emit runs;
  // then this stream waits for the row tiles
  int64_t num_row_tiles = 0;
  {
    const int64_t *ptrs[1] = {row_tile_counts};
    GIFT_TRY(read_scalars(side.s.stream, ptrs, 1, &num_row_tiles));
  }
  if (hipEventRecord(side.s.done, side.s.stream) != hipSuccess ||
      hipStreamWaitEvent(st, side.s.done, 0) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(GIFT_EDEVICE, "side stream ordering failed");
  }
  // row tile descriptors (key offsets fit int32: Z <= cap, checked above)
  TileDesc *row_descs = nullptr;
  GIFT_TRY(sc.get(&row_descs, num_row_tiles + 1, "row tile descriptors"));
  GIFT_TRY(tile_descs(row_tiles, zoff, num_row_tiles, st, row_descs));

  // 4. sort rows
  if (num_row_tiles > 0) {
    RowArgs ra{zoff, zkey, zsort, ucnt, row_descs, L};
    k_row_sort_tiles<<<static_cast<unsigned>(num_row_tiles), kBlock, 0, st>>>(ra);
    GIFT_TRY(check_launch("k_row_sort_tiles"));
  }
  // 5. row_ptr; the SpMM row tiles of every class on a side stream while
  //    this stream merges
  int64_t *rp64 = nullptr;
  GIFT_TRY(sc.get(&rp64, R + 1, "row offsets (64-bit)"));
  // (the 32-bit row_ptr is exact: the stored entries were bounded below 2^31)
  GIFT_TRY(scan_i32_to_i64(ucnt, rp64, R, st, g->row_ptr));
  int32_t *tstart[kTileClasses];
  int64_t *tile_counts = nullptr;
  GIFT_TRY(sc.get(&tile_counts, 2 * kTileClasses, "tile counts"));
  for (int c = 0; c < kTileClasses; ++c) GIFT_TRY(sc.get(&tstart[c], R + 2, "tile starts"));
  // everything the side stream reads or writes was allocated above, so it
  // is ordered after all earlier users of those blocks by this event
  gift_status ss = fork_to(st, side.s);
  // 6. merge the cell rows here; the star rows (a disjoint part of the CSR)
  //    on the side stream
  if (ss == GIFT_OK && V > 0) {
    k_star_rows<<<grid_for(V * kWave), kBlock, 0, side.s.stream>>>(
        virt_net, net_ptr, M, ucell, wnet, g->row_ptr, N, V, g->col, g->w, g->deg);
    ss = check_launch("k_star_rows");
  }
  static_assert(kTileClasses == 2, "both SpMM tile classes are built in one pass");
  if (ss == GIFT_OK)
    ss = build_tiles64_pair(rp64, R, N, kSpmmTiles[0], kSpmmTiles[1], side.s.stream, tstart[0],
                            tstart[1], tile_counts, tile_counts + 2);
  if (ss == GIFT_OK && num_row_tiles > 0) {
    MergeArgs ma{zoff, zsort, wnet, g->row_ptr, row_descs, g->col, g->w, g->deg,
                 L, N, d->weight_model};
    k_row_merge_tiles<<<static_cast<unsigned>(num_row_tiles), kBlock, 0, st>>>(ma);
    ss = check_launch("k_row_merge_tiles");
  }

  // CSR and tile counts, read from the side stream while the merge runs
  int64_t h2[2 + 2 * kTileClasses] = {};
  if (ss == GIFT_OK) {
    const int64_t *ptrs[2 + 2 * kTileClasses];
    ptrs[0] = rp64 + R;
    ptrs[1] = rp64 + N;
    for (int i = 0; i < 2 * kTileClasses; ++i) ptrs[2 + i] = tile_counts + i;
    ss = read_scalars(side.s.stream, ptrs, 2 + 2 * kTileClasses, h2);
  }
  // the side stream is idle once its readback returned; otherwise the guard
  // drains it
  GIFT_TRY(ss);
  side.idle = true;
  g->nnz = h2[0];
  g->nnz_cells = h2[1];
  // the side stream's work is complete (its readback returned), so this
  // stream may read the tile starts and the star rows without further
  // ordering
  for (int c = 0; c < kTileClasses; ++c) {
    g->num_tiles[c] = h2[2 + 2 * c];
    g->num_tiles_cells[c] = h2[3 + 2 * c];
    GIFT_TRY(dev_alloc(reinterpret_cast<void **>(&g->tiles[c]),
                       (g->num_tiles[c] + 1) * sizeof(TileDesc), st, "row tiles"));
    g->bytes += (g->num_tiles[c] + 1) * static_cast<int64_t>(sizeof(TileDesc));
    GIFT_TRY(tile_descs(tstart[c], rp64, g->num_tiles[c], st, g->tiles[c]));
  }

  // 7. normalisation
  for (int32_t i = 0; i < d->num_sigmas; ++i) GIFT_TRY(prepare_sigma(g, d->sigmas[i], st));
  return GIFT_OK;
}

}  // namespace
}  // namespace gift

using namespace gift;

extern "C" gift_status gift_build_graph(const gift_graph_desc *d, void *stream,
                                        gift_graph **out) {
  clear_error();
  if (!out) return set_error(GIFT_EINVAL, "gift_build_graph: out is NULL");
  *out = nullptr;
  if (!d) return set_error(GIFT_EINVAL, "gift_build_graph: desc is NULL");
  if (d->num_cells < 0 || d->num_nets < 0)
    return set_error(GIFT_EINVAL, "negative num_cells or num_nets");
  if (!d->net_ptr || (!d->pin_cell && d->num_nets > 0))
    return set_error(GIFT_EINVAL, "net_ptr / pin_cell is NULL");
  if (d->mem_space != GIFT_MEM_HOST && d->mem_space != GIFT_MEM_DEVICE)
    return set_error(GIFT_EINVAL, "bad mem_space %d", d->mem_space);
  if (d->weight_model != GIFT_W_INV_M1 && d->weight_model != GIFT_W_TWO_OVER_M)
    return set_error(GIFT_EINVAL, "bad weight_model %d", d->weight_model);
  if (d->star_threshold < 0) return set_error(GIFT_EINVAL, "star_threshold < 0");
  if (!dtype_valid(d->storage)) return set_error(GIFT_EINVAL, "bad storage dtype %d", d->storage);
  if (d->num_sigmas < 1 || !d->sigmas) return set_error(GIFT_EINVAL, "need at least one sigma");
  for (int32_t i = 0; i < d->num_sigmas; ++i)
    if (!(d->sigmas[i] >= 0.0) || !std::isfinite(d->sigmas[i]))
      return set_error(GIFT_EINVAL, "sigma[%d] = %g is not a finite value >= 0", i, d->sigmas[i]);
  if (d->num_pins < -1) return set_error(GIFT_EINVAL, "num_pins must be >= -1");
  if (d->mem_space == GIFT_MEM_HOST) {
    if (d->net_ptr[0] != 0) return set_error(GIFT_EINVAL, "net_ptr[0] must be 0");
    if (d->num_pins >= 0 && d->net_ptr[d->num_nets] != d->num_pins)
      return set_error(GIFT_EINVAL, "pin_cell has %lld entries but net_ptr[num_nets] = %lld",
                       (long long)d->num_pins, (long long)d->net_ptr[d->num_nets]);
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  gift_graph *g = new (std::nothrow) gift_graph();
  if (!g) return set_error(GIFT_ENOMEM, "host allocation failed");
  g->storage = d->storage;
  g->weight_model = d->weight_model;
  g->star_threshold = d->star_threshold;
  (void)hipGetDevice(&g->device);
  gift_status s;
  {
    ProfScope ps(st, GIFT_PROF_BUILD, 0.0);
    s = build_impl(d, st, g);
  }
  if (s != GIFT_OK) {
    std::string msg = gift_last_error();
    gift_destroy_graph(g, stream);
    set_error(s, "%s", msg.c_str());
    return s;
  }
  *out = g;
  return GIFT_OK;
}

extern "C" gift_status gift_graph_add_sigma(gift_graph *g, double sigma, void *stream) {
  clear_error();
  if (!g) return set_error(GIFT_EINVAL, "gift_graph_add_sigma: NULL graph");
  return prepare_sigma(g, sigma, static_cast<hipStream_t>(stream));
}

namespace gift {
namespace {

template <int D>
__global__ void k_widen(const typename Store<D>::T *val, int64_t nnz,
                        const typename Store<D>::A *diag, int64_t R, double *out) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < nnz) out[i] = static_cast<double>(Store<D>::load(val[i]));
  else if (i < nnz + R) out[i] = static_cast<double>(diag[i - nnz]);
}

template <int D>
gift_status widen(const gift_graph *g, const SigmaBlock *b, double *out, hipStream_t st) {
  using T = typename Store<D>::T;
  using A = typename Store<D>::A;
  k_widen<D><<<grid_for(g->nnz + g->num_rows), kBlock, 0, st>>>(
      static_cast<const T *>(b->val), g->nnz, static_cast<const A *>(b->diag), g->num_rows, out);
  return check_launch("k_widen");
}

}  // namespace
}  // namespace gift

extern "C" gift_status gift_graph_export_normalised(const gift_graph *g, double sigma,
                                                    double *val, double *diag, void *stream) {
  clear_error();
  if (!g) return set_error(GIFT_EINVAL, "gift_graph_export_normalised: NULL graph");
  const SigmaBlock *b = find_sigma(g, sigma);
  if (!b) return set_error(GIFT_EINVAL, "sigma %g was not prepared for this graph", sigma);
  hipStream_t st = static_cast<hipStream_t>(stream);
  Scratch sc(st);
  double *tmp = nullptr;
  GIFT_TRY(sc.get(&tmp, g->nnz + g->num_rows, "export buffer"));
  gift_status s = GIFT_OK;
  switch (g->storage) {
    case GIFT_F32: s = widen<GIFT_F32>(g, b, tmp, st); break;
    case GIFT_F64: s = widen<GIFT_F64>(g, b, tmp, st); break;
    case GIFT_BF16: s = widen<GIFT_BF16>(g, b, tmp, st); break;
    case GIFT_F16: s = widen<GIFT_F16>(g, b, tmp, st); break;
  }
  GIFT_TRY(s);
  if (val && g->nnz) GIFT_HIP(hipMemcpyAsync(val, tmp, g->nnz * 8, hipMemcpyDeviceToHost, st));
  if (diag && g->num_rows)
    GIFT_HIP(hipMemcpyAsync(diag, tmp + g->nnz, g->num_rows * 8, hipMemcpyDeviceToHost, st));
  GIFT_HIP(hipStreamSynchronize(st));
  return GIFT_OK;
}
