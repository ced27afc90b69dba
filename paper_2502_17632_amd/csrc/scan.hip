// Device-wide exclusive prefix sum (reduce / scan-of-tile-sums / scan), used
// for CSR row offsets and per-net output offsets.
#include "common.h"
#include "devutil.h"

namespace gift {
namespace {

constexpr int kItems = 8;
constexpr int64_t kTile = static_cast<int64_t>(kBlock) * kItems;

template <typename In>
__global__ __launch_bounds__(kBlock) void k_tile_sums(const In *__restrict__ in, int64_t n,
                                                      int64_t *__restrict__ sums) {
  __shared__ int64_t tmp[kBlock / kWave];
  int64_t base = static_cast<int64_t>(blockIdx.x) * kTile;
  int64_t v = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    int64_t i = base + k * kBlock + threadIdx.x;
    if (i < n) v += static_cast<int64_t>(in[i]);
  }
  int64_t t = block_sum<int64_t>(v, tmp);
  if (threadIdx.x == 0) sums[blockIdx.x] = t;
}

// out[i] = offs[tile] + exclusive prefix within the tile; the last tile also
// writes out[n] (the grand total).  With out32, the same values also go there
// narrowed to 32 bits (the caller knows that they fit, or never reads the copy
// otherwise).  Each wave scans a contiguous quarter of the tile, 64
// consecutive elements per step (coalesced loads and stores), carrying its
// running sum between steps; the waves' totals are combined once through LDS.
template <typename In>
__global__ __launch_bounds__(kBlock) void k_tile_scan(const In *__restrict__ in, int64_t n,
                                                      const int64_t *__restrict__ offs,
                                                      int64_t *__restrict__ out,
                                                      int32_t *__restrict__ out32) {
  constexpr int kWaves = kBlock / kWave;
  constexpr int64_t kPerWave = kTile / kWaves;
  __shared__ int64_t tmp[kWaves];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int64_t wbase = static_cast<int64_t>(blockIdx.x) * kTile + wid * kPerWave;
  int64_t v[kItems];
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t i = wbase + k * kWave + lane;
    v[k] = i < n ? static_cast<int64_t>(in[i]) : 0;
  }
  int64_t carry = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    int64_t x = v[k];
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const int64_t y = __shfl_up(x, off, kWave);
      if (lane >= off) x += y;
    }
    const int64_t incl = carry + x;
    v[k] = incl - v[k];  // exclusive prefix within the wave's quarter
    carry = __shfl(incl, kWave - 1, kWave);
  }
  if (lane == 0) tmp[wid] = carry;
  __syncthreads();
  int64_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    before += w < wid ? tmp[w] : 0;
    all += tmp[w];
  }
  const int64_t off = (offs ? offs[blockIdx.x] : 0) + before;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t i = wbase + k * kWave + lane;
    if (i < n) {
      out[i] = off + v[k];
      if (out32) out32[i] = static_cast<int32_t>(off + v[k]);
    }
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
    const int64_t total = (offs ? offs[blockIdx.x] : 0) + all;
    out[n] = total;
    if (out32) out32[n] = static_cast<int32_t>(total);
  }
}

template <typename In>
gift_status scan_impl(const In *in, int64_t *out, int64_t n, hipStream_t s,
                      int32_t *out32 = nullptr) {
  if (n <= kTile) {
    k_tile_scan<In><<<1, kBlock, 0, s>>>(in, n, nullptr, out, out32);
    return check_launch("k_tile_scan");
  }
  int64_t nb = (n + kTile - 1) / kTile;
  Scratch sc(s);
  int64_t *sums = nullptr, *offs = nullptr;
  GIFT_TRY(sc.get(&sums, nb, "scan tile sums"));
  GIFT_TRY(sc.get(&offs, nb + 1, "scan tile offsets"));
  k_tile_sums<In><<<static_cast<unsigned>(nb), kBlock, 0, s>>>(in, n, sums);
  GIFT_TRY(check_launch("k_tile_sums"));
  GIFT_TRY(scan_impl<int64_t>(sums, offs, nb, s));
  k_tile_scan<In><<<static_cast<unsigned>(nb), kBlock, 0, s>>>(in, n, offs, out, out32);
  return check_launch("k_tile_scan");
}

}  // namespace

gift_status scan_i32_to_i64(const int32_t *in, int64_t *out, int64_t n, hipStream_t s,
                            int32_t *out32) {
  return scan_impl<int32_t>(in, out, n, s, out32);
}

gift_status scan_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t s) {
  return scan_impl<int64_t>(in, out, n, s);
}

}  // namespace gift
