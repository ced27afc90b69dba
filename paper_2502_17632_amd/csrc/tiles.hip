// Row tiles: consecutive rows grouped so that one 256-thread block can stage
// all of a tile's entries in LDS.
//
// Row r starts a new tile when
//   - r = 0 or r = split (the first star row, so cell rows and star rows
//     never share a tile), or
//   - off[r] / entries differs from off[r-1] / entries (a new window of
//     entries begins), or
//   - r / rows differs from (r-1) / rows (at most `rows` rows per tile), or
//   - row r or row r-1 is long (more than long_row entries).
// A tile therefore holds either a single long row or rows that all start in
// one window of `entries` entries, each at most long_row long: at most
// entries + long_row - 1 entries.  The rule looks only at neighbouring
// rows, so tiles are built in parallel (flag, scan, scatter) and are
// deterministic.
#include "common.h"
#include "devutil.h"

namespace gift {
namespace {

// narrow (optional): off[0..R] copied to 32 bits (the caller has checked
// that off[R] < 2^31 before it reads the copy).
template <typename Off>
__global__ void k_tile_flags(const Off *off, int64_t R, int64_t split, TileShape sh,
                             int32_t *flag, int32_t *narrow) {
  int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (narrow && r <= R) narrow[r] = static_cast<int32_t>(off[r]);
  if (r >= R) return;
  int f = 1;
  if (r > 0 && r != split) {
    const int64_t a = off[r - 1], b = off[r], c = off[r + 1];
    const bool long_prev = b - a > sh.long_row, long_cur = c - b > sh.long_row;
    f = (a / sh.entries != b / sh.entries) || ((r - 1) / sh.rows != r / sh.rows) || long_prev ||
        long_cur;
  }
  flag[r] = f;
}

__global__ void k_tile_scatter(const int32_t *flag, const int64_t *pos, int64_t R, int64_t split,
                               int32_t *tile_row, int64_t *out_counts) {
  int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r < R && flag[r]) tile_row[pos[r]] = static_cast<int32_t>(r);
  if (r == 0) {
    const int64_t T = pos[R];
    tile_row[T] = static_cast<int32_t>(R);
    out_counts[0] = T;
    out_counts[1] = split < R ? pos[split] : T;  // tiles before the split row
  }
}

template <typename Off>
gift_status build_tiles_impl(const Off *off, int64_t R, int64_t split, TileShape sh,
                             hipStream_t st, int32_t *tile_row, int64_t *counts_dev,
                             int32_t *narrow) {
  Scratch sc(st);
  int32_t *flag = nullptr;
  int64_t *pos = nullptr;
  GIFT_TRY(sc.get(&flag, R, "tile flags"));
  GIFT_TRY(sc.get(&pos, R + 1, "tile positions"));
  k_tile_flags<Off><<<grid_for(R + 1), kBlock, 0, st>>>(off, R, split, sh, flag, narrow);
  GIFT_TRY(check_launch("k_tile_flags"));
  GIFT_TRY(scan_i32_to_i64(flag, pos, R, st));
  k_tile_scatter<<<grid_for(R > 0 ? R : 1), kBlock, 0, st>>>(flag, pos, R, split, tile_row,
                                                             counts_dev);
  return check_launch("k_tile_scatter");
}

// Both SpMM tile classes in one pass: per row the two start flags packed in
// one 64-bit word (class 0 in the low half, class 1 in the high half), so
// one 64-bit scan numbers the starts of both (the low half's total is at
// most R < 2^31 and never carries into the high half).
template <typename Off>
__global__ void k_tile_flags2(const Off *off, int64_t R, int64_t split, TileShape s0,
                              TileShape s1, int64_t *flag) {
  int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= R) return;
  int64_t f = 1 | (int64_t(1) << 32);
  if (r > 0 && r != split) {
    const int64_t a = off[r - 1], b = off[r], c = off[r + 1];
    const int64_t f0 = (a / s0.entries != b / s0.entries) || ((r - 1) / s0.rows != r / s0.rows) ||
                       b - a > s0.long_row || c - b > s0.long_row;
    const int64_t f1 = (a / s1.entries != b / s1.entries) || ((r - 1) / s1.rows != r / s1.rows) ||
                       b - a > s1.long_row || c - b > s1.long_row;
    f = f0 | (f1 << 32);
  }
  flag[r] = f;
}

__global__ void k_tile_scatter2(const int64_t *flag, const int64_t *pos, int64_t R, int64_t split,
                                int32_t *tile_row0, int32_t *tile_row1, int64_t *counts0,
                                int64_t *counts1) {
  int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r < R) {
    const int64_t f = flag[r], p = pos[r];
    if (f & 0xffffffff) tile_row0[p & 0xffffffff] = static_cast<int32_t>(r);
    if (f >> 32) tile_row1[p >> 32] = static_cast<int32_t>(r);
  }
  if (r == 0) {
    const int64_t T = pos[R];
    const int64_t T0 = T & 0xffffffff, T1 = T >> 32;
    const int64_t S = split < R ? pos[split] : T;
    tile_row0[T0] = static_cast<int32_t>(R);
    tile_row1[T1] = static_cast<int32_t>(R);
    counts0[0] = T0;
    counts0[1] = S & 0xffffffff;  // tiles before the split row
    counts1[0] = T1;
    counts1[1] = S >> 32;
  }
}

__global__ void k_tile_descs(const int32_t *tile_row, const int64_t *rp64, int64_t T,
                             TileDesc *out) {
  int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= T) return;
  const int32_t a = tile_row[t], b = tile_row[t + 1];
  out[t] = TileDesc{a, b, static_cast<int32_t>(rp64[a]), static_cast<int32_t>(rp64[b])};
}

}  // namespace

gift_status tile_descs(const int32_t *tile_row, const int64_t *rp64, int64_t T, hipStream_t st,
                       TileDesc *out) {
  if (T <= 0) return GIFT_OK;
  k_tile_descs<<<grid_for(T), kBlock, 0, st>>>(tile_row, rp64, T, out);
  return check_launch("k_tile_descs");
}

gift_status build_tiles64(const int64_t *off, int64_t R, int64_t split, TileShape sh,
                          hipStream_t st, int32_t *tile_row, int64_t *counts_dev,
                          int32_t *narrow) {
  return build_tiles_impl<int64_t>(off, R, split, sh, st, tile_row, counts_dev, narrow);
}

gift_status build_tiles64_pair(const int64_t *off, int64_t R, int64_t split, TileShape s0,
                               TileShape s1, hipStream_t st, int32_t *tile_row0,
                               int32_t *tile_row1, int64_t *counts0, int64_t *counts1) {
  Scratch sc(st);
  int64_t *flag = nullptr, *pos = nullptr;
  GIFT_TRY(sc.get(&flag, R, "tile flags"));
  GIFT_TRY(sc.get(&pos, R + 1, "tile positions"));
  k_tile_flags2<int64_t><<<grid_for(R), kBlock, 0, st>>>(off, R, split, s0, s1, flag);
  GIFT_TRY(check_launch("k_tile_flags2"));
  GIFT_TRY(scan_i64(flag, pos, R, st));
  k_tile_scatter2<<<grid_for(R > 0 ? R : 1), kBlock, 0, st>>>(flag, pos, R, split, tile_row0,
                                                              tile_row1, counts0, counts1);
  return check_launch("k_tile_scatter2");
}

}  // namespace gift
