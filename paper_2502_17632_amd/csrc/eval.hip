// Placement metrics of a signal g on a resident graph:
//   S(g)   = sum over edges w_ij (g_i - g_j)^2, per column: the smoothness of
//            Section 2.1 (eq. smoothness) and the weighted quadratic
//            wirelength of Section 2.2 (eq. wire_eq); with star nodes placed
//            at the mean of their cells, a star contributes exactly what its
//            clique would, so S is the clique-model value for any threshold;
//   |g|^2  per column, and R(g) = S / |g|^2, the Rayleigh quotient
//            (eq. smoothness_ray);
//   HPWL   = sum over nets of max - min of g over the net's pins.
// Everything is float64.  Sums are formed per row tile (S) or per block of
// nets (HPWL) in a fixed order and the partial sums are added in a fixed
// order too, so the results are deterministic.
#include "common.h"
#include "devutil.h"

namespace gift {
namespace {

__device__ __forceinline__ double load_x(const void *p, int32_t dt, int64_t i) {
  return dt == GIFT_F64 ? to_global(static_cast<const double *>(p))[i]
                        : static_cast<double>(to_global(static_cast<const float *>(p))[i]);
}

// Star rows: the mean of the net's cells (their columns), one wave per row.
__global__ __launch_bounds__(kBlock) void k_eval_star_means(const int32_t *row_ptr,
                                                            const int32_t *col, int64_t N,
                                                            int64_t V, const void *x,
                                                            int64_t ld, int32_t dt, int32_t C,
                                                            double *vx) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t v = static_cast<int64_t>(blockIdx.x) * (kBlock / kWave) + threadIdx.x / kWave;
  if (v >= V) return;
  const int32_t p0 = row_ptr[N + v], p1 = row_ptr[N + v + 1];
  for (int32_t q = 0; q < C; ++q) {
    double s = 0.0;
    for (int32_t p = p0 + lane; p < p1; p += kWave) s += load_x(x, dt, col[p] * ld + q);
    for (int off = kWave / 2; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) vx[v * C + q] = p1 > p0 ? s / static_cast<double>(p1 - p0) : 0.0;
  }
}

// One SpMM row tile (class 0) per block: sum over its entries of
// w_ij (g_i - g_j)^2 and, over its cell rows, g_i^2.  Columns go in rounds
// of kEvalCols: the rows' own values are staged in LDS, then each thread
// takes entries i, i + 256, ... of the tile, four at a time (their columns
// and weights loaded first, then their gathers), each thread's sums in a
// fixed order and a fixed tree over the block.  part[tile * 2C + q] = S part
// (each edge appears in both of its rows, so halved), [.. + C + q] = norm2.
constexpr int kEvalCols = 4;

__global__ __launch_bounds__(kBlock) void k_eval_smooth(const TileDesc *tiles,
                                                        const int32_t *row_ptr,
                                                        const int32_t *col, const double *w,
                                                        int64_t N, const void *x, int64_t ld,
                                                        int32_t dt, const double *vx,
                                                        int32_t C, double *part) {
  using TCL = TileClass<0>;
  __shared__ int32_t loff[TCL::kRows + 2];
  __shared__ uint16_t seg[TCL::kCap + 1];
  __shared__ double grow[TCL::kRows * kEvalCols];
  __shared__ double red[kBlock];
  const uint32_t tile = xcd_remap(blockIdx.x, gridDim.x);
  const TileDesc td = gload(tiles, tile);
  const gptr<const int32_t> rp = to_global(row_ptr), cl = to_global(col);
  const gptr<const double> wv = to_global(w), vxg = to_global(vx);
  const int ns = td.r1 - td.r0, n = td.p1 - td.p0;
  // a row longer than the tile class's limit has a tile of its own
  const bool long_row = ns == 1 && n > TCL::kLong;
  if (!long_row) {
    for (int k = threadIdx.x; k <= ns; k += kBlock) loff[k] = rp[td.r0 + k] - td.p0;
    __syncthreads();
    fill_segment_ids(loff, ns, seg);
  }
  auto gval = [&](int64_t r, int32_t q) -> double {
    return r < N ? load_x(x, dt, r * ld + q) : vxg[(r - N) * C + q];
  };
  for (int32_t q0 = 0; q0 < C; q0 += kEvalCols) {
    const int cb = C - q0 < kEvalCols ? C - q0 : kEvalCols;
    for (int k = threadIdx.x; k < ns * cb; k += kBlock)
      grow[(k / cb) * kEvalCols + k % cb] = gval(td.r0 + k / cb, q0 + k % cb);
    __syncthreads();
    double s[kEvalCols] = {}, n2[kEvalCols] = {};
    for (int r = threadIdx.x; r < ns; r += kBlock)
      if (td.r0 + r < N)
        for (int q = 0; q < cb; ++q) n2[q] += grow[r * kEvalCols + q] * grow[r * kEvalCols + q];
    int i = threadIdx.x;
    for (; i + 3 * kBlock < n; i += 4 * kBlock) {
      int32_t j[4];
      double wj[4], gj[4][kEvalCols];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        j[u] = cl[td.p0 + i + u * kBlock];
        wj[u] = wv[td.p0 + i + u * kBlock];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < kEvalCols; ++q) gj[u][q] = q < cb ? gval(j[u], q0 + q) : 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int r = long_row ? 0 : seg[i + u * kBlock];
#pragma unroll
        for (int q = 0; q < kEvalCols; ++q) {
          const double d = grow[r * kEvalCols + q] - gj[u][q];
          if (q < cb) s[q] += wj[u] * (d * d);
        }
      }
    }
    for (; i < n; i += kBlock) {
      const int32_t j = cl[td.p0 + i];
      const double wj = wv[td.p0 + i];
      const int r = long_row ? 0 : seg[i];
      for (int q = 0; q < cb; ++q) {
        const double d = grow[r * kEvalCols + q] - gval(j, q0 + q);
        s[q] += wj * (d * d);
      }
    }
    for (int q = 0; q < cb; ++q) {
      red[threadIdx.x] = 0.5 * s[q];
      __syncthreads();
      for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
      }
      if (threadIdx.x == 0) part[static_cast<int64_t>(tile) * 2 * C + q0 + q] = red[0];
      __syncthreads();
      red[threadIdx.x] = n2[q];
      __syncthreads();
      for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
      }
      if (threadIdx.x == 0) part[static_cast<int64_t>(tile) * 2 * C + C + q0 + q] = red[0];
      __syncthreads();
    }
  }
}

// 64 nets per wave, a lane per net: a net of at most kShortNet pins is
// handled by its lane (four pin loads in flight), every longer net of the
// wave by the whole wave (lanes over its pins, min and max by shuffles), so
// a 1000-pin net costs a few memory latencies instead of a thousand.  Min
// and max are exact, so each net's max - min does not depend on who formed
// it; a block sums its 256 nets by a fixed tree.  part[block * C + q].  Pin
// offsets are clamped to [0, P) and pins outside [0, N) are skipped, so a
// malformed netlist cannot lead to reads out of bounds.
constexpr int64_t kShortNet = 16;

__global__ __launch_bounds__(kBlock) void k_eval_hpwl(const int64_t *net_ptr,
                                                      const int32_t *pin, int64_t E, int64_t P,
                                                      int64_t N, const void *x, int64_t ld,
                                                      int32_t dt, int32_t C, double *part) {
  __shared__ double red[kBlock];
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  const gptr<const int64_t> np = to_global(net_ptr);
  const gptr<const int32_t> pc = to_global(pin);
  int64_t lo = 0, hi = 0;
  if (e < E) {
    lo = np[e];
    hi = np[e + 1];
    lo = lo < 0 ? 0 : (lo > P ? P : lo);
    hi = hi < lo ? lo : (hi > P ? P : hi);
  }
  const bool is_long = hi - lo > kShortNet;
  for (int32_t q = 0; q < C; ++q) {
    double h = 0.0;
    if (!is_long) {
      double mn = 0.0, mx = 0.0;
      bool any = false;
      int64_t p = lo;
      for (; p + 3 < hi; p += 4) {
        int64_t c[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) c[u] = pc[p + u];
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = (c[u] >= 0 && c[u] < N) ? load_x(x, dt, c[u] * ld + q) : 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (c[u] < 0 || c[u] >= N) continue;
          mn = !any || v[u] < mn ? v[u] : mn;
          mx = !any || v[u] > mx ? v[u] : mx;
          any = true;
        }
      }
      for (; p < hi; ++p) {
        const int64_t c = pc[p];
        if (c < 0 || c >= N) continue;
        const double v = load_x(x, dt, c * ld + q);
        mn = !any || v < mn ? v : mn;
        mx = !any || v > mx ? v : mx;
        any = true;
      }
      if (any) h = mx - mn;
    }
    // the wave's long nets, one after another, by all its lanes
    unsigned long long m = __ballot(is_long);
    while (m) {
      const int src = __builtin_ctzll(m);
      m &= m - 1;
      const int64_t plo = __shfl(lo, src), phi = __shfl(hi, src);
      double mn = 0.0, mx = 0.0;
      int any = 0;
      for (int64_t p = plo + lane; p < phi; p += kWave) {
        const int64_t c = pc[p];
        if (c < 0 || c >= N) continue;
        const double v = load_x(x, dt, c * ld + q);
        mn = !any || v < mn ? v : mn;
        mx = !any || v > mx ? v : mx;
        any = 1;
      }
      for (int off = kWave / 2; off > 0; off >>= 1) {
        const double omn = __shfl_xor(mn, off), omx = __shfl_xor(mx, off);
        const int oany = __shfl_xor(any, off);
        if (oany && (!any || omn < mn)) mn = omn;
        if (oany && (!any || omx > mx)) mx = omx;
        any = any | oany;
      }
      if (lane == src && any) h = mx - mn;
    }
    red[threadIdx.x] = h;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[static_cast<int64_t>(blockIdx.x) * C + q] = red[0];
    __syncthreads();
  }
}

// out[k] = sum over b < nb of part[b * stride + k]: one block per k, in a
// fixed order (block_sum_strided), the same on every run.
__global__ __launch_bounds__(kBlock) void k_eval_reduce(const double *part, int64_t nb,
                                                        int32_t stride, double *out) {
  __shared__ double red[kBlock];
  const double s = block_sum_strided(part + blockIdx.x, nb, stride, red);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// res[3C + q] = S / |g|^2 (the Rayleigh quotient of eq. smoothness_ray), 0
// for a zero signal.
__global__ void k_eval_rayleigh(double *res, int32_t C) {
  const int q = threadIdx.x;
  if (q >= C) return;
  const double n2 = res[C + q];
  res[3 * C + q] = n2 > 0.0 ? res[q] / n2 : 0.0;
}

}  // namespace
}  // namespace gift

using namespace gift;

extern "C" gift_status gift_evaluate_placement(const gift_graph *g, const void *x,
                                               int32_t num_cols, int64_t ld, int32_t dtype,
                                               const int64_t *net_ptr, const int32_t *pin_cell,
                                               int64_t num_nets, int64_t num_pins,
                                               double *smoothness, double *norm2,
                                               double *rayleigh, double *hpwl, void *stream) {
  clear_error();
  if (!g) return set_error(GIFT_EINVAL, "gift_evaluate_placement: NULL graph");
  if (num_cols < 1 || num_cols > 128) return set_error(GIFT_EINVAL, "num_cols %d not in [1, 128]", num_cols);
  if (ld < num_cols) return set_error(GIFT_EINVAL, "leading dimension smaller than num_cols");
  if (dtype != GIFT_F32 && dtype != GIFT_F64)
    return set_error(GIFT_EUNSUPPORTED, "dtype must be F32 or F64");
  if (hpwl && (num_nets < 0 || num_pins < 0 || !net_ptr || (num_pins > 0 && !pin_cell)))
    return set_error(GIFT_EINVAL, "hpwl needs the netlist (device net_ptr and pin_cell)");
  if (g->num_cells > 0 && !x) return set_error(GIFT_EINVAL, "x is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t N = g->num_cells, V = g->num_virtual;
  const int32_t C = num_cols;
  Scratch sc(st);
  double *vx = nullptr, *res = nullptr;
  GIFT_TRY(sc.get(&vx, (V > 0 ? V : 1) * C, "star means"));
  GIFT_TRY(sc.get(&res, 4 * C, "metrics"));
  GIFT_HIP(hipMemsetAsync(res, 0, sizeof(double) * 4 * C, st));
  const int64_t T = g->num_tiles[0];
  if (V > 0) {
    k_eval_star_means<<<grid_for(V * kWave), kBlock, 0, st>>>(g->row_ptr, g->col, N, V, x, ld,
                                                              dtype, C, vx);
    GIFT_TRY(check_launch("k_eval_star_means"));
  }
  if (T > 0) {
    double *part = nullptr;
    GIFT_TRY(sc.get(&part, T * 2 * C, "smoothness partial sums"));
    k_eval_smooth<<<static_cast<unsigned>(T), kBlock, 0, st>>>(g->tiles[0], g->row_ptr, g->col,
                                                              g->w, N, x, ld, dtype, vx, C, part);
    GIFT_TRY(check_launch("k_eval_smooth"));
    k_eval_reduce<<<static_cast<unsigned>(2 * C), kBlock, 0, st>>>(part, T, 2 * C, res);
    GIFT_TRY(check_launch("k_eval_reduce"));
  }
  if (hpwl && num_nets > 0) {
    const int64_t nb = (num_nets + kBlock - 1) / kBlock;
    double *part = nullptr;
    GIFT_TRY(sc.get(&part, nb * C, "hpwl partial sums"));
    k_eval_hpwl<<<static_cast<unsigned>(nb), kBlock, 0, st>>>(net_ptr, pin_cell, num_nets,
                                                              num_pins, N, x, ld, dtype, C, part);
    GIFT_TRY(check_launch("k_eval_hpwl"));
    k_eval_reduce<<<static_cast<unsigned>(C), kBlock, 0, st>>>(part, nb, C, res + 2 * C);
    GIFT_TRY(check_launch("k_eval_reduce"));
  }
  k_eval_rayleigh<<<1, C, 0, st>>>(res, C);
  GIFT_TRY(check_launch("k_eval_rayleigh"));
  std::vector<double> h(4 * C);
  GIFT_HIP(hipMemcpyAsync(h.data(), res, sizeof(double) * 4 * C, hipMemcpyDeviceToHost, st));
  GIFT_HIP(hipStreamSynchronize(st));
  for (int32_t q = 0; q < C; ++q) {
    if (smoothness) smoothness[q] = h[q];
    if (norm2) norm2[q] = h[C + q];
    if (rayleigh) rayleigh[q] = h[3 * C + q];
    if (hpwl) hpwl[q] = h[2 * C + q];
  }
  return GIFT_OK;
}
