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
// nets (HPWL) in a fixed order and the partial sums are added in tile order,
// so the results are deterministic.
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

// One row tile per block: sum over its rows of sum_j w_ij (g_i - g_j)^2 and,
// for cell rows, g_i^2; one thread per row, rows summed in order by a block
// tree of fixed shape.  part[tile * 2C + q] = S part, [.. + C + q] = norm2.
__global__ __launch_bounds__(kBlock) void k_eval_smooth(const TileDesc *tiles,
                                                        const int32_t *row_ptr,
                                                        const int32_t *col, const double *w,
                                                        int64_t N, const void *x, int64_t ld,
                                                        int32_t dt, const double *vx,
                                                        int32_t C, double *part) {
  __shared__ double red[kBlock];
  const uint32_t tile = xcd_remap(blockIdx.x, gridDim.x);
  const TileDesc td = gload(tiles, tile);
  const gptr<const int32_t> rp = to_global(row_ptr), cl = to_global(col);
  const gptr<const double> wv = to_global(w), vxg = to_global(vx);
  for (int32_t q = 0; q < C; ++q) {
    double s = 0.0, n2 = 0.0;
    for (int32_t r = td.r0 + threadIdx.x; r < td.r1; r += kBlock) {
      const double gi = r < N ? load_x(x, dt, r * ld + q) : vxg[(r - N) * C + q];
      if (r < N) n2 += gi * gi;
      for (int32_t p = rp[r]; p < rp[r + 1]; ++p) {
        const int32_t j = cl[p];
        const double gj = j < N ? load_x(x, dt, j * ld + q) : vxg[(j - N) * C + q];
        const double d = gi - gj;
        s += wv[p] * (d * d);
      }
    }
    // each edge appears in both of its rows
    s *= 0.5;
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[static_cast<int64_t>(tile) * 2 * C + q] = red[0];
    __syncthreads();
    red[threadIdx.x] = n2;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[static_cast<int64_t>(tile) * 2 * C + C + q] = red[0];
    __syncthreads();
  }
}

// One net per thread: max - min of g over its pins, per column; a block sums
// its nets by a fixed tree.  part[block * C + q].  Pin offsets are clamped to
// [0, P) and pins outside [0, N) are skipped, so a malformed netlist cannot
// lead to reads out of bounds.
__global__ __launch_bounds__(kBlock) void k_eval_hpwl(const int64_t *net_ptr,
                                                      const int32_t *pin, int64_t E, int64_t P,
                                                      int64_t N, const void *x, int64_t ld,
                                                      int32_t dt, int32_t C, double *part) {
  __shared__ double red[kBlock];
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const gptr<const int64_t> np = to_global(net_ptr);
  const gptr<const int32_t> pc = to_global(pin);
  int64_t lo = 0, hi = 0;
  if (e < E) {
    lo = np[e];
    hi = np[e + 1];
    lo = lo < 0 ? 0 : (lo > P ? P : lo);
    hi = hi < lo ? lo : (hi > P ? P : hi);
  }
  for (int32_t q = 0; q < C; ++q) {
    double h = 0.0, mn = 0.0, mx = 0.0;
    bool any = false;
    for (int64_t p = lo; p < hi; ++p) {
      const int64_t c = pc[p];
      if (c < 0 || c >= N) continue;
      const double v = load_x(x, dt, c * ld + q);
      mn = !any || v < mn ? v : mn;
      mx = !any || v > mx ? v : mx;
      any = true;
    }
    if (any) h = mx - mn;
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

// out[k] = sum over b of part[b * stride + k] for k < width, in order of b
// (one thread per k: a sequential sum, the same order on every run).
__global__ void k_eval_reduce(const double *part, int64_t nb, int32_t stride, int32_t width,
                              double *out) {
  const int k = threadIdx.x;
  if (k >= width) return;
  double s = 0.0;
  for (int64_t b = 0; b < nb; ++b) s += part[b * stride + k];
  out[k] = s;
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
    k_eval_reduce<<<1, 2 * C, 0, st>>>(part, T, 2 * C, 2 * C, res);
    GIFT_TRY(check_launch("k_eval_reduce"));
  }
  if (hpwl && num_nets > 0) {
    const int64_t nb = (num_nets + kBlock - 1) / kBlock;
    double *part = nullptr;
    GIFT_TRY(sc.get(&part, nb * C, "hpwl partial sums"));
    k_eval_hpwl<<<static_cast<unsigned>(nb), kBlock, 0, st>>>(net_ptr, pin_cell, num_nets,
                                                              num_pins, N, x, ld, dtype, C, part);
    GIFT_TRY(check_launch("k_eval_hpwl"));
    k_eval_reduce<<<1, C, 0, st>>>(part, nb, C, C, res + 2 * C);
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
