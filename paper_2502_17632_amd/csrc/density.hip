// Bin density of a placement (Section 2.2, eq. density_eq): the region
// [xl, xh] x [yl, yh] is cut into nbx x nby equal bins and every bin gets the
// overlap area of each object's rectangle (width w_v, height h_v, centred at
// the object's position) with it.  A block takes a contiguous range of
// objects, a thread per object adds its overlaps with the bins it covers into
// an LDS table of the block's bins, and the block then adds each of its bins
// to the map once (placements crowd many objects into few bins, and device
// atomics on one address serialise).  The sums are kept in 64-bit fixed
// point (2^-40 of a bin's area per unit), so the additions are exact and the
// result does not depend on their order; the map is then converted to
// float64.
#include <cmath>

#include "common.h"
#include "devutil.h"

namespace gift {
namespace {

constexpr double kFixScale = 1099511627776.0;  // 2^40 units per bin area

__device__ __forceinline__ double load_pos(const void *p, int32_t dt, int64_t i) {
  return dt == GIFT_F64 ? to_global(static_cast<const double *>(p))[i]
                        : static_cast<double>(to_global(static_cast<const float *>(p))[i]);
}

struct DensityArgs {
  const void *x;
  int64_t n, ld;
  int32_t dtype;
  const double *w, *h;  // per object, or NULL: w0 / h0
  double w0, h0;
  double xl, yl, bw, bh;
  int32_t nbx, nby;
  unsigned long long *acc;  // nby x nbx fixed-point sums
};

constexpr int kDensityBlocks = 2048;
constexpr int kDensitySlots = 1024;

__device__ __forceinline__ void add_object(const DensityArgs &a, int64_t v,
                                           LdsHash<unsigned long long, kDensitySlots> &h) {
  const double cx = load_pos(a.x, a.dtype, v * a.ld), cy = load_pos(a.x, a.dtype, v * a.ld + 1);
  const double wv = a.w ? to_global(a.w)[v] : a.w0, hv = a.h ? to_global(a.h)[v] : a.h0;
  if (!(wv > 0.0) || !(hv > 0.0) || !std::isfinite(cx) || !std::isfinite(cy)) return;
  const double x0 = cx - 0.5 * wv, x1 = cx + 0.5 * wv;
  const double y0 = cy - 0.5 * hv, y1 = cy + 0.5 * hv;
  // covered bin range, clamped to the grid
  const double fi0 = std::floor((x0 - a.xl) / a.bw), fi1 = std::floor((x1 - a.xl) / a.bw);
  const double fj0 = std::floor((y0 - a.yl) / a.bh), fj1 = std::floor((y1 - a.yl) / a.bh);
  if (fi1 < 0 || fj1 < 0 || fi0 >= a.nbx || fj0 >= a.nby) return;
  const int i0 = fi0 < 0 ? 0 : static_cast<int>(fi0);
  const int i1 = fi1 >= a.nbx ? a.nbx - 1 : static_cast<int>(fi1);
  const int j0 = fj0 < 0 ? 0 : static_cast<int>(fj0);
  const int j1 = fj1 >= a.nby ? a.nby - 1 : static_cast<int>(fj1);
  const double inv_area = 1.0 / (a.bw * a.bh);
  for (int j = j0; j <= j1; ++j) {
    const double b0 = a.yl + j * a.bh, b1 = b0 + a.bh;
    const double ly = fmin(y1, b1) - fmax(y0, b0);
    if (ly <= 0.0) continue;
    for (int i = i0; i <= i1; ++i) {
      const double c0 = a.xl + i * a.bw, c1 = c0 + a.bw;
      const double lx = fmin(x1, c1) - fmax(x0, c0);
      if (lx <= 0.0) continue;
      const unsigned long long q =
          static_cast<unsigned long long>(llrint(lx * ly * inv_area * kFixScale));
      h.add(j * a.nbx + i, q, a.acc);
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_density(DensityArgs a) {
  __shared__ LdsHash<unsigned long long, kDensitySlots> h;
  h.clear();
  __syncthreads();
  const int64_t per = (a.n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = static_cast<int64_t>(blockIdx.x) * per;
  const int64_t hi = lo + per < a.n ? lo + per : a.n;
  for (int64_t v = lo + threadIdx.x; v < hi; v += kBlock) add_object(a, v, h);
  __syncthreads();
  h.flush(a.acc);
}

__global__ void k_density_out(const unsigned long long *acc, int64_t nb, double area,
                              double *out) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k < nb) out[k] = static_cast<double>(acc[k]) / kFixScale * area;
}

// Overflow partial sums: block b sums max(0, rho_k - cap) over its fixed
// range of bins (a block tree of fixed shape), part[b].
constexpr int kOverflowBlocks = 256;
__global__ __launch_bounds__(kBlock) void k_overflow_part(const double *density, int64_t nb,
                                                          double cap, double *part) {
  __shared__ double red[kBlock];
  const int64_t per = (nb + gridDim.x - 1) / gridDim.x;
  const int64_t lo = static_cast<int64_t>(blockIdx.x) * per;
  const int64_t hi = lo + per < nb ? lo + per : nb;
  double s = 0.0;
  for (int64_t k = lo + threadIdx.x; k < hi; k += kBlock) {
    const double e = density[k] - cap;
    if (e > 0.0) s += e;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out = (sum of part in block order) / total_area
__global__ void k_overflow_total(const double *part, int nparts, double total_area,
                                 double *out) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < nparts; ++b) s += part[b];
  out[0] = s / total_area;
}

}  // namespace
}  // namespace gift

using namespace gift;

extern "C" gift_status gift_density_overflow(const double *density, int32_t nbx, int32_t nby,
                                             double xl, double yl, double xh, double yh,
                                             double target, double total_area,
                                             double *overflow, void *stream) {
  clear_error();
  if (!density || !overflow) return set_error(GIFT_EINVAL, "gift_density_overflow: NULL buffer");
  if (nbx < 1 || nby < 1 || static_cast<int64_t>(nbx) * nby > (int64_t(1) << 28))
    return set_error(GIFT_EINVAL, "bin grid %d x %d", nbx, nby);
  if (!(xh > xl) || !(yh > yl) || !std::isfinite(xh - xl) || !std::isfinite(yh - yl))
    return set_error(GIFT_EINVAL, "empty or infinite placement region");
  if (!(total_area > 0.0) || !std::isfinite(total_area) || !std::isfinite(target))
    return set_error(GIFT_EINVAL, "total_area must be finite and > 0, target finite");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t nb = static_cast<int64_t>(nbx) * nby;
  const double cap = target * (((xh - xl) / nbx) * ((yh - yl) / nby));
  Scratch sc(st);
  double *part = nullptr;
  GIFT_TRY(sc.get(&part, kOverflowBlocks + 1, "overflow partial sums"));
  k_overflow_part<<<kOverflowBlocks, kBlock, 0, st>>>(density, nb, cap, part);
  GIFT_TRY(check_launch("k_overflow_part"));
  k_overflow_total<<<1, kWave, 0, st>>>(part, kOverflowBlocks, total_area, part + kOverflowBlocks);
  GIFT_TRY(check_launch("k_overflow_total"));
  GIFT_HIP(hipMemcpyAsync(overflow, part + kOverflowBlocks, sizeof(double), hipMemcpyDeviceToHost,
                          st));
  GIFT_HIP(hipStreamSynchronize(st));
  return GIFT_OK;
}

extern "C" gift_status gift_bin_density(const void *x, int64_t num_objects, int64_t ld,
                                        int32_t dtype, const double *widths,
                                        const double *heights, double w0, double h0, double xl,
                                        double yl, double xh, double yh, int32_t nbx,
                                        int32_t nby, double *density, void *stream) {
  clear_error();
  if (num_objects < 0) return set_error(GIFT_EINVAL, "num_objects < 0");
  if (ld < 2) return set_error(GIFT_EINVAL, "ld must be >= 2 (x, y columns)");
  if (dtype != GIFT_F32 && dtype != GIFT_F64)
    return set_error(GIFT_EUNSUPPORTED, "dtype must be F32 or F64");
  if (nbx < 1 || nby < 1 || static_cast<int64_t>(nbx) * nby > (int64_t(1) << 28))
    return set_error(GIFT_EINVAL, "bin grid %d x %d", nbx, nby);
  if (!(xh > xl) || !(yh > yl) || !std::isfinite(xh - xl) || !std::isfinite(yh - yl))
    return set_error(GIFT_EINVAL, "empty or infinite placement region");
  if ((!widths && !(w0 > 0.0)) || (!heights && !(h0 > 0.0)))
    return set_error(GIFT_EINVAL, "object size must be > 0");
  if (!density || (num_objects > 0 && !x)) return set_error(GIFT_EINVAL, "NULL buffer");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t nb = static_cast<int64_t>(nbx) * nby;
  Scratch sc(st);
  unsigned long long *acc = nullptr;
  GIFT_TRY(sc.get(&acc, nb, "density sums"));
  GIFT_HIP(hipMemsetAsync(acc, 0, sizeof(unsigned long long) * nb, st));
  const double bw = (xh - xl) / nbx, bh = (yh - yl) / nby;
  if (num_objects > 0) {
    DensityArgs a{x, num_objects, ld, dtype, widths, heights, w0, h0, xl, yl, bw, bh, nbx, nby,
                  acc};
    const int64_t blocks = (num_objects + kBlock - 1) / kBlock;
    k_density<<<static_cast<unsigned>(blocks < kDensityBlocks ? blocks : kDensityBlocks), kBlock,
                0, st>>>(a);
    GIFT_TRY(check_launch("k_density"));
  }
  k_density_out<<<grid_for(nb), kBlock, 0, st>>>(acc, nb, bw * bh, density);
  return check_launch("k_density_out");
}
