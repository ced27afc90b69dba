// Import of a caller-supplied weighted graph: the undirected weighted graph of
// Section 2.1 (A = {w_ij}, D = diag(sum_j w_ij)) that Algorithm 1 takes as its
// input, given directly as a canonical CSR instead of a netlist.  The result
// is the same resident graph gift_build_graph makes (every row a cell, no
// star rows): degrees, SpMM row tiles and, per sigma, the normalised values
// of eq. A_formulation.
#include <cmath>

#include "common.h"
#include "devutil.h"

namespace gift {
namespace {

// One thread per row: checks the row (offsets non-decreasing and inside
// [0, nnz]; columns in [0, R), strictly ascending, never the row itself;
// weights finite and >= 0), writes its 32-bit offset and its float64 degree
// summed in ascending column.  Thread R writes the closing offset and checks
// that it equals nnz.  Any violation sets bit 0 of *flag.
__global__ void k_import_rows(const int64_t *rp, const int32_t *col, const double *w, int64_t R,
                              int64_t nnz, int32_t *rp32, double *deg,
                              unsigned long long *flag) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i > R) return;
  const int64_t a = rp[i];
  bool bad = a < 0 || a > nnz || (i == 0 && a != 0) || (i == R && a != nnz);
  rp32[i] = static_cast<int32_t>(bad ? 0 : a);
  if (i == R) {
    if (bad) atomicOr(flag, 1ull);
    return;
  }
  const int64_t b = rp[i + 1];
  double d = 0.0;
  if (bad || b < a || b > nnz) {
    bad = true;
  } else {
    int64_t prev = -1;
    for (int64_t p = a; p < b; ++p) {
      const int64_t c = col[p];
      const double v = w[p];
      if (c < 0 || c >= R || c == i || c <= prev || !(v >= 0.0) || !isfinite(v)) bad = true;
      prev = c;
      d = d + v;
    }
  }
  deg[i] = bad ? 0.0 : d;
  if (bad) atomicOr(flag, 1ull);
}

gift_status import_impl(const gift_csr_desc *d, hipStream_t st, gift_graph *g) {
  const int64_t R = d->num_rows, nnz = d->nnz;
  Scratch sc(st);
  const bool host = d->mem_space == GIFT_MEM_HOST;
  int64_t *rp64 = nullptr;
  GIFT_TRY(sc.get(&rp64, R + 1, "imported row offsets"));
  GIFT_TRY(dev_alloc(reinterpret_cast<void **>(&g->row_ptr), (R + 1) * sizeof(int32_t), st,
                     "row offsets"));
  GIFT_TRY(dev_alloc(reinterpret_cast<void **>(&g->col), (nnz > 0 ? nnz : 1) * sizeof(int32_t),
                     st, "columns"));
  GIFT_TRY(dev_alloc(reinterpret_cast<void **>(&g->w), (nnz > 0 ? nnz : 1) * sizeof(double), st,
                     "weights"));
  GIFT_TRY(dev_alloc(reinterpret_cast<void **>(&g->deg), (R > 0 ? R : 1) * sizeof(double), st,
                     "degrees"));
  g->bytes += (R + 1) * 4 + nnz * 12 + R * 8;
  const hipMemcpyKind kind = host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  GIFT_HIP(hipMemcpyAsync(rp64, d->row_ptr, (R + 1) * sizeof(int64_t), kind, st));
  if (nnz > 0) {
    GIFT_HIP(hipMemcpyAsync(g->col, d->col, nnz * sizeof(int32_t), kind, st));
    GIFT_HIP(hipMemcpyAsync(g->w, d->w, nnz * sizeof(double), kind, st));
  }
  unsigned long long *flag = nullptr;
  int64_t *tile_counts = nullptr;
  GIFT_TRY(sc.get(&flag, 1, "import check flag"));
  GIFT_TRY(sc.get(&tile_counts, 2 * kTileClasses, "tile counts"));
  GIFT_HIP(hipMemsetAsync(flag, 0, sizeof(*flag), st));
  k_import_rows<<<grid_for(R + 1), kBlock, 0, st>>>(rp64, g->col, g->w, R, nnz, g->row_ptr, g->deg,
                                                    flag);
  GIFT_TRY(check_launch("k_import_rows"));
  int32_t *tstart[kTileClasses];
  for (int c = 0; c < kTileClasses; ++c) GIFT_TRY(sc.get(&tstart[c], R + 2, "tile starts"));
  static_assert(kTileClasses == 2, "both SpMM tile classes are built in one pass");
  GIFT_TRY(build_tiles64_pair(rp64, R, R, kSpmmTiles[0], kSpmmTiles[1], st, tstart[0], tstart[1],
                              tile_counts, tile_counts + 2));
  int64_t h[1 + 2 * kTileClasses] = {};
  const int64_t *ptrs[1 + 2 * kTileClasses];
  ptrs[0] = reinterpret_cast<const int64_t *>(flag);
  for (int i = 0; i < 2 * kTileClasses; ++i) ptrs[1 + i] = tile_counts + i;
  GIFT_TRY(read_scalars(st, ptrs, 1 + 2 * kTileClasses, h));
  if (h[0] != 0)
    return set_error(GIFT_EINVAL,
                     "malformed CSR: row_ptr must start at 0, not decrease and end at nnz; "
                     "columns must lie in [0, R), ascend strictly within a row and avoid the "
                     "diagonal; weights must be finite and >= 0");
  for (int c = 0; c < kTileClasses; ++c) {
    g->num_tiles[c] = h[1 + 2 * c];
    g->num_tiles_cells[c] = h[2 + 2 * c];
    GIFT_TRY(dev_alloc(reinterpret_cast<void **>(&g->tiles[c]),
                       (g->num_tiles[c] + 1) * sizeof(TileDesc), st, "row tiles"));
    g->bytes += (g->num_tiles[c] + 1) * static_cast<int64_t>(sizeof(TileDesc));
    GIFT_TRY(tile_descs(tstart[c], rp64, g->num_tiles[c], st, g->tiles[c]));
  }
  for (int32_t i = 0; i < d->num_sigmas; ++i) GIFT_TRY(prepare_sigma(g, d->sigmas[i], st));
  return GIFT_OK;
}

}  // namespace
}  // namespace gift

using namespace gift;

extern "C" gift_status gift_graph_import_csr(const gift_csr_desc *d, void *stream,
                                             gift_graph **out) {
  clear_error();
  if (!out) return set_error(GIFT_EINVAL, "gift_graph_import_csr: out is NULL");
  *out = nullptr;
  if (!d) return set_error(GIFT_EINVAL, "gift_graph_import_csr: desc is NULL");
  if (d->num_rows < 0 || d->nnz < 0) return set_error(GIFT_EINVAL, "negative num_rows or nnz");
  if (d->num_rows >= (int64_t(1) << 31) - 1 || d->nnz >= (int64_t(1) << 31) - 1)
    return set_error(GIFT_EUNSUPPORTED, "graphs are limited to 2^31 - 2 rows and entries");
  if (!d->row_ptr || (d->nnz > 0 && (!d->col || !d->w)))
    return set_error(GIFT_EINVAL, "row_ptr / col / w is NULL");
  if (d->mem_space != GIFT_MEM_HOST && d->mem_space != GIFT_MEM_DEVICE)
    return set_error(GIFT_EINVAL, "bad mem_space %d", d->mem_space);
  if (!dtype_valid(d->storage)) return set_error(GIFT_EINVAL, "bad storage dtype %d", d->storage);
  if (d->reserved != 0) return set_error(GIFT_EINVAL, "reserved must be 0");
  if (d->num_sigmas < 1 || !d->sigmas) return set_error(GIFT_EINVAL, "need at least one sigma");
  for (int32_t i = 0; i < d->num_sigmas; ++i)
    if (!(d->sigmas[i] >= 0.0) || !std::isfinite(d->sigmas[i]))
      return set_error(GIFT_EINVAL, "sigma[%d] = %g is not a finite value >= 0", i, d->sigmas[i]);
  if (d->mem_space == GIFT_MEM_HOST && (d->row_ptr[0] != 0 || d->row_ptr[d->num_rows] != d->nnz))
    return set_error(GIFT_EINVAL, "row_ptr must start at 0 and end at nnz");
  hipStream_t st = static_cast<hipStream_t>(stream);
  gift_graph *g = new (std::nothrow) gift_graph();
  if (!g) return set_error(GIFT_ENOMEM, "host allocation failed");
  g->num_cells = d->num_rows;
  g->num_virtual = 0;
  g->num_rows = d->num_rows;
  g->nnz = d->nnz;
  g->nnz_cells = d->nnz;
  g->storage = d->storage;
  g->weight_model = -1;  // not built from a netlist
  g->star_threshold = 0;
  (void)hipGetDevice(&g->device);
  gift_status s = import_impl(d, st, g);
  if (s != GIFT_OK) {
    std::string msg = gift_last_error();
    gift_destroy_graph(g, stream);
    set_error(s, "%s", msg.c_str());
    return s;
  }
  *out = g;
  return GIFT_OK;
}
