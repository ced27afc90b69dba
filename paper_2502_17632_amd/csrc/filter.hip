// Multi-order graph filter g' = sum_t alpha_t A~_{sigma_t}^{k_t} g
// (Section 3.2.1, eq. proposed_filter; the powers are the repeated sparse
// products of the complexity paragraph in Section 3.2.2).
//
// Per distinct sigma the signal goes through k_max SpMM passes
//     x_k[i] = sum_j a_ij x_{k-1}[j] + diag_i x_{k-1}[i]
// (storage-type values and signals, float32 or float64 accumulation).  The
// last pass of the last sigma also forms the float64 combine of all terms, in
// term order, and writes the caller's output; iterates needed by earlier terms
// are kept in their own buffers.
//
// The pass is bound by memory traffic (about 0.4 flop per algorithmic byte):
// it streams each tile's col/values once and gathers signal rows.  One block
// per row tile: all of a thread's loads are issued at once (col/values, the
// rows' offsets and diagonal, then the gathers), products are staged in LDS
// and each row is summed by a group of lanes sized to the tile.  Blocks are
// remapped so each XCD works on chunks of consecutive tiles (xcd_remap).
//
// The same launch sequence serves one graph and a batch of graphs: in a batch
// every tile names its graph, whose CSR, values, I/O and row offset in the
// shared signal buffers come from a small device table.
//
// With BF16/F16 storage the iterates of each sigma group hold x - c v, v the
// eigenvalue-1 eigenvector sqrt(d + sigma) of A~_sigma (Theorem 1 with the
// self-loop) and c per graph and column, so the 16-bit rounding acts on the
// placement's deviation rather than on its absolute coordinates; the last
// pass adds c v back in its float64 combine (k_centre_part, k_centre_final).
#include <cmath>
#include <cstring>
#include <mutex>

#include "common.h"
#include "devutil.h"
#include "filter.h"

namespace gift {

namespace {

template <typename T, int C>
struct SigRow {
  static constexpr int kBytes = static_cast<int>(sizeof(T)) * C;
  static constexpr int kAlign = kBytes >= 16 ? 16 : kBytes;
  struct alignas(kAlign) V {
    T v[C];
  };
};

template <typename T, int C>
__device__ __forceinline__ typename SigRow<T, C>::V load_row(const T *x, int64_t r) {
  return gload(reinterpret_cast<const typename SigRow<T, C>::V *>(x), r);
}

__device__ __forceinline__ double load_in(const void *p, int32_t dt, int64_t i) {
  return dt == GIFT_F64 ? to_global(static_cast<const double *>(p))[i]
                        : static_cast<double>(to_global(static_cast<const float *>(p))[i]);
}

// Tiles and graphs of one launch: a single graph (`one`, kBatch false) or a
// batch (`graphs` indexed by `tile_graph`, kBatch true).
struct LaunchArgs {
  const TileDesc *tiles;
  const int32_t *tile_graph;
  const GraphDev *graphs;
  GraphDev one;
  // centring multipliers [graphs][groups][C] (16-bit storage), else NULL
  double *centre;
  // block b takes tile b (the list is laid out per XCD) rather than
  // xcd_remap(b)
  int32_t identity_map;
};

// Without the per-XCD layout, blocks take the tile list from its end, in
// chunks dealt to the XCDs: the star rows' tiles come last in the list, and
// each of their rows gathers its net's cells from around the design, so they
// start first instead of forming the launch's tail.  Every row is computed
// by the same arithmetic whichever block takes it.
__device__ __forceinline__ uint32_t tile_of_block(const LaunchArgs &l) {
  return l.identity_map ? blockIdx.x : gridDim.x - 1 - xcd_remap(blockIdx.x, gridDim.x);
}

template <bool kBatch>
__device__ __forceinline__ GraphDev graph_of(const LaunchArgs &l, uint32_t tile) {
  if constexpr (kBatch) return gload(l.graphs, to_global(l.tile_graph)[tile]);
  else return l.one;
}

template <bool kBatch>
__device__ __forceinline__ uint32_t graph_index(const LaunchArgs &l, uint32_t tile) {
  if constexpr (kBatch) return static_cast<uint32_t>(to_global(l.tile_graph)[tile]);
  else return 0;
}

struct FinalArgs {
  int32_t num_terms;
  int32_t in_dtype, out_dtype;
  int32_t col0;  // first column of this chunk in the caller's matrices
  const void *src[kMaxTerms];  // saved iterate of each term; NULL = this pass
  double alpha[kMaxTerms];
  // centring: each term's sigma group and sigma (the term's iterate holds
  // x - c v_sigma; the combine adds c v_sigma back)
  int32_t num_groups;
  int32_t term_group[kMaxTerms];
  double term_sigma[kMaxTerms];
};

// Writes local row `lr` of the pass result: the stored iterate, or (last
// pass) the float64 combine of all terms in term order.
template <int D, int C, bool kFinal>
__device__ __forceinline__ void emit_row(const FinalArgs &f, const GraphDev &gd,
                                         typename Store<D>::T *y, int64_t lr,
                                         const typename Store<D>::A *acc,
                                         const double *cen = nullptr) {
  using S = Store<D>;
  using T = typename S::T;
  if constexpr (!kFinal) {
    typename SigRow<T, C>::V out;
#pragma unroll
    for (int c = 0; c < C; ++c) out.v[c] = S::from_acc(acc[c]);
    gstore(reinterpret_cast<typename SigRow<T, C>::V *>(y), lr, out);
  } else {
    const GraphIO &io = gd.io;
    const bool fixed = io.fixed && to_global(io.fixed)[lr];
    const int64_t srow = gd.row_off + lr;
    double s[C];
    if (fixed) {
#pragma unroll
      for (int c = 0; c < C; ++c) s[c] = load_in(io.x_in, f.in_dtype, lr * io.ld_in + f.col0 + c);
    } else {
#pragma unroll
      for (int c = 0; c < C; ++c) s[c] = 0.0;
      const double dl = cen ? to_global(gd.deg)[lr] : 0.0;
      // every column sums the terms in term order; the saved rows of four
      // terms are loaded before any of them is added (one at a time above
      // four columns, where four would cost occupancy)
      constexpr int kTermBatch = C <= 4 ? 4 : 1;
      for (int t0 = 0; t0 < f.num_terms; t0 += kTermBatch) {
        double v[kTermBatch][C];
#pragma unroll
        for (int u = 0; u < kTermBatch; ++u) {
          const int t = t0 + u;
          const T *src = t < f.num_terms ? static_cast<const T *>(f.src[t]) : nullptr;
          if (src) {
            const auto row = load_row<T, C>(src, srow);
#pragma unroll
            for (int c = 0; c < C; ++c) v[u][c] = static_cast<double>(S::load(row.v[c]));
          } else {
#pragma unroll
            for (int c = 0; c < C; ++c) v[u][c] = static_cast<double>(acc[c]);
          }
        }
#pragma unroll
        for (int u = 0; u < kTermBatch; ++u) {
          const int t = t0 + u;
          if (t >= f.num_terms) break;
          if (cen) {
            const double vt = sqrt(dl + f.term_sigma[t]);
            const gptr<const double> ct = to_global(cen) + f.term_group[t] * C;
#pragma unroll
            for (int c = 0; c < C; ++c) v[u][c] = v[u][c] + ct[c] * vt;
          }
          const double a = f.alpha[t];
#pragma unroll
          for (int c = 0; c < C; ++c) s[c] = s[c] + a * v[u][c];
        }
      }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int64_t o = lr * io.ld_out + f.col0 + c;
      if (f.out_dtype == GIFT_F64) to_global(static_cast<double *>(io.y_out))[o] = s[c];
      else to_global(static_cast<float *>(io.y_out))[o] = static_cast<float>(s[c]);
    }
  }
}

// Lanes per row in the reduction of a tile with `rows` rows.
__device__ __forceinline__ int lanes_for(int rows) {
  int g = 1;
  while (g < 64 && rows * g * 2 <= kBlock) g <<= 1;
  return g;
}

// One SpMM pass over the tiles of this launch, one tile per block.
//
// Multi-row tile: every load is issued up front so a thread has all its
// col/value, offset and diagonal loads in flight at once, then all its
// gathers (an unused slot reads entry 0, which exists even in a graph without
// entries, and gathers row 0 of the tile's graph, not the column it read;
// unused row slots read row r0); the products are staged in LDS and each row is summed by a group
// of lanes sized to the tile's row count.  When the products would not fit
// the LDS budget (wide signal rows) the entries (col, value) are staged
// instead and the row groups gather the signal themselves.  Single long row:
// the whole block strides over the row and reduces across its waves.
template <int D, int C, bool kFinal, int TC, bool kBatch>
__global__ __launch_bounds__(kBlock) void k_spmm(LaunchArgs l, const void *xin, void *yout,
                                                 FinalArgs f) {
  using S = Store<D>;
  using T = typename S::T;
  using A = typename S::A;
  using TCL = TileClass<TC>;
  constexpr bool kStageProducts = C * sizeof(A) <= 8;
  constexpr int kStage = (TCL::kCap + kBlock - 1) / kBlock;
  __shared__ int32_t loff[TCL::kRows + 1];
  __shared__ A ldx[kStageProducts ? TCL::kRows * C : 1];
  __shared__ A lprod[kStageProducts ? TCL::kCap * C : 1];
  __shared__ int32_t lcol[kStageProducts ? 1 : TCL::kCap];
  __shared__ A lval[kStageProducts ? 1 : TCL::kCap];
  __shared__ A lred[kBlock / kWave][C];

  const uint32_t tile = tile_of_block(l);
  const int tid = threadIdx.x;
  const TileDesc td = gload(l.tiles, tile);
  const GraphDev gd = graph_of<kBatch>(l, tile);
  const int32_t r0 = td.r0, r1 = td.r1, p0 = td.p0, p1 = td.p1;
  const int nrows = r1 - r0;
  const int n = p1 - p0;
  const double *cen = kFinal && l.centre
                          ? l.centre + static_cast<int64_t>(graph_index<kBatch>(l, tile)) *
                                           f.num_groups * C
                          : nullptr;
  const T *x = static_cast<const T *>(xin) + gd.row_off * C;
  T *y = kFinal ? nullptr : static_cast<T *>(yout) + gd.row_off * C;
  const gptr<const T> val = to_global(static_cast<const T *>(gd.val));
  const gptr<const int32_t> col = to_global(gd.col);
  const gptr<const int32_t> row_ptr = to_global(gd.row_ptr);
  const gptr<const A> diag = to_global(static_cast<const A *>(gd.diag));

  if (nrows == 1 && n > TCL::kLong) {
    // single long row
    A acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0;
    int q = p0 + tid;
    for (; q + 3 * kBlock < p1; q += 4 * kBlock) {
      int32_t j[4];
      A v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        j[u] = col[q + u * kBlock];
        v[u] = S::load(val[q + u * kBlock]);
      }
      typename SigRow<T, C>::V xr[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) xr[u] = load_row<T, C>(x, j[u]);
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] += v[u] * S::load(xr[u].v[c]);
    }
    for (; q < p1; q += kBlock) {
      const auto xr = load_row<T, C>(x, col[q]);
      const A v = S::load(val[q]);
#pragma unroll
      for (int c = 0; c < C; ++c) acc[c] += v * S::load(xr.v[c]);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      for (int off = kWave / 2; off > 0; off >>= 1) acc[c] += __shfl_xor(acc[c], off);
      if ((tid & (kWave - 1)) == 0) lred[tid / kWave][c] = acc[c];
    }
    __syncthreads();
    if (tid == 0) {
      A tot[C];
      const A dg = diag[r0];
      const auto xi = load_row<T, C>(x, r0);
#pragma unroll
      for (int c = 0; c < C; ++c) {
        A s = lred[0][c];
        for (int w = 1; w < kBlock / kWave; ++w) s += lred[w][c];
        tot[c] = s + dg * S::load(xi.v[c]);
      }
      emit_row<D, C, kFinal>(f, gd, y, r0, tot, cen);
    }
    return;
  }

  // ---- multi-row tile (n <= kCap)
  {
    int32_t jj[kStage];
    A vv[kStage];
#pragma unroll
    for (int k = 0; k < kStage; ++k) {
      const int i = tid + k * kBlock;
      const int q = i < n ? p0 + i : 0;
      const int32_t c = col[q];
      jj[k] = i < n ? c : 0;  // an unused slot gathers row 0 of its graph
      vv[k] = S::load(val[q]);
    }
    constexpr int kRowIters = (TCL::kRows + 1 + kBlock - 1) / kBlock;
    int32_t ro[kRowIters];
#pragma unroll
    for (int k = 0; k < kRowIters; ++k) {
      const int i = tid + k * kBlock;
      ro[k] = row_ptr[i <= nrows ? r0 + i : r0];
    }
    constexpr int kDiagIters = (TCL::kRows + kBlock - 1) / kBlock;
    if constexpr (kStageProducts) {
      A dg[kDiagIters];
      typename SigRow<T, C>::V xr_row[kDiagIters];
#pragma unroll
      for (int k = 0; k < kDiagIters; ++k) {
        const int i = tid + k * kBlock;
        const int r = i < nrows ? r0 + i : r0;
        dg[k] = diag[r];
        xr_row[k] = load_row<T, C>(x, r);
      }
      typename SigRow<T, C>::V xv[kStage];
#pragma unroll
      for (int k = 0; k < kStage; ++k) xv[k] = load_row<T, C>(x, jj[k]);
#pragma unroll
      for (int k = 0; k < kStage; ++k) {
        const int i = tid + k * kBlock;
        if (i < n) {
#pragma unroll
          for (int c = 0; c < C; ++c) lprod[i * C + c] = vv[k] * S::load(xv[k].v[c]);
        }
      }
#pragma unroll
      for (int k = 0; k < kDiagIters; ++k) {
        const int i = tid + k * kBlock;
        if (i < nrows) {
#pragma unroll
          for (int c = 0; c < C; ++c) ldx[i * C + c] = dg[k] * S::load(xr_row[k].v[c]);
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < kStage; ++k) {
        const int i = tid + k * kBlock;
        if (i < n) {
          lcol[i] = jj[k];
          lval[i] = vv[k];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kRowIters; ++k) {
      const int i = tid + k * kBlock;
      if (i <= nrows) loff[i] = ro[k] - p0;
    }
  }
  __syncthreads();

  const int G = lanes_for(nrows);
  const int lane = tid & (G - 1);
  const int groups = kBlock / G;
  for (int base = 0; base < nrows; base += groups) {
    const int rr = base + tid / G;
    const bool live = rr < nrows;
    A acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0;
    if (live) {
      const int q1 = loff[rr + 1];
      if constexpr (kStageProducts) {
        for (int q = loff[rr] + lane; q < q1; q += G) {
#pragma unroll
          for (int c = 0; c < C; ++c) acc[c] += lprod[q * C + c];
        }
      } else {
        // four gathers in flight per lane, then their products in order
        int q = loff[rr] + lane;
        for (; q + 3 * G < q1; q += 4 * G) {
          typename SigRow<T, C>::V xr[4];
          A vr[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) xr[u] = load_row<T, C>(x, lcol[q + u * G]);
#pragma unroll
          for (int u = 0; u < 4; ++u) vr[u] = lval[q + u * G];
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < C; ++c) acc[c] += vr[u] * S::load(xr[u].v[c]);
        }
        for (; q < q1; q += G) {
          const auto xa = load_row<T, C>(x, lcol[q]);
          const A va = lval[q];
#pragma unroll
          for (int c = 0; c < C; ++c) acc[c] += va * S::load(xa.v[c]);
        }
      }
    }
    for (int off = G >> 1; off > 0; off >>= 1) {
#pragma unroll
      for (int c = 0; c < C; ++c) acc[c] += __shfl_xor(acc[c], off);
    }
    if (live && lane == 0) {
      if constexpr (kStageProducts) {
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] = acc[c] + ldx[rr * C + c];
      } else {
        const A dg = diag[r0 + rr];
        const auto xi = load_row<T, C>(x, r0 + rr);
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] = acc[c] + dg * S::load(xi.v[c]);
      }
      emit_row<D, C, kFinal>(f, gd, y, r0 + rr, acc, cen);
    }
  }
}

// x0 for the rows of one tile: cell rows are the caller's signal rounded to
// the storage type, star rows the float64 mean of their net's cells (a
// group of lanes per star row).  A tile never mixes cell rows and star rows.
//
// Centred (l.centre != NULL, 16-bit storage): every row stores x - c v with
// v = sqrt(d + sigma) of this sigma group and c = l.centre[graph][grp][col].
template <int D, int C, bool kBatch>
__global__ __launch_bounds__(kBlock) void k_prep(LaunchArgs l, int32_t in_dtype, int32_t col0,
                                                 void *x0v, int32_t grp, int32_t groups,
                                                 double sigma) {
  const uint32_t tile = tile_of_block(l);
  const TileDesc td = gload(l.tiles, tile);
  const GraphDev gd = graph_of<kBatch>(l, tile);
  const GraphIO &io = gd.io;
  const gptr<typename Store<D>::T> x0 =
      to_global(static_cast<typename Store<D>::T *>(x0v)) + gd.row_off * C;
  const gptr<const int32_t> row_ptr = to_global(gd.row_ptr), col = to_global(gd.col);
  const double *cen = l.centre ? l.centre +
                                     (static_cast<int64_t>(graph_index<kBatch>(l, tile)) * groups +
                                      grp) * C
                               : nullptr;
  using V = typename SigRow<typename Store<D>::T, C>::V;
  if (td.r0 < io.num_cells) {
    // a thread per row: all of its loads first (two rows at a time), one
    // square root per row, the row stored with one vector store
    for (int32_t r = td.r0 + threadIdx.x; r < td.r1; r += 2 * kBlock) {
      const int32_t r2 = r + kBlock;
      const bool two = r2 < td.r1;
      double v[2][C];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        v[0][c] = load_in(io.x_in, in_dtype, static_cast<int64_t>(r) * io.ld_in + col0 + c);
        v[1][c] = two ? load_in(io.x_in, in_dtype, static_cast<int64_t>(r2) * io.ld_in + col0 + c)
                      : 0.0;
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (h == 1 && !two) break;
        const int32_t rr = h ? r2 : r;
        V out;
        const double vr = cen ? sqrt(to_global(gd.deg)[rr] + sigma) : 0.0;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          double e = v[h][c];
          if (cen) e = e - to_global(cen)[c] * vr;
          out.v[c] = Store<D>::from_f64(e);
        }
        gstore(reinterpret_cast<V *>(static_cast<typename Store<D>::T *>(x0v) + gd.row_off * C),
               rr, out);
      }
    }
    return;
  }
  // star rows (more than 16 entries each): the tile's columns and row
  // offsets are staged in LDS first, with all of a thread's loads in flight
  // at once (a single row too long for the stage reads them in place); then
  // a group of at least 16 lanes per row, more when the tile has few rows,
  // gathers the cells' rows, several at a time per lane
  constexpr int kPrepCap = TileClass<0>::kCap;
  constexpr int kPrepStage = (kPrepCap + kBlock - 1) / kBlock;
  __shared__ int32_t pcol[kPrepCap];
  __shared__ int32_t poff[TileClass<0>::kRows + 1];
  const int nrows = td.r1 - td.r0;
  const int n = td.p1 - td.p0;
  const bool staged = n <= kPrepCap;
  if (staged) {
    int32_t cv[kPrepStage];
#pragma unroll
    for (int k = 0; k < kPrepStage; ++k) {
      const int i = static_cast<int>(threadIdx.x) + k * kBlock;
      cv[k] = i < n ? col[td.p0 + i] : 0;
    }
    for (int i = threadIdx.x; i <= nrows; i += kBlock) poff[i] = row_ptr[td.r0 + i] - td.p0;
#pragma unroll
    for (int k = 0; k < kPrepStage; ++k) {
      const int i = static_cast<int>(threadIdx.x) + k * kBlock;
      if (i < n) pcol[i] = cv[k];
    }
    __syncthreads();
  }
  auto col_at = [&](int32_t q) -> int64_t { return staged ? pcol[q] : col[td.p0 + q]; };
  const int G = lanes_for(nrows) > 16 ? lanes_for(nrows) : 16;
  const int lane = threadIdx.x & (G - 1);
  for (int base = 0; base < nrows; base += kBlock / G) {
    const int rr = base + static_cast<int>(threadIdx.x) / G;
    const bool live = rr < nrows;
    const int r = td.r0 + (live ? rr : 0);
    // entries of the row, local to the tile
    const int32_t p0 = live ? (staged ? poff[rr] : row_ptr[r] - td.p0) : 0;
    const int32_t p1 = live ? (staged ? poff[rr + 1] : row_ptr[r + 1] - td.p0) : 0;
    double s[C];
#pragma unroll
    for (int c = 0; c < C; ++c) s[c] = 0.0;
    // four cells per lane at a time: their columns, then their rows (held
    // as float32 when the input is float32, so that wide rows keep the
    // register count, and the occupancy, of narrow ones); the cells are
    // added one after another in entry order either way
    int32_t q = p0 + lane;
    if (in_dtype == GIFT_F32) {
      // (two cells at a time above four columns)
      constexpr int kU = C <= 4 ? 4 : 2;
      const gptr<const float> xf = to_global(static_cast<const float *>(io.x_in));
      for (; q + (kU - 1) * G < p1; q += kU * G) {
        int64_t j[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) j[u] = col_at(q + u * G);
        float xv[kU][C];
#pragma unroll
        for (int u = 0; u < kU; ++u)
#pragma unroll
          for (int c = 0; c < C; ++c) xv[u][c] = xf[j[u] * io.ld_in + col0 + c];
#pragma unroll
        for (int u = 0; u < kU; ++u)
#pragma unroll
          for (int c = 0; c < C; ++c) s[c] += static_cast<double>(xv[u][c]);
      }
    } else {
      for (; q + G < p1; q += 2 * G) {
        int64_t j[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) j[u] = col_at(q + u * G);
        double xv[2][C];
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
          for (int c = 0; c < C; ++c) xv[u][c] = load_in(io.x_in, in_dtype, j[u] * io.ld_in + col0 + c);
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
          for (int c = 0; c < C; ++c) s[c] += xv[u][c];
      }
    }
    for (; q < p1; q += G) {
      const int64_t j = col_at(q);
#pragma unroll
      for (int c = 0; c < C; ++c) s[c] += load_in(io.x_in, in_dtype, j * io.ld_in + col0 + c);
    }
#pragma unroll
    for (int c = 0; c < C; ++c)
      for (int off = G >> 1; off > 0; off >>= 1) s[c] += __shfl_xor(s[c], off);
    if (live && lane == 0) {
      const double m = static_cast<double>(p1 - p0);
      const double vr = cen ? sqrt(to_global(gd.deg)[r] + sigma) : 0.0;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        double v = m > 0 ? s[c] / m : 0.0;
        if (cen) v = v - to_global(cen)[c] * vr;
        x0[static_cast<int64_t>(r) * C + c] = Store<D>::from_f64(v);
      }
    }
  }
}

// The centring vectors.  With v = sqrt(d + sigma), A~_sigma v = v exactly
// (Theorem 1 with the self-loop), so A~^k (x - c v) + c v = A~^k x for any c.
// c = sum over cells of x / sum over cells of v (per graph, sigma group and
// column) makes c v match x on average; 16-bit iterates of x - c v then lose
// far less to rounding than iterates of x.
struct GroupSigmas {
  int32_t n;
  double s[kMaxTerms];
};

// Per tile of the all-rows list: sums over its cell rows of x (C columns)
// and of sqrt(d + sigma_g) (one per group); star-row tiles write zeros.
// One pass over the rows (each thread a fixed set of rows, accumulated in
// order), then per value a wave reduction by a fixed shuffle pattern and the
// waves' results added in wave order.  part[tile][C + groups].
template <int C, bool kBatch>
__global__ __launch_bounds__(kBlock) void k_centre_part(LaunchArgs l, int32_t in_dtype,
                                                        int32_t col0, GroupSigmas gs,
                                                        double *part) {
  constexpr int kGroupsInRegs = 4;
  __shared__ double wsum[kBlock / kWave][16 + kMaxTerms];
  const uint32_t tile = blockIdx.x;
  const TileDesc td = gload(l.tiles, tile);
  const GraphDev gd = graph_of<kBatch>(l, tile);
  const int nv = C + gs.n;
  const bool cells = td.r0 < gd.io.num_cells;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  double ax[C], av[kGroupsInRegs];
#pragma unroll
  for (int k = 0; k < C; ++k) ax[k] = 0.0;
#pragma unroll
  for (int g = 0; g < kGroupsInRegs; ++g) av[g] = 0.0;
  for (int g0 = 0; g0 < (gs.n > 0 ? gs.n : 1); g0 += kGroupsInRegs) {
    if (cells) {
      for (int32_t r = td.r0 + threadIdx.x; r < td.r1; r += kBlock) {
        if (g0 == 0) {
#pragma unroll
          for (int k = 0; k < C; ++k)
            ax[k] += load_in(gd.io.x_in, in_dtype, static_cast<int64_t>(r) * gd.io.ld_in + col0 + k);
        }
        const double d = to_global(gd.deg)[r];
#pragma unroll
        for (int g = 0; g < kGroupsInRegs; ++g)
          if (g0 + g < gs.n) av[g] += sqrt(d + gs.s[g0 + g]);
      }
    }
    // reduce this round's values: x columns (first round) and its groups
#pragma unroll
    for (int k = 0; k < C + kGroupsInRegs; ++k) {
      const bool isx = k < C;
      if (!isx && g0 + (k - C) >= gs.n) continue;
      if (isx && g0 != 0) continue;
      double v = isx ? ax[k] : av[k - C];
      for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
      if (lane == 0) wsum[wave][isx ? k : C + g0 + (k - C)] = v;
    }
#pragma unroll
    for (int g = 0; g < kGroupsInRegs; ++g) av[g] = 0.0;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nv; k += kBlock) {
    double t = 0.0;
    for (int w = 0; w < kBlock / kWave; ++w) t += wsum[w][k];
    part[static_cast<int64_t>(tile) * nv + k] = t;
  }
}

// One block per graph: sums its tiles' partials (strided per thread, then a
// block tree: a fixed order) and writes centre[graph][g][q] = sum x_q /
// sum v_g (0 when the graph has no cells).
template <int C, bool kBatch>
__global__ __launch_bounds__(kBlock) void k_centre_final(LaunchArgs l, const double *part,
                                                         int32_t groups, double *centre) {
  __shared__ double red[kBlock];
  __shared__ double tot[16 + kMaxTerms];
  const GraphDev gd = kBatch ? gload(l.graphs, blockIdx.x) : l.one;
  const int nv = C + groups;
  for (int k = 0; k < nv; ++k) {
    double a = 0.0;
    for (int32_t t = gd.tile_lo + threadIdx.x; t < gd.tile_hi; t += kBlock)
      a += part[static_cast<int64_t>(t) * nv + k];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) tot[k] = red[0];
    __syncthreads();
  }
  // a column whose sum is not finite (a NaN or infinite input) is not
  // centred, so the bad value reaches only the rows the filter carries it
  // to, as without centring
  for (int i = threadIdx.x; i < groups * C; i += kBlock) {
    const int g = i / C, q = i % C;
    const double sv = tot[C + g];
    const double c = sv > 0.0 ? tot[q] / sv : 0.0;
    centre[(static_cast<int64_t>(blockIdx.x) * groups + g) * C + q] = isfinite(c) ? c : 0.0;
  }
}

// Algorithmic bytes of one SpMM pass: row_ptr, col and values of the rows it
// covers, their diagonal, every signal row read once, the iterate written.
// The last pass covers the cell rows only, reads the saved iterates of the
// other terms and writes the output instead.
double pass_bytes(const FilterPlan &pl, int C, bool fin) {
  const double bt = static_cast<double>(dtype_size(pl.storage));
  const double ba = static_cast<double>(accum_size(pl.storage));
  const double rows = static_cast<double>(fin ? pl.cell_rows : pl.R);
  const double nnz = static_cast<double>(fin ? pl.nnz_cells : pl.nnz);
  const double R = static_cast<double>(pl.R);
  const double b = 4.0 * (rows + 1) + (4.0 + bt) * nnz + ba * rows + bt * C * R;
  if (!fin) return b + bt * C * rows;
  return b + (pl.num_terms - 1) * bt * C * rows +
         (pl.out_dtype == GIFT_F64 ? 8.0 : 4.0) * C * rows;
}

LaunchArgs launch_args(const FilterPlan &pl, const PlanGroup &grp, bool fin) {
  LaunchArgs l{};
  l.tiles = fin ? pl.final_tiles : pl.tiles;
  l.tile_graph = fin ? pl.final_tile_graph : pl.tile_graph;
  l.graphs = grp.graphs;
  l.one = pl.one;
  l.one.val = grp.val;
  l.one.diag = grp.diag;
  l.identity_map = pl.identity_map ? 1 : 0;
  return l;
}

template <int D, int C, int TC, bool kBatch>
gift_status enqueue_chunk(const FilterPlan &pl, const ChunkBuffers &bf, int32_t col0,
                          hipStream_t st) {
  using T = typename Store<D>::T;
  T *x0 = static_cast<T *>(bf.x0), *ping = static_cast<T *>(bf.ping),
    *pong = static_cast<T *>(bf.pong);
  const int32_t G = static_cast<int32_t>(pl.groups.size());
  auto args = [&](const PlanGroup &grp, bool fin) {
    LaunchArgs l = launch_args(pl, grp, fin);
    l.centre = pl.centre ? bf.centre : nullptr;
    return l;
  };
  const unsigned prep_grid = static_cast<unsigned>(pl.num_tiles);
  if (pl.centre && pl.num_tiles > 0) {
    GroupSigmas gs{};
    gs.n = G;
    for (int32_t g = 0; g < G; ++g) gs.s[g] = pl.groups[g].sigma;
    // the sums run over every graph's contiguous tiles
    LaunchArgs lc = args(pl.groups.front(), false);
    int64_t nct = pl.num_tiles;
    if (pl.centre_tiles) {
      lc.tiles = pl.centre_tiles;
      lc.tile_graph = pl.centre_tile_graph;
      nct = pl.num_centre_tiles;
    }
    k_centre_part<C, kBatch><<<static_cast<unsigned>(nct), kBlock, 0, st>>>(
        lc, pl.in_dtype, col0, gs, bf.centre_part);
    GIFT_TRY(check_launch("k_centre_part"));
    k_centre_final<C, kBatch><<<static_cast<unsigned>(pl.num_graphs), kBlock, 0, st>>>(
        lc, bf.centre_part, G, bf.centre);
    GIFT_TRY(check_launch("k_centre_final"));
  }
  if (!pl.centre && pl.num_tiles > 0) {
    // one x0 serves every sigma group
    k_prep<D, C, kBatch><<<prep_grid, kBlock, 0, st>>>(args(pl.groups.front(), false),
                                                       pl.in_dtype, col0, x0, 0, G, 0.0);
    GIFT_TRY(check_launch("k_prep"));
  }
  FinalArgs fa{};
  fa.num_terms = pl.num_terms;
  fa.in_dtype = pl.in_dtype;
  fa.out_dtype = pl.out_dtype;
  fa.col0 = col0;
  fa.num_groups = G;
  for (int32_t t = 0; t < pl.num_terms; ++t) {
    fa.src[t] = bf.saved[t];
    fa.alpha[t] = pl.terms[t].alpha;
    fa.term_sigma[t] = pl.terms[t].sigma;
    for (int32_t g = 0; g < G; ++g)
      if (pl.groups[g].sigma == pl.terms[t].sigma) fa.term_group[t] = g;
  }
  const size_t ng = pl.groups.size();
  for (size_t gi = 0; gi < ng; ++gi) {
    const PlanGroup &grp = pl.groups[gi];
    if (pl.centre && pl.num_tiles > 0) {
      // x0 - c v of this group's sigma
      k_prep<D, C, kBatch><<<prep_grid, kBlock, 0, st>>>(args(grp, false), pl.in_dtype, col0, x0,
                                                         static_cast<int32_t>(gi), G, grp.sigma);
      GIFT_TRY(check_launch("k_prep"));
    }
    const T *cur = x0;
    for (int32_t k = 1; k <= grp.kmax; ++k) {
      const bool fin = gi + 1 == ng && k == grp.kmax;
      T *dst = nullptr;
      if (!fin) {
        for (int32_t t = 0; t < pl.num_terms; ++t)
          if (pl.terms[t].sigma == grp.sigma && pl.terms[t].order == k)
            dst = static_cast<T *>(bf.saved[t]);
        if (!dst) dst = (cur == ping) ? pong : ping;
      }
      const int64_t tiles = fin ? pl.num_final_tiles : pl.num_tiles;
      if (tiles > 0) {
        const LaunchArgs l = args(grp, fin);
        const unsigned grid = static_cast<unsigned>(tiles);
        const void *x = cur;
        void *y = dst;
        if (fin)
          GIFT_TRY(launch_timed(k_spmm<D, C, true, TC, kBatch>, grid, st, pl.profile,
                                GIFT_PROF_SPMM_FINAL, pass_bytes(pl, C, true), "k_spmm", l, x,
                                y, fa));
        else
          GIFT_TRY(launch_timed(k_spmm<D, C, false, TC, kBatch>, grid, st, pl.profile,
                                GIFT_PROF_SPMM, pass_bytes(pl, C, false), "k_spmm", l, x, y,
                                fa));
      }
      if (!fin) cur = dst;
    }
  }
  return GIFT_OK;
}

template <int D, int C>
gift_status enqueue_chunk_tc(const FilterPlan &pl, const ChunkBuffers &bf, int32_t col0,
                             hipStream_t st) {
  const bool batch = pl.groups.front().graphs != nullptr;
  if (pl.tile_class == 1)
    return batch ? enqueue_chunk<D, C, 1, true>(pl, bf, col0, st)
                 : enqueue_chunk<D, C, 1, false>(pl, bf, col0, st);
  return batch ? enqueue_chunk<D, C, 0, true>(pl, bf, col0, st)
               : enqueue_chunk<D, C, 0, false>(pl, bf, col0, st);
}

template <int D>
gift_status enqueue_chunk_c(const FilterPlan &pl, const ChunkBuffers &bf, int C, int32_t col0,
                            hipStream_t st) {
  switch (C) {
    case 1: return enqueue_chunk_tc<D, 1>(pl, bf, col0, st);
    case 2: return enqueue_chunk_tc<D, 2>(pl, bf, col0, st);
    case 4: return enqueue_chunk_tc<D, 4>(pl, bf, col0, st);
    case 8: return enqueue_chunk_tc<D, 8>(pl, bf, col0, st);
    case 16: return enqueue_chunk_tc<D, 16>(pl, bf, col0, st);
  }
  return set_error(GIFT_EUNSUPPORTED, "column chunk %d", C);
}

size_t round_up(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

int chunk_width(int remaining) {
  return remaining >= 16 ? 16 : remaining >= 8 ? 8 : remaining >= 4 ? 4 : remaining >= 2 ? 2 : 1;
}

gift_status enqueue_filter_chunk(const FilterPlan &pl, const ChunkBuffers &bf, int C, int32_t col0,
                                 hipStream_t st) {
  if (pl.tile_class < 0 || pl.tile_class >= kTileClasses)
    return set_error(GIFT_EINVAL, "tile class %d", pl.tile_class);
  switch (pl.storage) {
    case GIFT_F32: return enqueue_chunk_c<GIFT_F32>(pl, bf, C, col0, st);
    case GIFT_F64: return enqueue_chunk_c<GIFT_F64>(pl, bf, C, col0, st);
    case GIFT_BF16: return enqueue_chunk_c<GIFT_BF16>(pl, bf, C, col0, st);
    case GIFT_F16: return enqueue_chunk_c<GIFT_F16>(pl, bf, C, col0, st);
  }
  return set_error(GIFT_EUNSUPPORTED, "storage %d", pl.storage);
}

gift_status plan_groups(const gift_graph *g, const gift_term *terms, int32_t nt,
                        std::vector<PlanGroup> *out) {
  out->clear();
  for (int32_t t = 0; t < nt; ++t) {
    const gift_term &tm = terms[t];
    if (!(tm.sigma >= 0.0) || !std::isfinite(tm.sigma))
      return set_error(GIFT_EINVAL, "term %d: sigma %g", t, tm.sigma);
    if (tm.order < 1) return set_error(GIFT_EINVAL, "term %d: order %d < 1", t, tm.order);
    if (!std::isfinite(tm.alpha)) return set_error(GIFT_EINVAL, "term %d: alpha not finite", t);
    if (tm.reserved != 0) return set_error(GIFT_EINVAL, "term %d: reserved field not 0", t);
    const SigmaBlock *b = find_sigma(g, tm.sigma);
    if (!b)
      return set_error(GIFT_EINVAL, "term %d: sigma %g was not prepared for this graph", t,
                       tm.sigma);
    bool found = false;
    for (PlanGroup &gr : *out)
      if (gr.sigma == tm.sigma) {
        if (tm.order > gr.kmax) gr.kmax = tm.order;
        found = true;
      }
    if (!found) out->push_back(PlanGroup{tm.sigma, tm.order, b->val, b->diag, nullptr});
  }
  for (size_t i = 1; i < out->size(); ++i)
    for (size_t j = i; j > 0 && (*out)[j].sigma < (*out)[j - 1].sigma; --j)
      std::swap((*out)[j], (*out)[j - 1]);
  return GIFT_OK;
}

// Buffers x0, ping, pong and one saved iterate per distinct (sigma, order)
// term other than the one the last pass forms, each rounded to 256 bytes.
size_t carve_chunk_buffers(const FilterPlan &pl, int C, unsigned char *base, ChunkBuffers *bf) {
  const size_t rb = round_up(dtype_size(pl.storage) * C * static_cast<size_t>(pl.R));
  const uintptr_t b = reinterpret_cast<uintptr_t>(base);
  size_t off = 0;
  auto slot = [&]() {
    void *p = reinterpret_cast<void *>(b + off);
    off += rb;
    return p;
  };
  bf->x0 = slot();
  bf->ping = slot();
  bf->pong = slot();
  const PlanGroup &last = pl.groups.back();
  for (int32_t t = 0; t < pl.num_terms; ++t) {
    bf->saved[t] = nullptr;
    const gift_term &tm = pl.terms[t];
    if (tm.sigma == last.sigma && tm.order == last.kmax) continue;
    int32_t same = -1;
    for (int32_t u = 0; u < t && same < 0; ++u)
      if (pl.terms[u].sigma == tm.sigma && pl.terms[u].order == tm.order) same = u;
    bf->saved[t] = same >= 0 ? bf->saved[same] : slot();
  }
  bf->centre_part = nullptr;
  bf->centre = nullptr;
  if (pl.centre) {
    const size_t G = pl.groups.size();
    const int64_t ct = pl.centre_tiles ? pl.num_centre_tiles : pl.num_tiles;
    bf->centre_part = reinterpret_cast<double *>(b + off);
    off += round_up(sizeof(double) * (C + G) * static_cast<size_t>(ct + 1));
    bf->centre = reinterpret_cast<double *>(b + off);
    off += round_up(sizeof(double) * G * C * static_cast<size_t>(pl.num_graphs));
  }
  return off;
}

size_t chunk_buffer_bytes(const FilterPlan &pl, int C) {
  ChunkBuffers bf;
  return carve_chunk_buffers(pl, C, nullptr, &bf);
}

// ---------------------------------------------------------------------------
// The exact filter g' = (I + L~_sigma)^-1 g (Section 3.2.2, eq. derivative
// and eq. spectral) that the paper's filter approximates: conjugate gradients
// on (2 I - A~_sigma) g' = g over all R rows, per column, from g' = 0.  One
// iteration is an SpMM pass (the same kernel as the filter) and three fused
// vector kernels; dot products are float64, summed per block over fixed
// ranges and then across blocks in a fixed order (deterministic).  The scalars stay on the
// device; the host reads the residuals every few iterations to stop.
// ---------------------------------------------------------------------------
namespace {

constexpr int kCgBlocks = 1024;  // blocks of the vector kernels (fixed ranges)

__device__ __forceinline__ void cg_range(int64_t n, int64_t *lo, int64_t *hi) {
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  *lo = static_cast<int64_t>(blockIdx.x) * per;
  *hi = *lo + per < n ? *lo + per : n;
}

// Sums v[C] over the block (fixed tree) and writes part[block * C + q].
template <int C>
__device__ __forceinline__ void cg_block_sum(double (&v)[C], double *red, double *part) {
#pragma unroll
  for (int q = 0; q < C; ++q) {
    red[threadIdx.x] = v[q];
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x * C + q] = red[0];
    __syncthreads();
  }
}

// out[q] = sum of part[b * C + q] over b < nb: block q, in the fixed order of
// block_sum_strided.
template <int C>
__global__ __launch_bounds__(kBlock) void k_cg_reduce(const double *part, int nb, double *out) {
  __shared__ double red[kBlock];
  const double s = block_sum_strided(part + blockIdx.x, nb, C, red);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// x = 0, r = p = b; part = b . b
template <int D, int C>
__global__ __launch_bounds__(kBlock) void k_cg_init(const typename Store<D>::T *b,
                                                    typename Store<D>::T *x,
                                                    typename Store<D>::T *r,
                                                    typename Store<D>::T *p, int64_t R,
                                                    double *part) {
  __shared__ double red[kBlock];
  int64_t lo, hi;
  cg_range(R, &lo, &hi);
  double acc[C] = {};
  for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
#pragma unroll
    for (int q = 0; q < C; ++q) {
      const auto v = b[i * C + q];
      x[i * C + q] = Store<D>::from_f64(0.0);
      r[i * C + q] = v;
      p[i * C + q] = v;
      const double d = static_cast<double>(Store<D>::load(v));
      acc[q] += d * d;
    }
  }
  cg_block_sum<C>(acc, red, part);
}

// q = 2 p - q (q holds A~ p); part = p . q
template <int D, int C>
__global__ __launch_bounds__(kBlock) void k_cg_q(const typename Store<D>::T *p,
                                                 typename Store<D>::T *q, int64_t R,
                                                 double *part) {
  using S = Store<D>;
  __shared__ double red[kBlock];
  int64_t lo, hi;
  cg_range(R, &lo, &hi);
  double acc[C] = {};
  for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const typename S::A pv = S::load(p[i * C + c]);
      const typename S::A qv = 2 * pv - S::load(q[i * C + c]);
      q[i * C + c] = S::from_acc(qv);
      acc[c] += static_cast<double>(pv) * static_cast<double>(qv);
    }
  }
  cg_block_sum<C>(acc, red, part);
}

// alpha = rho / pq; x += alpha p; r -= alpha q; part = r . r
template <int D, int C>
__global__ __launch_bounds__(kBlock) void k_cg_update(typename Store<D>::T *x,
                                                      typename Store<D>::T *r,
                                                      const typename Store<D>::T *p,
                                                      const typename Store<D>::T *q,
                                                      const double *rho, const double *pq,
                                                      int64_t R, double *part) {
  using S = Store<D>;
  using A = typename S::A;
  __shared__ double red[kBlock];
  A alpha[C];
#pragma unroll
  for (int c = 0; c < C; ++c) alpha[c] = static_cast<A>(pq[c] > 0.0 ? rho[c] / pq[c] : 0.0);
  int64_t lo, hi;
  cg_range(R, &lo, &hi);
  double acc[C] = {};
  for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int64_t k = i * C + c;
      x[k] = S::from_acc(S::load(x[k]) + alpha[c] * S::load(p[k]));
      const A rv = S::load(r[k]) - alpha[c] * S::load(q[k]);
      r[k] = S::from_acc(rv);
      acc[c] += static_cast<double>(rv) * static_cast<double>(rv);
    }
  }
  cg_block_sum<C>(acc, red, part);
}

// beta = rho_new / rho; p = r + beta p
template <int D, int C>
__global__ __launch_bounds__(kBlock) void k_cg_p(const typename Store<D>::T *r,
                                                 typename Store<D>::T *p, const double *rho,
                                                 const double *rho_new, int64_t R) {
  using S = Store<D>;
  using A = typename S::A;
  A beta[C];
#pragma unroll
  for (int c = 0; c < C; ++c) beta[c] = static_cast<A>(rho[c] > 0.0 ? rho_new[c] / rho[c] : 0.0);
  int64_t lo, hi;
  cg_range(R, &lo, &hi);
  for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int64_t k = i * C + c;
      p[k] = S::from_acc(S::load(r[k]) + beta[c] * S::load(p[k]));
    }
  }
}

// y_out[cells] = x (fixed rows copied from x_in)
template <int D, int C>
__global__ void k_cg_out(const typename Store<D>::T *x, int64_t N, GraphIO io, int32_t in_dt,
                         int32_t out_dt, int32_t col0) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N * C) return;
  const int64_t r = i / C;
  const int c = static_cast<int>(i % C);
  double v = static_cast<double>(Store<D>::load(x[i]));
  if (io.fixed && to_global(io.fixed)[r]) v = load_in(io.x_in, in_dt, r * io.ld_in + col0 + c);
  const int64_t o = r * io.ld_out + col0 + c;
  if (out_dt == GIFT_F64) to_global(static_cast<double *>(io.y_out))[o] = v;
  else to_global(static_cast<float *>(io.y_out))[o] = static_cast<float>(v);
}

template <int D, int C>
gift_status exact_chunk(const gift_graph *g, const FilterPlan &pl, double tol, int64_t max_iter,
                        int32_t col0, hipStream_t st, int64_t *iters) {
  using T = typename Store<D>::T;
  const int64_t R = pl.R;
  const size_t vb = static_cast<size_t>(R) * C;
  Scratch sc(st);
  T *b = nullptr, *x = nullptr, *r = nullptr, *p = nullptr, *q = nullptr;
  double *part = nullptr, *dots = nullptr;
  GIFT_TRY(sc.get(&b, vb, "cg right-hand side"));
  GIFT_TRY(sc.get(&x, vb, "cg solution"));
  GIFT_TRY(sc.get(&r, vb, "cg residual"));
  GIFT_TRY(sc.get(&p, vb, "cg direction"));
  GIFT_TRY(sc.get(&q, vb, "cg product"));
  GIFT_TRY(sc.get(&part, static_cast<size_t>(kCgBlocks) * C, "cg partial dots"));
  // dots: bb | rho (two slots, swapped every iteration) | pq
  GIFT_TRY(sc.get(&dots, 4 * C, "cg scalars"));
  double *bb = dots, *rho[2] = {dots + C, dots + 2 * C}, *pq = dots + 3 * C;
  const unsigned nb = static_cast<unsigned>(std::min<int64_t>(kCgBlocks, (R + kBlock - 1) / kBlock));
  k_prep<D, C, false><<<static_cast<unsigned>(pl.num_tiles), kBlock, 0, st>>>(
      launch_args(pl, pl.groups.front(), false), pl.in_dtype, col0, b, 0, 1, 0.0);
  GIFT_TRY(check_launch("k_prep"));
  k_cg_init<D, C><<<nb, kBlock, 0, st>>>(b, x, r, p, R, part);
  GIFT_TRY(check_launch("k_cg_init"));
  k_cg_reduce<C><<<C, kBlock, 0, st>>>(part, nb, bb);
  GIFT_TRY(check_launch("k_cg_reduce"));
  GIFT_HIP(hipMemcpyAsync(rho[0], bb, sizeof(double) * C, hipMemcpyDeviceToDevice, st));
  const LaunchArgs l = launch_args(pl, pl.groups.front(), false);
  std::vector<double> h(2 * C);
  int64_t it = 0;
  int cur = 0;
  bool done = false;
  while (!done && it < max_iter) {
    GIFT_TRY(launch_timed(k_spmm<D, C, false, 0, false>, static_cast<unsigned>(pl.num_tiles), st,
                          pl.profile, GIFT_PROF_SPMM, pass_bytes(pl, C, false), "k_spmm", l,
                          static_cast<const void *>(p), static_cast<void *>(q), FinalArgs{}));
    k_cg_q<D, C><<<nb, kBlock, 0, st>>>(p, q, R, part);
    GIFT_TRY(check_launch("k_cg_q"));
    k_cg_reduce<C><<<C, kBlock, 0, st>>>(part, nb, pq);
    k_cg_update<D, C><<<nb, kBlock, 0, st>>>(x, r, p, q, rho[cur], pq, R, part);
    GIFT_TRY(check_launch("k_cg_update"));
    k_cg_reduce<C><<<C, kBlock, 0, st>>>(part, nb, rho[cur ^ 1]);
    k_cg_p<D, C><<<nb, kBlock, 0, st>>>(r, p, rho[cur], rho[cur ^ 1], R);
    GIFT_TRY(check_launch("k_cg_p"));
    cur ^= 1;
    ++it;
    if (it % 4 == 0 || it == max_iter) {
      GIFT_HIP(hipMemcpyAsync(h.data(), bb, sizeof(double) * C, hipMemcpyDeviceToHost, st));
      GIFT_HIP(hipMemcpyAsync(h.data() + C, rho[cur], sizeof(double) * C,
                              hipMemcpyDeviceToHost, st));
      GIFT_HIP(hipStreamSynchronize(st));
      done = true;
      for (int c = 0; c < C; ++c)
        if (h[C + c] > tol * tol * h[c]) done = false;
    }
  }
  if (it > *iters) *iters = it;
  const int64_t N = pl.cell_rows;
  if (N > 0) {
    k_cg_out<D, C><<<grid_for(N * C), kBlock, 0, st>>>(x, N, pl.one.io, pl.in_dtype,
                                                         pl.out_dtype, col0);
    GIFT_TRY(check_launch("k_cg_out"));
  }
  GIFT_HIP(hipStreamSynchronize(st));
  return GIFT_OK;
}

template <int D>
gift_status exact_chunk_c(const gift_graph *g, const FilterPlan &pl, int C, double tol,
                          int64_t max_iter, int32_t col0, hipStream_t st, int64_t *iters) {
  switch (C) {
    case 1: return exact_chunk<D, 1>(g, pl, tol, max_iter, col0, st, iters);
    case 2: return exact_chunk<D, 2>(g, pl, tol, max_iter, col0, st, iters);
    case 4: return exact_chunk<D, 4>(g, pl, tol, max_iter, col0, st, iters);
    case 8: return exact_chunk<D, 8>(g, pl, tol, max_iter, col0, st, iters);
    case 16: return exact_chunk<D, 16>(g, pl, tol, max_iter, col0, st, iters);
  }
  return set_error(GIFT_EUNSUPPORTED, "column chunk %d", C);
}

}  // namespace

}  // namespace gift

using namespace gift;

namespace gift {
namespace {

// The allocation-free variant's scratch: the chunk signal buffers (x0, ping,
// pong and the saved iterates) live in this file-scope array instead of the
// caching allocator.  Every GPU the library runs on holds its own copy until
// the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for the current device.
constexpr size_t kNoAllocScratchBytes = size_t(128) << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (with that device current).
gift_status scratch_address(void **out) {
  int dev = 0;
  GIFT_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return set_error(GIFT_EUNSUPPORTED, "device %d beyond the %d the scratch table holds", dev,
                     kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    GIFT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return set_error(GIFT_EDEVICE, "hipGetSymbolAddress returned NULL for the scratch");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GIFT_OK;
}

// Shared by gift_filter_placement and its allocation-free variant.  With
// `fixed_buf` NULL the chunk buffers come from the caching allocator;
// otherwise they are carved from fixed_buf (cap bytes) and nothing is
// allocated.
gift_status filter_impl(const gift_graph *g, const gift_term *terms, int32_t nt, const void *x_in,
                        int32_t num_cols, int64_t ld_in, int32_t in_dt, void *y_out,
                        int64_t ld_out, int32_t out_dt, const uint8_t *fixed, void *stream,
                        unsigned char *fixed_buf, size_t cap) {
  if (!g || !terms) return set_error(GIFT_EINVAL, "gift_filter_placement: NULL graph or terms");
  if (nt < 1 || nt > kMaxTerms) return set_error(GIFT_EINVAL, "num_terms %d not in [1, 64]", nt);
  if (num_cols < 1) return set_error(GIFT_EINVAL, "num_cols %d < 1", num_cols);
  if (ld_in < num_cols || ld_out < num_cols)
    return set_error(GIFT_EINVAL, "leading dimension smaller than num_cols");
  if (in_dt != GIFT_F32 && in_dt != GIFT_F64)
    return set_error(GIFT_EUNSUPPORTED, "in_dtype must be F32 or F64");
  if (out_dt != GIFT_F32 && out_dt != GIFT_F64)
    return set_error(GIFT_EUNSUPPORTED, "out_dtype must be F32 or F64");
  FilterPlan pl;
  GIFT_TRY(plan_groups(g, terms, nt, &pl.groups));
  if (g->num_cells == 0) return GIFT_OK;
  if (!x_in || !y_out) return set_error(GIFT_EINVAL, "x_in / y_out is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int tc = g->tile_class;
  pl.storage = g->storage;
  pl.tile_class = tc;
  pl.R = g->num_rows;
  pl.nnz = g->nnz;
  pl.cell_rows = g->num_cells;
  pl.nnz_cells = g->nnz_cells;
  pl.tiles = g->tiles[tc];
  pl.num_tiles = g->num_tiles[tc];
  pl.final_tiles = g->tiles[tc];
  pl.num_final_tiles = g->num_tiles_cells[tc];
  pl.terms = terms;
  pl.num_terms = nt;
  pl.in_dtype = in_dt;
  pl.out_dtype = out_dt;
  pl.one = GraphDev{g->row_ptr, g->col, nullptr, nullptr, 0,
                    GraphIO{x_in, ld_in, y_out, ld_out, fixed, g->num_cells}, g->deg, 0,
                    static_cast<int32_t>(pl.num_tiles)};
  pl.centre = centred_storage(g->storage);
  pl.num_graphs = 1;
  if (fixed_buf) {
    // the profiler creates events on first use; this path creates nothing
    pl.profile = false;
    const size_t need = chunk_buffer_bytes(pl, chunk_width(num_cols));
    if (need > cap)
      return set_error(GIFT_EUNSUPPORTED,
                       "the allocation-free filter needs %zu bytes of signal buffers "
                       "(%lld rows x %d columns, %d terms); its scratch holds %zu",
                       need, static_cast<long long>(pl.R), chunk_width(num_cols), nt, cap);
  }
  for (int32_t col0 = 0; col0 < num_cols;) {
    const int C = chunk_width(num_cols - col0);
    Scratch sc(st);
    unsigned char *buf = fixed_buf;
    if (!buf) GIFT_TRY(sc.get(&buf, chunk_buffer_bytes(pl, C), "filter signal buffers"));
    ChunkBuffers bf;
    carve_chunk_buffers(pl, C, buf, &bf);
    GIFT_TRY(enqueue_filter_chunk(pl, bf, C, col0, st));
    col0 += C;
  }
  return GIFT_OK;
}

}  // namespace
}  // namespace gift

extern "C" gift_status gift_filter_placement(const gift_graph *g, const gift_term *terms,
                                             int32_t nt, const void *x_in, int32_t num_cols,
                                             int64_t ld_in, int32_t in_dt, void *y_out,
                                             int64_t ld_out, int32_t out_dt,
                                             const uint8_t *fixed, void *stream) {
  clear_error();
  return filter_impl(g, terms, nt, x_in, num_cols, ld_in, in_dt, y_out, ld_out, out_dt, fixed,
                     stream, nullptr, 0);
}

extern "C" gift_status gift_filter_placement_noalloc(const gift_graph *g, const gift_term *terms,
                                                     int32_t nt, const void *x_in,
                                                     int32_t num_cols, int64_t ld_in,
                                                     int32_t in_dt, void *y_out, int64_t ld_out,
                                                     int32_t out_dt, const uint8_t *fixed,
                                                     void *stream) {
  clear_error();
  void *p = nullptr;
  GIFT_TRY(scratch_address(&p));
  return filter_impl(g, terms, nt, x_in, num_cols, ld_in, in_dt, y_out, ld_out, out_dt, fixed,
                     stream, static_cast<unsigned char *>(p), kNoAllocScratchBytes);
}

extern "C" gift_status gift_filter_exact(const gift_graph *g, double sigma, const void *x_in,
                                         int32_t num_cols, int64_t ld_in, int32_t in_dt,
                                         void *y_out, int64_t ld_out, int32_t out_dt,
                                         const uint8_t *fixed, double tol, int64_t max_iter,
                                         int64_t *iterations, void *stream) {
  clear_error();
  if (iterations) *iterations = 0;
  if (!g) return set_error(GIFT_EINVAL, "gift_filter_exact: NULL graph");
  if (num_cols < 1) return set_error(GIFT_EINVAL, "num_cols %d < 1", num_cols);
  if (ld_in < num_cols || ld_out < num_cols)
    return set_error(GIFT_EINVAL, "leading dimension smaller than num_cols");
  if (in_dt != GIFT_F32 && in_dt != GIFT_F64)
    return set_error(GIFT_EUNSUPPORTED, "in_dtype must be F32 or F64");
  if (out_dt != GIFT_F32 && out_dt != GIFT_F64)
    return set_error(GIFT_EUNSUPPORTED, "out_dtype must be F32 or F64");
  if (g->storage != GIFT_F32 && g->storage != GIFT_F64)
    return set_error(GIFT_EUNSUPPORTED, "the exact filter needs F32 or F64 storage");
  if (!(tol > 0.0) || max_iter < 1) return set_error(GIFT_EINVAL, "tol must be > 0, max_iter >= 1");
  gift_term term{sigma, 1, 0, 1.0};
  FilterPlan pl;
  GIFT_TRY(plan_groups(g, &term, 1, &pl.groups));
  if (g->num_cells == 0) return GIFT_OK;
  if (!x_in || !y_out) return set_error(GIFT_EINVAL, "x_in / y_out is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  pl.storage = g->storage;
  pl.tile_class = 0;
  pl.R = g->num_rows;
  pl.nnz = g->nnz;
  pl.cell_rows = g->num_cells;
  pl.nnz_cells = g->nnz_cells;
  pl.tiles = g->tiles[0];
  pl.num_tiles = g->num_tiles[0];
  pl.terms = &term;
  pl.num_terms = 1;
  pl.in_dtype = in_dt;
  pl.out_dtype = out_dt;
  pl.one = GraphDev{g->row_ptr, g->col, nullptr, nullptr, 0,
                    GraphIO{x_in, ld_in, y_out, ld_out, fixed, g->num_cells}, g->deg, 0,
                    static_cast<int32_t>(pl.num_tiles)};
  int64_t its = 0;
  for (int32_t col0 = 0; col0 < num_cols;) {
    const int C = chunk_width(num_cols - col0);
    if (g->storage == GIFT_F64) GIFT_TRY(exact_chunk_c<GIFT_F64>(g, pl, C, tol, max_iter, col0, st, &its));
    else GIFT_TRY(exact_chunk_c<GIFT_F32>(g, pl, C, tol, max_iter, col0, st, &its));
    col0 += C;
  }
  if (iterations) *iterations = its;
  return GIFT_OK;
}
