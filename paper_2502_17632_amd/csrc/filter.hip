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
// The pass is bound by HBM bandwidth (about 0.4 flop per byte): it streams
// row_ptr, col and the values once and gathers signal rows.  A group of G
// lanes works on one row (G per row segment: cell rows are short, star rows
// long), the lanes of a group read consecutive entries, and the group's
// partial sums are combined with cross-lane shuffles.  Blocks are remapped so
// each XCD works on one contiguous range of rows.
#include <cmath>
#include <cstring>

#include "common.h"
#include "devutil.h"

namespace gift {

constexpr int kMaxTerms = 64;

struct PassArgs {
  const int32_t *row_ptr;
  const int32_t *col;
  const void *val;
  const void *diag;
  const void *x;
  void *y;
  const int32_t *tile_row;  // tiles [0, num_tiles) of this launch
  const int32_t *tile_ptr;  // first entry of every tile
};

struct FinalArgs {
  int32_t num_terms;
  int32_t in_dtype, out_dtype;
  int32_t col0;  // first column of this chunk in the caller's matrices
  const void *src[kMaxTerms];  // saved iterate of each term; NULL = this pass
  double alpha[kMaxTerms];
  const void *x_in;
  int64_t ld_in;
  void *y_out;
  int64_t ld_out;
  const uint8_t *fixed;
};

template <typename T, int C>
struct SigRow {
  static constexpr int kBytes = static_cast<int>(sizeof(T)) * C;
  static constexpr int kAlign = kBytes >= 16 ? 16 : kBytes;
  struct alignas(kAlign) V {
    T v[C];
  };
};

template <typename T, int C>
__device__ __forceinline__ typename SigRow<T, C>::V load_row(const T *__restrict__ x, int64_t r) {
  return reinterpret_cast<const typename SigRow<T, C>::V *>(x)[r];
}

__device__ __forceinline__ double load_in(const void *p, int32_t dt, int64_t i) {
  return dt == GIFT_F64 ? static_cast<const double *>(p)[i]
                        : static_cast<double>(static_cast<const float *>(p)[i]);
}

// Writes row `row` of the pass result: the stored iterate, or (last pass) the
// float64 combine of all terms in term order.
template <int D, int C, bool kFinal>
__device__ __forceinline__ void emit_row(const PassArgs &p, const FinalArgs &f, int64_t row,
                                         const typename Store<D>::A *acc) {
  using S = Store<D>;
  using T = typename S::T;
  if constexpr (!kFinal) {
    typename SigRow<T, C>::V out;
#pragma unroll
    for (int c = 0; c < C; ++c) out.v[c] = S::from_acc(acc[c]);
    reinterpret_cast<typename SigRow<T, C>::V *>(p.y)[row] = out;
  } else {
    const bool fixed = f.fixed && f.fixed[row];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      double s = 0.0;
      if (fixed) {
        s = load_in(f.x_in, f.in_dtype, row * f.ld_in + f.col0 + c);
      } else {
        for (int t = 0; t < f.num_terms; ++t) {
          const T *src = static_cast<const T *>(f.src[t]);
          double v = src ? static_cast<double>(S::load(src[row * C + c]))
                         : static_cast<double>(acc[c]);
          s = s + f.alpha[t] * v;
        }
      }
      const int64_t o = row * f.ld_out + f.col0 + c;
      if (f.out_dtype == GIFT_F64) static_cast<double *>(f.y_out)[o] = s;
      else static_cast<float *>(f.y_out)[o] = static_cast<float>(s);
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
// Multi-row tile: all entries are fetched at once (coalesced col/value loads,
// then the signal gathers, up to kStage per thread in flight), their products
// staged in LDS, then each row is summed by a group of lanes sized to the
// tile's row count.  When the products would not fit the LDS budget (wide
// signal rows) the entries (col, value) are staged instead and the row groups
// gather the signal themselves.  Single long row: the whole block strides
// over the row and reduces across its waves.
template <int D, int C, bool kFinal>
__global__ __launch_bounds__(kBlock) void k_spmm(PassArgs p, FinalArgs f) {
  using S = Store<D>;
  using T = typename S::T;
  using A = typename S::A;
  constexpr bool kStageProducts = C * sizeof(A) <= 8;
  constexpr int kStage = (kTileCap + kBlock - 1) / kBlock;
  __shared__ int32_t loff[kTileRows + 1];
  __shared__ A ldx[kStageProducts ? kTileRows * C : 1];
  __shared__ A lprod[kStageProducts ? kTileCap * C : 1];
  __shared__ int32_t lcol[kStageProducts ? 1 : kTileCap];
  __shared__ A lval[kStageProducts ? 1 : kTileCap];
  __shared__ A lred[kBlock / kWave][C];

  const uint32_t tile = xcd_remap(blockIdx.x, gridDim.x);
  const int tid = threadIdx.x;
  const int64_t r0 = p.tile_row[tile], r1 = p.tile_row[tile + 1];
  const int64_t p0 = p.tile_ptr[tile], p1 = p.tile_ptr[tile + 1];
  const int nrows = static_cast<int>(r1 - r0);
  const int64_t n = p1 - p0;
  const T *__restrict__ x = static_cast<const T *>(p.x);
  const T *__restrict__ val = static_cast<const T *>(p.val);
  const int32_t *__restrict__ col = p.col;
  const A *__restrict__ diag = static_cast<const A *>(p.diag);

  if (nrows == 1 && n > kLongRow) {
    // single long row
    A acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0;
    int64_t q = p0 + tid;
    for (; q + 3 * kBlock < p1; q += 4 * kBlock) {
      int32_t j[4];
      A v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        j[u] = col[q + u * kBlock];
        v[u] = S::load(val[q + u * kBlock]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const auto xr = load_row<T, C>(x, j[u]);
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] += v[u] * S::load(xr.v[c]);
      }
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
      emit_row<D, C, kFinal>(p, f, r0, tot);
    }
    return;
  }

  // ---- multi-row tile (n <= kTileCap)
  // Every load is issued unconditionally (inactive slots read entry p0 or
  // row 0, always valid) so that all of a thread's loads are in flight at
  // once: first col/value and the rows' offsets and diagonal terms, then the
  // signal gathers; only then are results written to LDS.
  {
    int32_t jj[kStage];
    A vv[kStage];
#pragma unroll
    for (int k = 0; k < kStage; ++k) {
      const int i = tid + k * kBlock;
      const int64_t q = i < n ? p0 + i : 0;
      jj[k] = col[q];
      vv[k] = S::load(val[q]);
    }
    constexpr int kRowIters = (kTileRows + 1 + kBlock - 1) / kBlock;
    int32_t ro[kRowIters];
#pragma unroll
    for (int k = 0; k < kRowIters; ++k) {
      const int i = tid + k * kBlock;
      ro[k] = p.row_ptr[i <= nrows ? r0 + i : r0];
    }
    constexpr int kDiagIters = kTileRows / kBlock;
    A dg[kDiagIters];
    typename SigRow<T, C>::V xr_row[kDiagIters];
    if constexpr (kStageProducts) {
#pragma unroll
      for (int k = 0; k < kDiagIters; ++k) {
        const int i = tid + k * kBlock;
        const int64_t r = i < nrows ? r0 + i : r0;
        dg[k] = diag[r];
        xr_row[k] = load_row<T, C>(x, r);
      }
    }
    if constexpr (kStageProducts) {
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
      if (i <= nrows) loff[i] = static_cast<int32_t>(ro[k] - p0);
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
        int q = loff[rr] + lane;
        for (; q + G < q1; q += 2 * G) {
          const auto xa = load_row<T, C>(x, lcol[q]);
          const auto xb = load_row<T, C>(x, lcol[q + G]);
          const A va = lval[q], vb = lval[q + G];
#pragma unroll
          for (int c = 0; c < C; ++c) acc[c] += va * S::load(xa.v[c]);
#pragma unroll
          for (int c = 0; c < C; ++c) acc[c] += vb * S::load(xb.v[c]);
        }
        if (q < q1) {
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
      emit_row<D, C, kFinal>(p, f, r0 + rr, acc);
    }
  }
}

// Rows [0, N): the caller's signal, rounded to the storage type.
template <int D, int C>
__global__ void k_prep_cells(const void *x_in, int64_t ld_in, int32_t in_dtype, int32_t col0,
                             int64_t N, typename Store<D>::T *x0) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N * C) return;
  int64_t r = i / C;
  int c = static_cast<int>(i - r * C);
  x0[i] = Store<D>::from_f64(load_in(x_in, in_dtype, r * ld_in + col0 + c));
}

// Star rows [N, R): the mean of the net's cells (float64 sum), one wave each.
template <int D, int C>
__global__ __launch_bounds__(kBlock) void k_prep_stars(const int32_t *row_ptr,
                                                       const int32_t *col, const void *x_in,
                                                       int64_t ld_in, int32_t in_dtype,
                                                       int32_t col0, int64_t N, int64_t V,
                                                       typename Store<D>::T *x0) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t waves = static_cast<int64_t>(gridDim.x) * (kBlock / kWave);
  for (int64_t v = static_cast<int64_t>(blockIdx.x) * (kBlock / kWave) + threadIdx.x / kWave;
       v < V; v += waves) {
    const int64_t r = N + v;
    const int32_t p0 = row_ptr[r], p1 = row_ptr[r + 1];
    double s[C];
#pragma unroll
    for (int c = 0; c < C; ++c) s[c] = 0.0;
    for (int32_t q = p0 + lane; q < p1; q += kWave) {
      const int64_t j = col[q];
#pragma unroll
      for (int c = 0; c < C; ++c) s[c] += load_in(x_in, in_dtype, j * ld_in + col0 + c);
    }
#pragma unroll
    for (int c = 0; c < C; ++c)
      for (int off = kWave / 2; off > 0; off >>= 1) s[c] += __shfl_xor(s[c], off);
    if (lane == 0) {
      const double m = static_cast<double>(p1 - p0);
#pragma unroll
      for (int c = 0; c < C; ++c) x0[r * C + c] = Store<D>::from_f64(m > 0 ? s[c] / m : 0.0);
    }
  }
}

namespace {

struct Group {
  double sigma;
  int32_t kmax;
  const SigmaBlock *blk;
};

// Algorithmic bytes of one SpMM pass: row_ptr, col and values of the rows it
// covers, their diagonal, every signal row read once, the iterate written.
// The last pass covers the cell rows only, reads the saved iterates of the
// other terms and writes the output instead.
template <int D, int C>
double pass_bytes(const gift_graph *g, bool fin, int32_t nt, int32_t out_dt) {
  const double bt = sizeof(typename Store<D>::T), ba = sizeof(typename Store<D>::A);
  const double rows = static_cast<double>(fin ? g->num_cells : g->num_rows);
  const double nnz = static_cast<double>(fin ? g->nnz_cells : g->nnz);
  const double R = static_cast<double>(g->num_rows);
  double b = 4.0 * (rows + 1) + (4.0 + bt) * nnz + ba * rows + bt * C * R;
  if (!fin) return b + bt * C * rows;
  return b + (nt - 1) * bt * C * rows + (out_dt == GIFT_F64 ? 8.0 : 4.0) * C * rows;
}

template <int D, int C>
gift_status run_chunk(const gift_graph *g, const std::vector<Group> &groups,
                      const gift_term *terms, int32_t nt, const void *x_in, int64_t ld_in,
                      int32_t in_dt, void *y_out, int64_t ld_out, int32_t out_dt,
                      const uint8_t *fixed, int32_t col0, hipStream_t st) {
  using T = typename Store<D>::T;
  const int64_t N = g->num_cells, V = g->num_virtual, R = g->num_rows;
  Scratch sc(st);
  T *x0 = nullptr, *ping = nullptr, *pong = nullptr;
  GIFT_TRY(sc.get(&x0, R * C, "signal x0"));
  GIFT_TRY(sc.get(&ping, R * C, "signal ping"));
  GIFT_TRY(sc.get(&pong, R * C, "signal pong"));
  // saved iterate for every term that is not the very last pass
  std::vector<T *> saved(nt, nullptr);
  const Group &last = groups.back();
  for (int32_t t = 0; t < nt; ++t) {
    bool is_final = terms[t].sigma == last.sigma && terms[t].order == last.kmax;
    if (is_final) continue;
    for (int32_t u = 0; u < t; ++u)
      if (terms[u].sigma == terms[t].sigma && terms[u].order == terms[t].order) saved[t] = saved[u];
    if (!saved[t]) GIFT_TRY(sc.get(&saved[t], R * C, "saved iterate"));
  }

  k_prep_cells<D, C><<<grid_for(N * C), kBlock, 0, st>>>(x_in, ld_in, in_dt, col0, N, x0);
  GIFT_TRY(check_launch("k_prep_cells"));
  if (V > 0) {
    k_prep_stars<D, C><<<grid_for(V * kWave), kBlock, 0, st>>>(g->row_ptr, g->col, x_in, ld_in,
                                                                in_dt, col0, N, V, x0);
    GIFT_TRY(check_launch("k_prep_stars"));
  }

  FinalArgs fa{};
  fa.num_terms = nt;
  fa.in_dtype = in_dt;
  fa.out_dtype = out_dt;
  fa.col0 = col0;
  fa.x_in = x_in;
  fa.ld_in = ld_in;
  fa.y_out = y_out;
  fa.ld_out = ld_out;
  fa.fixed = fixed;
  for (int32_t t = 0; t < nt; ++t) {
    fa.src[t] = saved[t];
    fa.alpha[t] = terms[t].alpha;
  }

  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const Group &grp = groups[gi];
    const T *cur = x0;
    for (int32_t k = 1; k <= grp.kmax; ++k) {
      const bool fin = gi + 1 == groups.size() && k == grp.kmax;
      T *dst = nullptr;
      if (!fin) {
        for (int32_t t = 0; t < nt; ++t)
          if (terms[t].sigma == grp.sigma && terms[t].order == k) dst = saved[t];
        if (!dst) dst = (cur == ping) ? pong : ping;
      }
      PassArgs pa{};
      pa.row_ptr = g->row_ptr;
      pa.col = g->col;
      pa.val = grp.blk->val;
      pa.diag = grp.blk->diag;
      pa.x = cur;
      pa.y = dst;
      pa.tile_row = g->tile_row;
      pa.tile_ptr = g->tile_ptr;
      const int64_t tiles = fin ? g->num_tiles_cells : g->num_tiles;
      if (tiles == 0) continue;
      const unsigned grid = static_cast<unsigned>(tiles);
      {
        ProfScope ps(st, fin ? GIFT_PROF_SPMM_FINAL : GIFT_PROF_SPMM,
                     pass_bytes<D, C>(g, fin, nt, out_dt));
        if (fin) k_spmm<D, C, true><<<grid, kBlock, 0, st>>>(pa, fa);
        else k_spmm<D, C, false><<<grid, kBlock, 0, st>>>(pa, fa);
      }
      GIFT_TRY(check_launch("k_spmm"));
      cur = dst;
    }
  }
  return GIFT_OK;
}

template <int D>
gift_status run_chunk_c(int C, const gift_graph *g, const std::vector<Group> &groups,
                        const gift_term *terms, int32_t nt, const void *x_in, int64_t ld_in,
                        int32_t in_dt, void *y_out, int64_t ld_out, int32_t out_dt,
                        const uint8_t *fixed, int32_t col0, hipStream_t st) {
  switch (C) {
    case 1: return run_chunk<D, 1>(g, groups, terms, nt, x_in, ld_in, in_dt, y_out, ld_out, out_dt, fixed, col0, st);
    case 2: return run_chunk<D, 2>(g, groups, terms, nt, x_in, ld_in, in_dt, y_out, ld_out, out_dt, fixed, col0, st);
    case 4: return run_chunk<D, 4>(g, groups, terms, nt, x_in, ld_in, in_dt, y_out, ld_out, out_dt, fixed, col0, st);
    case 8: return run_chunk<D, 8>(g, groups, terms, nt, x_in, ld_in, in_dt, y_out, ld_out, out_dt, fixed, col0, st);
    case 16: return run_chunk<D, 16>(g, groups, terms, nt, x_in, ld_in, in_dt, y_out, ld_out, out_dt, fixed, col0, st);
  }
  return set_error(GIFT_EUNSUPPORTED, "column chunk %d", C);
}

}  // namespace

// Terms grouped by distinct sigma (ascending), each with its highest order.
gift_status plan_groups(const gift_graph *g, const gift_term *terms, int32_t nt,
                        std::vector<Group> *out);

gift_status plan_groups(const gift_graph *g, const gift_term *terms, int32_t nt,
                        std::vector<Group> *out) {
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
    for (Group &gr : *out)
      if (gr.sigma == tm.sigma) {
        if (tm.order > gr.kmax) gr.kmax = tm.order;
        found = true;
      }
    if (!found) out->push_back(Group{tm.sigma, tm.order, b});
  }
  for (size_t i = 1; i < out->size(); ++i)
    for (size_t j = i; j > 0 && (*out)[j].sigma < (*out)[j - 1].sigma; --j)
      std::swap((*out)[j], (*out)[j - 1]);
  return GIFT_OK;
}

}  // namespace gift

using namespace gift;

extern "C" gift_status gift_filter_placement(const gift_graph *g, const gift_term *terms,
                                             int32_t nt, const void *x_in, int32_t num_cols,
                                             int64_t ld_in, int32_t in_dt, void *y_out,
                                             int64_t ld_out, int32_t out_dt,
                                             const uint8_t *fixed, void *stream) {
  clear_error();
  if (!g || !terms) return set_error(GIFT_EINVAL, "gift_filter_placement: NULL graph or terms");
  if (nt < 1 || nt > kMaxTerms) return set_error(GIFT_EINVAL, "num_terms %d not in [1, 64]", nt);
  if (num_cols < 1) return set_error(GIFT_EINVAL, "num_cols %d < 1", num_cols);
  if (ld_in < num_cols || ld_out < num_cols)
    return set_error(GIFT_EINVAL, "leading dimension smaller than num_cols");
  if (in_dt != GIFT_F32 && in_dt != GIFT_F64)
    return set_error(GIFT_EUNSUPPORTED, "in_dtype must be F32 or F64");
  if (out_dt != GIFT_F32 && out_dt != GIFT_F64)
    return set_error(GIFT_EUNSUPPORTED, "out_dtype must be F32 or F64");
  std::vector<gift::Group> groups;
  GIFT_TRY(plan_groups(g, terms, nt, &groups));
  if (g->num_cells == 0) return GIFT_OK;
  if (!x_in || !y_out) return set_error(GIFT_EINVAL, "x_in / y_out is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  int32_t col0 = 0;
  while (col0 < num_cols) {
    int rem = num_cols - col0;
    int C = rem >= 16 ? 16 : rem >= 8 ? 8 : rem >= 4 ? 4 : rem >= 2 ? 2 : 1;
    gift_status s = GIFT_OK;
    switch (g->storage) {
      case GIFT_F32: s = run_chunk_c<GIFT_F32>(C, g, groups, terms, nt, x_in, ld_in, in_dt, y_out, ld_out, out_dt, fixed, col0, st); break;
      case GIFT_F64: s = run_chunk_c<GIFT_F64>(C, g, groups, terms, nt, x_in, ld_in, in_dt, y_out, ld_out, out_dt, fixed, col0, st); break;
      case GIFT_BF16: s = run_chunk_c<GIFT_BF16>(C, g, groups, terms, nt, x_in, ld_in, in_dt, y_out, ld_out, out_dt, fixed, col0, st); break;
      case GIFT_F16: s = run_chunk_c<GIFT_F16>(C, g, groups, terms, nt, x_in, ld_in, in_dt, y_out, ld_out, out_dt, fixed, col0, st); break;
    }
    if (s != GIFT_OK) return s;
    col0 += C;
  }
  return GIFT_OK;
}
