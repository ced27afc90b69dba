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
// Pipeline (all device work on the caller's stream):
//   1. per net: distinct cells, ascending (tiers by pin count: 16-lane group,
//      wave, block + LDS bitonic sort, block merge sort through global memory)
//   2. per net: clique or star, virtual id, weight
//   3. per cell row: number of directed entries, exclusive scan -> offsets
//   4. emit (col, net) keys into each row's slice (atomic slot reservation
//      per pin, so the order inside a slice is arbitrary)
//   5. per row: sort keys by (col, net) (same four tiers) and count distinct
//      columns; the sorted order fixes the summation order, so the result
//      does not depend on the emission order
//   6. scan of distinct counts -> row_ptr; merge runs of equal col summing
//      weights in ascending net id (float64); degree summed in ascending col
//   7. star rows: the net's sorted cells with weight M w(M)
//   8. per sigma: s_i = 1/sqrt(d_i + sigma), a_ij = (w_ij s_i) s_j,
//      diag_i = (sigma s_i) s_i
#include <cmath>
#include <cstring>
#include <new>

#include "common.h"
#include "devutil.h"

namespace gift {
namespace {

enum : uint32_t { kFlagBadNetPtr = 1u, kFlagBadPin = 2u };

constexpr int kBigCap32 = 8192;    // largest net sorted in LDS (32-bit keys)
constexpr int kBigCap64 = 4096;    // largest row sorted in LDS (64-bit keys)
constexpr int kChunk32 = 8192;     // LDS chunk of the global merge sort (u32)
constexpr int kChunk64 = 4096;     // LDS chunk of the global merge sort (u64)

__device__ __forceinline__ uint64_t group_mask(uint64_t ballot, int width) {
  if (width == 64) return ballot;
  int base = (threadIdx.x & 63) & ~(width - 1);
  return (ballot >> base) & ((1ull << width) - 1ull);
}

__device__ __forceinline__ double clique_weight(int64_t m, int model) {
  return model == GIFT_W_TWO_OVER_M ? 2.0 / static_cast<double>(m)
                                    : 1.0 / static_cast<double>(m - 1);
}
__device__ __forceinline__ double star_weight(int64_t m, int model) {
  return model == GIFT_W_TWO_OVER_M ? 2.0
                                    : static_cast<double>(m) / static_cast<double>(m - 1);
}

// ---------------------------------------------------------------------------
// 0. netlist checks that need no per-net work
// ---------------------------------------------------------------------------
__global__ void k_check_ends(const int64_t *net_ptr, int64_t E, int64_t P, uint32_t *flag) {
  if (threadIdx.x == 0 && blockIdx.x == 0)
    if (net_ptr[0] != 0 || net_ptr[E] != P) atomicOr(flag, kFlagBadNetPtr);
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
  int32_t *list_out; // nets handed to the next tier
  int32_t *count_out;
};

// Group of W lanes per net (nets with at most W pins); `list_in` NULL means
// "net e = group index" (first tier), else the nets listed there.
template <int W>
__global__ __launch_bounds__(kBlock) void k_net_group(NetArgs a, const int32_t *list_in,
                                                      const int32_t *count_in) {
  const int t = threadIdx.x & (W - 1);
  const int64_t groups = static_cast<int64_t>(gridDim.x) * (kBlock / W);
  const int64_t n_items = list_in ? static_cast<int64_t>(*count_in) : a.E;
  for (int64_t gi = static_cast<int64_t>(blockIdx.x) * (kBlock / W) + threadIdx.x / W;
       gi < n_items; gi += groups) {
    const int64_t e = list_in ? list_in[gi] : gi;
    const int64_t lo = a.net_ptr[e], hi = a.net_ptr[e + 1];
    if (lo < 0 || hi < lo || hi > a.P) {  // group-uniform
      if (t == 0) {
        atomicOr(a.flag, kFlagBadNetPtr);
        a.M[e] = 0;
      }
      continue;
    }
    const int64_t m_raw = hi - lo;
    if (m_raw > W) {
      if (t == 0) a.list_out[atomicAdd(a.count_out, 1)] = static_cast<int32_t>(e);
      continue;
    }
    const bool live = t < m_raw;
    int32_t c = live ? a.pin[lo + t] : 0;
    const bool bad = live && (c < 0 || c >= a.N);
    const uint64_t badm = group_mask(__ballot(bad), W);
    if (live) a.pin_net[lo + t] = static_cast<int32_t>(e);
    if (badm) {
      if (t == 0) {
        atomicOr(a.flag, kFlagBadPin);
        a.M[e] = 0;
      }
      continue;
    }
    // first occurrence of each cell, then its rank among distinct cells
    bool first = live;
    for (int s = 0; s < W; ++s) {
      int32_t oc = __shfl(c, s, W);
      if (s < t && s < m_raw && oc == c) first = false;
    }
    int less = 0;
    for (int s = 0; s < W; ++s) {
      int32_t oc = __shfl(c, s, W);
      int of = __shfl(static_cast<int>(first), s, W);
      if (s < m_raw && of && oc < c) ++less;
    }
    if (first) a.ucell[lo + less] = c;
    const uint64_t fm = group_mask(__ballot(first), W);
    if (t == 0) a.M[e] = __popcll(fm);
  }
}

// One block per net, pins sorted in LDS (nets with at most kBigCap pins).
__global__ __launch_bounds__(kBlock) void k_net_block(NetArgs a, const int32_t *list_in,
                                                      const int32_t *count_in) {
  __shared__ uint32_t keys[kBigCap32];
  __shared__ int32_t tmp[kBlock / kWave];
  __shared__ int bad_s;
  const int64_t n_items = *count_in;
  for (int64_t gi = blockIdx.x; gi < n_items; gi += gridDim.x) {
    const int64_t e = list_in[gi];
    const int64_t lo = a.net_ptr[e], hi = a.net_ptr[e + 1];
    const int64_t m_raw = hi - lo;  // checked by the first tier
    if (m_raw > kBigCap32) {
      if (threadIdx.x == 0) a.list_out[atomicAdd(a.count_out, 1)] = static_cast<int32_t>(e);
      continue;
    }
    if (threadIdx.x == 0) bad_s = 0;
    __syncthreads();
    const int np = next_pow2_i(static_cast<int>(m_raw));
    for (int i = threadIdx.x; i < np; i += kBlock) {
      uint32_t k = 0xffffffffu;
      if (i < m_raw) {
        int32_t c = a.pin[lo + i];
        a.pin_net[lo + i] = static_cast<int32_t>(e);
        if (c < 0 || c >= a.N) bad_s = 1;
        k = static_cast<uint32_t>(c);
      }
      keys[i] = k;
    }
    __syncthreads();
    if (bad_s) {
      if (threadIdx.x == 0) {
        atomicOr(a.flag, kFlagBadPin);
        a.M[e] = 0;
      }
      __syncthreads();
      continue;
    }
    lds_bitonic_sort<uint32_t>(keys, np);
    int32_t base = 0;
    for (int c0 = 0; c0 < m_raw; c0 += kBlock) {
      int i = c0 + threadIdx.x;
      int f = (i < m_raw && (i == 0 || keys[i] != keys[i - 1])) ? 1 : 0;
      int32_t total;
      int32_t pos = block_excl_scan<int32_t>(f, &total, tmp);
      if (f) a.ucell[lo + base + pos] = static_cast<int32_t>(keys[i]);
      base += total;
    }
    if (threadIdx.x == 0) a.M[e] = base;
    __syncthreads();
  }
}

// One block per net, merge sort through global memory (any size).
__global__ __launch_bounds__(kBlock) void k_net_huge(NetArgs a, const int32_t *list_in,
                                                     const int32_t *count_in, uint32_t *tmpbuf) {
  __shared__ uint32_t lds[kChunk32];
  __shared__ int32_t tmp[kBlock / kWave];
  __shared__ int bad_s;
  const int64_t n_items = *count_in;
  for (int64_t gi = blockIdx.x; gi < n_items; gi += gridDim.x) {
    const int64_t e = list_in[gi];
    const int64_t lo = a.net_ptr[e], hi = a.net_ptr[e + 1];
    const int64_t m_raw = hi - lo;
    uint32_t *ka = reinterpret_cast<uint32_t *>(a.ucell) + lo;
    uint32_t *kb = tmpbuf + lo;
    if (threadIdx.x == 0) bad_s = 0;
    __syncthreads();
    for (int64_t i = threadIdx.x; i < m_raw; i += kBlock) {
      int32_t c = a.pin[lo + i];
      a.pin_net[lo + i] = static_cast<int32_t>(e);
      if (c < 0 || c >= a.N) bad_s = 1;
      ka[i] = static_cast<uint32_t>(c);
    }
    __syncthreads();
    if (bad_s) {
      if (threadIdx.x == 0) {
        atomicOr(a.flag, kFlagBadPin);
        a.M[e] = 0;
      }
      __syncthreads();
      continue;
    }
    bool in_b = block_merge_sort_global<uint32_t, kChunk32>(ka, kb, m_raw, lds, 0xffffffffu);
    if (!in_b) {
      for (int64_t i = threadIdx.x; i < m_raw; i += kBlock) kb[i] = ka[i];
      __syncthreads();
    }
    int64_t base = 0;
    for (int64_t c0 = 0; c0 < m_raw; c0 += kBlock) {
      int64_t i = c0 + threadIdx.x;
      int f = (i < m_raw && (i == 0 || kb[i] != kb[i - 1])) ? 1 : 0;
      int32_t total;
      int32_t pos = block_excl_scan<int32_t>(f, &total, tmp);
      if (f) ka[base + pos] = kb[i];
      base += total;
    }
    if (threadIdx.x == 0) a.M[e] = static_cast<int32_t>(base);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// 2. classify nets
// ---------------------------------------------------------------------------
__global__ void k_classify(const int32_t *M, int64_t E, int64_t T, int model,
                           int32_t *is_star, double *wnet) {
  int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= E) return;
  int64_t m = M[e];
  bool star = m >= 2 && T > 0 && m > T;
  is_star[e] = star ? 1 : 0;
  wnet[e] = m < 2 ? 0.0 : (star ? star_weight(m, model) : clique_weight(m, model));
}

__global__ void k_virtual_map(const int32_t *is_star, const int64_t *vrank, int64_t E,
                              int32_t *virt_net) {
  int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < E && is_star[e]) virt_net[vrank[e]] = static_cast<int32_t>(e);
}

// ---------------------------------------------------------------------------
// 3./4. count and emit the directed entries of cell rows
// ---------------------------------------------------------------------------
struct EmitArgs {
  const int64_t *net_ptr;
  const int32_t *ucell, *pin_net, *M, *is_star;
  const int64_t *vrank;
  int64_t E, P, N;
};

__global__ void k_count(EmitArgs a, int32_t *cnt) {
  int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= a.P) return;
  int64_t e = a.pin_net[p];
  if (e < 0 || e >= a.E) return;
  int64_t i = p - a.net_ptr[e];
  int64_t m = a.M[e];
  if (m < 2 || i < 0 || i >= m) return;
  int32_t c = a.ucell[p];
  if (c < 0 || c >= a.N) return;
  atomicAdd(&cnt[c], a.is_star[e] ? 1 : static_cast<int32_t>(m - 1));
}

__global__ void k_emit(EmitArgs a, const int64_t *zoff, int32_t *cursor, uint64_t *zkey) {
  int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= a.P) return;
  int64_t e = a.pin_net[p];
  int64_t lo = a.net_ptr[e];
  int64_t i = p - lo;
  int64_t m = a.M[e];
  if (m < 2 || i >= m) return;
  int32_t c = a.ucell[p];
  const uint64_t net = static_cast<uint64_t>(e);
  if (a.is_star[e]) {
    int32_t slot = atomicAdd(&cursor[c], 1);
    uint64_t v = static_cast<uint64_t>(a.N + a.vrank[e]);
    zkey[zoff[c] + slot] = (v << 32) | net;
  } else {
    int32_t slot = atomicAdd(&cursor[c], static_cast<int32_t>(m - 1));
    uint64_t *dst = zkey + zoff[c] + slot;
    for (int64_t j = 0; j < m; ++j) {
      if (j == i) continue;
      uint64_t b = static_cast<uint32_t>(a.ucell[lo + j]);
      *dst++ = (b << 32) | net;
    }
  }
}

// ---------------------------------------------------------------------------
// 5. sort each cell row's keys by (col, net); count distinct columns
// ---------------------------------------------------------------------------
struct RowArgs {
  const int64_t *zoff;
  uint64_t *zkey;   // emitted keys (also scratch of the huge tier)
  uint64_t *zsort;  // sorted keys
  int32_t *ucnt;    // distinct columns per row
  int64_t N;
  int32_t *list_out;
  int32_t *count_out;
};

__device__ __forceinline__ uint32_t key_col(uint64_t k) { return static_cast<uint32_t>(k >> 32); }

template <int W>
__global__ __launch_bounds__(kBlock) void k_row_group(RowArgs a, const int32_t *list_in,
                                                      const int32_t *count_in) {
  const int t = threadIdx.x & (W - 1);
  const int64_t groups = static_cast<int64_t>(gridDim.x) * (kBlock / W);
  const int64_t n_items = list_in ? static_cast<int64_t>(*count_in) : a.N;
  for (int64_t gi = static_cast<int64_t>(blockIdx.x) * (kBlock / W) + threadIdx.x / W;
       gi < n_items; gi += groups) {
    const int64_t r = list_in ? list_in[gi] : gi;
    const int64_t lo = a.zoff[r], L = a.zoff[r + 1] - lo;
    if (L > W) {
      if (t == 0) a.list_out[atomicAdd(a.count_out, 1)] = static_cast<int32_t>(r);
      continue;
    }
    if (L == 0) {
      if (t == 0) a.ucnt[r] = 0;
      continue;
    }
    const bool live = t < L;
    const uint64_t k = live ? a.zkey[lo + t] : ~0ull;
    int rank = 0;
    for (int s = 0; s < W; ++s) {
      uint64_t o = __shfl(k, s, W);
      if (s < L && o < k) ++rank;
    }
    // column of the key ranked just below this one
    uint64_t prev = ~0ull;
    for (int s = 0; s < W; ++s) {
      int orank = __shfl(rank, s, W);
      uint64_t o = __shfl(k, s, W);
      if (s < L && orank == rank - 1) prev = o;
    }
    if (live) a.zsort[lo + rank] = k;
    const bool head = live && (rank == 0 || key_col(prev) != key_col(k));
    const uint64_t hm = group_mask(__ballot(head), W);
    if (t == 0) a.ucnt[r] = __popcll(hm);
  }
}

__global__ __launch_bounds__(kBlock) void k_row_block(RowArgs a, const int32_t *list_in,
                                                      const int32_t *count_in) {
  __shared__ uint64_t keys[kBigCap64];
  __shared__ int32_t tmp[kBlock / kWave];
  const int64_t n_items = *count_in;
  for (int64_t gi = blockIdx.x; gi < n_items; gi += gridDim.x) {
    const int64_t r = list_in[gi];
    const int64_t lo = a.zoff[r], L = a.zoff[r + 1] - lo;
    if (L > kBigCap64) {
      if (threadIdx.x == 0) a.list_out[atomicAdd(a.count_out, 1)] = static_cast<int32_t>(r);
      continue;
    }
    const int np = next_pow2_i(static_cast<int>(L));
    for (int i = threadIdx.x; i < np; i += kBlock) keys[i] = i < L ? a.zkey[lo + i] : ~0ull;
    __syncthreads();
    lds_bitonic_sort<uint64_t>(keys, np);
    int32_t heads = 0;
    for (int i = threadIdx.x; i < L; i += kBlock) {
      a.zsort[lo + i] = keys[i];
      if (i == 0 || key_col(keys[i]) != key_col(keys[i - 1])) ++heads;
    }
    int32_t total = block_sum<int32_t>(heads, tmp);
    if (threadIdx.x == 0) a.ucnt[r] = total;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void k_row_huge(RowArgs a, const int32_t *list_in,
                                                     const int32_t *count_in) {
  __shared__ uint64_t lds[kChunk64];
  __shared__ int32_t tmp[kBlock / kWave];
  const int64_t n_items = *count_in;
  for (int64_t gi = blockIdx.x; gi < n_items; gi += gridDim.x) {
    const int64_t r = list_in[gi];
    const int64_t lo = a.zoff[r], L = a.zoff[r + 1] - lo;
    uint64_t *ka = a.zkey + lo, *kb = a.zsort + lo;
    bool in_b = block_merge_sort_global<uint64_t, kChunk64>(ka, kb, L, lds, ~0ull);
    if (!in_b) {
      for (int64_t i = threadIdx.x; i < L; i += kBlock) kb[i] = ka[i];
      __syncthreads();
    }
    int32_t heads = 0;
    for (int64_t i = threadIdx.x; i < L; i += kBlock)
      if (i == 0 || key_col(kb[i]) != key_col(kb[i - 1])) ++heads;
    int32_t total = block_sum<int32_t>(heads, tmp);
    if (threadIdx.x == 0) a.ucnt[r] = total;
    __syncthreads();
  }
}

__global__ void k_virtual_counts(const int32_t *virt_net, const int32_t *M, int64_t N,
                                 int64_t V, int32_t *ucnt) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < V) ucnt[N + i] = M[virt_net[i]];
}

__global__ void k_row_ptr32(const int64_t *rp64, int64_t n, int32_t *rp32) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i <= n) rp32[i] = static_cast<int32_t>(rp64[i]);
}

// ---------------------------------------------------------------------------
// 6./7. merge into the CSR of A, degrees
// ---------------------------------------------------------------------------
__global__ void k_merge_cells(const int64_t *zoff, const uint64_t *zsort, const double *wnet,
                              const int32_t *row_ptr, int64_t N, int32_t *col, double *w,
                              double *deg) {
  int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= N) return;
  const int64_t lo = zoff[r], hi = zoff[r + 1];
  int64_t out = row_ptr[r];
  double d = 0.0;
  uint32_t cur = 0;
  double acc = 0.0;
  for (int64_t p = lo; p < hi; ++p) {
    uint64_t k = zsort[p];
    uint32_t c = key_col(k);
    double wk = wnet[static_cast<uint32_t>(k)];
    if (p == lo) {
      cur = c;
      acc = wk;
    } else if (c == cur) {
      acc = acc + wk;
    } else {
      col[out] = static_cast<int32_t>(cur);
      w[out] = acc;
      ++out;
      d = d + acc;
      cur = c;
      acc = wk;
    }
  }
  if (hi > lo) {
    col[out] = static_cast<int32_t>(cur);
    w[out] = acc;
    d = d + acc;
  }
  deg[r] = d;
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
    for (int32_t i = lane; i < m; i += kWave) {
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
// 8. normalisation for one sigma
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

template <int D>
__global__ __launch_bounds__(kBlock) void k_sigma_values(const int32_t *row_ptr,
                                                         const int32_t *col, const double *w,
                                                         const double *s, int64_t R,
                                                         typename Store<D>::T *val) {
  constexpr int G = 8;
  const int t = threadIdx.x & (G - 1);
  const int64_t r = (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) / G;
  if (r >= R) return;
  const double si = s[r];
  for (int64_t p = row_ptr[r] + t; p < row_ptr[r + 1]; p += G)
    val[p] = Store<D>::from_f64((w[p] * si) * s[col[p]]);
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
  k_sigma_values<D><<<grid_for(g->num_rows * 8), kBlock, 0, st>>>(
      g->row_ptr, g->col, g->w, s, g->num_rows, static_cast<T *>(b.val));
  return check_launch("k_sigma_values");
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

unsigned list_grid() { return 2048; }

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
  } else {
    GIFT_HIP(hipMemcpyAsync(&P, d->net_ptr + E, 8, hipMemcpyDeviceToHost, st));
    GIFT_HIP(hipStreamSynchronize(st));
    if (P < 0) return set_error(GIFT_EINVAL, "net_ptr[num_nets] is negative");
  }
  if (P >= (int64_t(1) << 31) || N + E >= (int64_t(1) << 31))
    return set_error(GIFT_EUNSUPPORTED, "netlist too large (pins %lld, cells+nets %lld)",
                     (long long)P, (long long)(N + E));

  uint32_t *flag = nullptr;
  int32_t *M = nullptr, *ucell = nullptr, *pin_net = nullptr, *lists = nullptr, *counts = nullptr;
  uint32_t *tmp32 = nullptr;
  GIFT_TRY(sc.get(&flag, 1, "flag"));
  GIFT_TRY(sc.get(&M, E, "net sizes"));
  GIFT_TRY(sc.get(&ucell, P, "distinct cells"));
  GIFT_TRY(sc.get(&pin_net, P, "pin nets"));
  GIFT_TRY(sc.get(&tmp32, P, "net sort scratch"));
  const int64_t list_cap = (E > N ? E : N) + 1;
  GIFT_TRY(sc.get(&lists, 3 * list_cap, "tier lists"));
  GIFT_TRY(sc.get(&counts, 8, "tier counts"));
  GIFT_HIP(hipMemsetAsync(flag, 0, 4, st));
  GIFT_HIP(hipMemsetAsync(counts, 0, 8 * 4, st));
  GIFT_HIP(hipMemsetAsync(pin_net, 0xff, P * 4 + 4, st));

  k_check_ends<<<1, 64, 0, st>>>(net_ptr, E, P, flag);
  GIFT_TRY(check_launch("k_check_ends"));

  // 1. distinct cells per net, four tiers
  NetArgs na{net_ptr, pin, E, P, N, M, ucell, pin_net, flag, nullptr, nullptr};
  int32_t *l1 = lists, *l2 = lists + list_cap, *l3 = lists + 2 * list_cap;
  na.list_out = l1;
  na.count_out = counts + 0;
  k_net_group<16><<<grid_for(E * 16), kBlock, 0, st>>>(na, nullptr, nullptr);
  GIFT_TRY(check_launch("k_net_group<16>"));
  na.list_out = l2;
  na.count_out = counts + 1;
  k_net_group<64><<<list_grid(), kBlock, 0, st>>>(na, l1, counts + 0);
  GIFT_TRY(check_launch("k_net_group<64>"));
  na.list_out = l3;
  na.count_out = counts + 2;
  k_net_block<<<list_grid(), kBlock, 0, st>>>(na, l2, counts + 1);
  GIFT_TRY(check_launch("k_net_block"));
  k_net_huge<<<256, kBlock, 0, st>>>(na, l3, counts + 2, tmp32);
  GIFT_TRY(check_launch("k_net_huge"));

  // 2. classify
  int32_t *is_star = nullptr, *virt_net = nullptr;
  int64_t *vrank = nullptr;
  double *wnet = nullptr;
  GIFT_TRY(sc.get(&is_star, E, "star flags"));
  GIFT_TRY(sc.get(&vrank, E + 1, "virtual ranks"));
  GIFT_TRY(sc.get(&wnet, E, "net weights"));
  GIFT_TRY(sc.get(&virt_net, E, "virtual nets"));
  k_classify<<<grid_for(E), kBlock, 0, st>>>(M, E, d->star_threshold, d->weight_model, is_star,
                                             wnet);
  GIFT_TRY(check_launch("k_classify"));
  GIFT_TRY(scan_i32_to_i64(is_star, vrank, E, st));
  k_virtual_map<<<grid_for(E), kBlock, 0, st>>>(is_star, vrank, E, virt_net);
  GIFT_TRY(check_launch("k_virtual_map"));

  // 3. entries per cell row
  int32_t *cnt = nullptr;
  int64_t *zoff = nullptr;
  GIFT_TRY(sc.get(&cnt, N, "row counts"));
  GIFT_TRY(sc.get(&zoff, N + 1, "row offsets"));
  GIFT_HIP(hipMemsetAsync(cnt, 0, N * 4 + 4, st));
  EmitArgs ea{net_ptr, ucell, pin_net, M, is_star, vrank, E, P, N};
  k_count<<<grid_for(P), kBlock, 0, st>>>(ea, cnt);
  GIFT_TRY(check_launch("k_count"));
  GIFT_TRY(scan_i32_to_i64(cnt, zoff, N, st));

  // sizes back to the host
  struct Sizes {
    uint32_t flag;
    uint32_t pad;
    int64_t V, Z;
  } hs{};
  GIFT_HIP(hipMemcpyAsync(&hs.flag, flag, 4, hipMemcpyDeviceToHost, st));
  GIFT_HIP(hipMemcpyAsync(&hs.V, vrank + E, 8, hipMemcpyDeviceToHost, st));
  GIFT_HIP(hipMemcpyAsync(&hs.Z, zoff + N, 8, hipMemcpyDeviceToHost, st));
  GIFT_HIP(hipStreamSynchronize(st));
  if (hs.flag & kFlagBadNetPtr)
    return set_error(GIFT_EINVAL, "net_ptr must start at 0, end at the pin count and not decrease");
  if (hs.flag & kFlagBadPin) return set_error(GIFT_EINVAL, "a pin names a cell outside [0, num_cells)");
  const int64_t V = hs.V, Z = hs.Z, R = N + V;
  if (R >= (int64_t(1) << 31))
    return set_error(GIFT_EUNSUPPORTED, "too many rows (%lld)", (long long)R);
  g->num_cells = N;
  g->num_virtual = V;
  g->num_rows = R;

  // 4. emit
  uint64_t *zkey = nullptr, *zsort = nullptr;
  int32_t *cursor = nullptr, *ucnt = nullptr;
  GIFT_TRY(sc.get(&zkey, Z, "emitted keys"));
  GIFT_TRY(sc.get(&zsort, Z, "sorted keys"));
  GIFT_TRY(sc.get(&cursor, N, "row cursors"));
  GIFT_TRY(sc.get(&ucnt, R, "distinct counts"));
  GIFT_HIP(hipMemsetAsync(cursor, 0, N * 4 + 4, st));
  k_emit<<<grid_for(P), kBlock, 0, st>>>(ea, zoff, cursor, zkey);
  GIFT_TRY(check_launch("k_emit"));

  // 5. sort rows, four tiers
  RowArgs ra{zoff, zkey, zsort, ucnt, N, nullptr, nullptr};
  ra.list_out = l1;
  ra.count_out = counts + 3;
  k_row_group<16><<<grid_for(N * 16), kBlock, 0, st>>>(ra, nullptr, nullptr);
  GIFT_TRY(check_launch("k_row_group<16>"));
  ra.list_out = l2;
  ra.count_out = counts + 4;
  k_row_group<64><<<list_grid(), kBlock, 0, st>>>(ra, l1, counts + 3);
  GIFT_TRY(check_launch("k_row_group<64>"));
  ra.list_out = l3;
  ra.count_out = counts + 5;
  k_row_block<<<list_grid(), kBlock, 0, st>>>(ra, l2, counts + 4);
  GIFT_TRY(check_launch("k_row_block"));
  k_row_huge<<<256, kBlock, 0, st>>>(ra, l3, counts + 5);
  GIFT_TRY(check_launch("k_row_huge"));
  k_virtual_counts<<<grid_for(V), kBlock, 0, st>>>(virt_net, M, N, V, ucnt);
  GIFT_TRY(check_launch("k_virtual_counts"));

  // 6. row_ptr
  int64_t *rp64 = nullptr;
  GIFT_TRY(sc.get(&rp64, R + 1, "row offsets (64-bit)"));
  GIFT_TRY(scan_i32_to_i64(ucnt, rp64, R, st));
  int64_t nnz = 0, nnz_cells = 0;
  GIFT_HIP(hipMemcpyAsync(&nnz, rp64 + R, 8, hipMemcpyDeviceToHost, st));
  GIFT_HIP(hipMemcpyAsync(&nnz_cells, rp64 + N, 8, hipMemcpyDeviceToHost, st));
  GIFT_HIP(hipStreamSynchronize(st));
  g->nnz_cells = nnz_cells;
  if (nnz >= (int64_t(1) << 31))
    return set_error(GIFT_EUNSUPPORTED, "too many stored entries (%lld)", (long long)nnz);
  g->nnz = nnz;
  GIFT_TRY(dev_alloc(reinterpret_cast<void **>(&g->row_ptr), (R + 1) * 4, st, "row_ptr"));
  GIFT_TRY(dev_alloc(reinterpret_cast<void **>(&g->col), nnz * 4, st, "col"));
  GIFT_TRY(dev_alloc(reinterpret_cast<void **>(&g->w), nnz * 8, st, "weights"));
  GIFT_TRY(dev_alloc(reinterpret_cast<void **>(&g->deg), R * 8, st, "degrees"));
  g->bytes = (R + 1) * 4 + nnz * 12 + R * 8;
  k_row_ptr32<<<grid_for(R + 1), kBlock, 0, st>>>(rp64, R, g->row_ptr);
  GIFT_TRY(check_launch("k_row_ptr32"));

  // 7. merge
  k_merge_cells<<<grid_for(N), kBlock, 0, st>>>(zoff, zsort, wnet, g->row_ptr, N, g->col, g->w,
                                                g->deg);
  GIFT_TRY(check_launch("k_merge_cells"));
  k_star_rows<<<grid_for(V * kWave), kBlock, 0, st>>>(virt_net, net_ptr, M, ucell, wnet,
                                                       g->row_ptr, N, V, g->col, g->w, g->deg);
  GIFT_TRY(check_launch("k_star_rows"));

  // 8. normalisation
  for (int32_t i = 0; i < d->num_sigmas; ++i) GIFT_TRY(prepare_sigma(g, d->sigmas[i], st));

  // choose the SpMM row split from the mean row lengths
  double mean_cells = N ? static_cast<double>(nnz) / static_cast<double>(R) : 0.0;
  g->group_cells = mean_cells > 24 ? 8 : 4;
  g->group_virtual = 16;
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
  if (d->mem_space == GIFT_MEM_HOST) {
    if (d->net_ptr[0] != 0) return set_error(GIFT_EINVAL, "net_ptr[0] must be 0");
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
    // algorithmic bytes: the netlist in, the graph out (structure, float64
    // weights and degrees, values and diagonal per sigma)
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
