// Eigenvector placement: the classic placer that Section 3.3.1 analyses as
// the ideal low-pass filter of eq. ideal_filter.  Its placement is [u_2, u_3],
// the eigenvectors of the second and third smallest eigenvalues of the graph
// Laplacian L = D - A (Section 2.1, where U diagonalises L), here of the
// clique net model.
//
// A netlist graph is usually disconnected and every component adds a zero
// eigenvalue, so the eigenvectors are taken on the largest connected
// component (most cells; ties: smallest cell index), with its constant
// vector (eigenvalue 0) projected out; cells outside it get 0.
//
// Steps, all on the device:
//   1. components: every row starts with its own index as label; sweeps
//      lower each row's label to the smallest among itself and its
//      neighbours (and push it to them) until nothing changes, so every row
//      ends with the smallest row index of its component (a cell index);
//   2. the giant component: cell counts per label, the largest by a
//      fixed-shape reduction;
//   3. L x for a block of K vectors on the resident star graph: star rows
//      take the mean of their cells, which eliminates them exactly (the Schur
//      complement of a star of weight M w(M) is the clique of weight w(M)),
//      then y_i = d_i x_i - sum_j w_ij x_j on the cell rows;
//   4. Chebyshev-filtered subspace iteration: each outer step applies
//      T_m((L - c I) / e), with [c - e, c + e] = [theta_K, b] the interval to
//      damp (theta_K the largest Ritz value of the block, b = 2 max degree >=
//      lambda_max), projects out the constant, orthonormalises the block by
//      Cholesky QR twice, and takes the Ritz pairs of the 4 x 4 projected
//      matrix (cyclic Jacobi).  It stops when the residuals of u_2 and u_3
//      are at most tol * b.
// Every reduction is formed per block over a fixed row range, and the
// blocks' partial sums are added in a fixed order, so results are
// deterministic.
#include <cmath>
#include <cstring>

#include "common.h"
#include "devutil.h"

namespace gift {
namespace {

constexpr int K = 4;               // block size: u_2, u_3 and two guard vectors
constexpr int kFilterDegree = 16;  // Chebyshev degree per outer step
constexpr int kRedBlocks = 1024;   // blocks of the row reductions
constexpr int kMaxSweeps = 4096;   // component sweeps before giving up

// Layout of the small device array of K x K matrices and K-vectors.
constexpr int kG = 0;            // Gram matrix / projected L (K x K)
constexpr int kT = kG + K * K;   // transform applied to the block (K x K)
constexpr int kTheta = kT + K * K;  // Ritz values, ascending
constexpr int kSum = kTheta + K;    // column sums over the component
constexpr int kRes = kSum + K;      // squared residual norms
constexpr int kSign = kRes + K;     // output signs
constexpr int kSmall = kSign + K;

// ---------------------------------------------------------------------------
// 1-2. components and the giant component
// ---------------------------------------------------------------------------
__global__ void k_cc_init(int32_t *label, int64_t R) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < R) label[i] = static_cast<int32_t>(i);
}

// One sweep: row i takes the smallest label among itself, its neighbours and
// its label's label, and lowers its neighbours' labels to it.  Labels only
// decrease and always name a row of the same component.
__global__ void k_cc_sweep(const int32_t *row_ptr, const int32_t *col, int64_t R,
                           int32_t *label, uint32_t *changed) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= R) return;
  const int32_t p0 = row_ptr[i], p1 = row_ptr[i + 1];
  int32_t m = label[i];
  for (int32_t p = p0; p < p1; ++p) {
    const int32_t l = label[col[p]];
    m = l < m ? l : m;
  }
  const int32_t jump = label[m];
  m = jump < m ? jump : m;
  bool ch = false;
  if (m < label[i]) {
    atomicMin(label + i, m);
    ch = true;
  }
  for (int32_t p = p0; p < p1; ++p) {
    const int32_t j = col[p];
    if (label[j] > m) {
      atomicMin(label + j, m);
      ch = true;
    }
  }
  if (ch) atomicOr(changed, 1u);
}

// Component sizes: count[label[i]] += 1 over the cell rows.  Block b takes a
// contiguous range of cells and adds into an LDS table first: nearly every
// cell of a placement graph is in one component, and one address taking N
// device atomics in a row costs milliseconds.
constexpr int kCountSlots = 1024;
__global__ __launch_bounds__(kBlock) void k_cc_count(const int32_t *label, int64_t N,
                                                     int32_t *count) {
  __shared__ LdsHash<int32_t, kCountSlots> h;
  h.clear();
  __syncthreads();
  const int64_t per = (N + gridDim.x - 1) / gridDim.x;
  const int64_t lo = static_cast<int64_t>(blockIdx.x) * per;
  const int64_t hi = lo + per < N ? lo + per : N;
  const gptr<const int32_t> lb = to_global(label);
  for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) h.add(lb[i], 1, count);
  __syncthreads();
  h.flush(count);
}

// key = count << 32 | (2^31 - 1 - label): the largest key is the largest
// component, ties to the smallest label.  Per block of labels, then one
// block over the partial maxima.
__global__ __launch_bounds__(kBlock) void k_cc_best(const int32_t *count, int64_t N,
                                                    int64_t *part) {
  __shared__ int64_t red[kBlock];
  int64_t best = 0;
  for (int64_t l = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; l < N;
       l += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int64_t c = count[l];
    if (c > 0) {
      const int64_t key = (c << 32) | (0x7fffffff - l);
      best = key > best ? key : best;
    }
  }
  red[threadIdx.x] = best;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off && red[threadIdx.x + off] > red[threadIdx.x])
      red[threadIdx.x] = red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out[0] = the best key (one block over the per-block maxima).
__global__ __launch_bounds__(kBlock) void k_cc_key(const int64_t *part, int nb, int64_t *out) {
  __shared__ int64_t red[kBlock];
  int64_t best = 0;
  for (int b = threadIdx.x; b < nb; b += kBlock) best = part[b] > best ? part[b] : best;
  red[threadIdx.x] = best;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off && red[threadIdx.x + off] > red[threadIdx.x])
      red[threadIdx.x] = red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// dpart[b] = the largest degree over block b's range of the giant
// component's cells (the component named by key[0]).
__global__ __launch_bounds__(kBlock) void k_cc_dmax(const int32_t *label, const double *deg,
                                                    int64_t N, const int64_t *key,
                                                    double *dpart) {
  __shared__ double red[kBlock];
  const int32_t g = static_cast<int32_t>(0x7fffffff - (key[0] & 0xffffffff));
  const int64_t per = (N + gridDim.x - 1) / gridDim.x;
  const int64_t lo = static_cast<int64_t>(blockIdx.x) * per;
  const int64_t hi = lo + per < N ? lo + per : N;
  double dmax = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock)
    if (label[i] == g) dmax = deg[i] > dmax ? deg[i] : dmax;
  red[threadIdx.x] = dmax;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off && red[threadIdx.x + off] > red[threadIdx.x])
      red[threadIdx.x] = red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) dpart[blockIdx.x] = red[0];
}

// out[1] = bits of 2 max degree over the giant component's cells (an upper
// bound on lambda_max by Gershgorin).  Maxima are exact, so the split over
// blocks does not change the value.
__global__ __launch_bounds__(kBlock) void k_cc_bound(const double *dpart, int nb, int64_t *out) {
  __shared__ double red[kBlock];
  double dmax = 0.0;
  for (int b = threadIdx.x; b < nb; b += kBlock) dmax = dpart[b] > dmax ? dpart[b] : dmax;
  red[threadIdx.x] = dmax;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off && red[threadIdx.x + off] > red[threadIdx.x])
      red[threadIdx.x] = red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double b = 2.0 * red[0];
    int64_t bits;
    memcpy(&bits, &b, 8);
    out[1] = bits;
  }
}

// ---------------------------------------------------------------------------
// 3. L x on the star graph, for a block of K vectors (row-major N x K)
// ---------------------------------------------------------------------------
// Star rows: the mean of their cells (one wave per star row).
__global__ __launch_bounds__(kBlock) void k_eig_star_means(const int32_t *row_ptr,
                                                           const int32_t *col, int64_t N,
                                                           int64_t V, const double *x,
                                                           double *ext) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t v = static_cast<int64_t>(blockIdx.x) * (kBlock / kWave) + threadIdx.x / kWave;
  if (v >= V) return;
  const int32_t p0 = row_ptr[N + v], p1 = row_ptr[N + v + 1];
  double s[K] = {};
  for (int32_t p = p0 + lane; p < p1; p += kWave) {
    const int64_t c = col[p];
#pragma unroll
    for (int q = 0; q < K; ++q) s[q] += x[c * K + q];
  }
#pragma unroll
  for (int q = 0; q < K; ++q)
    for (int off = kWave / 2; off > 0; off >>= 1) s[q] += __shfl_xor(s[q], off);
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < K; ++q) ext[v * K + q] = p1 > p0 ? s[q] / static_cast<double>(p1 - p0) : 0.0;
  }
}

// out = alpha (L x) + beta x + gamma prev on the giant component's cells, 0
// elsewhere (prev may be NULL).  One block per SpMM row tile of cell rows
// (class 0): the tile's columns and weights are staged in LDS with every
// load in flight at once, then each row is taken by a group of lanes (one
// lane when the tile has many rows), four gathers of 32-byte rows in flight
// per lane, the group's partial sums combined by a fixed shuffle tree.  A
// row longer than the class's limit has a tile of its own and the whole
// block: lanes over its entries, then a fixed tree over the block.  The
// order is the same on every run.
__device__ __forceinline__ int eig_lanes_for(int rows) {
  int g = 1;
  while (g < 64 && rows * g * 2 <= kBlock) g <<= 1;
  return g;
}

__device__ __forceinline__ void eig_row_out(int64_t i, const double (&acc)[K], bool in,
                                            const double *deg, const double *x,
                                            const double *prev, double alpha, double beta,
                                            double gamma, double *out) {
  double o[K] = {};
  if (in) {
    const double d = to_global(deg)[i];
#pragma unroll
    for (int q = 0; q < K; ++q) {
      const double xi = to_global(x)[i * K + q];
      o[q] = alpha * (d * xi - acc[q]) + beta * xi;
      if (prev) o[q] += gamma * to_global(prev)[i * K + q];
    }
  }
#pragma unroll
  for (int q = 0; q < K; ++q) out[i * K + q] = o[q];
}

__global__ __launch_bounds__(kBlock) void k_eig_apply(const TileDesc *tiles,
                                                      const int32_t *row_ptr, const int32_t *col,
                                                      const double *w, const double *deg,
                                                      const int32_t *label, int32_t giant,
                                                      int64_t N, const double *x,
                                                      const double *ext, const double *prev,
                                                      double alpha, double beta, double gamma,
                                                      double *out) {
  using TCL = TileClass<0>;
  constexpr int kStage = (TCL::kCap + kBlock - 1) / kBlock;
  __shared__ int32_t loff[TCL::kRows + 1];
  __shared__ int32_t lcol[TCL::kCap];
  __shared__ double lw[TCL::kCap];
  __shared__ double red[kBlock / kWave][K];
  const TileDesc td = gload(tiles, xcd_remap(blockIdx.x, gridDim.x));
  const gptr<const double> xg = to_global(x), eg = to_global(ext), wg = to_global(w);
  const gptr<const int32_t> cg = to_global(col), rp = to_global(row_ptr);
  const int ns = td.r1 - td.r0, n = td.p1 - td.p0;
  const int tid = threadIdx.x;
  auto src_of = [&](int64_t j) { return j < N ? xg + j * K : eg + (j - N) * K; };
  if (ns == 1 && n > TCL::kLong) {
    const int64_t i = td.r0;
    const bool in = to_global(label)[i] == giant;
    double acc[K] = {};
    if (in) {
      int q = td.p0 + tid;
      for (; q + 3 * kBlock < td.p1; q += 4 * kBlock) {
        int64_t j[4];
        double wj[4], v[4][K];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          j[u] = cg[q + u * kBlock];
          wj[u] = wg[q + u * kBlock];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const gptr<const double> src = src_of(j[u]);
#pragma unroll
          for (int k = 0; k < K; ++k) v[u][k] = src[k];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int k = 0; k < K; ++k) acc[k] += wj[u] * v[u][k];
      }
      for (; q < td.p1; q += kBlock) {
        const double wj = wg[q];
        const gptr<const double> src = src_of(cg[q]);
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] += wj * src[k];
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      for (int off = kWave / 2; off > 0; off >>= 1) acc[k] += __shfl_xor(acc[k], off);
      if ((tid & (kWave - 1)) == 0) red[tid / kWave][k] = acc[k];
    }
    __syncthreads();
    if (tid == 0) {
      double tot[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        tot[k] = red[0][k];
        for (int wv = 1; wv < kBlock / kWave; ++wv) tot[k] += red[wv][k];
      }
      eig_row_out(i, tot, in, deg, x, prev, alpha, beta, gamma, out);
    }
    return;
  }
  {
    int32_t cj[kStage];
    double wv[kStage];
#pragma unroll
    for (int k = 0; k < kStage; ++k) {
      const int i = tid + k * kBlock;
      const int q = i < n ? td.p0 + i : 0;  // unused slots read entry 0, which always exists
      cj[k] = cg[q];
      wv[k] = wg[q];
    }
    for (int i = tid; i <= ns; i += kBlock) loff[i] = rp[td.r0 + i] - td.p0;
#pragma unroll
    for (int k = 0; k < kStage; ++k) {
      const int i = tid + k * kBlock;
      if (i < n) {
        lcol[i] = cj[k];
        lw[i] = wv[k];
      }
    }
  }
  __syncthreads();
  const int G = eig_lanes_for(ns);
  const int lane = tid & (G - 1);
  for (int base = 0; base < ns; base += kBlock / G) {
    const int rr = base + tid / G;
    const bool live = rr < ns;
    const int64_t i = td.r0 + (live ? rr : 0);
    const bool in = live && to_global(label)[i] == giant;
    double acc[K] = {};
    if (in) {
      const int q1 = loff[rr + 1];
      int q = loff[rr] + lane;
      for (; q + 3 * G < q1; q += 4 * G) {
        double v[4][K];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const gptr<const double> src = src_of(lcol[q + u * G]);
#pragma unroll
          for (int k = 0; k < K; ++k) v[u][k] = src[k];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int k = 0; k < K; ++k) acc[k] += lw[q + u * G] * v[u][k];
      }
      for (; q < q1; q += G) {
        const gptr<const double> src = src_of(lcol[q]);
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] += lw[q] * src[k];
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
      for (int off = G >> 1; off > 0; off >>= 1) acc[k] += __shfl_xor(acc[k], off);
    if (live && lane == 0) eig_row_out(i, acc, in, deg, x, prev, alpha, beta, gamma, out);
  }
}

// ---------------------------------------------------------------------------
// block reductions over the N rows (fixed ranges; partials added in a fixed
// order)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void row_range(int64_t n, int64_t *lo, int64_t *hi) {
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  *lo = static_cast<int64_t>(blockIdx.x) * per;
  *hi = *lo + per < n ? *lo + per : n;
}

template <int M>
__device__ __forceinline__ void block_sums(double (&v)[M], double *red, double *part) {
#pragma unroll
  for (int q = 0; q < M; ++q) {
    red[threadIdx.x] = v[q];
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x * M + q] = red[0];
    __syncthreads();
  }
}

// part = per-block a^T b (K x K, row-major), over all N rows
__global__ __launch_bounds__(kBlock) void k_eig_gram(const double *a, const double *b, int64_t N,
                                                     double *part) {
  __shared__ double red[kBlock];
  int64_t lo, hi;
  row_range(N, &lo, &hi);
  double s[K * K] = {};
  for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
    double ai[K], bi[K];
#pragma unroll
    for (int q = 0; q < K; ++q) {
      ai[q] = a[i * K + q];
      bi[q] = b[i * K + q];
    }
#pragma unroll
    for (int q = 0; q < K; ++q)
#pragma unroll
      for (int r = 0; r < K; ++r) s[q * K + r] += ai[q] * bi[r];
  }
  block_sums<K * K>(s, red, part);
}

// part = per-block column sums of x over the giant component
__global__ __launch_bounds__(kBlock) void k_eig_colsum(const double *x, const int32_t *label,
                                                       int32_t giant, int64_t N, double *part) {
  __shared__ double red[kBlock];
  int64_t lo, hi;
  row_range(N, &lo, &hi);
  double s[K] = {};
  for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock)
    if (label[i] == giant)
#pragma unroll
      for (int q = 0; q < K; ++q) s[q] += x[i * K + q];
  block_sums<K>(s, red, part);
}

// part = per-block sums of (w_q - theta_q x_q)^2 over all rows
__global__ __launch_bounds__(kBlock) void k_eig_resid(const double *x, const double *wv,
                                                      const double *small, int64_t N,
                                                      double *part) {
  __shared__ double red[kBlock];
  int64_t lo, hi;
  row_range(N, &lo, &hi);
  double theta[K];
#pragma unroll
  for (int q = 0; q < K; ++q) theta[q] = small[kTheta + q];
  double s[K] = {};
  for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock)
#pragma unroll
    for (int q = 0; q < K; ++q) {
      const double r = wv[i * K + q] - theta[q] * x[i * K + q];
      s[q] += r * r;
    }
  block_sums<K>(s, red, part);
}
// out[q] = sum over b of part[b * M + q]: block q, in the fixed order of
// block_sum_strided
__global__ __launch_bounds__(kBlock) void k_eig_sum(const double *part, int nb, int M,
                                                    double *out) {
  __shared__ double red[kBlock];
  const double s = block_sum_strided(part + blockIdx.x, nb, M, red);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// A reproducible start: a hash of (seed, row, column) mapped to [-1, 1) on
// the giant component, 0 elsewhere (splitmix64 finaliser).
__global__ void k_eig_rand(double *x, const int32_t *label, int32_t giant, int64_t N,
                           uint64_t seed) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N) return;
#pragma unroll
  for (int q = 0; q < K; ++q) {
    uint64_t z = seed + 0x9e3779b97f4a7c15ull * static_cast<uint64_t>(i * K + q + 1);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    const double u = static_cast<double>(z >> 11) * (1.0 / 9007199254740992.0);
    x[i * K + q] = label[i] == giant ? 2.0 * u - 1.0 : 0.0;
  }
}

// x -= mean over the component (from the column sums), 0 outside it
__global__ void k_eig_deflate(double *x, const int32_t *label, int32_t giant, int64_t N,
                              const double *small, double count) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const bool in = label[i] == giant;
#pragma unroll
  for (int q = 0; q < K; ++q) x[i * K + q] = in ? x[i * K + q] - small[kSum + q] / count : 0.0;
}

// out = x T (T row-major K x K at small[kT]); out may be x
__global__ void k_eig_mul(const double *x, const double *small, int64_t N, double *out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double xi[K], o[K] = {};
#pragma unroll
  for (int q = 0; q < K; ++q) xi[q] = x[i * K + q];
#pragma unroll
  for (int r = 0; r < K; ++r)
#pragma unroll
    for (int q = 0; q < K; ++q) o[q] += xi[r] * small[kT + r * K + q];
#pragma unroll
  for (int q = 0; q < K; ++q) out[i * K + q] = o[q];
}

// T = R^-1 with R^T R = G + eps tr(G) I (Cholesky; the small shift keeps it
// positive definite when the block is nearly dependent, and a second pass of
// Cholesky QR restores orthonormality).  One thread.
__global__ void k_eig_cholinv(double *small) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double g[K][K], r[K][K] = {}, t[K][K] = {};
  double tr = 0.0;
  for (int a = 0; a < K; ++a)
    for (int b = 0; b < K; ++b) g[a][b] = 0.5 * (small[kG + a * K + b] + small[kG + b * K + a]);
  for (int a = 0; a < K; ++a) tr += g[a][a];
  if (!(tr > 0.0)) {
    for (int a = 0; a < K; ++a)
      for (int b = 0; b < K; ++b) small[kT + a * K + b] = a == b ? 1.0 : 0.0;
    return;
  }
  for (int a = 0; a < K; ++a) g[a][a] += 1e-14 * tr;
  for (int j = 0; j < K; ++j) {
    double d = g[j][j];
    for (int k = 0; k < j; ++k) d -= r[k][j] * r[k][j];
    r[j][j] = sqrt(d > 1e-300 ? d : 1e-300);
    for (int i = j + 1; i < K; ++i) {
      double v = g[j][i];
      for (int k = 0; k < j; ++k) v -= r[k][j] * r[k][i];
      r[j][i] = v / r[j][j];
    }
  }
  // R upper triangular: solve R T = I column by column
  for (int c = 0; c < K; ++c)
    for (int i = K - 1; i >= 0; --i) {
      double v = i == c ? 1.0 : 0.0;
      for (int k = i + 1; k < K; ++k) v -= r[i][k] * t[k][c];
      t[i][c] = v / r[i][i];
    }
  for (int a = 0; a < K; ++a)
    for (int b = 0; b < K; ++b) small[kT + a * K + b] = t[a][b];
}

// Eigenpairs of the symmetric K x K matrix at small[kG] by cyclic Jacobi:
// eigenvectors (columns) to small[kT], eigenvalues ascending to small[kTheta].
// One thread.
__global__ void k_eig_rr(double *small) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double a[K][K], v[K][K];
  for (int i = 0; i < K; ++i)
    for (int j = 0; j < K; ++j) {
      a[i][j] = 0.5 * (small[kG + i * K + j] + small[kG + j * K + i]);
      v[i][j] = i == j ? 1.0 : 0.0;
    }
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int i = 0; i < K; ++i) {
      dia += a[i][i] * a[i][i];
      for (int j = i + 1; j < K; ++j) off += a[i][j] * a[i][j];
    }
    if (off <= 1e-32 * dia || off == 0.0) break;
    for (int p = 0; p < K; ++p)
      for (int q = p + 1; q < K; ++q) {
        if (a[p][q] == 0.0) continue;
        const double th = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
        const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < K; ++k) {  // columns p, q
          const double akp = a[k][p], akq = a[k][q];
          a[k][p] = c * akp - s * akq;
          a[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < K; ++k) {  // rows p, q
          const double apk = a[p][k], aqk = a[q][k];
          a[p][k] = c * apk - s * aqk;
          a[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < K; ++k) {
          const double vkp = v[k][p], vkq = v[k][q];
          v[k][p] = c * vkp - s * vkq;
          v[k][q] = s * vkp + c * vkq;
        }
      }
  }
  int order[K];
  for (int i = 0; i < K; ++i) order[i] = i;
  for (int i = 1; i < K; ++i)  // insertion sort by eigenvalue
    for (int j = i; j > 0 && a[order[j]][order[j]] < a[order[j - 1]][order[j - 1]]; --j) {
      const int t = order[j];
      order[j] = order[j - 1];
      order[j - 1] = t;
    }
  for (int c = 0; c < K; ++c) {
    small[kTheta + c] = a[order[c]][order[c]];
    for (int r = 0; r < K; ++r) small[kT + r * K + c] = v[r][order[c]];
  }
}

// Per block and column q < 2: the largest |x| (ties: smallest row) as
// (|x| bits, row) pairs; then one block picks the winners and sets the
// output signs so that each vector's largest-magnitude entry is positive.
__global__ __launch_bounds__(kBlock) void k_eig_argmax(const double *x, int64_t N,
                                                       double *vpart, int64_t *ipart) {
  __shared__ double rv[kBlock];
  __shared__ int64_t ri[kBlock];
  int64_t lo, hi;
  row_range(N, &lo, &hi);
  for (int q = 0; q < 2; ++q) {
    double bv = -1.0;
    int64_t bi = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
      const double a = fabs(x[i * K + q]);
      if (a > bv) {
        bv = a;
        bi = i;
      }
    }
    rv[threadIdx.x] = bv;
    ri[threadIdx.x] = bi;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off) {
        const double ov = rv[threadIdx.x + off];
        const int64_t oi = ri[threadIdx.x + off];
        if (ov > rv[threadIdx.x] || (ov == rv[threadIdx.x] && oi < ri[threadIdx.x])) {
          rv[threadIdx.x] = ov;
          ri[threadIdx.x] = oi;
        }
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      vpart[blockIdx.x * 2 + q] = rv[0];
      ipart[blockIdx.x * 2 + q] = ri[0];
    }
    __syncthreads();
  }
}

__global__ void k_eig_sign(const double *x, const double *vpart, const int64_t *ipart, int nb,
                           double *small) {
  const int q = threadIdx.x;
  if (q >= 2) return;
  double bv = -1.0;
  int64_t bi = 0;
  for (int b = 0; b < nb; ++b) {
    const double v = vpart[b * 2 + q];
    const int64_t i = ipart[b * 2 + q];
    if (v > bv || (v == bv && i < bi)) {
      bv = v;
      bi = i;
    }
  }
  small[kSign + q] = x[bi * K + q] < 0.0 ? -1.0 : 1.0;
}

__global__ void k_eig_out(const double *x, const double *small, int64_t N, double *y,
                          int64_t ld) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N) return;
  y[i * ld] = small[kSign] * x[i * K];
  y[i * ld + 1] = small[kSign + 1] * x[i * K + 1];
}

// dst[i] = the bits of src[i] (doubles read back through int64 slots)
__global__ void k_eig_bits(const double *src, int n, int64_t *dst) {
  const int i = threadIdx.x;
  if (i >= n) return;
  int64_t b;
  const double v = src[i];
  memcpy(&b, &v, 8);
  dst[i] = b;
}

__global__ void k_eig_copy_i64(const int64_t *src, int n, int64_t *dst) {
  const int i = threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__global__ void k_eig_flag_i64(const uint32_t *flag, int64_t *dst) { dst[0] = *flag; }

}  // namespace
}  // namespace gift

using namespace gift;

namespace gift {
namespace {

// Reads n device doubles (bit patterns) or int64 values through a pinned
// slot: one launch and one wait.
gift_status read_back(hipStream_t st, const double *dsrc, const int64_t *isrc,
                      const uint32_t *flag, int n, int64_t *out) {
  Readback rb{};
  GIFT_TRY(readback_acquire(&rb));
  if (dsrc) k_eig_bits<<<1, 64, 0, st>>>(dsrc, n, rb.dev);
  else if (isrc) k_eig_copy_i64<<<1, 64, 0, st>>>(isrc, n, rb.dev);
  else k_eig_flag_i64<<<1, 1, 0, st>>>(flag, rb.dev);
  gift_status s = check_launch("eigen readback");
  if (s != GIFT_OK) {
    readback_release(rb);
    return s;
  }
  GIFT_TRY(readback_wait(rb, st));
  const volatile int64_t *h = rb.host;
  for (int i = 0; i < n; ++i) out[i] = h[i];
  readback_release(rb);
  return GIFT_OK;
}

double as_double(int64_t bits) {
  double d;
  memcpy(&d, &bits, 8);
  return d;
}

struct EigenRun {
  const gift_graph *g;
  hipStream_t st;
  int64_t N, V;
  const int32_t *label;
  int32_t giant;
  double count;
  double *ext, *part, *small;

  gift_status star(const double *x) {
    if (V == 0) return GIFT_OK;
    k_eig_star_means<<<grid_for(V * kWave), kBlock, 0, st>>>(g->row_ptr, g->col, N, V, x, ext);
    return check_launch("k_eig_star_means");
  }
  // out = alpha L x + beta x + gamma prev
  gift_status apply(const double *x, const double *prev, double alpha, double beta, double gamma,
                    double *out) {
    GIFT_TRY(star(x));
    // the cell tiles of class 0 cover rows 0..N-1 (star rows come after)
    const int64_t T = g->num_tiles_cells[0];
    if (T == 0) return GIFT_OK;
    k_eig_apply<<<static_cast<unsigned>(T), kBlock, 0, st>>>(
        g->tiles[0], g->row_ptr, g->col, g->w, g->deg, label, giant, N, x, ext, prev, alpha,
        beta, gamma, out);
    return check_launch("k_eig_apply");
  }
  gift_status gram(const double *a, const double *b) {
    k_eig_gram<<<kRedBlocks, kBlock, 0, st>>>(a, b, N, part);
    GIFT_TRY(check_launch("k_eig_gram"));
    k_eig_sum<<<K * K, kBlock, 0, st>>>(part, kRedBlocks, K * K, small + kG);
    return check_launch("k_eig_sum");
  }
  gift_status deflate(double *x) {
    k_eig_colsum<<<kRedBlocks, kBlock, 0, st>>>(x, label, giant, N, part);
    GIFT_TRY(check_launch("k_eig_colsum"));
    k_eig_sum<<<K, kBlock, 0, st>>>(part, kRedBlocks, K, small + kSum);
    GIFT_TRY(check_launch("k_eig_sum"));
    k_eig_deflate<<<grid_for(N), kBlock, 0, st>>>(x, label, giant, N, small, count);
    return check_launch("k_eig_deflate");
  }
  // Cholesky QR, twice
  gift_status orth(double *x) {
    for (int pass = 0; pass < 2; ++pass) {
      GIFT_TRY(gram(x, x));
      k_eig_cholinv<<<1, 1, 0, st>>>(small);
      GIFT_TRY(check_launch("k_eig_cholinv"));
      k_eig_mul<<<grid_for(N), kBlock, 0, st>>>(x, small, N, x);
      GIFT_TRY(check_launch("k_eig_mul"));
    }
    return GIFT_OK;
  }
  // Ritz pairs of the block: w = L x, H = x^T w, x <- x V, w <- w V; then
  // the Ritz values and squared residual norms back to the host
  gift_status rayleigh_ritz(double *x, double *w, double *theta, double *res) {
    GIFT_TRY(apply(x, nullptr, 1.0, 0.0, 0.0, w));
    GIFT_TRY(gram(x, w));
    k_eig_rr<<<1, 1, 0, st>>>(small);
    GIFT_TRY(check_launch("k_eig_rr"));
    k_eig_mul<<<grid_for(N), kBlock, 0, st>>>(x, small, N, x);
    GIFT_TRY(check_launch("k_eig_mul"));
    k_eig_mul<<<grid_for(N), kBlock, 0, st>>>(w, small, N, w);
    GIFT_TRY(check_launch("k_eig_mul"));
    k_eig_resid<<<kRedBlocks, kBlock, 0, st>>>(x, w, small, N, part);
    GIFT_TRY(check_launch("k_eig_resid"));
    k_eig_sum<<<K, kBlock, 0, st>>>(part, kRedBlocks, K, small + kRes);
    GIFT_TRY(check_launch("k_eig_sum"));
    int64_t bits[3 * K];
    static_assert(kRes == kTheta + 2 * K, "Ritz values and residuals are read together");
    GIFT_TRY(read_back(st, small + kTheta, nullptr, nullptr, 3 * K, bits));
    for (int q = 0; q < K; ++q) {
      theta[q] = as_double(bits[q]);
      res[q] = sqrt(as_double(bits[2 * K + q]));
    }
    return GIFT_OK;
  }
};

}  // namespace
}  // namespace gift

extern "C" gift_status gift_eigen_placement(const gift_graph *g, double tol, int32_t max_iter,
                                            uint64_t seed, double *y_out, int64_t ld_out,
                                            int32_t *labels, gift_eigen_result *result,
                                            void *stream) {
  clear_error();
  if (!g) return set_error(GIFT_EINVAL, "gift_eigen_placement: NULL graph");
  if (!result) return set_error(GIFT_EINVAL, "gift_eigen_placement: NULL result");
  if (!(tol > 0.0) || !std::isfinite(tol)) return set_error(GIFT_EINVAL, "tol must be > 0");
  if (max_iter < 1) return set_error(GIFT_EINVAL, "max_iter must be >= 1");
  if (ld_out < 2) return set_error(GIFT_EINVAL, "ld_out must be >= 2");
  const int64_t N = g->num_cells, V = g->num_virtual, R = g->num_rows;
  if (N < K + 2) return set_error(GIFT_EINVAL, "the graph has fewer than %d cells", K + 2);
  if (!y_out) return set_error(GIFT_EINVAL, "y_out is NULL");
  std::memset(result, 0, sizeof(*result));
  hipStream_t st = static_cast<hipStream_t>(stream);
  Scratch sc(st);

  // 1. components
  int32_t *label = nullptr, *count = nullptr;
  uint32_t *changed = nullptr;
  GIFT_TRY(sc.get(&label, R, "component labels"));
  GIFT_TRY(sc.get(&count, N, "component sizes"));
  GIFT_TRY(sc.get(&changed, 1, "change flag"));
  k_cc_init<<<grid_for(R), kBlock, 0, st>>>(label, R);
  GIFT_TRY(check_launch("k_cc_init"));
  int sweeps = 0;
  for (;;) {
    if (sweeps == kMaxSweeps)
      return set_error(GIFT_EUNSUPPORTED, "components did not settle in %d sweeps", kMaxSweeps);
    GIFT_HIP(hipMemsetAsync(changed, 0, 4, st));
    k_cc_sweep<<<grid_for(R), kBlock, 0, st>>>(g->row_ptr, g->col, R, label, changed);
    GIFT_TRY(check_launch("k_cc_sweep"));
    ++sweeps;
    int64_t ch = 0;
    GIFT_TRY(read_back(st, nullptr, nullptr, changed, 1, &ch));
    if (ch == 0) break;
  }

  // 2. the giant component and the spectral bound
  int64_t *bpart = nullptr, *pick = nullptr;
  double *dpart = nullptr;
  GIFT_TRY(sc.get(&bpart, kRedBlocks, "component maxima"));
  GIFT_TRY(sc.get(&dpart, kRedBlocks, "degree maxima"));
  GIFT_TRY(sc.get(&pick, 2, "giant component"));
  GIFT_HIP(hipMemsetAsync(count, 0, N * 4, st));
  k_cc_count<<<kRedBlocks, kBlock, 0, st>>>(label, N, count);
  GIFT_TRY(check_launch("k_cc_count"));
  k_cc_best<<<kRedBlocks, kBlock, 0, st>>>(count, N, bpart);
  GIFT_TRY(check_launch("k_cc_best"));
  k_cc_key<<<1, kBlock, 0, st>>>(bpart, kRedBlocks, pick);
  GIFT_TRY(check_launch("k_cc_key"));
  k_cc_dmax<<<kRedBlocks, kBlock, 0, st>>>(label, g->deg, N, pick, dpart);
  GIFT_TRY(check_launch("k_cc_dmax"));
  k_cc_bound<<<1, kBlock, 0, st>>>(dpart, kRedBlocks, pick);
  GIFT_TRY(check_launch("k_cc_bound"));
  int64_t hp[2];
  GIFT_TRY(read_back(st, nullptr, pick, nullptr, 2, hp));
  const int64_t cells = hp[0] >> 32;
  const int32_t giant = static_cast<int32_t>(0x7fffffff - (hp[0] & 0xffffffff));
  const double b = as_double(hp[1]);
  result->component_label = giant;
  result->component_cells = cells;
  result->sweeps = sweeps;
  if (labels) GIFT_HIP(hipMemcpyAsync(labels, label, R * 4, hipMemcpyDeviceToDevice, st));
  if (cells < K + 2)
    return set_error(GIFT_EINVAL, "the largest connected component has %lld cells (< %d)",
                     (long long)cells, K + 2);

  // 3-4. filtered subspace iteration
  double *buf[3] = {}, *w = nullptr, *ext = nullptr, *part = nullptr, *small = nullptr;
  for (int i = 0; i < 3; ++i) GIFT_TRY(sc.get(&buf[i], N * K, "eigen block"));
  GIFT_TRY(sc.get(&w, N * K, "L times the block"));
  GIFT_TRY(sc.get(&ext, (V > 0 ? V : 1) * K, "star means"));
  GIFT_TRY(sc.get(&part, kRedBlocks * K * K, "block partial sums"));
  GIFT_TRY(sc.get(&small, kSmall, "projected matrices"));
  double *vpart = nullptr;
  int64_t *ipart = nullptr;
  GIFT_TRY(sc.get(&vpart, kRedBlocks * 2, "largest entries"));
  GIFT_TRY(sc.get(&ipart, kRedBlocks * 2, "largest entry rows"));
  EigenRun run{g, st, N, V, label, giant, static_cast<double>(cells), ext, part, small};

  double *x = buf[0];
  k_eig_rand<<<grid_for(N), kBlock, 0, st>>>(x, label, giant, N, seed);
  GIFT_TRY(check_launch("k_eig_rand"));
  GIFT_TRY(run.deflate(x));
  GIFT_TRY(run.orth(x));
  double theta[K], res[K];
  GIFT_TRY(run.rayleigh_ritz(x, w, theta, res));
  int32_t it = 0;
  auto converged = [&]() { return res[0] <= tol * b && res[1] <= tol * b; };
  while (!converged() && it < max_iter) {
    // damp [a, b]: a = the block's largest Ritz value, kept inside (theta_2, b)
    double a = theta[K - 1];
    if (!(a < 0.99 * b)) a = 0.99 * b;
    if (!(a > theta[1])) a = theta[1] + 0.01 * (b - theta[1]);
    const double c = 0.5 * (a + b), e = 0.5 * (b - a);
    // the two buffers other than x hold the recurrence's next terms
    double *others[2];
    for (int i = 0, k = 0; i < 3; ++i)
      if (buf[i] != x) others[k++] = buf[i];
    double *prev = x, *cur = others[0], *spare = others[1];
    GIFT_TRY(run.apply(x, nullptr, 1.0 / e, -c / e, 0.0, cur));
    for (int j = 2; j <= kFilterDegree; ++j) {
      GIFT_TRY(run.apply(cur, prev, 2.0 / e, -2.0 * c / e, -1.0, spare));
      double *t = prev;
      prev = cur;
      cur = spare;
      spare = t;
    }
    x = cur;
    GIFT_TRY(run.deflate(x));
    GIFT_TRY(run.orth(x));
    GIFT_TRY(run.rayleigh_ritz(x, w, theta, res));
    ++it;
  }

  k_eig_argmax<<<kRedBlocks, kBlock, 0, st>>>(x, N, vpart, ipart);
  GIFT_TRY(check_launch("k_eig_argmax"));
  k_eig_sign<<<1, kWave, 0, st>>>(x, vpart, ipart, kRedBlocks, small);
  GIFT_TRY(check_launch("k_eig_sign"));
  k_eig_out<<<grid_for(N), kBlock, 0, st>>>(x, small, N, y_out, ld_out);
  GIFT_TRY(check_launch("k_eig_out"));
  GIFT_HIP(hipStreamSynchronize(st));
  result->lambda[0] = theta[0];
  result->lambda[1] = theta[1];
  result->residual[0] = res[0];
  result->residual[1] = res[1];
  result->spectral_bound = b;
  result->iterations = it;
  result->converged = converged() ? 1 : 0;
  return GIFT_OK;
}
