// Device-side building blocks: block scans, LDS bitonic sort, block-level
// merge sort through global memory.  All functions assume a 1-D block of
// kBlock threads that all reach every call (block-uniform control flow).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gift {

constexpr int kBlock = 256;
constexpr int kWave = 64;

// Exclusive scan of one value per thread across the block.  *total receives
// the block sum.  Uses `tmp` (kBlock/kWave entries of LDS).
template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T *total, T *tmp) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  T x = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    T y = __shfl_up(x, off, kWave);
    if (lane >= off) x += y;
  }
  if (lane == kWave - 1) tmp[wid] = x;
  __syncthreads();
  T before = 0, all = 0;
#pragma unroll
  for (int i = 0; i < kBlock / kWave; ++i) {
    T t = tmp[i];
    if (i < wid) before += t;
    all += t;
  }
  __syncthreads();
  *total = all;
  return before + x - v;
}

template <typename T>
__device__ __forceinline__ T block_sum(T v, T *tmp) {
  T total;
  (void)block_excl_scan<T>(v, &total, tmp);
  return total;
}

// Fills seg[i] = k for every entry i of segment k (segments given by
// local offsets loff[0..ns]); one thread per segment.
__device__ __forceinline__ void fill_segment_ids(const int32_t *loff, int ns, uint16_t *seg) {
  for (int k = threadIdx.x; k < ns; k += kBlock)
    for (int i = loff[k]; i < loff[k + 1]; ++i) seg[i] = static_cast<uint16_t>(k);
}

// Sum of part[b * stride] over b < nb by one block, in a fixed order:
// thread t adds the contiguous run [t * per, (t + 1) * per) in order, then a
// fixed tree adds the threads' sums.  The same order on every run, and every
// thread's loads are independent of each other (no serial chain over nb).
// `red` is kBlock doubles of LDS; every thread gets the result.
__device__ __forceinline__ double block_sum_strided(const double *part, int64_t nb,
                                                    int64_t stride, double *red) {
  const int64_t per = (nb + kBlock - 1) / kBlock;
  const int64_t b0 = static_cast<int64_t>(threadIdx.x) * per;
  const int64_t b1 = b0 + per < nb ? b0 + per : nb;
  double s = 0.0;
#pragma unroll 4
  for (int64_t b = b0; b < b1; ++b) s += part[b * stride];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Per-block accumulation of (key, amount) pairs before they reach global
// memory: an LDS table of S slots (S a power of two), open addressing with
// linear probing over at most kProbes slots; a pair that finds no slot goes
// straight to global memory.  Many additions to one key inside a block thus
// cost one global atomic (flush), not one each: device-scope atomics on one
// address serialise in the memory system, LDS ones stay inside the CU.
// Integer amounts only, so the totals do not depend on the order.  Usage:
// clear(); __syncthreads(); add(...)...; __syncthreads(); flush().
template <typename V, int S>
struct LdsHash {
  static_assert((S & (S - 1)) == 0, "slot count must be a power of two");
  static constexpr int kProbes = 8;
  int32_t key[S];
  V val[S];
  __device__ __forceinline__ void clear() {
    for (int k = threadIdx.x; k < S; k += blockDim.x) {
      key[k] = -1;
      val[k] = 0;
    }
  }
  __device__ __forceinline__ void add(int32_t k, V v, V *global) {
    uint32_t h = (static_cast<uint32_t>(k) * 2654435761u) >> 7 & (S - 1);
    for (int p = 0; p < kProbes; ++p) {
      const int32_t prev = atomicCAS(&key[h], -1, k);
      if (prev == -1 || prev == k) {
        atomicAdd(&val[h], v);
        return;
      }
      h = (h + 1) & (S - 1);
    }
    atomicAdd(global + k, v);
  }
  __device__ __forceinline__ void flush(V *global) {
    for (int k = threadIdx.x; k < S; k += blockDim.x)
      if (key[k] >= 0 && val[k] != 0) atomicAdd(global + key[k], val[k]);
  }
};

// Ascending bitonic sort of s[0..n) in LDS, n a power of two.
template <typename K>
__device__ void lds_bitonic_sort(K *s, int n) {
  for (int k = 2; k <= n; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n; i += kBlock) {
        int ixj = i ^ j;
        if (ixj > i) {
          K a = s[i], b = s[ixj];
          bool up = (i & k) == 0;
          if ((a > b) == up) {
            s[i] = b;
            s[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
  }
}

__host__ __device__ constexpr int next_pow2_i(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Sorts a[0..n) ascending with one block, using b[0..n) as scratch and `lds`
// (kChunk keys of LDS) for the first pass.  Returns true when the sorted
// keys end in b, false when they end in a.
template <typename K, int kChunk>
__device__ bool block_merge_sort_global(K *a, K *b, int64_t n, K *lds, K pad) {
  // First pass: sort chunks of kChunk keys in LDS, in place in a.
  for (int64_t c0 = 0; c0 < n; c0 += kChunk) {
    int len = static_cast<int>((n - c0) < kChunk ? (n - c0) : kChunk);
    int np = next_pow2_i(len);
    for (int i = threadIdx.x; i < np; i += kBlock) lds[i] = (i < len) ? a[c0 + i] : pad;
    __syncthreads();
    lds_bitonic_sort<K>(lds, np);
    for (int i = threadIdx.x; i < len; i += kBlock) a[c0 + i] = lds[i];
    __syncthreads();
  }
  // Merge passes: runs of width w -> 2w, ping-ponging between a and b.
  K *src = a, *dst = b;
  bool in_b = false;
  constexpr int kItems = 8;
  for (int64_t w = kChunk; w < n; w <<= 1) {
    for (int64_t lo = 0; lo < n; lo += 2 * w) {
      int64_t mid = lo + w < n ? lo + w : n;
      int64_t hi = lo + 2 * w < n ? lo + 2 * w : n;
      const K *A = src + lo, *B = src + mid;
      int64_t la = mid - lo, lb = hi - mid, tot = hi - lo;
      for (int64_t o0 = 0; o0 < tot; o0 += static_cast<int64_t>(kBlock) * kItems) {
        int64_t d = o0 + static_cast<int64_t>(threadIdx.x) * kItems;
        if (d < tot) {
          int64_t l = d - lb > 0 ? d - lb : 0, h = d < la ? d : la;
          while (l < h) {
            int64_t m = (l + h) >> 1;
            if (A[m] <= B[d - m - 1]) l = m + 1; else h = m;
          }
          int64_t i = l, j = d - l;
          for (int k = 0; k < kItems && d + k < tot; ++k) {
            bool takeA = j >= lb || (i < la && A[i] <= B[j]);
            dst[lo + d + k] = takeA ? A[i++] : B[j++];
          }
        }
      }
    }
    __syncthreads();
    K *t = src; src = dst; dst = t;
    in_b = !in_b;
  }
  return in_b;
}

}  // namespace gift
