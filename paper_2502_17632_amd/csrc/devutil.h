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
