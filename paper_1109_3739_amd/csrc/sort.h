// Ascending sort of 64-bit keys on the device (bitonic network; stages
// whose partner distance fits a 4096-key tile run in LDS).  Used for small
// auxiliary orderings (index vectors), not on the SpGEMM hot path.
#pragma once

#include "common.h"

namespace spx {

constexpr int kSortTile = 4096;
constexpr int kSortThreads = 512;

// All stages k <= kSortTile of the network, per tile.
static __global__ void __launch_bounds__(kSortThreads) k_bitonic_tile_full(uint64_t* keys) {
  __shared__ uint64_t s[kSortTile];
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int i = threadIdx.x; i < kSortTile; i += kSortThreads) s[i] = keys[base + i];
  __syncthreads();
  for (int k = 2; k <= kSortTile; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < kSortTile / 2; i += kSortThreads) {
        const int lo = 2 * i - (i & (j - 1));
        const int hi = lo + j;
        const bool asc = ((base + lo) & k) == 0;
        const uint64_t x = s[lo], y = s[hi];
        if ((x > y) == asc) {
          s[lo] = y;
          s[hi] = x;
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < kSortTile; i += kSortThreads) keys[base + i] = s[i];
}

// One stage (k, j) with j >= kSortTile, over global memory.
static __global__ void k_bitonic_global(uint64_t* keys, int64_t n, int64_t k, int64_t j) {
  const int64_t half = n >> 1;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < half; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t lo = 2 * i - (i & (j - 1));
    const int64_t hi = lo + j;
    const bool asc = (lo & k) == 0;
    const uint64_t x = keys[lo], y = keys[hi];
    if ((x > y) == asc) {
      keys[lo] = y;
      keys[hi] = x;
    }
  }
}

// Remaining stages j < kSortTile of merge step k > kSortTile, per tile.
static __global__ void __launch_bounds__(kSortThreads) k_bitonic_tile_merge(uint64_t* keys, int64_t k) {
  __shared__ uint64_t s[kSortTile];
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int i = threadIdx.x; i < kSortTile; i += kSortThreads) s[i] = keys[base + i];
  __syncthreads();
  const bool asc = (base & k) == 0;  // constant over the tile since k > tile
  for (int j = kSortTile >> 1; j > 0; j >>= 1) {
    for (int i = threadIdx.x; i < kSortTile / 2; i += kSortThreads) {
      const int lo = 2 * i - (i & (j - 1));
      const int hi = lo + j;
      const uint64_t x = s[lo], y = s[hi];
      if ((x > y) == asc) {
        s[lo] = y;
        s[hi] = x;
      }
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < kSortTile; i += kSortThreads) keys[base + i] = s[i];
}

static __global__ void k_pad_u64(uint64_t* keys, int64_t from, int64_t to) {
  for (int64_t i = from + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < to; i += (int64_t)gridDim.x * blockDim.x)
    keys[i] = ~0ull;
}

// Sorts keys[0, n) ascending in place; the buffer must hold
// sort_capacity(n) elements (entries past n are overwritten).
inline int64_t sort_capacity(int64_t n) {
  int64_t p = kSortTile;
  while (p < n) p <<= 1;
  return p;
}

inline int sort_u64(uint64_t* keys, int64_t n, hipStream_t st) {
  if (n <= 1) return SPX_OK;
  const int64_t N = sort_capacity(n);
  k_pad_u64<<<grid_for(N - n, 256, 4096), 256, 0, st>>>(keys, n, N);
  SPX_HIP(hipGetLastError());
  const unsigned tiles = (unsigned)(N / kSortTile);
  k_bitonic_tile_full<<<tiles, kSortThreads, 0, st>>>(keys);
  SPX_HIP(hipGetLastError());
  for (int64_t k = 2 * kSortTile; k <= N; k <<= 1) {
    for (int64_t j = k >> 1; j >= kSortTile; j >>= 1) {
      k_bitonic_global<<<grid_for(N / 2, 256, 65536), 256, 0, st>>>(keys, N, k, j);
      SPX_HIP(hipGetLastError());
    }
    k_bitonic_tile_merge<<<tiles, kSortThreads, 0, st>>>(keys, k);
    SPX_HIP(hipGetLastError());
  }
  return SPX_OK;
}

}  // namespace spx
