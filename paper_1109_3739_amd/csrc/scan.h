// Device-wide exclusive prefix sum over int64 values produced by a functor.
//   out[i] = sum_{t < i} f(t) for i = 0..n  (n+1 entries; out[n] = total)
// Block sums, then a block scan with carry-in.  Up to kFusedCarry blocks,
// each block adds up the sums of the blocks before it itself (two
// launches); above that the sums are scanned first, recursively (three).
// Used for column pointers and work-list offsets.
#pragma once

#include "common.h"

namespace spx {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int64_t kScanTile = kScanThreads * kScanItems;

template <class F>
__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(F f, int64_t n, int64_t* sums) {
  __shared__ int64_t red[kScanThreads / kWave + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + (int64_t)k * kScanThreads + threadIdx.x;
    if (i < n) s += f(i);
  }
  s = wave_sum(s);
  if (lane_id() == 0) red[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int w = 0; w < kScanThreads / kWave; ++w) t += red[w];
    sums[blockIdx.x] = t;
  }
}

constexpr int64_t kFusedCarry = 1024;

// The carry-in of block b read straight from the block sums: the workgroup
// adds up sums[0, b).
__device__ __forceinline__ int64_t carry_from_sums(const int64_t* sums, int64_t b, int64_t* red) {
  int64_t s = 0;
  for (int64_t i = threadIdx.x; i < b; i += blockDim.x) s += sums[i];
  int64_t total;
  (void)block_excl_scan(s, red, &total);
  return total;
}

// carry: the scanned block sums; else sums: the block sums themselves; else
// a single block.
template <class F>
__global__ void __launch_bounds__(kScanThreads) k_scan_apply(F f, int64_t n, const int64_t* carry, const int64_t* sums,
                                                             int64_t* out) {
  __shared__ int64_t red[kScanThreads / kWave + 1];
  const int64_t cin = carry ? carry[blockIdx.x] : sums ? carry_from_sums(sums, blockIdx.x, red) : 0;
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int64_t v[kScanItems];
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + k;
    v[k] = i < n ? f(i) : 0;
    s += v[k];
  }
  int64_t total;
  int64_t run = block_excl_scan(s, red, &total) + cin;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + k;
    if (i < n) out[i] = run;
    run += v[k];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == blockDim.x - 1) out[n] = run;
}

struct LoadI64 {
  const int64_t* p;
  __device__ int64_t operator()(int64_t i) const { return p[i]; }
};

// Enqueues the scan on `stream`; temporary block sums come from `scr` (any
// type with Scratch's get_n: the context's allocator, or a fixed buffer).
template <class F, class S>
int exclusive_scan(F f, int64_t n, int64_t* out, S& scr, hipStream_t stream) {
  if (n <= 0) return fill_i64(out, 1, 0, stream);
  const int64_t nblocks = ceil_div(n, kScanTile);
  if (nblocks == 1) {
    k_scan_apply<F><<<1, kScanThreads, 0, stream>>>(f, n, nullptr, nullptr, out);
    SPX_HIP(hipGetLastError());
    return SPX_OK;
  }
  int64_t* sums = nullptr;
  int64_t* carry = nullptr;
  SPX_TRY(scr.get_n(nblocks, &sums));
  if (nblocks > kFusedCarry) SPX_TRY(scr.get_n(nblocks + 1, &carry));
  k_scan_reduce<F><<<(unsigned)nblocks, kScanThreads, 0, stream>>>(f, n, sums);
  SPX_HIP(hipGetLastError());
  if (carry) SPX_TRY(exclusive_scan(LoadI64{sums}, nblocks, carry, scr, stream));
  k_scan_apply<F><<<(unsigned)nblocks, kScanThreads, 0, stream>>>(f, n, carry, carry ? nullptr : sums, out);
  SPX_HIP(hipGetLastError());
  return SPX_OK;
}

}  // namespace spx
